"""Python binding of libhh.so (include/hh.h): argument marshalling only.

Every entry point takes torch tensors on the current GPU, enqueues the HIP
kernels on torch's current stream and returns without synchronising.  There
is no fallback: if libhh.so is missing or the device is not a gfx950 the
calls raise.

Tensor conventions (uint64 quantities may be given as int64 or uint64):
    keys      (n_keys, 4)   key k, word i = lane i
    data      (data_bytes,) uint8, the packed messages
    offsets   (n,)          byte offset of message j in data
    lengths   (n,)          byte length of message j
    key_idx   (n,) int32/uint32, or None for key 0 everywhere
    result    (n, width) int64 -- the bits of the uint64 hash words
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, List

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhh.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED_DEVICE, ERR_OUT_OF_MEMORY, ERR_LAUNCH, ERR_BUSY = range(6)
PATHS = {"auto": 0, "lane1": 1, "lane4": 2, "bucketed": 3}
STATE_WORDS = 16


class HHError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s (status %d)" % (what, status))
        self.status = status


class _Tuning(ctypes.Structure):
    _fields_ = [("lane4_min_bytes", ctypes.c_uint32), ("waves_per_cu", ctypes.c_uint32),
                ("use_graph", ctypes.c_uint32), ("long_ring", ctypes.c_uint32),
                ("isolate_long", ctypes.c_uint32)]


_lib = None
_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64


def lib() -> ctypes.CDLL:
    """Load libhh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhh.so is not built (%s); run `python -m "
                               "paper_1612_06257_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        L.hh_status_string.argtypes = [ctypes.c_int]
        L.hh_status_string.restype = ctypes.c_char_p
        L.hh_version.restype = ctypes.c_int
        L.hh_get_constants.argtypes = [_vp, _vp]
        L.hh_get_constants.restype = None
        hash_args = [_vp, _u32, _vp, _vp, _u64, _vp, _vp, _u64, _vp, _vp]
        for name in ("hh_hash64", "hh_hash128", "hh_hash256"):
            getattr(L, name).argtypes = hash_args
            getattr(L, name).restype = ctypes.c_int
        L.hh_hash_path.argtypes = [ctypes.c_int, _u32] + hash_args
        L.hh_hash_path.restype = ctypes.c_int
        L.hh_hash_noalloc.argtypes = [_u32] + hash_args
        L.hh_hash_noalloc.restype = ctypes.c_int
        L.hh_hash64_uniform.argtypes = [_vp, _u32, _vp, _vp, _u64, _vp, _u64, _u64, _vp, _vp]
        L.hh_hash64_uniform.restype = ctypes.c_int
        L.hh_prf.argtypes = [_u32, _vp, _u32, _u64, _u64, _vp, _vp]
        L.hh_prf.restype = ctypes.c_int
        L.hh_avalanche.argtypes = [ctypes.c_int, _u32, _u32, _u64, _vp, _u64, _u32, _u32, _vp,
                                   _vp]
        L.hh_avalanche.restype = ctypes.c_int
        L.hh_copy_segments.argtypes = [_vp, _u64, _vp, _u64, _vp, _vp, _vp, _u64, _u64, _vp]
        L.hh_pinned_device_pointer.argtypes = [_vp, ctypes.POINTER(_vp)]
        L.hh_pinned_device_pointer.restype = ctypes.c_int
        L.hh_copy_segments.restype = ctypes.c_int
        L.hh_state_init.argtypes = [_vp, _u32, _vp, _vp, _u64, _vp, _u64, _vp]
        L.hh_state_init.restype = ctypes.c_int
        L.hh_state_update.argtypes = [_vp, _u64, _vp, _vp, _u64, _vp, _vp, _u64, _vp]
        L.hh_state_update.restype = ctypes.c_int
        L.hh_state_final.argtypes = [_vp, _u64, _vp, _vp, _u64, _vp, _vp, _vp, _vp, _u64, _vp, _u64, _vp]
        L.hh_state_final.restype = ctypes.c_int
        L.hh_state_step.argtypes = L.hh_state_final.argtypes
        L.hh_state_step.restype = ctypes.c_int
        L.hh_get_tuning.argtypes = [ctypes.POINTER(_Tuning)]
        L.hh_get_tuning.restype = None
        L.hh_set_tuning.argtypes = [ctypes.POINTER(_Tuning)]
        L.hh_set_tuning.restype = ctypes.c_int
        L.hh_release.restype = ctypes.c_int
        L.hh_timing_enable.argtypes = [ctypes.c_int]
        L.hh_timing_enable.restype = ctypes.c_int
        L.hh_timing_collect.argtypes = [ctypes.POINTER(ctypes.c_uint32),
                                        ctypes.POINTER(ctypes.c_double)]
        L.hh_timing_collect.restype = ctypes.c_int
        L.hh_feed_open.argtypes = [_vp, _u32, _vp, _u64, _u32, _u32, _u32, _vp, ctypes.POINTER(_vp)]
        L.hh_feed_open.restype = ctypes.c_int
        L.hh_feed_submit.argtypes = [_vp, _u32, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_u64)]
        L.hh_feed_submit.restype = ctypes.c_int
        L.hh_feed_poll.argtypes = [_vp]
        L.hh_feed_poll.restype = ctypes.c_int
        L.hh_feed_results.argtypes = [_vp]
        L.hh_feed_results.restype = _vp
        L.hh_feed_close.argtypes = [_vp]
        L.hh_feed_close.restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    """Text for a status code returned by the library."""
    return lib().hh_status_string(status).decode()


def _check(status: int) -> None:
    if status != OK:
        raise HHError(status, status_string(status))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else _vp(t.data_ptr())


def _stream() -> _vp:
    return _vp(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str, dtypes, ndim: int) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU" % name)
    if t.dtype not in dtypes:
        raise TypeError("%s has dtype %s, expected one of %s" % (name, t.dtype, dtypes))
    if t.dim() != ndim or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %d-d tensor" % (name, ndim))
    return t


_W64 = (torch.int64, torch.uint64)
_W32 = (torch.int32, torch.uint32)


def _msg_args(keys, data, offsets, lengths, key_idx):
    _dev(keys, "keys", _W64, 2)
    if keys.shape[1] != 4 or keys.shape[0] < 1:
        raise ValueError("keys must have shape (n_keys >= 1, 4)")
    _dev(data, "data", (torch.uint8,), 1)
    _dev(offsets, "offsets", _W64, 1)
    if lengths is not None:
        _dev(lengths, "lengths", _W64, 1)
        if lengths.numel() != offsets.numel():
            raise ValueError("offsets and lengths differ in size")
    if key_idx is not None:
        _dev(key_idx, "key_idx", _W32, 1)
        if key_idx.numel() != offsets.numel():
            raise ValueError("key_idx and offsets differ in size")


def _hash_call(keys, data, offsets, lengths, key_idx, width, path, out):
    """Checked arguments of hh_hash_path (all but the stream) and the output."""
    if width not in (1, 2, 4):
        raise ValueError("width must be 1, 2 or 4 words")
    if path not in PATHS:
        raise ValueError("path must be one of %s" % sorted(PATHS))
    _msg_args(keys, data, offsets, lengths, key_idx)
    n = offsets.numel()
    if out is None:
        out = torch.empty((n, width), dtype=torch.int64, device=offsets.device)
    else:
        _dev(out, "out", _W64, 2)
        if tuple(out.shape) != (n, width):
            raise ValueError("out must have shape (n, width)")
    args = (PATHS[path], width, _ptr(keys), keys.shape[0], _ptr(key_idx), _ptr(data),
            data.numel(), _ptr(offsets), _ptr(lengths), n, _ptr(out))
    return args, out


def hash(keys: torch.Tensor, data: torch.Tensor, offsets: torch.Tensor, lengths: torch.Tensor,
         key_idx: Optional[torch.Tensor] = None, width: int = 1, path: str = "auto",
         out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """HighwayHash of every message; returns (n, width) int64 hash words."""
    args, out = _hash_call(keys, data, offsets, lengths, key_idx, width, path, out)
    _check(lib().hh_hash_path(*args, _stream()))
    return out


def prepare(keys: torch.Tensor, data: torch.Tensor, offsets: torch.Tensor,
            lengths: torch.Tensor, key_idx: Optional[torch.Tensor] = None, width: int = 1,
            path: str = "auto", out: Optional[torch.Tensor] = None, stream=None):
    """The hash call of hash(...), with its arguments checked and marshalled
    once: returns call(), which makes the same hh_hash_path call on `stream`
    (a torch.cuda.Stream, fixed now; None: the current stream at each call)
    and returns `out`.  For callers that repeat one call on resident tensors,
    so that each repetition costs one foreign call instead of the argument
    checks.  The tensors must stay alive and in place while call() is used."""
    args, out = _hash_call(keys, data, offsets, lengths, key_idx, width, path, out)
    fn = lib().hh_hash_path
    handle = None if stream is None else _vp(stream.cuda_stream)
    keep = (keys, data, offsets, lengths, key_idx)

    def call():
        status = fn(*args, handle if handle is not None else _stream())
        if status != OK:
            raise HHError(status, status_string(status))
        return out

    call.out = out
    call.tensors = keep
    return call


# most messages per hh_hash_noalloc call (HH_NOALLOC_MAX_MSGS in hh.h)
NOALLOC_MAX_MSGS = 1 << 20


def hash_noalloc(keys: torch.Tensor, data: torch.Tensor, offsets: torch.Tensor,
                 lengths: torch.Tensor, key_idx: Optional[torch.Tensor] = None, width: int = 1,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """hh_hash_noalloc: the bucketed path with the planner's lists in the
    library's fixed per-GPU array, for at most NOALLOC_MAX_MSGS messages.
    Pass `out` to keep the call free of allocations (torch's included)."""
    if width not in (1, 2, 4):
        raise ValueError("width must be 1, 2 or 4 words")
    _msg_args(keys, data, offsets, lengths, key_idx)
    n = offsets.numel()
    if out is None:
        out = torch.empty((n, width), dtype=torch.int64, device=offsets.device)
    else:
        _dev(out, "out", _W64, 2)
        if tuple(out.shape) != (n, width):
            raise ValueError("out must have shape (n, width)")
    _check(lib().hh_hash_noalloc(width, _ptr(keys), keys.shape[0], _ptr(key_idx), _ptr(data),
                                 data.numel(), _ptr(offsets), _ptr(lengths), n, _ptr(out),
                                 _stream()))
    return out


def hash64(keys, data, offsets, lengths, key_idx=None, out=None) -> torch.Tensor:
    """hash(..., width=1) on the AUTO path: one 64-bit word per message."""
    return hash(keys, data, offsets, lengths, key_idx, 1, "auto", out)


def hash128(keys, data, offsets, lengths, key_idx=None, out=None) -> torch.Tensor:
    """hash(..., width=2) on the AUTO path: two 64-bit words per message."""
    return hash(keys, data, offsets, lengths, key_idx, 2, "auto", out)


def hash256(keys, data, offsets, lengths, key_idx=None, out=None) -> torch.Tensor:
    """hash(..., width=4) on the AUTO path: four 64-bit words per message."""
    return hash(keys, data, offsets, lengths, key_idx, 4, "auto", out)


def hash64_uniform(keys, data, offsets, length: int, key_idx=None, out=None) -> torch.Tensor:
    """The plain kernel: all messages have the same length (one launch)."""
    _msg_args(keys, data, offsets, None, key_idx)
    n = offsets.numel()
    if out is None:
        out = torch.empty((n, 1), dtype=torch.int64, device=offsets.device)
    else:
        _dev(out, "out", _W64, 2)
        if out.shape[0] != n or out.shape[1] != 1:
            raise ValueError("out must have shape (n, 1)")
    _check(lib().hh_hash64_uniform(_ptr(keys), keys.shape[0], _ptr(key_idx), _ptr(data),
                                   data.numel(), _ptr(offsets), int(length), n, _ptr(out),
                                   _stream()))
    return out


def prf(keys: torch.Tensor, n: int, counter_base: int = 0, width: int = 1,
        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Counter-mode PRF: row j is the hash of the 8-byte little-endian counter
    counter_base + j under key (counter_base + j) mod n_keys."""
    _dev(keys, "keys", _W64, 2)
    if keys.shape[1] != 4 or keys.shape[0] < 1:
        raise ValueError("keys must have shape (n_keys >= 1, 4)")
    if width not in (1, 2, 4):
        raise ValueError("width must be 1, 2 or 4 words")
    if out is None:
        out = torch.empty((n, width), dtype=torch.int64, device=keys.device)
    else:
        _dev(out, "out", _W64, 2)
        if tuple(out.shape) != (n, width):
            raise ValueError("out must have shape (n, width)")
    _check(lib().hh_prf(width, _ptr(keys), keys.shape[0], int(counter_base) % (1 << 64), n,
                        _ptr(out), _stream()))
    return out


def avalanche_counts(msg_bytes: int, n_samples: int, rounds: int = 4, seed: int = 0,
                     key=None, bits=None) -> torch.Tensor:
    """Flip counts of output bits (64 columns) per flipped input bit (rows),
    int64 tensor on the GPU.  key=None: SplitMix64 keys and messages from
    `seed`; else the messages enumerate little-endian sample indices under
    that key (4 words)."""
    bits = range(8 * msg_bytes) if bits is None else bits
    bits = list(bits)
    counts = torch.zeros((len(bits), 64), dtype=torch.int64, device="cuda")
    kbuf = None
    if key is not None:
        kbuf = (ctypes.c_uint64 * 4)(*[int(x) % (1 << 64) for x in key])
    mode = 0 if key is None else 1
    i = 0
    while i < len(bits):
        first = bits[i]
        cnt = 1
        while cnt < 32 and i + cnt < len(bits) and bits[i + cnt] == first + cnt:
            cnt += 1
        view = counts[i:i + cnt]
        _check(lib().hh_avalanche(mode, msg_bytes, rounds, int(seed) % (1 << 64),
                                  None if kbuf is None else ctypes.cast(kbuf, _vp), n_samples,
                                  first, cnt, _ptr(view), _stream()))
        i += cnt
    return counts


def state_init(keys, n: int, key_idx=None, states=None, state_idx=None) -> torch.Tensor:
    """Reset (Sec. 4.4) n states: state state_idx[k] (k if None) from key
    key_idx[k] (0 if None).  Returns the (rows, 16) state tensor."""
    _dev(keys, "keys", _W64, 2)
    if key_idx is not None:
        _dev(key_idx, "key_idx", _W32, 1)
        if key_idx.numel() != n:
            raise ValueError("key_idx must have n entries")
    if state_idx is not None:
        _dev(state_idx, "state_idx", _W32, 1)
        if state_idx.numel() != n:
            raise ValueError("state_idx must have n entries")
        if states is None:
            raise ValueError("states is required with state_idx")
    if states is None:
        states = torch.empty((n, STATE_WORDS), dtype=torch.int64, device=keys.device)
    else:
        _dev(states, "states", _W64, 2)
        if states.shape[1] != STATE_WORDS or (state_idx is None and states.shape[0] < n):
            raise ValueError("states must have shape (>= n, 16)")
    _check(lib().hh_state_init(_ptr(keys), keys.shape[0], _ptr(key_idx), _ptr(states),
                               states.shape[0], _ptr(state_idx), n, _stream()))
    return states


def copy_segments(dst: torch.Tensor, src: torch.Tensor, src_offs: torch.Tensor,
                  dst_offs: torch.Tensor, lens: torch.Tensor, max_len: int = 1 << 16) -> None:
    """dst[dst_offs[k]:+lens[k]] = src[src_offs[k]:+lens[k]] for every k, one
    launch.  max_len (the longest segment) only sizes the launch."""
    _dev(dst, "dst", (torch.uint8,), 1)
    _dev(src, "src", (torch.uint8,), 1)
    for t, nm in ((src_offs, "src_offs"), (dst_offs, "dst_offs"), (lens, "lens")):
        _dev(t, nm, _W64, 1)
    n = lens.numel()
    if src_offs.numel() != n or dst_offs.numel() != n:
        raise ValueError("segment arrays differ in size")
    _check(lib().hh_copy_segments(_ptr(dst), dst.numel(), _ptr(src), src.numel(), _ptr(src_offs),
                                  _ptr(dst_offs), _ptr(lens), n, max_len, _stream()))


def state_update(states, data, offsets, lengths, state_idx=None) -> None:
    """Fold whole packets (lengths multiples of 32) into states."""
    _dev(states, "states", _W64, 2)
    _dev(data, "data", (torch.uint8,), 1)
    _dev(offsets, "offsets", _W64, 1)
    _dev(lengths, "lengths", _W64, 1)
    n = offsets.numel()
    if lengths.numel() != n:
        raise ValueError("offsets and lengths differ in size")
    if state_idx is not None:
        _dev(state_idx, "state_idx", _W32, 1)
        if state_idx.numel() != n:
            raise ValueError("state_idx must have one entry per item")
    _check(lib().hh_state_update(_ptr(states), states.shape[0], _ptr(state_idx), _ptr(data),
                                 data.numel(), _ptr(offsets), _ptr(lengths), n, _stream()))


def state_final(states, data, offsets, lengths, width_words=None, out=None, out_offsets=None,
                state_idx=None) -> torch.Tensor:
    """Fold the last bytes, finalize (Sec. 4.3) and write the hashes.  Without
    out_offsets item k's words go to out[4k ..] (out has shape (n, 4))."""
    _dev(states, "states", _W64, 2)
    _dev(data, "data", (torch.uint8,), 1)
    _dev(offsets, "offsets", _W64, 1)
    _dev(lengths, "lengths", _W64, 1)
    n = offsets.numel()
    if lengths.numel() != n:
        raise ValueError("offsets and lengths differ in size")
    for t, nm, dt in ((width_words, "width_words", (torch.uint8,)), (state_idx, "state_idx", _W32),
                      (out_offsets, "out_offsets", _W64)):
        if t is not None:
            _dev(t, nm, dt, 1)
            if t.numel() != n:
                raise ValueError("%s must have one entry per item" % nm)
    if out_offsets is not None and out is None:
        raise ValueError("out is required with out_offsets")
    if out is None:
        out = torch.zeros((n, 4), dtype=torch.int64, device=offsets.device)
    else:
        if out.dtype not in _W64 or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous 64-bit device tensor")
        if out_offsets is None and out.numel() < 4 * n:
            raise ValueError("out must hold 4 words per item")
    _check(lib().hh_state_final(_ptr(states), states.shape[0], _ptr(state_idx), _ptr(data),
                                data.numel(), _ptr(offsets), _ptr(lengths), _ptr(width_words),
                                _ptr(out), out.numel(), _ptr(out_offsets), n, _stream()))
    return out


def state_step(states, data, offsets, lengths, width_words, out=None, out_offsets=None,
               state_idx=None) -> None:
    """Mixed items in one launch: width_words[k] == 0 folds whole packets into
    the state (as state_update), any other width finishes (as state_final)."""
    _dev(states, "states", _W64, 2)
    _dev(data, "data", (torch.uint8,), 1)
    _dev(offsets, "offsets", _W64, 1)
    _dev(lengths, "lengths", _W64, 1)
    n = offsets.numel()
    if lengths.numel() != n:
        raise ValueError("offsets and lengths differ in size")
    for t, nm, dt in ((width_words, "width_words", (torch.uint8,)), (state_idx, "state_idx", _W32),
                      (out_offsets, "out_offsets", _W64)):
        if t is not None:
            _dev(t, nm, dt, 1)
            if t.numel() != n:
                raise ValueError("%s must have one entry per item" % nm)
    if width_words is None:
        raise ValueError("width_words is required")
    if out is not None and (out.dtype not in _W64 or not out.is_cuda or not out.is_contiguous()):
        raise ValueError("out must be a contiguous 64-bit device tensor")
    _check(lib().hh_state_step(_ptr(states), states.shape[0], _ptr(state_idx), _ptr(data),
                               data.numel(), _ptr(offsets), _ptr(lengths), _ptr(width_words),
                               _ptr(out), 0 if out is None else out.numel(), _ptr(out_offsets), n,
                               _stream()))


def constants():
    """The library's Sec. 4.4 constants (host copy of what the kernels use)."""
    c0 = (ctypes.c_uint64 * 4)()
    c1 = (ctypes.c_uint64 * 4)()
    lib().hh_get_constants(ctypes.cast(c0, _vp), ctypes.cast(c1, _vp))
    return [int(x) for x in c0], [int(x) for x in c1]


def get_tuning() -> dict:
    """The library's tuning of the bucketed path, as a dict of hh_tuning fields."""
    t = _Tuning()
    lib().hh_get_tuning(ctypes.byref(t))
    return {f: int(getattr(t, f)) for f, _ in _Tuning._fields_}


def set_tuning(**kw) -> None:
    """Set the given hh_tuning fields (the others keep their values); invalid values raise."""
    cur = get_tuning()
    cur.update(kw)
    t = _Tuning(**cur)
    _check(lib().hh_set_tuning(ctypes.byref(t)))


def release() -> None:
    """Free the library's per-stream workspaces and cached graphs (no call may be in flight)."""
    _check(lib().hh_release())


class Feed:
    """hh_feed_*: a persistent kernel that hashes long messages as they are
    submitted (see hh.h).  `keys` (n_keys x 4, device) and `data` (uint8,
    device) stay fixed and alive while the feed is open.  rows is a
    (slots, 5) uint64 view of the feed's host result rows: four hash words,
    then the ticket of the message they belong to."""

    def __init__(self, keys: torch.Tensor, data: torch.Tensor, slots: int, waves: int = 256,
                 max_ms: int = 2000, stream=None):
        _dev(keys, "keys", _W64, 2)
        if keys.shape[1] != 4 or keys.shape[0] < 1:
            raise ValueError("keys must have shape (n_keys >= 1, 4)")
        _dev(data, "data", (torch.uint8,), 1)
        self.keys, self.data, self.slots = keys, data, int(slots)
        h = _vp()
        st = _vp(stream.cuda_stream) if stream is not None else _stream()
        _check(lib().hh_feed_open(_ptr(keys), keys.shape[0], _ptr(data), data.numel(),
                                  self.slots, int(waves), int(max_ms), st, ctypes.byref(h)))
        self._h = h
        base = lib().hh_feed_results(h)
        self.rows = np.ctypeslib.as_array(
            (ctypes.c_uint64 * (5 * self.slots)).from_address(base)).reshape(self.slots, 5)

    def submit(self, offsets, lengths, key_idx, widths, slots) -> int:
        """Queue messages (host arrays, taken in this order); returns the
        first message's ticket (message i: ticket + i), or 0 when the queue
        has no room for them yet (submit again later)."""
        o = np.ascontiguousarray(offsets, np.uint64)
        L = np.ascontiguousarray(lengths, np.uint64)
        k = np.ascontiguousarray(key_idx, np.uint32)
        w = np.ascontiguousarray(widths, np.uint8)
        s = np.ascontiguousarray(slots, np.uint32)
        n = o.size
        if not (L.size == k.size == w.size == s.size == n):
            raise ValueError("message arrays must have equal lengths")
        t = _u64()
        st = lib().hh_feed_submit(self._h, n, o.ctypes.data, L.ctypes.data, k.ctypes.data,
                                  w.ctypes.data, s.ctypes.data, ctypes.byref(t))
        if st == ERR_BUSY:
            return 0
        _check(st)
        return int(t.value)

    def poll(self) -> None:
        """Relaunch the kernel if it has ended while submitted groups wait."""
        _check(lib().hh_feed_poll(self._h))

    def close(self) -> None:
        if self._h is not None:
            h, self._h = self._h, None
            self.rows = None
            _check(lib().hh_feed_close(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pinned_device_pointer(t: torch.Tensor) -> int:
    """Device address of a pinned host tensor's storage (kernels may read and
    write it directly)."""
    if not isinstance(t, torch.Tensor) or t.is_cuda or not t.is_pinned():
        raise ValueError("expected a pinned host tensor")
    d = _vp()
    _check(lib().hh_pinned_device_pointer(_vp(t.data_ptr()), ctypes.byref(d)))
    return int(d.value)


def independent_streams(n: int, avoid=None, probe_bytes: int = 1 << 22,
                        max_tries: int = 16) -> List[torch.cuda.Stream]:
    """n streams whose work runs concurrently with each other and with the
    streams in `avoid` (default: the current stream).

    The runtime puts streams on a few hardware queues (GPU_MAX_HW_QUEUES,
    4 by default), which one decided at a stream's first launch by how many
    streams the process used before; kernels on one queue run in order, so a
    stream that shares a queue with a busy one waits behind its work.  Each
    candidate is tested: a one-message hash of probe_bytes (one quad, a few
    milliseconds) runs on an already chosen or avoided stream, then a tiny
    kernel on the candidate; the candidate is kept if that kernel completes
    while the hash still runs.  A candidate's first launch happens here, so
    its one-time set-up cost is paid here too.  Returns the best streams found
    if fewer than n independent ones exist."""
    import time
    dev = torch.device("cuda", torch.cuda.current_device())
    busy = list(avoid) if avoid is not None else [torch.cuda.current_stream()]
    buf = torch.zeros(probe_bytes, dtype=torch.uint8, device=dev)
    keys = torch.zeros((1, 4), dtype=torch.int64, device=dev)
    off = torch.zeros(1, dtype=torch.int64, device=dev)
    ln = torch.full((1,), probe_bytes, dtype=torch.int64, device=dev)
    out = torch.empty((1, 1), dtype=torch.int64, device=dev)
    tick = torch.zeros(1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize(dev)

    def overlaps(cand, other) -> bool:
        with torch.cuda.stream(other):
            hash(keys, buf, off, ln, None, 1, "lane4", out)
            done_other = torch.cuda.Event()
            done_other.record(other)
        with torch.cuda.stream(cand):
            tick.add_(1)
            done_cand = torch.cuda.Event()
            done_cand.record(cand)
        t0 = time.perf_counter()
        while not done_cand.query() and time.perf_counter() - t0 < 2e-3:
            time.sleep(5e-5)
        ok = done_cand.query() and not done_other.query()
        torch.cuda.synchronize(dev)
        return ok

    chosen: List[torch.cuda.Stream] = []
    spare: List[torch.cuda.Stream] = []
    for _ in range(max_tries):
        if len(chosen) == n:
            break
        cand = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(cand):   # first launch: binds the stream
            tick.add_(1)
        torch.cuda.synchronize(dev)
        if all(overlaps(cand, other) for other in busy + chosen):
            chosen.append(cand)
        else:
            spare.append(cand)
    while len(chosen) < n and spare:
        chosen.append(spare.pop(0))
    return chosen


_MANY_STREAMS: dict = {}


def hash_many(batches, width: int = 1, n_streams: int = 3, path: str = "auto") -> list:
    """Hash several independent batches, each (keys, data, offsets, lengths,
    key_idx), round-robin on up to n_streams streams that run concurrently
    (chosen once per device by independent_streams).  One batch cannot finish
    before its longest message's serial chain of Updates, which leaves most
    of the GPU idle for the end of a batch; the next batches fill it.  Work
    queued on the current stream before the call is visible to every batch,
    and the current stream waits for all of them; returns the (n_i, width)
    outputs in order, usable on the current stream."""
    if width not in (1, 2, 4):
        raise ValueError("width must be 1, 2 or 4 words")
    batches = list(batches)
    if not batches:
        return []
    dev = torch.cuda.current_device()
    streams = _MANY_STREAMS.get((dev, n_streams))
    if streams is None:
        streams = independent_streams(n_streams, avoid=[])
        _MANY_STREAMS[(dev, n_streams)] = streams
    cur = torch.cuda.current_stream()
    ready = torch.cuda.Event()
    ready.record(cur)
    used = streams[:len(batches)]
    for s in used:
        s.wait_event(ready)
    outs = []
    for i, (keys, data, offsets, lengths, key_idx) in enumerate(batches):
        s = used[i % len(used)]
        with torch.cuda.stream(s):
            out = torch.empty((offsets.numel(), width), dtype=torch.int64, device=offsets.device)
            hash(keys, data, offsets, lengths, key_idx, width, path, out)
        # the caching allocator must not hand these blocks to other work
        # before the streams that use them are done with them
        for t in (keys, data, offsets, lengths, key_idx):
            if t is not None:
                t.record_stream(s)
        out.record_stream(cur)
        outs.append(out)
    for s in used:
        done = torch.cuda.Event()
        done.record(s)
        cur.wait_event(done)
    return outs


def state_step_raw(states: torch.Tensor, data: torch.Tensor, offsets: int, lengths: int,
                   width_words: int, out: int, out_words: int, out_offsets: int, state_idx: int,
                   n: int, stream: int) -> None:
    """state_step with the item arrays and the output given as device
    addresses (e.g. from pinned_device_pointer) and an explicit stream
    handle; states and data are device tensors as for state_step."""
    _dev(states, "states", _W64, 2)
    _dev(data, "data", (torch.uint8,), 1)
    if not (offsets and lengths and width_words and out and out_offsets and state_idx):
        raise ValueError("every item array must be given")
    _check(lib().hh_state_step(_ptr(states), states.shape[0], _vp(state_idx), _ptr(data),
                               data.numel(), _vp(offsets), _vp(lengths), _vp(width_words),
                               _vp(out), out_words, _vp(out_offsets), n, _vp(stream)))


def hash_raw(keys: torch.Tensor, data: torch.Tensor, key_idx: int, offsets: int, lengths: int,
             n: int, out: int, width: int = 4, path: str = "lane4", stream: int = 0) -> None:
    """hash(...) with the message arrays and the output given as device
    addresses (e.g. from pinned_device_pointer; key_idx 0: key 0 for every
    message), n messages, out n * width words, and an explicit stream
    handle; keys and data are device tensors as for hash."""
    _dev(keys, "keys", _W64, 2)
    _dev(data, "data", (torch.uint8,), 1)
    if width not in (1, 2, 4):
        raise ValueError("width must be 1, 2 or 4 words")
    if path not in PATHS:
        raise ValueError("path must be one of %s" % sorted(PATHS))
    if not (offsets and lengths and out):
        raise ValueError("offsets, lengths and out must be given")
    _check(lib().hh_hash_path(PATHS[path], width, _ptr(keys), keys.shape[0], _vp(key_idx or None),
                              _ptr(data), data.numel(), _vp(offsets), _vp(lengths), n, _vp(out),
                              _vp(stream)))


def state_init_raw(keys: torch.Tensor, n: int, key_idx: int, states: torch.Tensor,
                   state_idx: int, stream: int) -> None:
    """state_init with key_idx and state_idx given as device addresses (e.g.
    from pinned_device_pointer) and an explicit stream handle; keys and
    states are device tensors as for state_init."""
    _dev(keys, "keys", _W64, 2)
    _dev(states, "states", _W64, 2)
    if not (key_idx and state_idx):
        raise ValueError("key_idx and state_idx must be given")
    if states.shape[1] != STATE_WORDS:
        raise ValueError("states must have shape (rows, 16)")
    _check(lib().hh_state_init(_ptr(keys), keys.shape[0], _vp(key_idx), _ptr(states),
                               states.shape[0], _vp(state_idx), n, _vp(stream)))


def timing_enable(on: bool = True) -> None:
    """Record HIP events around each bucketed call's long-message kernel."""
    _check(lib().hh_timing_enable(int(bool(on))))


def timing_collect():
    """(launches, total_ms) of the long-message kernels recorded so far."""
    n = ctypes.c_uint32()
    ms = ctypes.c_double()
    _check(lib().hh_timing_collect(ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def to_u64(t: torch.Tensor):
    """Hash words as a numpy uint64 array (copies to the host)."""
    return t.detach().cpu().numpy().view("uint64")
