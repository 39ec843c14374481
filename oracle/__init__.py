"""CPU oracle for HighwayHash (arXiv:1612.06257, Sec. 4) -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package.  The product library never does, and this package
imports nothing from the product.  The arithmetic lives in ``hh_oracle.c``
(plain scalar C); this module only compiles it with gcc and marshals arguments
through ctypes.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hh_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libhh_oracle.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)

# Layout of hh_ref_state in hh_oracle.c: v0[4], v1[4], mul0[4], mul1[4].
STATE_WORDS = 16


def build(force: bool = True) -> str:
    """Compile hh_oracle.c into libhh_oracle.so with gcc (plain -O2 C99)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
             "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load(path: str) -> ctypes.CDLL:
    L = ctypes.CDLL(path)
    _declare(L)
    return L


@contextlib.contextmanager
def using(path: str):
    """Temporarily route every call to another build of the oracle (the tests
    use this to check that deliberately broken copies fail the pins)."""
    global _lib
    saved = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


def compile_source(src_path: str, out_path: str) -> str:
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-shared", "-fPIC", "-pthread", "-w",
                           "-o", out_path, src_path])
    return out_path


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _load(_LIB_PATH)
    return _lib


def _declare(L: ctypes.CDLL) -> None:
    L.hh_ref_constants.argtypes = [_u64p, _u64p]
    L.hh_ref_reset.argtypes = [_u64p, _u64p]
    L.hh_ref_zipper_merge.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _u64p, _u64p]
    L.hh_ref_update.argtypes = [_u64p, _u64p]
    L.hh_ref_permute.argtypes = [_u64p, _u64p]
    L.hh_ref_remainder.argtypes = [_u64p, _u8p, ctypes.c_size_t]
    L.hh_ref_finalize.argtypes = [_u64p, ctypes.c_int, _u64p]
    L.hh_ref_hash_rounds.argtypes = [_u64p, _u8p, ctypes.c_size_t, ctypes.c_int, _u64p]
    L.hh_ref_hash64.argtypes = [_u64p, _u8p, ctypes.c_size_t]
    L.hh_ref_hash64.restype = ctypes.c_uint64
    L.hh_ref_hash128.argtypes = [_u64p, _u8p, ctypes.c_size_t, _u64p]
    L.hh_ref_hash256.argtypes = [_u64p, _u8p, ctypes.c_size_t, _u64p]
    L.hh_ref_cat_size.restype = ctypes.c_size_t
    L.hh_ref_cat_init.argtypes = [ctypes.c_void_p, _u64p]
    L.hh_ref_cat_append.argtypes = [ctypes.c_void_p, _u8p, ctypes.c_size_t]
    L.hh_ref_cat_finish.argtypes = [ctypes.c_void_p, ctypes.c_int, _u64p]
    L.hh_ref_batch.argtypes = [_u64p, _u32p, _u8p, _u64p, _u64p, ctypes.c_uint64,
                               ctypes.c_int, _u64p, ctypes.c_int]
    L.hh_ref_batch.restype = ctypes.c_int


def _p(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _key(key) -> np.ndarray:
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64).reshape(4))
    return k


def _bytes(msg) -> np.ndarray:
    if isinstance(msg, (bytes, bytearray)):
        a = np.frombuffer(bytes(msg), dtype=np.uint8)
    else:
        a = np.asarray(msg, dtype=np.uint8)
    # one spare byte so that an empty message still has a valid pointer
    buf = np.zeros(a.size + 1, dtype=np.uint8)
    buf[: a.size] = a
    return buf


def constants():
    c0 = np.zeros(4, np.uint64)
    c1 = np.zeros(4, np.uint64)
    lib().hh_ref_constants(_p(c0, ctypes.c_uint64), _p(c1, ctypes.c_uint64))
    return [int(x) for x in c0], [int(x) for x in c1]


def hash_words(key, msg, width_words: int = 1, rounds: int = 4) -> list:
    """Hash one message; returns `width_words` 64-bit words (lane 0 first)."""
    k = _key(key)
    m = _bytes(msg)
    out = np.zeros(4, np.uint64)
    lib().hh_ref_hash_rounds(_p(k, ctypes.c_uint64), _p(m, ctypes.c_uint8), m.size - 1,
                             rounds, _p(out, ctypes.c_uint64))
    return [int(x) for x in out[:width_words]]


def hash64(key, msg) -> int:
    k = _key(key)
    m = _bytes(msg)
    return int(lib().hh_ref_hash64(_p(k, ctypes.c_uint64), _p(m, ctypes.c_uint8), m.size - 1))


def hash128(key, msg) -> list:
    k = _key(key)
    m = _bytes(msg)
    out = np.zeros(2, np.uint64)
    lib().hh_ref_hash128(_p(k, ctypes.c_uint64), _p(m, ctypes.c_uint8), m.size - 1,
                         _p(out, ctypes.c_uint64))
    return [int(x) for x in out]


def hash256(key, msg) -> list:
    k = _key(key)
    m = _bytes(msg)
    out = np.zeros(4, np.uint64)
    lib().hh_ref_hash256(_p(k, ctypes.c_uint64), _p(m, ctypes.c_uint8), m.size - 1,
                         _p(out, ctypes.c_uint64))
    return [int(x) for x in out]


# --- single steps, for the tests that pin each step to the paper -------------

def reset(key) -> np.ndarray:
    s = np.zeros(STATE_WORDS, np.uint64)
    k = _key(key)
    lib().hh_ref_reset(_p(k, ctypes.c_uint64), _p(s, ctypes.c_uint64))
    return s


def update(state, packet) -> np.ndarray:
    s = np.array(state, dtype=np.uint64).reshape(STATE_WORDS).copy()
    p = np.ascontiguousarray(np.asarray(packet, dtype=np.uint64).reshape(4))
    lib().hh_ref_update(_p(s, ctypes.c_uint64), _p(p, ctypes.c_uint64))
    return s


def zipper_merge(a: int, b: int):
    ra = ctypes.c_uint64()
    rb = ctypes.c_uint64()
    lib().hh_ref_zipper_merge(ctypes.c_uint64(a), ctypes.c_uint64(b), ctypes.byref(ra),
                              ctypes.byref(rb))
    return int(ra.value), int(rb.value)


def permute(v0) -> list:
    v = np.ascontiguousarray(np.asarray(v0, dtype=np.uint64).reshape(4))
    out = np.zeros(4, np.uint64)
    lib().hh_ref_permute(_p(v, ctypes.c_uint64), _p(out, ctypes.c_uint64))
    return [int(x) for x in out]


def remainder(state, tail) -> np.ndarray:
    s = np.array(state, dtype=np.uint64).reshape(STATE_WORDS).copy()
    t = _bytes(tail)
    lib().hh_ref_remainder(_p(s, ctypes.c_uint64), _p(t, ctypes.c_uint8), t.size - 1)
    return s


def finalize(state, rounds: int = 4):
    s = np.array(state, dtype=np.uint64).reshape(STATE_WORDS).copy()
    out = np.zeros(4, np.uint64)
    lib().hh_ref_finalize(_p(s, ctypes.c_uint64), rounds, _p(out, ctypes.c_uint64))
    return s, [int(x) for x in out]


class Cat:
    """Incremental hashing (Sec. 4.5): append any chunks, finish any time."""

    def __init__(self, key):
        self._buf = ctypes.create_string_buffer(lib().hh_ref_cat_size())
        self._key = _key(key)
        lib().hh_ref_cat_init(self._buf, _p(self._key, ctypes.c_uint64))

    def append(self, chunk) -> "Cat":
        m = _bytes(chunk)
        lib().hh_ref_cat_append(self._buf, _p(m, ctypes.c_uint8), m.size - 1)
        return self

    def finish(self, width_words: int = 1) -> list:
        out = np.zeros(4, np.uint64)
        lib().hh_ref_cat_finish(self._buf, width_words, _p(out, ctypes.c_uint64))
        return [int(x) for x in out[:width_words]]


def batch(keys, key_idx, data, offsets, lengths, width_words: int = 1,
          n_threads: int | None = None) -> np.ndarray:
    """Hash many messages: message j = data[offsets[j]:offsets[j]+lengths[j]]
    under keys[key_idx[j]] (key 0 if key_idx is None).  Returns a uint64 array
    of shape (n, width_words)."""
    keys = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64).reshape(-1, 4))
    data = np.ascontiguousarray(np.asarray(data, dtype=np.uint8))
    if data.size == 0:
        data = np.zeros(1, np.uint8)
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    lengths = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint64))
    n = offsets.size
    if lengths.size != n:
        raise ValueError("offsets and lengths differ in size")
    if n and int((offsets + lengths).max()) > data.size:
        raise ValueError("a message runs past the end of data")
    if key_idx is not None:
        key_idx = np.ascontiguousarray(np.asarray(key_idx, dtype=np.uint32))
        if key_idx.size != n:
            raise ValueError("key_idx size differs from the message count")
        if n and int(key_idx.max()) >= keys.shape[0]:
            raise ValueError("key index out of range")
        kip = _p(key_idx, ctypes.c_uint32)
    else:
        kip = None
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    out = np.zeros((max(n, 1), width_words), np.uint64)
    rc = lib().hh_ref_batch(_p(keys, ctypes.c_uint64), kip, _p(data, ctypes.c_uint8),
                            _p(offsets, ctypes.c_uint64), _p(lengths, ctypes.c_uint64), n,
                            width_words, _p(out, ctypes.c_uint64), int(n_threads))
    if rc != 0:
        raise ValueError("hh_ref_batch rejected its arguments")
    return out[:n]
