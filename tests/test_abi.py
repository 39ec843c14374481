"""CPU-side checks of the C ABI: the library loads, exports every entry point
that include/hh.h declares, rejects bad arguments before touching a device,
and carries the Sec. 4.4 constants derived from pi."""
import ctypes
import os
import re

import pytest

from test_oracle_steps import _fourth_lane, _pi_fraction_words

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hh.h")


def _hh():
    from paper_1612_06257_amd import hh
    return hh


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:volatile\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*"
                       r"(hh_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("hh_hash64", "hh_hash128", "hh_hash256", "hh_hash64_uniform", "hh_hash_path",
                 "hh_state_init", "hh_state_update", "hh_state_final", "hh_status_string",
                 "hh_feed_open", "hh_feed_submit", "hh_feed_poll", "hh_feed_results",
                 "hh_feed_close"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = _hh().lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    hh = _hh()
    for s in range(6):
        assert hh.status_string(s) != "unknown status"
    assert hh.status_string(0) == "ok"
    assert hh.lib().hh_version() >= 100


def test_invalid_arguments_rejected_without_device():
    L = _hh().lib()
    vp = ctypes.c_void_p
    dummy = vp(16)
    # n > 0 with NULL keys / offsets / out
    assert L.hh_hash64(None, 1, None, dummy, 8, dummy, dummy, 3, dummy, None) == 1
    assert L.hh_hash64(dummy, 0, None, dummy, 8, dummy, dummy, 3, dummy, None) == 1
    assert L.hh_hash64(dummy, 1, None, dummy, 8, None, dummy, 3, dummy, None) == 1
    assert L.hh_hash64(dummy, 1, None, dummy, 8, dummy, dummy, 3, None, None) == 1
    assert L.hh_hash64(dummy, 1, None, None, 8, dummy, dummy, 3, dummy, None) == 1
    assert L.hh_hash_path(0, 3, dummy, 1, None, dummy, 8, dummy, dummy, 3, dummy, None) == 1
    assert L.hh_hash_path(9, 1, dummy, 1, None, dummy, 8, dummy, dummy, 3, dummy, None) in (1, 2)
    assert L.hh_state_update(None, 4, None, dummy, 8, dummy, dummy, 2, None) == 1
    assert L.hh_state_final(dummy, 4, None, dummy, 8, dummy, dummy, None, None, 8, None, 2,
                            None) == 1
    # n == 0 is a no-op that succeeds even with NULL pointers
    assert L.hh_hash64(None, 0, None, None, 0, None, None, 0, None, None) == 0
    assert L.hh_state_init(None, 0, None, None, 0, None, 0, None) == 0
    assert L.hh_state_init(None, 1, None, dummy, 4, None, 1, None) == 1
    assert L.hh_copy_segments(None, 0, None, 0, None, None, None, 0, 0, None) == 0
    assert L.hh_copy_segments(None, 8, dummy, 8, dummy, dummy, dummy, 1, 8, None) == 1
    assert L.hh_copy_segments(dummy, 8, dummy, 8, dummy, None, dummy, 1, 8, None) == 1
    # the allocation-free entry point: the same checks, plus its size limit
    # (HH_NOALLOC_MAX_MSGS = 2^20 messages per call)
    assert L.hh_hash_noalloc(1, None, 0, None, None, 0, None, None, 0, None, None) == 0
    assert L.hh_hash_noalloc(3, dummy, 1, None, dummy, 8, dummy, dummy, 3, dummy, None) == 1
    assert L.hh_hash_noalloc(1, dummy, 0, None, dummy, 8, dummy, dummy, 3, dummy, None) == 1
    assert L.hh_hash_noalloc(1, dummy, 1, None, dummy, 8, dummy, dummy, 3, None, None) == 1
    assert L.hh_hash_noalloc(1, dummy, 1, None, dummy, 8, dummy, dummy, (1 << 20) + 1, dummy,
                             None) == 1
    assert _hh().NOALLOC_MAX_MSGS == 1 << 20
    # the feed: every argument error is found before any device call
    h = vp()
    assert L.hh_feed_open(dummy, 1, dummy, 8, 16, 4, 100, None, None) == 1
    assert L.hh_feed_open(None, 1, dummy, 8, 16, 4, 100, None, ctypes.byref(h)) == 1
    assert L.hh_feed_open(dummy, 0, dummy, 8, 16, 4, 100, None, ctypes.byref(h)) == 1
    assert L.hh_feed_open(dummy, 1, None, 8, 16, 4, 100, None, ctypes.byref(h)) == 1
    assert L.hh_feed_open(dummy, 1, dummy, 8, 0, 4, 100, None, ctypes.byref(h)) == 1
    assert L.hh_feed_open(dummy, 1, dummy, 8, 65537, 4, 100, None, ctypes.byref(h)) == 1
    assert L.hh_feed_open(dummy, 1, dummy, 8, 16, 1, 100, None, ctypes.byref(h)) == 1
    assert L.hh_feed_open(dummy, 1, dummy, 8, 16, 66, 100, None, ctypes.byref(h)) == 1
    assert L.hh_feed_open(dummy, 1, dummy, 8, 16, 4, 0, None, ctypes.byref(h)) == 1
    assert L.hh_feed_open(dummy, 1, dummy, 8, 16, 4, 60001, None, ctypes.byref(h)) == 1
    assert h.value is None
    t = ctypes.c_uint64()
    assert L.hh_feed_submit(None, 1, dummy, dummy, None, dummy, dummy, ctypes.byref(t)) == 1
    assert L.hh_feed_poll(None) == 1
    assert L.hh_feed_results(None) is None
    assert L.hh_feed_close(None) == 1


def test_no_device_reported_as_unsupported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = _hh().lib()
    vp = ctypes.c_void_p
    dummy = vp(16)
    assert L.hh_hash64(dummy, 1, None, dummy, 8, dummy, dummy, 3, dummy, None) == 2
    assert L.hh_hash_noalloc(1, dummy, 1, None, dummy, 8, dummy, dummy, 1 << 20, dummy,
                             None) == 2


def test_library_constants_follow_pi_derivation():
    w = _pi_fraction_words(8)
    c0, c1 = _hh().constants()
    assert c0 == [_fourth_lane(w[0], w[1], w[2]), w[2], w[1], w[0]]
    assert c1 == [_fourth_lane(w[4], w[5], w[6]), w[6], w[5], w[4]]


def test_tuning_roundtrip():
    hh = _hh()
    t = hh.get_tuning()
    hh.set_tuning(**t)
    assert hh.get_tuning() == t
    with pytest.raises(hh.HHError):
        hh.set_tuning(waves_per_cu=0)
    with pytest.raises(hh.HHError):
        hh.set_tuning(**dict(t, isolate_long=2))
    for bad in (dict(long_ring=60), dict(long_ring=0), dict(waves_per_cu=33),
                dict(use_graph=2)):
        with pytest.raises(hh.HHError):
            hh.set_tuning(**dict(t, **bad))
        assert hh.get_tuning() == t  # a rejected setting changes nothing
    for ring in (36, 48, 72, 96):
        hh.set_tuning(**dict(t, long_ring=ring))
        assert hh.get_tuning()["long_ring"] == ring
    hh.set_tuning(**t)
    assert hh.get_tuning() == t
