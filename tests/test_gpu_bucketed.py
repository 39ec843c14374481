"""The bucketed path under every tuning setting and as a replayed hipGraph:
bit-exact with the oracle on a batch that mixes empty, short and long
messages at every alignment."""
import numpy as np
import pytest
import torch

from _gpu import announce, assert_same, batch_to_device, oracle_ref, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh():
    h = require_gpu()
    saved = h.get_tuning()
    yield h
    h.set_tuning(**saved)


def _batch(seed=31, n=2500):
    rng = np.random.default_rng(seed)
    lens = np.concatenate([np.zeros(40), rng.integers(1, 200, n // 2),
                           rng.integers(200, 20000, n // 2 - 60),
                           rng.integers(100000, 400000, 20)]).astype(np.uint64)
    rng.shuffle(lens)
    gaps = rng.integers(0, 16, lens.size).astype(np.uint64)
    offsets = np.cumsum(lens + gaps) - lens
    data = np.frombuffer(rng.bytes(int(offsets[-1] + lens[-1]) + 8), np.uint8).copy()
    keys = rng.integers(0, 2**64, size=(5, 4), dtype=np.uint64)
    key_idx = rng.integers(0, 5, lens.size, dtype=np.uint32)
    return keys, key_idx, data, offsets.astype(np.uint64), lens


@pytest.mark.parametrize("tuning", [
    dict(long_ring=24), dict(long_ring=48), dict(long_ring=64), dict(waves_per_cu=8),
    dict(waves_per_cu=12, long_ring=32), dict(lane4_min_bytes=0), dict(lane4_min_bytes=1),
    dict(lane4_min_bytes=4096), dict(lane4_min_bytes=1 << 30)])
def test_tuning_variants_bit_exact(hh, tuning):
    base = hh.get_tuning()
    keys, key_idx, data, offsets, lengths = _batch()
    want = oracle_ref(2, keys, key_idx, data, offsets, lengths)
    try:
        hh.set_tuning(**dict(base, **tuning))
        announce("tuning", tuning)
        k, ki, d, o, L = batch_to_device(keys, key_idx, data, offsets, lengths)
        got = hh.to_u64(hh.hash(k, d, o, L, ki, 2, "auto"))
        torch.cuda.synchronize()
        assert_same(got, want, str(tuning))
    finally:
        hh.set_tuning(**base)


def test_graph_replays_match_eager(hh):
    base = hh.get_tuning()
    keys, key_idx, data, offsets, lengths = _batch(seed=41)
    want = oracle_ref(1, keys, key_idx, data, offsets, lengths)
    k, ki, d, o, L = batch_to_device(keys, key_idx, data, offsets, lengths)
    side = torch.cuda.Stream()
    out = torch.empty((lengths.size, 1), dtype=torch.int64, device="cuda")
    try:
        hh.set_tuning(**dict(base, use_graph=1))
        for rep in range(4):
            announce("graph replay", rep)
            with torch.cuda.stream(side):
                out.zero_()
                hh.hash(k, d, o, L, ki, 1, "auto", out)
            side.synchronize()
            assert_same(hh.to_u64(out), want, "replay %d" % rep)
            # eager work between replays, on the default stream
            hh.set_tuning(**dict(base, use_graph=0))
            eager = hh.to_u64(hh.hash(k, d, o, L, ki, 1, "auto"))
            assert_same(eager, want, "eager %d" % rep)
            hh.set_tuning(**dict(base, use_graph=1))
        # same pointers, new contents: the replay must hash the new bytes
        data2 = data.copy()
        data2[::3] ^= 0x5A
        d.copy_(torch.from_numpy(data2))
        want2 = oracle_ref(1, keys, key_idx, data2, offsets, lengths)
        with torch.cuda.stream(side):
            hh.hash(k, d, o, L, ki, 1, "auto", out)
        side.synchronize()
        assert_same(hh.to_u64(out), want2, "replay after data change")
    finally:
        hh.set_tuning(**base)


def test_autotune_caches_and_stays_bit_exact(hh, tmp_path):
    from paper_1612_06257_amd import autotune
    base = hh.get_tuning()
    keys, key_idx, data, offsets, lengths = _batch(seed=53, n=800)
    want = oracle_ref(1, keys, key_idx, data, offsets, lengths)
    k, ki, d, o, L = batch_to_device(keys, key_idx, data, offsets, lengths)
    cache = str(tmp_path / "tune.json")
    try:
        best = autotune.tune(k, d, o, L, ki, 1, reps=2, cache_path=cache)
        assert best["candidates"] >= 3 and best["ms"] > 0
        assert autotune.lookup(L, 1, cache) == best
        got = hh.to_u64(autotune.hash(k, d, o, L, ki, 1, cache_path=cache))
        assert_same(got, want, "autotuned " + str(best))
    finally:
        hh.set_tuning(**base)
