"""Seeded random batches through every path and tuning: message counts,
length mixes (empty, short, power-law, a few long ones near each other),
alignments, key pools, output widths and tuning settings are drawn per case,
and every result must equal the oracle's bit for bit."""
import numpy as np
import pytest
import torch

from _gpu import announce, assert_same, batch_to_device, oracle_ref, require_gpu

pytestmark = pytest.mark.gpu

RINGS = (36, 48, 72, 96)
WAVES = (1, 2, 4, 8)
THRESHOLDS = (0, 1, 33, 128, 700)


@pytest.fixture(scope="module")
def hh():
    h = require_gpu()
    saved = h.get_tuning()
    yield h
    h.set_tuning(**saved)


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.choice([1, 2, 15, 16, 17, 63, 64, 65, 300, 1000, 3000]))
    kind = seed % 4
    if kind == 0:      # power law up to 300 KB
        lens = np.floor(8 * (1 - rng.random(n)) ** (-1 / 1.1)).clip(0, 300000)
    elif kind == 1:    # short and empty
        lens = rng.integers(0, 100, n)
    elif kind == 2:    # a few long ones of nearly equal length among short ones
        lens = rng.integers(0, 5000, n)
        k = max(1, n // 50)
        lens[rng.choice(n, k, replace=False)] = 200000 + rng.integers(0, 64, k)
    else:              # uniform over packet boundaries
        lens = 32 * rng.integers(0, 400, n) + rng.integers(0, 32, n)
    lens = lens.astype(np.uint64)
    gaps = rng.integers(0, 8, n).astype(np.uint64)
    offsets = np.cumsum(lens + gaps) - lens
    total = int(offsets[-1] + lens[-1]) if n else 0
    data = np.frombuffer(rng.bytes(total + 1), np.uint8).copy()
    n_keys = int(rng.choice([1, 3, 64]))
    keys = rng.integers(0, 2**64, size=(n_keys, 4), dtype=np.uint64)
    key_idx = None if n_keys == 1 else rng.integers(0, n_keys, n, dtype=np.uint32)
    width = int(rng.choice([1, 2, 4]))
    tuning = dict(long_ring=int(rng.choice(RINGS)), waves_per_cu=int(rng.choice(WAVES)),
                  lane4_min_bytes=int(rng.choice(THRESHOLDS)),
                  isolate_long=int(rng.integers(0, 2)), use_graph=0)
    path = str(rng.choice(["bucketed", "bucketed", "auto", "lane4", "lane1"]))
    return keys, key_idx, data, offsets.astype(np.uint64), lens, width, tuning, path


@pytest.mark.parametrize("seed", range(32))
def test_random_batch_bit_exact(hh, seed):
    keys, key_idx, data, offsets, lengths, width, tuning, path = _case(seed)
    announce("random", seed, lengths.size, width, path, tuning)
    want = oracle_ref(width, keys, key_idx, data, offsets, lengths)
    base = hh.get_tuning()
    try:
        hh.set_tuning(**dict(base, **tuning))
        k, ki, d, o, L = batch_to_device(keys, key_idx, data, offsets, lengths)
        got = hh.to_u64(hh.hash(k, d, o, L, ki, width, path))
        torch.cuda.synchronize()
        assert_same(got, want, "seed %d" % seed)
    finally:
        hh.set_tuning(**base)
