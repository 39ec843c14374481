"""The GPU avalanche kernel counts exactly what the oracle counts on the same
SplitMix64 (or enumerated) inputs, for several sizes and round counts."""
import numpy as np
import pytest
import torch

import oracle
from _gpu import announce, require_gpu
from paper_1612_06257_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh():
    return require_gpu()


def _cpu_counts(keys, msgs, rounds):
    n, size = msgs.shape
    counts = np.zeros((8 * size, 64), np.int64)
    for s in range(n):
        h0 = oracle.hash_words(keys[s], msgs[s], 1, rounds)[0]
        for b in range(8 * size):
            m2 = msgs[s].copy()
            m2[b // 8] ^= np.uint8(1 << (b % 8))
            d = h0 ^ oracle.hash_words(keys[s], m2, 1, rounds)[0]
            for k in range(64):
                counts[b, k] += (d >> k) & 1
    return counts


@pytest.mark.parametrize("size,rounds,n", [(3, 2, 130), (3, 4, 100), (13, 4, 70), (32, 3, 65),
                                           (8, 1, 64)])
def test_random_inputs_counts_match_oracle(hh, size, rounds, n):
    announce("avalanche", size, rounds, n)
    seed = 777 + size
    keys, msgs = W.avalanche_inputs(seed, n, size)
    want = _cpu_counts(keys, msgs, rounds)
    got = hh.avalanche_counts(size, n, rounds, seed=seed).cpu().numpy()
    assert np.array_equal(got, want)


def test_enumerated_inputs_counts_match_oracle(hh):
    key = [11, 22, 33, 44]
    n = 300
    msgs = np.arange(n, dtype="<u8").view(np.uint8).reshape(n, 8)[:, :2].copy()
    keys = np.tile(np.array(key, np.uint64), (n, 1))
    want = _cpu_counts(keys, msgs, 3)
    got = hh.avalanche_counts(2, n, 3, key=key).cpu().numpy()
    assert np.array_equal(got, want)


def test_bit_groups_split_and_subset(hh):
    # more than 32 input bits are processed in groups; a subset of bits gives
    # the same rows as the full run
    full = hh.avalanche_counts(9, 200, 4, seed=5).cpu().numpy()
    sub = hh.avalanche_counts(9, 200, 4, seed=5, bits=range(40, 72)).cpu().numpy()
    assert np.array_equal(full[40:72], sub)
