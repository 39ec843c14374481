"""Whole-hash properties the paper fixes, checked on the CPU oracle.

* Sec. 4.5: incremental hashing equals one-shot hashing for any chunking.
* Sec. 4.5 / 6.3: zero-valued inputs of different lengths, and inputs with
  different numbers of trailing zeros, hash differently.
* Sec. 4.3: the upper lanes reach the 64-bit result (via Permute), so every
  key bit and every input bit changes it.
* Sec. 6.1: avalanche -- each output bit flips with probability 1/2 when one
  input bit flips; the measured bias is compared with its null distribution.
* Sec. 4.3: two finalization rounds leave strong biases, four do not.
* Sec. 4.3: 64-, 128- and 256-bit results come from the same final sum.
"""
import numpy as np
import pytest
from scipy import stats

import oracle

RNG_SEED = 20161219


def _rand_key(rng):
    return rng.integers(0, 2**64, size=4, dtype=np.uint64)


def _batch_fixed(keys, key_idx, msgs, width=1):
    """Hash an (n, L) array of equal-length messages through the oracle."""
    n, L = msgs.shape
    data = np.ascontiguousarray(msgs).reshape(-1)
    offsets = np.arange(n, dtype=np.uint64) * np.uint64(L)
    lengths = np.full(n, L, dtype=np.uint64)
    return oracle.batch(keys, key_idx, data, offsets, lengths, width)


# --------------------------------------------------------------------------
# Sec. 4.5 incremental hashing


@pytest.mark.parametrize("width", [1, 2, 4])
def test_streaming_equals_one_shot(width):
    rng = np.random.default_rng(RNG_SEED)
    for L in list(range(0, 70)) + [95, 96, 97, 300, 1000]:
        key = _rand_key(rng)
        msg = rng.integers(0, 256, size=L, dtype=np.uint8)
        want = oracle.hash_words(key, msg, width)
        # random split points
        for _ in range(3):
            cuts = sorted(rng.integers(0, L + 1, size=int(rng.integers(0, 6))))
            c = oracle.Cat(key)
            prev = 0
            for x in list(cuts) + [L]:
                c.append(msg[prev:x])
                prev = x
            assert c.finish(width) == want
        # byte by byte, and around the packet boundary
        c = oracle.Cat(key)
        for b in msg:
            c.append(bytes([int(b)]))
        assert c.finish(width) == want
        for cut in (31, 32, 33):
            if cut <= L:
                assert oracle.Cat(key).append(msg[:cut]).append(msg[cut:]).finish(width) == want


def test_finish_leaves_stream_usable():
    rng = np.random.default_rng(RNG_SEED + 1)
    key = _rand_key(rng)
    msg = rng.integers(0, 256, size=77, dtype=np.uint8)
    c = oracle.Cat(key)
    c.append(msg[:40])
    assert c.finish() == oracle.hash_words(key, msg[:40])
    c.append(msg[40:])
    assert c.finish() == oracle.hash_words(key, msg)


# --------------------------------------------------------------------------
# Sec. 4.5, Sec. 6.3 zero-valued inputs


def test_zero_messages_of_different_lengths_differ():
    rng = np.random.default_rng(RNG_SEED + 2)
    key = _rand_key(rng)
    n = 4097
    lengths = np.arange(n, dtype=np.uint64)
    offsets = np.zeros(n, dtype=np.uint64)
    data = np.zeros(n, dtype=np.uint8)
    for width in (1, 2, 4):
        h = oracle.batch(key, None, data, offsets, lengths, width)
        assert len({tuple(int(x) for x in row) for row in h}) == n


def test_trailing_zeros_change_the_hash():
    rng = np.random.default_rng(RNG_SEED + 3)
    for base_len in (0, 1, 5, 31, 32, 33, 64, 100):
        key = _rand_key(rng)
        base = rng.integers(0, 256, size=base_len, dtype=np.uint8)
        hs = {oracle.hash64(key, np.concatenate([base, np.zeros(k, np.uint8)]))
              for k in range(0, 97)}
        assert len(hs) == 97


# --------------------------------------------------------------------------
# Sec. 4.3 every key and input bit reaches the 64-bit result


def test_every_key_bit_changes_h64():
    rng = np.random.default_rng(RNG_SEED + 4)
    for L in (0, 3, 32, 45):
        key = _rand_key(rng)
        msg = rng.integers(0, 256, size=L, dtype=np.uint8)
        h = oracle.hash64(key, msg)
        keys = np.repeat(key[None, :], 256, axis=0)
        for b in range(256):
            keys[b, b // 64] ^= np.uint64(1) << np.uint64(b % 64)
        msgs = np.repeat(msg[None, :], 256, axis=0) if L else np.zeros((256, 0), np.uint8)
        hf = _batch_fixed(keys, np.arange(256, dtype=np.uint32), msgs)[:, 0]
        assert np.all(hf != np.uint64(h))


def test_every_input_bit_changes_h64():
    rng = np.random.default_rng(RNG_SEED + 5)
    key = _rand_key(rng)
    for L in range(1, 97):
        msg = rng.integers(0, 256, size=L, dtype=np.uint8)
        h = oracle.hash64(key, msg)
        msgs = np.repeat(msg[None, :], 8 * L, axis=0)
        for b in range(8 * L):
            msgs[b, b // 8] ^= np.uint8(1 << (b % 8))
        hf = _batch_fixed(key, None, msgs)[:, 0]
        assert np.all(hf != np.uint64(h)), L


def test_upper_half_of_packet_reaches_h64():
    # bytes 16..31 feed lanes 2 and 3, which reach lane 0 only through Permute
    rng = np.random.default_rng(RNG_SEED + 6)
    key = _rand_key(rng)
    msg = rng.integers(0, 256, size=32, dtype=np.uint8)
    h = oracle.hash64(key, msg)
    for byte in range(16, 32):
        m2 = msg.copy()
        m2[byte] ^= 0x80
        assert oracle.hash64(key, m2) != h


# --------------------------------------------------------------------------
# Sec. 6.1 avalanche, Sec. 4.3 finalization rounds


def _flip_counts(keys, msgs, rounds=4):
    """For each (input bit, output bit of H64) the number of the N inputs for
    which flipping that input bit flips that output bit."""
    n, L = msgs.shape
    nbits = 8 * L
    counts = np.zeros((nbits, 64), dtype=np.int64)
    chunk = max(1, 2**20 // (nbits + 1))
    for s in range(0, n, chunk):
        m = msgs[s:s + chunk]
        k = keys[s:s + chunk]
        c = m.shape[0]
        allm = np.repeat(m[:, None, :], nbits + 1, axis=1)
        for b in range(nbits):
            allm[:, b + 1, b // 8] ^= np.uint8(1 << (b % 8))
        flat = allm.reshape(-1, L)
        kidx = np.repeat(np.arange(c, dtype=np.uint32), nbits + 1)
        if rounds == 4:
            h = _batch_fixed(k, kidx, flat)[:, 0].reshape(c, nbits + 1)
        else:
            h = np.array([oracle.hash_words(k[kidx[i]], flat[i], 1, rounds)[0]
                          for i in range(flat.shape[0])], dtype=np.uint64).reshape(c, nbits + 1)
        x = h[:, 1:] ^ h[:, :1]
        bits = np.unpackbits(x.view(np.uint8).reshape(c, nbits, 8), axis=2,
                             bitorder="little")
        counts += bits.sum(axis=0, dtype=np.int64)
    return counts


def _max_bias(counts, n):
    return float(np.max(np.abs(2.0 * counts / n - 1.0)))


def _null_threshold(n, cells, alpha=1e-6):
    """Bias level that the max over `cells` independent fair-coin cells with
    n trials each exceeds with probability below alpha (normal approx.)."""
    z = stats.norm.isf(alpha / (2 * cells))
    return z / np.sqrt(n)


@pytest.mark.parametrize("size", [4, 7, 8, 16, 17, 31, 32])
def test_avalanche_bias_matches_random_null(size):
    rng = np.random.default_rng(RNG_SEED + 100 + size)
    n = 2**14
    keys = rng.integers(0, 2**64, size=(n, 4), dtype=np.uint64)
    msgs = rng.integers(0, 256, size=(n, size), dtype=np.uint8)
    counts = _flip_counts(keys, msgs)
    bias = _max_bias(counts, n)
    thr = _null_threshold(n, counts.size)
    assert bias < thr, (size, bias, thr)


def test_two_finalization_rounds_are_biased_four_are_not():
    # Sec. 4.3: strong biases remain after two rounds on 3-byte inputs
    rng = np.random.default_rng(RNG_SEED + 200)
    n = 2**11
    keys = rng.integers(0, 2**64, size=(n, 4), dtype=np.uint64)
    msgs = rng.integers(0, 256, size=(n, 3), dtype=np.uint8)
    thr = _null_threshold(n, 24 * 64)
    b2 = _max_bias(_flip_counts(keys, msgs, rounds=2), n)
    b4 = _max_bias(_flip_counts(keys, msgs, rounds=4), n)
    assert b4 < thr, b4
    assert b2 > 3 * thr, (b2, thr)


# --------------------------------------------------------------------------
# Sec. 4.3 output widths; brute force on a tiny domain; batch driver


def test_wide_outputs_share_the_final_sum():
    rng = np.random.default_rng(RNG_SEED + 7)
    for L in (0, 1, 31, 32, 33, 200):
        key = _rand_key(rng)
        msg = rng.integers(0, 256, size=L, dtype=np.uint8)
        h64 = oracle.hash64(key, msg)
        h128 = oracle.hash128(key, msg)
        h256 = oracle.hash256(key, msg)
        assert h64 == h128[0] == h256[0]
        assert h128 == h256[:2]


def test_all_two_byte_messages_distinct():
    rng = np.random.default_rng(RNG_SEED + 8)
    key = _rand_key(rng)
    msgs = np.stack(np.meshgrid(np.arange(256), np.arange(256), indexing="ij"),
                    axis=-1).reshape(-1, 2).astype(np.uint8)
    h = _batch_fixed(key, None, msgs)[:, 0]
    assert np.unique(h).size == 65536


def test_batch_matches_single_calls_and_thread_counts():
    rng = np.random.default_rng(RNG_SEED + 9)
    n = 500
    keys = rng.integers(0, 2**64, size=(7, 4), dtype=np.uint64)
    key_idx = rng.integers(0, 7, size=n, dtype=np.uint32)
    lengths = rng.integers(0, 300, size=n).astype(np.uint64)
    offsets = rng.integers(0, 5000, size=n).astype(np.uint64)
    data = rng.integers(0, 256, size=5300, dtype=np.uint8)
    for width in (1, 2, 4):
        ref = oracle.batch(keys, key_idx, data, offsets, lengths, width, n_threads=1)
        for t in (2, 3, 16):
            assert np.array_equal(oracle.batch(keys, key_idx, data, offsets, lengths, width,
                                               n_threads=t), ref)
        for j in range(0, n, 37):
            o, L = int(offsets[j]), int(lengths[j])
            assert [int(x) for x in ref[j]] == oracle.hash_words(keys[key_idx[j]],
                                                                  data[o:o + L], width)
