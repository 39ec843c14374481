"""Seeded synthetic workloads (no hashing in here).

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` and returns a
``Batch``: a packed byte buffer plus per-message uint64 offsets and lengths,
a pool of 256-bit keys (four uint64 words each, word i = lane i) and an
optional per-message key index.  Both the oracle-side tests and the HIP path
consume these arrays; nothing here depends on either.

The shapes follow the paper's workloads (single messages of 8..1024 bytes,
sizes 32i+{0,9,18,27}, the keyed-PRF use case of Sec. 1) scaled up to batches:

* ``plain_fixed``     n messages of exactly L bytes, aligned offsets L*j.
* ``short_mixed``     lengths uniform on {0..64}; messages 0..64 are all-zero
                      messages of lengths 0..64, a further 1/64 are zeroed.
* ``lognormal``       lengths round(exp(N(ln median, sigma))) clipped to
                      [1, max_len], packed back to back (unaligned starts).
* ``prf_counters``    message j is the 8-byte little-endian counter j, hashed
                      under key j mod n_keys from a pool.
* ``serving_trace``   Poisson arrivals; bounded power-law (Zipf-like) lengths;
                      per-request key from a pool and output width 1/2/4 words.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

SEED_BASE = 161206257


@dataclasses.dataclass
class Batch:
    name: str
    seed: int
    keys: np.ndarray                 # (n_keys, 4) uint64
    key_idx: Optional[np.ndarray]    # (n,) uint32 or None (all key 0)
    data: np.ndarray                 # (data_bytes,) uint8
    offsets: np.ndarray              # (n,) uint64
    lengths: np.ndarray              # (n,) uint64

    @property
    def n(self) -> int:
        return int(self.lengths.size)

    @property
    def total_bytes(self) -> int:
        return int(self.lengths.sum()) if self.lengths.size else 0

    def describe(self) -> dict:
        L = self.lengths
        return {
            "workload": self.name,
            "seed": self.seed,
            "n_msgs": self.n,
            "bytes": self.total_bytes,
            "n_keys": int(self.keys.shape[0]),
            "min_len": int(L.min()) if L.size else 0,
            "max_len": int(L.max()) if L.size else 0,
        }


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _keys(rng: np.random.Generator, n_keys: int) -> np.ndarray:
    return rng.integers(0, 2**64, size=(n_keys, 4), dtype=np.uint64, endpoint=False)


def _random_bytes(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniform random bytes: uniform 64-bit draws viewed as little-endian
    bytes (a writable array)."""
    words = rng.integers(0, 2**64, size=(n + 7) // 8, dtype=np.uint64)
    return words.astype("<u8", copy=False).view(np.uint8)[:n]


def _packed_offsets(lengths: np.ndarray) -> np.ndarray:
    off = np.zeros(lengths.size, dtype=np.uint64)
    if lengths.size > 1:
        np.cumsum(lengths[:-1], out=off[1:])
    return off


def plain_fixed(n: int = 4096, length: int = 1024, seed: int = SEED_BASE + 1) -> Batch:
    """n messages of exactly `length` uniform random bytes, one key."""
    rng = _rng(seed)
    keys = _keys(rng, 1)
    lengths = np.full(n, length, dtype=np.uint64)
    offsets = np.arange(n, dtype=np.uint64) * np.uint64(length)
    data = _random_bytes(rng, n * length)
    return Batch(f"plain_fixed(n={n},L={length})", seed, keys, None, data, offsets, lengths)


def short_mixed(n: int = 2**20, max_len: int = 64, seed: int = SEED_BASE + 2) -> Batch:
    """Lengths uniform on {0..max_len}; messages 0..max_len are all-zero
    messages of lengths 0..max_len; a further seeded 1/64 are zeroed."""
    rng = _rng(seed)
    keys = _keys(rng, 1)
    lengths = rng.integers(0, max_len + 1, size=n, dtype=np.uint64)
    k = min(n, max_len + 1)
    lengths[:k] = np.arange(k, dtype=np.uint64)
    offsets = _packed_offsets(lengths)
    total = int(lengths.sum())
    data = _random_bytes(rng, total)
    zero = np.zeros(n, dtype=bool)
    zero[:k] = True
    zero |= rng.random(n) < (1.0 / 64.0)
    for j in np.nonzero(zero)[0]:
        o, L = int(offsets[j]), int(lengths[j])
        data[o:o + L] = 0
    return Batch(f"short_mixed(n={n},L=0..{max_len})", seed, keys, None, data, offsets, lengths)


def lognormal_lengths(rng: np.random.Generator, n: int, median: float, sigma: float,
                      max_len: int) -> np.ndarray:
    x = np.exp(rng.normal(np.log(median), sigma, size=n))
    return np.clip(np.rint(x), 1, max_len).astype(np.uint64)


def lognormal(n: int = 2**16, median: float = 4096.0, sigma: float = 2.15,
              max_len: int = 2**20, seed: int = SEED_BASE + 3) -> Batch:
    """Log-normal lengths (median 4 KiB, sigma 2.15 so the total is about
    2 GiB at n = 2^16), clipped to [1, max_len], packed back to back."""
    rng = _rng(seed)
    keys = _keys(rng, 1)
    lengths = lognormal_lengths(rng, n, median, sigma, max_len)
    offsets = _packed_offsets(lengths)
    data = _random_bytes(rng, int(lengths.sum()))
    return Batch(f"lognormal(n={n},median={int(median)},sigma={sigma},max={max_len})", seed,
                 keys, None, data, offsets, lengths)


def prf_counters(n: int = 2**24, n_keys: int = 1024, seed: int = SEED_BASE + 4) -> Batch:
    """Message j is the 8-byte little-endian encoding of j, under key
    j mod n_keys drawn from a seeded pool."""
    rng = _rng(seed)
    keys = _keys(rng, n_keys)
    ctr = np.arange(n, dtype=np.uint64)
    data = ctr.astype("<u8").view(np.uint8).copy()
    offsets = np.arange(n, dtype=np.uint64) * np.uint64(8)
    lengths = np.full(n, 8, dtype=np.uint64)
    key_idx = (ctr % np.uint64(n_keys)).astype(np.uint32)
    return Batch(f"prf_counters(n={n},keys={n_keys})", seed, keys, key_idx, data, offsets,
                 lengths)


def power_law_lengths(rng: np.random.Generator, n: int, s: float = 1.1, lo: int = 8,
                      hi: int = 2**24) -> np.ndarray:
    """Bounded power law: a continuous density proportional to x^-s on
    [lo, hi+1), floored to an integer (a Zipf(s) law on lo..hi up to the
    discretisation).  Requires lo >= 1."""
    if lo < 1:
        raise ValueError("lo must be at least 1")
    u = rng.random(n)
    a = float(lo) ** (1.0 - s)
    b = float(hi + 1) ** (1.0 - s)
    x = (a + u * (b - a)) ** (1.0 / (1.0 - s))
    return np.clip(np.floor(x), lo, hi).astype(np.uint64)


@dataclasses.dataclass
class Trace:
    """A serving trace: request r arrives at arrival_s[r] (seconds from the
    start), carries data[offsets[r]:offsets[r]+lengths[r]], is hashed under
    keys[key_idx[r]] and wants width_words[r] output words (1, 2 or 4)."""
    seed: int
    rate: float
    arrival_s: np.ndarray
    keys: np.ndarray
    key_idx: np.ndarray
    width_words: np.ndarray
    data: np.ndarray
    offsets: np.ndarray
    lengths: np.ndarray

    @property
    def n(self) -> int:
        return int(self.lengths.size)


def serving_trace(n_requests: int, rate_per_s: float, s: float = 1.1, lo: int = 8,
                  hi: int = 2**24, n_keys: int = 64, seed: int = SEED_BASE + 5,
                  materialize: bool = True) -> Trace:
    """Poisson arrivals at `rate_per_s`, power-law lengths on [lo, hi],
    keys from a pool of n_keys, output width uniform on {1, 2, 4} words."""
    rng = _rng(seed)
    keys = _keys(rng, n_keys)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    arrival = np.cumsum(gaps) - gaps[0]
    lengths = power_law_lengths(rng, n_requests, s, lo, hi)
    key_idx = rng.integers(0, n_keys, size=n_requests, dtype=np.uint32)
    width = np.array([1, 2, 4], dtype=np.uint8)[rng.integers(0, 3, size=n_requests)]
    offsets = _packed_offsets(lengths)
    data = _random_bytes(rng, int(lengths.sum())) if materialize else np.zeros(0, np.uint8)
    return Trace(seed, rate_per_s, arrival, keys, key_idx, width, data, offsets, lengths)


# --- SplitMix64 inputs for the avalanche studies ----------------------------
# SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
# generators", OOPSLA 2014): the state advances by the golden gamma
# 0x9e3779b97f4a7c15 and each output is mix(state).  Output number i (i >= 1)
# of the generator seeded with `seed` is mix(seed + i * gamma).

_SM_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_SM_M1 = np.uint64(0xBF58476D1CE4E5B9)
_SM_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_outputs(seed: int, index: np.ndarray) -> np.ndarray:
    """Outputs number `index` (uint64 array, >= 1) of SplitMix64(seed)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed % 2**64) + np.asarray(index, np.uint64) * _SM_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _SM_M1
        z = (z ^ (z >> np.uint64(27))) * _SM_M2
        return z ^ (z >> np.uint64(31))


def avalanche_inputs(seed: int, n: int, msg_bytes: int):
    """Keys (n, 4) and messages (n, msg_bytes) of the SplitMix64 avalanche
    stream: key word w of sample s is output 8s+w+1, message word w output
    8s+4+w+1 (little-endian bytes, cut to msg_bytes)."""
    s = np.arange(n, dtype=np.uint64)[:, None]
    keys = splitmix64_outputs(seed, 8 * s + np.arange(4, dtype=np.uint64) + 1)
    words = splitmix64_outputs(seed, 8 * s + 4 + np.arange(4, dtype=np.uint64) + 1)
    msgs = words.astype("<u8").view(np.uint8).reshape(n, 32)[:, :msg_bytes].copy()
    return keys, msgs
