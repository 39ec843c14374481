"""Counter-mode PRF (hh_prf): bit-exact with the batch path and the oracle,
and its output stream statistically indistinguishable from uniform bits."""
import numpy as np
import pytest
import torch
from scipy import stats

import oracle
from _gpu import announce, require_gpu
from paper_1612_06257_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh():
    return require_gpu()


@pytest.fixture(scope="module")
def prf_batch():
    return W.prf_counters()


@pytest.fixture(scope="module")
def prf_out(hh, prf_batch):
    keys = torch.from_numpy(prf_batch.keys).view(torch.int64).cuda()
    out = hh.prf(keys, prf_batch.n)
    torch.cuda.synchronize()
    return out


def test_prf_equals_batch_path_on_all_counters(hh, prf_batch, prf_out):
    announce("prf vs batch", prf_batch.n)
    b = prf_batch
    keys = torch.from_numpy(b.keys).view(torch.int64).cuda()
    ref = hh.hash(keys, torch.from_numpy(b.data).cuda(),
                  torch.from_numpy(b.offsets).view(torch.int64).cuda(),
                  torch.from_numpy(b.lengths).view(torch.int64).cuda(),
                  torch.from_numpy(b.key_idx).view(torch.int32).cuda(), 1)
    assert torch.equal(ref, prf_out)


def test_prf_matches_oracle_samples_widths_and_wraparound(hh):
    rng = np.random.default_rng(61)
    keys = rng.integers(0, 2**64, size=(37, 4), dtype=np.uint64)
    kt = torch.from_numpy(keys).view(torch.int64).cuda()
    for base in (0, 12345678901234567890, 2**64 - 150):
        for width in (1, 2, 4):
            got = hh.to_u64(hh.prf(kt, 300, base, width))
            for j in range(0, 300, 7):
                c = (base + j) % 2**64
                msg = np.frombuffer(int(c).to_bytes(8, "little"), np.uint8)
                assert [int(x) for x in got[j]] == oracle.hash_words(keys[c % 37], msg, width)


def _bit_freqs(x: torch.Tensor) -> torch.Tensor:
    return torch.stack([((x >> b) & 1).sum(dim=0) for b in range(64)]).double()


def test_prf_output_bits_are_unbiased(prf_out):
    x = prf_out[:, 0]
    n = x.numel()
    freq = _bit_freqs(x) / n
    sigma = 0.5 / np.sqrt(n)
    assert float((freq - 0.5).abs().max()) < 6 * sigma
    # per key class (key = counter mod 1024): 64 bits x 1024 classes
    per = _bit_freqs(x.view(n // 1024, 1024)) / (n // 1024)
    cells = per.numel()
    z = stats.norm.isf(1e-6 / (2 * cells))
    assert float((per - 0.5).abs().max()) < z * 0.5 / np.sqrt(n // 1024)


def test_prf_top16_histogram_chi_square(prf_out):
    x = prf_out[:, 0]
    top = ((x >> 48) & 0xFFFF).long()
    counts = torch.bincount(top, minlength=65536).double()
    expected = x.numel() / 65536.0
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    p = stats.chi2.sf(chi2, 65535)
    assert 1e-6 < p < 1 - 1e-6, (chi2, p)


@pytest.mark.parametrize("n_keys,n,base", [(37, 3_000_001, 5), (1, 1_000_003, 2**64 - 1000),
                                           (1024, 1_500_000, 77), (700_001, 2_000_000, 0)])
def test_prf_every_launch_shape(hh, n_keys, n, base):
    # the grid keeps one key per thread when its thread count can be made a
    # multiple of n_keys (37, 1, 1024 here), else takes the key per counter
    # (700001 keys, more than the resident threads); both against the batch
    # path on every counter and the oracle on samples
    rng = np.random.default_rng(62)
    keys = rng.integers(0, 2**64, size=(n_keys, 4), dtype=np.uint64)
    kt = torch.from_numpy(keys).view(torch.int64).cuda()
    announce("prf shape", n_keys, n, base)
    for width in (1, 4):
        got = hh.prf(kt, n, base, width)
        c = (np.uint64(base) + np.arange(n, dtype=np.uint64))   # wraps mod 2^64
        ref = hh.hash(kt, torch.from_numpy(c.view(np.uint8)).cuda(),
                      torch.arange(0, 8 * n, 8, dtype=torch.int64, device="cuda"),
                      torch.full((n,), 8, dtype=torch.int64, device="cuda"),
                      torch.from_numpy((c % np.uint64(n_keys)).astype(np.uint32)).view(
                          torch.int32).cuda(), width)
        torch.cuda.synchronize()
        assert torch.equal(ref, got), (n_keys, n, width)
        g = hh.to_u64(got)
        for j in list(rng.integers(0, n, 20)) + [0, n - 1]:
            cj = int(c[j])
            msg = np.frombuffer(cj.to_bytes(8, "little"), np.uint8)
            assert [int(x) for x in g[j]] == oracle.hash_words(keys[cj % n_keys], msg, width)
