"""hh_hash_noalloc: the bucketed path with its planner lists in the library's
fixed per-GPU array.  Through the C ABI, two calls in a row (the second with
a smaller batch), each compared with hh_hash_path(HH_PATH_BUCKETED) and the
oracle, bit for bit; then a batch of the largest allowed size."""
import numpy as np
import pytest
import torch

from _gpu import announce, assert_same, batch_to_device, oracle_ref, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh():
    return require_gpu()


def _batch(seed, n, long_n):
    """Empty, short and long messages at every alignment; a few long enough
    (>= 100 KB) to run on CUs of their own."""
    rng = np.random.default_rng(seed)
    lens = np.concatenate([np.zeros(7), rng.integers(1, 128, n // 2),
                           rng.integers(128, 9000, n - n // 2 - 7 - long_n),
                           rng.integers(100_000, 300_000, long_n)]).astype(np.uint64)
    rng.shuffle(lens)
    gaps = rng.integers(0, 9, lens.size).astype(np.uint64)
    offsets = (np.cumsum(lens + gaps) - lens).astype(np.uint64)
    data = np.frombuffer(rng.bytes(int(offsets[-1] + lens[-1]) + 5), np.uint8)
    keys = rng.integers(0, 2**64, size=(3, 4), dtype=np.uint64)
    key_idx = rng.integers(0, 3, lens.size, dtype=np.uint32)
    return keys, key_idx, data, offsets, lens


def _both(hh, width, batch):
    """(no-alloc result, bucketed result) on the current stream, outputs
    preallocated so the no-alloc call allocates nothing."""
    k, ki, d, o, L = batch_to_device(*batch)
    n = o.numel()
    out_na = torch.full((n, width), -1, dtype=torch.int64, device="cuda")
    out_bk = torch.full((n, width), -2, dtype=torch.int64, device="cuda")
    hh.hash_noalloc(k, d, o, L, ki, width, out_na)
    hh.hash(k, d, o, L, ki, width, "bucketed", out_bk)
    torch.cuda.synchronize()
    return hh.to_u64(out_na), hh.to_u64(out_bk)


def test_two_calls_in_a_row_match_bucketed_and_oracle(hh):
    first = _batch(seed=71, n=3000, long_n=6)
    second = _batch(seed=72, n=700, long_n=2)
    for width, batch, tag in ((4, first, "first call"), (1, second, "second, smaller call"),
                              (2, first, "third call, larger again")):
        announce("noalloc", tag, "n=%d" % batch[3].size, "width", width)
        got, bucketed = _both(hh, width, batch)
        want = oracle_ref(width, *batch)
        assert_same(bucketed, want, "bucketed " + tag)
        assert_same(got, want, "noalloc " + tag)


def test_same_stream_back_to_back_without_sync(hh):
    # one stream orders the calls: the second call's plan reset runs after
    # the first call's kernels, whatever their sizes
    a, b = _batch(seed=73, n=2000, long_n=4), _batch(seed=74, n=300, long_n=1)
    da, db = batch_to_device(*a), batch_to_device(*b)
    oa = torch.empty((a[3].size, 2), dtype=torch.int64, device="cuda")
    ob = torch.empty((b[3].size, 2), dtype=torch.int64, device="cuda")
    announce("noalloc back-to-back", a[3].size, b[3].size)
    for _ in range(3):
        hh.hash_noalloc(da[0], da[2], da[3], da[4], da[1], 2, oa)
        hh.hash_noalloc(db[0], db[2], db[3], db[4], db[1], 2, ob)
    torch.cuda.synchronize()
    assert_same(hh.to_u64(oa), oracle_ref(2, *a), "first batch")
    assert_same(hh.to_u64(ob), oracle_ref(2, *b), "second batch")


def test_largest_allowed_batch(hh):
    n = hh.NOALLOC_MAX_MSGS
    rng = np.random.default_rng(75)
    lens = rng.integers(0, 300, n).astype(np.uint64)
    lens[rng.integers(0, n, 4)] = 200_000
    offsets = (np.cumsum(lens) - lens).astype(np.uint64)
    data = np.frombuffer(rng.bytes(int(lens.sum()) + 3), np.uint8)
    keys = rng.integers(0, 2**64, size=(1, 4), dtype=np.uint64)
    batch = (keys, None, data, offsets, lens)
    announce("noalloc largest batch", n)
    got, bucketed = _both(hh, 1, batch)
    assert np.array_equal(got, bucketed)
    want = oracle_ref(1, *batch)
    assert_same(got, want, "noalloc largest batch")
    k, ki, d, o, L = batch_to_device(*batch)
    with pytest.raises(hh.HHError):
        over = torch.cat([o, o[:1]])
        hh.hash_noalloc(k, d, over, torch.cat([L, L[:1]]), None, 1)
