"""Bit-exact parity of every HIP path with the CPU oracle (GPU required).

HighwayHash is integer arithmetic with exactly one correct output per
(key, message, width), so the tolerance is zero bits everywhere."""
import numpy as np
import pytest
import torch

import oracle
from _golden import load_vectors
from _gpu import (PATHS, announce, assert_same, batch_to_device, oracle_ref, require_gpu, run)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh():
    return require_gpu()


def _pack(msgs, gap_rng=None):
    """Pack byte arrays into one buffer, optionally with random gaps so that
    starts take every alignment."""
    offsets, lengths, chunks, pos = [], [], [], 0
    for m in msgs:
        if gap_rng is not None:
            g = int(gap_rng.integers(0, 16))
            chunks.append(np.full(g, 0xA5, np.uint8))
            pos += g
        offsets.append(pos)
        lengths.append(m.size)
        chunks.append(m)
        pos += m.size
    data = np.concatenate(chunks) if chunks else np.zeros(0, np.uint8)
    return data, np.array(offsets, np.uint64), np.array(lengths, np.uint64)


def test_golden_vectors_every_path(hh):
    vecs = load_vectors()
    keys = np.stack([v[0] for v in vecs])
    key_idx = np.arange(len(vecs), dtype=np.uint32)
    data, offsets, lengths = _pack([v[1] for v in vecs], np.random.default_rng(1))
    want = np.array([v[2] for v in vecs], dtype=np.uint64)
    for path in PATHS:
        for width in (1, 2, 4):
            announce("golden", path, width)
            got = run(hh, path, width, keys, key_idx, data, offsets, lengths)
            assert_same(got, want[:, :width], "golden %s w%d" % (path, width))


@pytest.mark.parametrize("path", PATHS)
def test_mixed_lengths_and_alignments(hh, path):
    rng = np.random.default_rng(2)
    n = 3000
    lengths = np.concatenate([np.arange(0, 700), rng.integers(0, 300, n - 700 - 20),
                              rng.integers(1000, 100000, 20)]).astype(np.uint64)
    rng.shuffle(lengths)
    msgs = [np.frombuffer(rng.bytes(int(L)), np.uint8) for L in lengths]
    data, offsets, lengths = _pack(msgs, rng)
    keys = rng.integers(0, 2**64, size=(37, 4), dtype=np.uint64)
    key_idx = rng.integers(0, 37, size=n, dtype=np.uint32)
    for width in (1, 2, 4):
        announce("mixed", path, width)
        want = oracle_ref(width, keys, key_idx, data, offsets, lengths)
        got = run(hh, path, width, keys, key_idx, data, offsets, lengths)
        assert_same(got, want, "mixed %s w%d" % (path, width))


@pytest.mark.parametrize("path", PATHS)
def test_packet_counts_around_prefetch_depths(hh, path):
    # whole-packet counts 0..80 times several tail sizes, then 81..400 (the
    # loop/drain boundaries of every ring depth up to 96 packets in flight:
    # the loop runs from 5/3 of a ring and steps by a ring) at every start
    # misalignment
    rng = np.random.default_rng(3)
    lens = []
    for k in range(0, 81):
        for r in (0, 1, 3, 4, 5, 28, 29, 31):
            lens.append(32 * k + r)
    for k in range(81, 401):
        for r in (0, 5, 31):
            lens.append(32 * k + r)
    msgs = [np.frombuffer(rng.bytes(L), np.uint8) for L in lens]
    data, offsets, lengths = _pack(msgs, rng)
    keys = rng.integers(0, 2**64, size=(1, 4), dtype=np.uint64)
    announce("prefetch-depths", path)
    want = oracle_ref(1, keys, None, data, offsets, lengths)
    got = run(hh, path, 1, keys, None, data, offsets, lengths)
    assert_same(got, want, "depths " + path)


@pytest.mark.parametrize("path", PATHS)
def test_messages_ending_at_end_of_buffer(hh, path):
    rng = np.random.default_rng(4)
    key = rng.integers(0, 2**64, size=(1, 4), dtype=np.uint64)
    for L in list(range(0, 70)) + [95, 96, 97, 255, 256, 257, 1023]:
        for mis in range(4):
            data = np.frombuffer(rng.bytes(L + mis), np.uint8)
            offsets = np.array([mis], np.uint64)
            lengths = np.array([L], np.uint64)
            want = oracle_ref(1, key, None, data, offsets, lengths)
            got = run(hh, path, 1, key, None, data, offsets, lengths)
            assert_same(got, want, "end-of-buffer L=%d mis=%d %s" % (L, mis, path))


def test_empty_batch_and_empty_messages(hh):
    k, ki, d, o, L = batch_to_device(np.ones((1, 4), np.uint64), None, np.zeros(4, np.uint8),
                                     np.zeros(0, np.uint64), np.zeros(0, np.uint64))
    out = hh.hash(k, d, o, L)
    assert out.shape == (0, 1)
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 2**64, size=(5, 4), dtype=np.uint64)
    key_idx = np.arange(100, dtype=np.uint32) % 5
    offsets = rng.integers(0, 4, 100).astype(np.uint64)
    lengths = np.zeros(100, np.uint64)
    data = np.zeros(4, np.uint8)
    want = oracle_ref(4, keys, key_idx, data, offsets, lengths)
    for path in PATHS:
        got = run(hh, path, 4, keys, key_idx, data, offsets, lengths)
        assert_same(got, want, "empty messages " + path)


def test_out_of_contract_inputs_are_clamped(hh):
    rng = np.random.default_rng(6)
    keys = rng.integers(0, 2**64, size=(3, 4), dtype=np.uint64)
    data = np.frombuffer(rng.bytes(100), np.uint8)
    offsets = np.array([0, 90, 150, 10], np.uint64)
    lengths = np.array([10, 50, 5, 20], np.uint64)   # 2nd runs past the end, 3rd starts past it
    key_idx = np.array([0, 1, 2, 7], np.uint32)       # 7 >= n_keys: clamped to 2
    c_off = np.minimum(offsets, 100)
    c_len = np.minimum(lengths, 100 - c_off)
    c_idx = np.minimum(key_idx, 2)
    want = oracle_ref(1, keys, c_idx, data, c_off, c_len)
    for path in PATHS:
        got = run(hh, path, 1, keys, key_idx, data, offsets, lengths)
        assert_same(got, want, "clamped " + path)


def test_uniform_plain_kernel(hh):
    # lengths of 8 packets or more take the deep-ring kernel: cover the switch,
    # every loop/drain boundary of its 8-packet ring after the 2 packets loaded
    # up front, and a few long lengths
    rng = np.random.default_rng(7)
    deep = [32 * k + r for k in (7, 8, 9, 17, 18, 19, 25, 26, 27, 34, 35, 36) for r in (0, 13)]
    for L in [0, 1, 8, 31, 32, 33, 64, 100, 1024] + deep + [4097, 65541, 300007]:
        n = 777 if L <= 4097 else 40
        keys = rng.integers(0, 2**64, size=(4, 4), dtype=np.uint64)
        key_idx = rng.integers(0, 4, n, dtype=np.uint32)
        data = np.frombuffer(rng.bytes(n * L + 3), np.uint8)
        offsets = (np.arange(n, dtype=np.uint64) * np.uint64(L) + np.uint64(3 if L else 0))
        lengths = np.full(n, L, np.uint64)
        want = oracle_ref(1, keys, key_idx, data, offsets, lengths)
        k, ki, d, o, _ = batch_to_device(keys, key_idx, data, offsets, lengths)
        out = hh.hash64_uniform(k, d, o, L, ki)
        torch.cuda.synchronize()
        assert_same(hh.to_u64(out), want, "uniform L=%d" % L)


def test_state_api_equals_one_shot(hh):
    rng = np.random.default_rng(8)
    n = 300
    keys = rng.integers(0, 2**64, size=(9, 4), dtype=np.uint64)
    key_idx = rng.integers(0, 9, n, dtype=np.uint32)
    lens = rng.integers(0, 5000, n).astype(np.uint64)
    msgs = [np.frombuffer(rng.bytes(int(L)), np.uint8) for L in lens]
    data, offsets, lengths = _pack(msgs, rng)
    widths = np.array([1, 2, 4], np.uint8)[rng.integers(0, 3, n)]
    want = {w: oracle_ref(w, keys, key_idx, data, offsets, lengths) for w in (1, 2, 4)}
    k, ki, d, o, L = batch_to_device(keys, key_idx, data, offsets, lengths)
    states = hh.state_init(k, n, ki)
    # feed each message in chunks of 32*c bytes; messages finish at random steps
    pos = np.zeros(n, np.uint64)
    active = np.ones(n, bool)
    step = 0
    out = torch.zeros((n, 4), dtype=torch.int64, device="cuda")
    while active.any():
        step += 1
        upd_idx, upd_off, upd_len, fin_idx, fin_off, fin_len = [], [], [], [], [], []
        for j in np.nonzero(active)[0]:
            remaining = int(lengths[j] - pos[j])
            chunk = 32 * int(rng.integers(0, 40))
            if chunk >= remaining or rng.random() < 0.1:
                fin_idx.append(j)
                fin_off.append(int(offsets[j] + pos[j]))
                fin_len.append(remaining)
                active[j] = False
            else:
                upd_idx.append(j)
                upd_off.append(int(offsets[j] + pos[j]))
                upd_len.append(chunk)
                pos[j] += chunk
        if upd_idx:
            hh.state_update(states, d, torch.tensor(upd_off, dtype=torch.int64, device="cuda"),
                            torch.tensor(upd_len, dtype=torch.int64, device="cuda"),
                            torch.tensor(upd_idx, dtype=torch.int32, device="cuda"))
        if fin_idx:
            fi = np.array(fin_idx)
            hh.state_final(states, d, torch.tensor(fin_off, dtype=torch.int64, device="cuda"),
                           torch.tensor(fin_len, dtype=torch.int64, device="cuda"),
                           torch.from_numpy(widths[fi]).cuda(),
                           out.view(-1), torch.from_numpy(4 * fi.astype(np.uint64)).view(
                               torch.int64).cuda(),
                           torch.tensor(fin_idx, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    got = hh.to_u64(out)
    for j in range(n):
        w = int(widths[j])
        assert [int(x) for x in got[j, :w]] == [int(x) for x in want[w][j]], j


@pytest.mark.parametrize("path", PATHS)
def test_prepared_call_repeats_the_same_hash(hh, path):
    # hh.prepare checks and marshals once; each call() makes the same C call
    # on the given stream and writes the same exact results
    rng = np.random.default_rng(21)
    lengths = rng.integers(0, 3000, 900).astype(np.uint64)
    msgs = [np.frombuffer(rng.bytes(int(L)), np.uint8) for L in lengths]
    data, offsets, lengths = _pack(msgs, rng)
    keys = rng.integers(0, 2**64, size=(3, 4), dtype=np.uint64)
    key_idx = rng.integers(0, 3, lengths.size, dtype=np.uint32)
    want = oracle_ref(2, keys, key_idx, data, offsets, lengths)
    k, ki, d, o, L = batch_to_device(keys, key_idx, data, offsets, lengths)
    stream = torch.cuda.Stream()
    announce("prepared", path)
    call = hh.prepare(k, d, o, L, ki, 2, path, None, stream)
    for _ in range(3):
        call.out.fill_(-1)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            got = call()
        stream.synchronize()
        assert_same(hh.to_u64(got), want, "prepared " + path)
