"""The serving loop on the GPU: every request's result in the mixed,
continuously batched run equals the same request hashed alone (one-shot
kernel) and the oracle, bit for bit; admission stays within the budget."""
import numpy as np
import pytest
import torch

import oracle
from _gpu import announce, require_gpu
from paper_1612_06257_amd import serve, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh():
    return require_gpu()


@pytest.mark.parametrize("source,long_chunk,long_mode,whole_max", [
    ("device", 1 << 20, "feed", None), ("host", 1 << 20, "feed", None),
    ("device", 1 << 20, "chunks", None), ("host", 1 << 20, "chunks", None),
    ("device", 8192, "chunks", None), ("device", 1 << 20, "feed", 0),
    ("device", 1 << 20, "feed", 16384)])
def test_serving_results_match_alone_and_oracle(hh, source, long_chunk, long_mode, whole_max):
    # requests over four chunks (16 KiB; chunked: sixteen, 64 KiB) take the
    # long lane (its own stream): whole, in the feed's persistent kernel, or
    # in chunked iterations (with 8 KiB chunks, several long-lane iterations
    # beside the short ones); with device ingress, requests up to 8 KiB (or
    # whole_max; 0: none) take the whole lane
    announce("serving", source, long_chunk, long_mode, whole_max)
    tr = workloads.serving_trace(400, 20000.0, lo=1, hi=200000, n_keys=16, seed=99)
    tr.lengths[::23] = 0
    budget = 8 << 20
    backend = serve.GpuBackend(tr.keys, tr.data, budget, 256, source)
    srv = serve.Server(backend, budget_bytes=budget, chunk_bytes=4096,
                       long_chunk_bytes=long_chunk, long_mode=long_mode,
                       whole_max_bytes=whole_max)
    reqs = serve.requests_from_trace(tr)
    try:
        m = srv.run(reqs)
    finally:
        backend.close()
    assert m["completed"] == len(reqs)
    assert m["max_bytes_in_flight"] <= budget
    assert (m["whole_launches"] > 0) == (source == "device" and whole_max != 0)
    # alone: each request through the one-shot batched kernel, one message per call
    keys = torch.from_numpy(tr.keys).view(torch.int64).cuda()
    data = torch.from_numpy(tr.data).cuda()
    for r in reqs:
        msg = tr.data[r.src:r.src + r.length]
        want = tuple(oracle.hash_words(tr.keys[r.key_idx], msg, r.width))
        assert r.result == want, r.rid
    sample = reqs[::7]
    offs = torch.tensor([r.src for r in sample], dtype=torch.int64, device="cuda")
    lens = torch.tensor([r.length for r in sample], dtype=torch.int64, device="cuda")
    kidx = torch.tensor([r.key_idx for r in sample], dtype=torch.int32, device="cuda")
    one = hh.to_u64(hh.hash(keys, data, offs, lens, kidx, 4))
    for i, r in enumerate(sample):
        assert tuple(int(x) for x in one[i][:r.width]) == r.result


def test_copy_segments_matches_slices(hh):
    announce("copy_segments")
    rng = np.random.default_rng(5)
    src = rng.integers(0, 256, 1 << 20, dtype=np.uint8)
    n = 700
    lens = rng.integers(0, 9000, n)
    lens[::50] = 0
    lens[1::50] = 7                               # shorter than one word
    soff = rng.integers(0, src.size - 9000, n)
    # disjoint destinations at odd offsets, one segment running past the end
    dst_size = int(lens.sum()) + 3 * n + 100
    doff = np.cumsum(np.concatenate([[1], lens[:-1] + 3]))
    doff_last = dst_size - 5
    doff[-1] = doff_last
    lens[-1] = 40                                  # clamped to the 5 bytes left
    want = np.zeros(dst_size, np.uint8)
    for s, d_, L in zip(soff, doff, lens):
        L = min(L, dst_size - d_)
        want[d_:d_ + L] = src[s:s + L]
    dst = torch.zeros(dst_size, dtype=torch.uint8, device="cuda")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int64)).cuda()
    s_dev = torch.from_numpy(src).cuda()
    # the launch-shape hint changes nothing but speed
    for hint in (0, 9000, 1 << 30):
        dst.zero_()
        hh.copy_segments(dst, s_dev, t(soff), t(doff), t(lens), hint)
        assert np.array_equal(dst.cpu().numpy(), want), hint


def test_state_init_into_slots(hh):
    announce("state_init slots")
    rng = np.random.default_rng(6)
    keys = torch.from_numpy(rng.integers(0, 2**64, (5, 4), dtype=np.uint64)).view(
        torch.int64).cuda()
    n = 90
    kidx = torch.from_numpy(rng.integers(0, 5, n).astype(np.int32)).cuda()
    slots = torch.from_numpy(rng.permutation(200)[:n].astype(np.int32)).cuda()
    dense = hh.state_init(keys, n, kidx)
    states = torch.full((200, hh.STATE_WORDS), 7, dtype=torch.int64, device="cuda")
    hh.state_init(keys, n, kidx, states, slots)
    torch.cuda.synchronize()
    assert torch.equal(states[slots.long()], dense)
    untouched = torch.ones(200, dtype=torch.bool, device="cuda")
    untouched[slots.long()] = False
    assert bool((states[untouched] == 7).all())


def test_raw_calls_on_pinned_item_lists_match_tensor_calls(hh):
    # the serving loop passes the device addresses of pinned host arrays
    # (item lists in, hashes out) to hh_hash_path and hh_state_init: same
    # results as the tensor calls on device arrays
    announce("raw calls on pinned memory")
    rng = np.random.default_rng(13)
    n = 300
    keys_np = rng.integers(0, 2**64, (7, 4), dtype=np.uint64)
    keys = torch.from_numpy(keys_np).view(torch.int64).cuda()
    lens = rng.integers(0, 9000, n)
    lens[::31] = 0
    offs = np.concatenate([[0], np.cumsum(lens[:-1] + 5)])
    data_np = rng.integers(0, 256, int(offs[-1] + lens[-1] + 5), dtype=np.uint8)
    data = torch.from_numpy(data_np).cuda()
    kidx = rng.integers(0, 7, n).astype(np.int32)
    pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
    p_offs, p_lens, p_kidx = pin(offs.astype(np.int64)), pin(lens.astype(np.int64)), pin(kidx)
    p_out = torch.zeros((n, 4), dtype=torch.int64).pin_memory()
    dev = hh.pinned_device_pointer
    stream = torch.cuda.current_stream().cuda_stream
    hh.hash_raw(keys, data, dev(p_kidx), dev(p_offs), dev(p_lens), n, dev(p_out), 4, "lane4",
                stream)
    want = hh.hash(keys, data, p_offs.cuda(), p_lens.cuda(), p_kidx.cuda(), 4)
    torch.cuda.synchronize()
    assert torch.equal(p_out, want.cpu())
    for j in range(0, n, 37):
        msg = data_np[offs[j]:offs[j] + lens[j]]
        assert [int(x) for x in p_out[j].numpy().view(np.uint64)] == \
            oracle.hash_words(keys_np[kidx[j]], msg, 4)
    slots = pin(rng.permutation(500)[:n].astype(np.int32))
    states = torch.full((500, hh.STATE_WORDS), 3, dtype=torch.int64, device="cuda")
    hh.state_init_raw(keys, n, dev(p_kidx), states, dev(slots), stream)
    dense = hh.state_init(keys, n, p_kidx.cuda())
    torch.cuda.synchronize()
    assert torch.equal(states[slots.cuda().long()], dense)
    with pytest.raises(ValueError):
        hh.hash_raw(keys, data, 0, 0, dev(p_lens), n, dev(p_out), 4, "lane4", stream)


def test_state_indices_past_the_array_are_skipped(hh):
    announce("state bounds")
    rng = np.random.default_rng(12)
    keys = torch.from_numpy(rng.integers(0, 2**64, (2, 4), dtype=np.uint64)).view(
        torch.int64).cuda()
    data = torch.from_numpy(rng.integers(0, 256, 4096, dtype=np.uint8)).cuda()
    states = torch.full((8, hh.STATE_WORDS), 3, dtype=torch.int64, device="cuda")
    slots = torch.tensor([0, 8, 5, 1 << 30], dtype=torch.int32, device="cuda")
    hh.state_init(keys, 4, None, states, slots)
    offs = torch.tensor([0, 64, 128, 192], dtype=torch.int64, device="cuda")
    lens = torch.full((4,), 64, dtype=torch.int64, device="cuda")
    hh.state_update(states, data, offs, lens, slots)
    # out holds 6 words: item 0 (offset 0) fits, item 2 (offset 4) is cut to 2 words
    out = torch.full((6,), -1, dtype=torch.int64, device="cuda")
    oo = torch.tensor([0, 0, 4, 0], dtype=torch.int64, device="cuda")
    ww = torch.full((4,), 4, dtype=torch.uint8, device="cuda")
    hh.state_final(states, data, offs + 64, lens - 1, ww, out, oo, slots)
    torch.cuda.synchronize()
    rest = [i for i in range(8) if i not in (0, 5)]
    assert bool((states[rest] == 3).all())
    key = keys.cpu().numpy().view(np.uint64)[0]
    d = data.cpu().numpy()
    h0 = oracle.hash_words(key, d[0:64].tobytes() + d[64:127].tobytes(), 4)
    h2 = oracle.hash_words(key, d[128:192].tobytes() + d[192:255].tobytes(), 4)
    got = hh.to_u64(out).tolist()
    assert got[:4] == [int(x) for x in h0]
    assert got[4:6] == [int(x) for x in h2[:2]]


def test_state_step_mixed_equals_separate_calls(hh):
    announce("state_step mixed")
    rng = np.random.default_rng(13)
    keys = torch.from_numpy(rng.integers(0, 2**64, (3, 4), dtype=np.uint64)).view(
        torch.int64).cuda()
    data = torch.from_numpy(rng.integers(0, 256, 1 << 16, dtype=np.uint8)).cuda()
    n = 300
    kidx = torch.from_numpy(rng.integers(0, 3, n).astype(np.int32)).cuda()
    offs = torch.from_numpy(rng.integers(0, 60000, n).astype(np.int64)).cuda()
    widths = np.array([0, 1, 2, 4], np.uint8)[rng.integers(0, 4, n)]
    lens_np = rng.integers(0, 3000, n).astype(np.int64)
    lens_np[widths == 0] &= ~31                      # updates take whole packets
    lens = torch.from_numpy(lens_np).cuda()
    ww = torch.from_numpy(widths).cuda()
    a = hh.state_init(keys, n, kidx)
    b = a.clone()
    out_a = torch.full((n, 4), -1, dtype=torch.int64, device="cuda")
    out_b = out_a.clone()
    hh.state_step(a, data, offs, lens, ww, out_a.view(-1))
    upd = torch.from_numpy(np.flatnonzero(widths == 0).astype(np.int32)).cuda()
    fin = torch.from_numpy(np.flatnonzero(widths != 0).astype(np.int32)).cuda()
    hh.state_update(b, data, offs[upd.long()], lens[upd.long()], upd)
    hh.state_final(b, data, offs[fin.long()], lens[fin.long()], ww[fin.long()], out_b.view(-1),
                   4 * fin.long(), fin)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(out_a, out_b)
    # an update-only call needs no output buffer
    hh.state_step(a, data, offs[upd.long()], lens[upd.long()], ww[upd.long()], None, None, upd)
    hh.state_update(b, data, offs[upd.long()], lens[upd.long()], upd)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_widths_other_than_1_2_4_write_nothing(hh):
    # hh_state_final and hh_state_step: an item of width 3, 5, 8 or 255
    # writes no output word and leaves its state as it is; the valid items
    # of the same launch are unaffected
    announce("state widths out of contract")
    rng = np.random.default_rng(14)
    keys = torch.from_numpy(rng.integers(0, 2**64, (1, 4), dtype=np.uint64)).view(
        torch.int64).cuda()
    d_np = rng.integers(0, 256, 1 << 14, dtype=np.uint8)
    data = torch.from_numpy(d_np).cuda()
    widths = np.array([3, 1, 255, 2, 5, 4, 8, 0], np.uint8)
    n = widths.size
    offs_np = rng.integers(0, 10000, n).astype(np.int64)
    lens_np = rng.integers(1, 3000, n).astype(np.int64)
    lens_np[widths == 0] &= ~31
    offs, lens = torch.from_numpy(offs_np).cuda(), torch.from_numpy(lens_np).cuda()
    ww = torch.from_numpy(widths).cuda()
    key = keys.cpu().numpy().view(np.uint64)[0]
    for fn in ("final", "step"):
        states = hh.state_init(keys, n)
        before = states.clone()
        out = torch.full((n, 4), -7, dtype=torch.int64, device="cuda")
        if fn == "final":
            hh.state_final(states, data, offs, lens, ww, out.view(-1))
        else:
            hh.state_step(states, data, offs, lens, ww, out.view(-1))
        torch.cuda.synchronize()
        got = hh.to_u64(out)
        for k, w in enumerate(widths.tolist()):
            if w in (1, 2, 4):
                msg = d_np[offs_np[k]:offs_np[k] + lens_np[k]].tobytes()
                want = [int(x) for x in oracle.hash_words(key, msg, w)]
                assert got[k][:w].tolist() == want, (fn, k, w)
                assert (out[k, w:] == -7).all(), (fn, k, w)
            elif fn == "final" or w != 0:
                assert (out[k] == -7).all(), (fn, k, w)
        fin = torch.from_numpy(widths != 0).cuda() if fn == "step" else torch.ones(
            n, dtype=torch.bool, device="cuda")
        assert torch.equal(states[fin], before[fin]), fn


@pytest.mark.parametrize("arrivals,long_mode", [("saturation", "feed"), ("poisson", "feed"),
                                               ("saturation", "chunks"), ("poisson", "chunks")])
def test_serving_at_benchmark_settings(hh, arrivals, long_mode):
    # the settings the benchmark's serving runs use: 64 KiB chunks, 1 MiB
    # long-lane chunks, power-law lengths on [8 B, 16 MiB], 64 keys, widths
    # 1/2/4, device ingress (requests up to 8 KiB in the whole lane); a few
    # requests of 4-16 MiB span many long-lane iterations beside the short
    # ones.  Every result equals the oracle and
    # the request hashed on its own by the one-shot batched path.
    from paper_1612_06257_amd import workloads as W
    announce("serving at bench settings", arrivals, long_mode)
    tr = W.serving_trace(500, 40000.0, seed=W.SEED_BASE + 77, materialize=False)
    lens = tr.lengths.copy()
    lens[[3, 97, 211, 402]] = [1 << 24, (1 << 24) - 1, (5 << 20) + 17, (4 << 20) + 32]
    lens[[5, 6]] = [8, 31]
    rng = np.random.default_rng(77)
    tr.lengths = lens
    tr.offsets = (np.cumsum(lens) - lens).astype(np.uint64)
    tr.data = rng.integers(0, 256, int(lens.sum()), dtype=np.uint8)
    if arrivals == "saturation":
        tr.arrival_s[:] = 0.0
    m, reqs = serve.serve_trace(tr, chunk_bytes=1 << 16, long_chunk_bytes=1 << 20,
                                long_mode=long_mode)
    assert m["completed"] == len(reqs) == tr.n
    got = {r.rid: r.result for r in reqs}
    keys = torch.from_numpy(tr.keys).view(torch.int64).cuda()
    data = torch.from_numpy(tr.data).cuda()
    for w in (1, 2, 4):
        idx = np.flatnonzero(tr.width_words == w)
        want = oracle.batch(tr.keys, tr.key_idx[idx], tr.data, tr.offsets[idx], tr.lengths[idx],
                            w)
        alone = hh.to_u64(hh.hash(keys, data, torch.from_numpy(tr.offsets[idx].astype(
            np.int64)).cuda(), torch.from_numpy(tr.lengths[idx].astype(np.int64)).cuda(),
            torch.from_numpy(tr.key_idx[idx].astype(np.int32)).cuda(), w))
        torch.cuda.synchronize()
        for row, i in enumerate(idx.tolist()):
            assert got[i] == tuple(int(x) for x in want[row]), ("oracle", i, w, tr.lengths[i])
            assert got[i] == tuple(int(x) for x in alone[row]), ("alone", i, w, tr.lengths[i])
