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
    dict(long_ring=36), dict(long_ring=48), dict(long_ring=96), dict(waves_per_cu=8),
    dict(waves_per_cu=12, long_ring=48), dict(lane4_min_bytes=0), dict(lane4_min_bytes=1),
    dict(lane4_min_bytes=4096), dict(lane4_min_bytes=1 << 30), dict(isolate_long=0),
    dict(isolate_long=1, waves_per_cu=2), dict(isolate_long=1, waves_per_cu=8)])
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


def _isolation_batch(n_top, top_lo, top_hi, n_rest, rest_hi, seed):
    rng = np.random.default_rng(seed)
    lens = np.concatenate([rng.integers(top_lo, top_hi, n_top),
                           rng.integers(0, rest_hi, n_rest)]).astype(np.uint64)
    rng.shuffle(lens)
    offsets = (np.cumsum(lens) - lens).astype(np.uint64) + rng.integers(0, 3, lens.size).astype(
        np.uint64)
    data = np.frombuffer(rng.bytes(int(offsets[-1] + lens[-1]) + 8), np.uint8).copy()
    keys = rng.integers(0, 2**64, size=(3, 4), dtype=np.uint64)
    key_idx = rng.integers(0, 3, lens.size, dtype=np.uint32)
    return keys, key_idx, data, offsets, lens


@pytest.mark.parametrize("case", [
    # several critical items (top octave spans 4 items of 16)
    dict(n_top=50, top_lo=200000, top_hi=400000, n_rest=3000, rest_hi=20000, seed=3),
    # one critical item that is not full
    dict(n_top=5, top_lo=300000, top_hi=310000, n_rest=500, rest_hi=5000, seed=4),
    # more top-octave items than a quarter of the CUs: isolation switches off
    dict(n_top=1500, top_lo=4096, top_hi=8192, n_rest=3000, rest_hi=4096, seed=5),
    # a batch too heavy for the CUs left over: isolation switches off
    dict(n_top=20, top_lo=1024, top_hi=1100, n_rest=40000, rest_hi=500, seed=6),
])
def test_isolation_regimes_bit_exact(hh, case):
    announce("isolation", case)
    keys, key_idx, data, offsets, lengths = _isolation_batch(**case)
    want = oracle_ref(4, keys, key_idx, data, offsets, lengths)
    k, ki, d, o, L = batch_to_device(keys, key_idx, data, offsets, lengths)
    base = hh.get_tuning()
    try:
        for iso in (1, 0):
            hh.set_tuning(**dict(base, isolate_long=iso, waves_per_cu=4))
            got = hh.to_u64(hh.hash(k, d, o, L, ki, 4, "bucketed"))
            assert_same(got, want, "isolate_long=%d" % iso)
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


def test_calls_after_release_allocate_afresh(hh):
    # hh_release frees every workspace and cached graph; the next calls, on
    # the stream used before and on another one, build new ones and hash
    # exactly, eagerly and as replayed graphs
    base = hh.get_tuning()
    keys, key_idx, data, offsets, lengths = _batch(seed=61)
    want = oracle_ref(1, keys, key_idx, data, offsets, lengths)
    k, ki, d, o, L = batch_to_device(keys, key_idx, data, offsets, lengths)
    side = torch.cuda.Stream()
    try:
        for use_graph in (0, 1):
            hh.set_tuning(**dict(base, use_graph=use_graph))
            for rep in range(2):
                announce("release", use_graph, rep)
                with torch.cuda.stream(side):
                    before = hh.hash(k, d, o, L, ki, 1, "auto")
                torch.cuda.synchronize()
                hh.release()
                with torch.cuda.stream(side):
                    after_side = hh.hash(k, d, o, L, ki, 1, "auto")
                after_default = hh.hash(k, d, o, L, ki, 1, "auto")
                torch.cuda.synchronize()
                for name, got in (("before", before), ("side", after_side),
                                  ("default", after_default)):
                    assert_same(hh.to_u64(got), want, "graph %d rep %d %s" % (use_graph, rep,
                                                                               name))
    finally:
        hh.set_tuning(**base)
        torch.cuda.synchronize()


def test_back_to_back_calls_share_the_plan(hh):
    # consecutive calls on one stream reuse one workspace; each call's last
    # wave leaves the plan zeroed for the next one, so batches of different
    # sizes and mixes queued without any synchronisation must all be exact
    announce("back-to-back")
    batches = []
    for seed, n in ((51, 300), (52, 2500), (53, 200), (54, 1200), (55, 2500)):
        keys, key_idx, data, offsets, lengths = _batch(seed=seed, n=n)
        want = oracle_ref(1, keys, key_idx, data, offsets, lengths)
        batches.append((batch_to_device(keys, key_idx, data, offsets, lengths), want))
    torch.cuda.synchronize()
    outs = []
    for _ in range(3):
        for (k, ki, d, o, L), _w in batches:
            outs.append(hh.hash(k, d, o, L, ki, 1, "bucketed"))
    torch.cuda.synchronize()
    for i, out in enumerate(outs):
        assert_same(hh.to_u64(out), batches[i % len(batches)][1], "call %d" % i)


@pytest.mark.parametrize("n_streams", [2, 3, 4, 6])
def test_concurrent_calls_on_several_streams(hh, n_streams):
    # independent batches issued round-robin on several streams overlap on
    # the GPU; each stream has its own workspace, and a stream's first call
    # (which zeroes its new plan on that stream) runs while the others are in
    # flight.  Every call writes its own output; every output is exact.
    keys, key_idx, data, offsets, lengths = _batch(seed=40 + n_streams, n=1600)
    base = hh.get_tuning()
    hh.set_tuning(**dict(base, lane4_min_bytes=0, use_graph=0))
    try:
        want = oracle_ref(2, keys, key_idx, data, offsets, lengths)
        k, ki, d, o, L = batch_to_device(keys, key_idx, data, offsets, lengths)
        streams = [torch.cuda.Stream() for _ in range(n_streams)]
        n_calls = 4 * n_streams
        outs = [torch.full((lengths.size, 2), -1, dtype=torch.int64, device="cuda")
                for _ in range(n_calls)]
        torch.cuda.synchronize()
        announce("concurrent streams", n_streams, n_calls)
        for i in range(n_calls):
            with torch.cuda.stream(streams[i % n_streams]):
                hh.hash(k, d, o, L, ki, 2, "bucketed", outs[i])
        torch.cuda.synchronize()
        for i, out in enumerate(outs):
            assert_same(hh.to_u64(out), want, "streams %d call %d" % (n_streams, i))
    finally:
        hh.set_tuning(**base)


def test_independent_streams_overlap_and_hash_exactly(hh):
    # streams chosen by measured concurrency: distinct, and a tiny kernel on
    # one completes while a few-millisecond hash runs on another
    import time
    streams = hh.independent_streams(2, avoid=[])
    assert len(streams) == 2
    assert streams[0].cuda_stream != streams[1].cuda_stream
    n = 1 << 22
    buf = torch.zeros(n, dtype=torch.uint8, device="cuda")
    keys = torch.zeros((1, 4), dtype=torch.int64, device="cuda")
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    ln = torch.full((1,), n, dtype=torch.int64, device="cuda")
    out = torch.empty((1, 1), dtype=torch.int64, device="cuda")
    tick = torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(streams[0]):
        hh.hash(keys, buf, off, ln, None, 1, "lane4", out)
        e0 = torch.cuda.Event()
        e0.record()
    with torch.cuda.stream(streams[1]):
        tick.add_(1)
        e1 = torch.cuda.Event()
        e1.record()
    t0 = time.perf_counter()
    while not e1.query() and time.perf_counter() - t0 < 0.5:
        time.sleep(1e-4)
    assert e1.query()
    assert not e0.query(), "the tiny kernel waited for the long hash"
    torch.cuda.synchronize()
    keys_, key_idx, data, offsets, lengths = _batch(seed=77, n=600)
    want = oracle_ref(1, keys_, key_idx, data, offsets, lengths)
    k, ki, d, o, L = batch_to_device(keys_, key_idx, data, offsets, lengths)
    for s in streams:
        with torch.cuda.stream(s):
            got = hh.hash(k, d, o, L, ki, 1, "bucketed")
        s.synchronize()
        assert_same(hh.to_u64(got), want, "stream %x" % s.cuda_stream)


def test_hash_many_equals_each_batch_alone(hh):
    # independent batches of different shapes hashed concurrently on several
    # streams give exactly what each batch gives alone (and the oracle)
    batches, wants = [], []
    for seed, n in ((81, 900), (82, 50), (83, 2500), (84, 1), (85, 700)):
        keys, key_idx, data, offsets, lengths = _batch(seed=seed, n=max(n, 300))
        keys_, key_idx_, offsets_, lengths_ = keys, key_idx[:n], offsets[:n], lengths[:n]
        wants.append(oracle_ref(2, keys_, key_idx_, data, offsets_, lengths_))
        k, ki, d, o, L = batch_to_device(keys_, key_idx_, data, offsets_, lengths_)
        batches.append((k, d, o, L, ki))
    outs = hh.hash_many(batches, width=2, n_streams=3)
    torch.cuda.synchronize()
    assert len(outs) == len(batches)
    for i, (got, want) in enumerate(zip(outs, wants)):
        assert_same(hh.to_u64(got), want, "batch %d" % i)
    # twice in a row on the same streams
    outs2 = hh.hash_many(batches[::-1], width=2, n_streams=3)
    torch.cuda.synchronize()
    for i, (got, want) in enumerate(zip(outs2, wants[::-1])):
        assert_same(hh.to_u64(got), want, "second call batch %d" % i)


def test_calls_from_several_host_threads(hh):
    # four host threads, each with its own stream, call the bucketed path at
    # the same time (ctypes releases the GIL): workspaces are created and
    # looked up concurrently, every result is exact
    import threading
    keys, key_idx, data, offsets, lengths = _batch(seed=91, n=1200)
    want = oracle_ref(1, keys, key_idx, data, offsets, lengths)
    k, ki, d, o, L = batch_to_device(keys, key_idx, data, offsets, lengths)
    results, errors = {}, []

    def work(t):
        try:
            s = torch.cuda.Stream()
            outs = []
            with torch.cuda.stream(s):
                for _ in range(5):
                    outs.append(hh.hash(k, d, o, L, ki, 1, "bucketed"))
            s.synchronize()
            results[t] = [hh.to_u64(x) for x in outs]
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    assert not errors, errors
    assert sorted(results) == [0, 1, 2, 3]
    for t, outs in results.items():
        for i, got in enumerate(outs):
            assert_same(got, want, "thread %d call %d" % (t, i))


@pytest.mark.parametrize("shared", ["stream", "null"])
def test_host_threads_sharing_one_stream(hh, shared):
    # four host threads call the bucketed path on ONE stream (a shared torch
    # stream, or the null stream that is every thread's default), each with
    # its own batch of a different size, so the workspace is looked up, grown
    # and enqueued against from several threads at once; each call's
    # sequence must stay whole on the stream and every result exact
    import threading
    announce("threads sharing", shared)
    batches = [_batch(seed=95 + t, n=600 + 900 * t) for t in range(4)]
    wants = [oracle_ref(1, *b) for b in batches]
    devs = [batch_to_device(*b) for b in batches]
    stream = torch.cuda.Stream() if shared == "stream" else None
    results, errors = {}, []
    start = threading.Barrier(4)

    def work(t):
        try:
            k, ki, d, o, L = devs[t]
            outs = []
            start.wait(timeout=30)
            if stream is None:
                for _ in range(6):
                    outs.append(hh.hash(k, d, o, L, ki, 1, "bucketed"))
            else:
                with torch.cuda.stream(stream):
                    for _ in range(6):
                        outs.append(hh.hash(k, d, o, L, ki, 1, "bucketed"))
            results[t] = outs
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    torch.cuda.synchronize()
    assert not errors, errors
    assert sorted(results) == [0, 1, 2, 3]
    for t, outs in results.items():
        for i, got in enumerate(outs):
            assert_same(hh.to_u64(got), wants[t], "%s: thread %d call %d" % (shared, t, i))
