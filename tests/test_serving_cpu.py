"""The serving scheduler on a CPU stand-in backend: continuous batching gives
every request the same hash as hashing it alone, admission never exceeds the
budget, oversized requests are refused, and the arena allocator never hands
out overlapping regions."""
import numpy as np
import pytest

import oracle
from _serve_cpu import CpuBackend, VirtualClock
from paper_1612_06257_amd import serve, workloads


def _trace(n, rate, hi, seed=7):
    tr = workloads.serving_trace(n, rate, lo=1, hi=hi, n_keys=8, seed=seed)
    tr.lengths[::17] = 0  # some empty requests
    return tr


def _run(tr, budget, chunk, max_slots=64, reads_source=False):
    clock = VirtualClock()
    reqs = serve.requests_from_trace(tr)
    arena = budget
    be = CpuBackend(tr.keys, tr.data, arena, max_slots, clock, reads_source=reads_source)
    srv = serve.Server(be, budget_bytes=budget, chunk_bytes=chunk, clock=clock, sleep=clock.sleep)
    m = srv.run(reqs)
    return m, reqs, be


def test_arena_allocator_no_overlap_and_coalesces():
    rng = np.random.default_rng(1)
    a = serve.Arena(1 << 20)
    live = {}
    for step in range(2000):
        if live and (rng.random() < 0.45 or len(live) > 50):
            k = list(live)[int(rng.integers(0, len(live)))]
            off, n = live.pop(k)
            a.release(off, n)
        else:
            n = int(rng.integers(1, 40000))
            off = a.alloc(n)
            if off is not None:
                for o2, n2 in live.values():
                    r1 = (off, off + (n + 255) // 256 * 256)
                    r2 = (o2, o2 + (n2 + 255) // 256 * 256)
                    assert r1[1] <= r2[0] or r2[1] <= r1[0]
                live[step] = (off, n)
    for off, n in live.values():
        a.release(off, n)
    assert a.free == [(0, a.capacity)] and a.used == 0


def test_arena_batched_release_equals_one_by_one():
    # the scheduler returns a whole harvest at once: the free list after a
    # batched release equals the one after releasing the same spans singly
    rng = np.random.default_rng(2)
    a, b = serve.Arena(1 << 22), serve.Arena(1 << 22)
    live = []
    for step in range(3000):
        if live and rng.random() < 0.4:
            k = int(rng.integers(1, min(len(live), 40) + 1))
            idx = set(rng.choice(len(live), k, replace=False).tolist())
            out = [live[i] for i in sorted(idx)]
            live = [x for i, x in enumerate(live) if i not in idx]
            a.release_many(out)
            for off, n in out:
                b.release(off, n)
            assert a.free == b.free and a.used == b.used
        else:
            n = int(rng.integers(0, 30000))
            off_a, off_b = a.alloc(n), b.alloc(n)
            assert off_a == off_b
            if off_a is not None:
                live.append((off_a, n))
    a.release_many(live)
    assert a.free == [(0, a.capacity)] and a.used == 0


@pytest.mark.parametrize("chunk,reads_source", [(32, False), (256, False), (4096, False),
                                                (256, True)])
def test_results_equal_one_shot_hashes(chunk, reads_source):
    # reads_source: the kernels read each request where it arrived (device
    # ingress); the arena then only keeps the budget's books
    tr = _trace(250, 2000.0, hi=6000)
    m, reqs, be = _run(tr, budget=1 << 16, chunk=chunk, reads_source=reads_source)
    assert m["completed"] + m["rejected"] == len(reqs)
    assert m["rejected"] == 0
    for r in reqs:
        msg = tr.data[r.src:r.src + r.length]
        assert r.result == tuple(oracle.hash_words(tr.keys[r.key_idx], msg, r.width)), r.rid
    assert m["max_bytes_in_flight"] <= 1 << 16
    assert be.launches == m["iterations"]


@pytest.mark.parametrize("reads_source", [False, True])
def test_admission_respects_budget_and_back_pressure(reads_source):
    # with payloads copied into the arena, or read where they arrived (then
    # the budget's sum alone binds, with no arena range)
    tr = _trace(200, 1e6, hi=20000, seed=3)   # everything arrives at once
    budget = 40000
    m, reqs, be = _run(tr, budget=budget, chunk=512, reads_source=reads_source)
    assert m["max_bytes_in_flight"] <= budget
    assert m["max_bytes_in_flight"] > budget // 2   # the budget did bind
    big = [r for r in reqs if serve.Server.reservation(r.length) > budget]
    assert all(r.status == "rejected" for r in big)
    assert all(r.status == "done" for r in reqs if r not in big)
    for r in reqs:
        if r.status == "done":
            msg = tr.data[r.src:r.src + r.length]
            assert r.result == tuple(oracle.hash_words(tr.keys[r.key_idx], msg, r.width))


def test_result_alone_equals_result_in_mix():
    tr = _trace(60, 500.0, hi=3000, seed=11)
    m, reqs, _ = _run(tr, budget=1 << 15, chunk=64)
    for r in reqs[:12]:
        solo = workloads.Trace(tr.seed, tr.rate, np.zeros(1), tr.keys,
                               np.array([r.key_idx], np.uint32), np.array([r.width], np.uint8),
                               tr.data, np.array([r.src], np.uint64),
                               np.array([r.length], np.uint64))
        m1, reqs1, _ = _run(solo, budget=1 << 15, chunk=64)
        assert reqs1[0].result == r.result


def test_chunk_must_be_packet_multiple():
    clock = VirtualClock()
    be = CpuBackend(np.zeros((1, 4), np.uint64), np.zeros(0, np.uint8), 1024, 4, clock)
    with pytest.raises(ValueError):
        serve.Server(be, budget_bytes=1024, chunk_bytes=100)


def test_long_lane_results_equal_one_shot():
    # requests over 2 KiB advance in the long lane, 256 bytes per iteration,
    # beside the short ones (64 bytes per iteration); every result is exact
    # and a request never changes lane
    tr = _trace(200, 3000.0, hi=9000, seed=21)
    clock = VirtualClock()
    reqs = serve.requests_from_trace(tr)
    be = CpuBackend(tr.keys, tr.data, 1 << 17, 64, clock)
    srv = serve.Server(be, budget_bytes=1 << 17, chunk_bytes=64, long_chunk_bytes=256,
                       long_min_bytes=2048, clock=clock, sleep=clock.sleep)
    m = srv.run(reqs)
    assert m["completed"] == len(reqs)
    assert be.lane_launches[1] > 0 and be.lane_launches[0] > 0
    for r in reqs:
        msg = tr.data[r.src:r.src + r.length]
        assert r.result == tuple(oracle.hash_words(tr.keys[r.key_idx], msg, r.width)), r.rid


def test_collector_off_during_the_loop_and_restored():
    # the loop runs with Python's cyclic collector off (a full pass can stop
    # it for tens of milliseconds) and leaves the collector as it found it
    import gc

    class Recording(CpuBackend):
        def launch(self, *a, **k):
            self.gc_states.add(gc.isenabled())
            return super().launch(*a, **k)

    tr = _trace(60, 2000.0, hi=3000, seed=41)
    for enabled in (True, False):
        (gc.enable if enabled else gc.disable)()
        try:
            clock = VirtualClock()
            reqs = serve.requests_from_trace(tr)
            be = Recording(tr.keys, tr.data, 1 << 16, 64, clock)
            be.gc_states = set()
            srv = serve.Server(be, budget_bytes=1 << 16, chunk_bytes=64, clock=clock,
                               sleep=clock.sleep)
            assert srv.run(reqs)["completed"] == len(reqs)
            assert be.gc_states == {False}
            assert gc.isenabled() == enabled
        finally:
            gc.enable()


@pytest.mark.parametrize("reads_source", [False, True])
def test_feed_mode_results_equal_one_shot(reads_source):
    # long requests go whole to the feed, longest first, each exactly once,
    # from the arena after admission or straight from where they arrived;
    # every result is exact
    from _serve_cpu import FeedCpuBackend
    tr = _trace(300, 3000.0, hi=9000, seed=51)
    clock = VirtualClock()
    reqs = serve.requests_from_trace(tr)
    be = FeedCpuBackend(tr.keys, tr.data, 1 << 18, 128, clock, reads_source=reads_source)
    srv = serve.Server(be, budget_bytes=1 << 18, chunk_bytes=64, long_min_bytes=2048,
                       clock=clock, sleep=clock.sleep)
    assert srv.long_mode == "feed"
    m = srv.run(reqs)
    assert m["completed"] == len(reqs)
    assert be.submits and be.lane_launches[1] == 0
    n_long = sum(r.length > 2048 for r in reqs)
    assert sum(len(g) for g, _ in be.submits) == n_long
    for g, lens in be.submits:
        assert np.all(np.diff(lens.astype(np.int64)) <= 0)   # longest first
    for r in reqs:
        msg = tr.data[r.src:r.src + r.length]
        assert r.result == tuple(oracle.hash_words(tr.keys[r.key_idx], msg, r.width)), r.rid


@pytest.mark.parametrize("feed", [False, True])
def test_whole_lane_results_equal_one_shot(feed):
    # requests up to whole_max_bytes are hashed whole in one launch each pass,
    # from where they arrived, with no admission and no state; the others
    # take lane 0 (and the feed); every result is exact
    from _serve_cpu import FeedCpuBackend
    tr = _trace(300, 3000.0, hi=9000, seed=57)
    clock = VirtualClock()
    reqs = serve.requests_from_trace(tr)
    cls = FeedCpuBackend if feed else CpuBackend
    be = cls(tr.keys, tr.data, 1 << 18, 128, clock, reads_source=True, whole=True)
    srv = serve.Server(be, budget_bytes=1 << 18, chunk_bytes=64, long_min_bytes=2048,
                       whole_max_bytes=256, clock=clock, sleep=clock.sleep)
    m = srv.run(reqs)
    assert m["completed"] == len(reqs) and m["whole_launches"] == len(be.whole_launched)
    lens = np.concatenate(be.whole_launched)
    assert lens.size == sum(r.length <= 256 for r in reqs) and lens.max() <= 256
    # whole-lane requests were never admitted (no state was reset for
    # them), nor were the feed's, which it also reads where they arrived
    admitted = sum(256 < r.length and (r.length <= 2048 or not feed) for r in reqs)
    assert be.admitted == admitted
    for r in reqs:
        msg = tr.data[r.src:r.src + r.length]
        assert r.result == tuple(oracle.hash_words(tr.keys[r.key_idx], msg, r.width)), r.rid
    with pytest.raises(ValueError):   # the whole lane needs a backend that has one
        serve.Server(CpuBackend(tr.keys, tr.data, 1 << 17, 64, clock), budget_bytes=1 << 17,
                     whole_max_bytes=256)


def test_chunked_long_lane_still_selectable():
    from _serve_cpu import FeedCpuBackend
    tr = _trace(80, 3000.0, hi=9000, seed=53)
    clock = VirtualClock()
    reqs = serve.requests_from_trace(tr)
    be = FeedCpuBackend(tr.keys, tr.data, 1 << 17, 64, clock)
    srv = serve.Server(be, budget_bytes=1 << 17, chunk_bytes=64, long_chunk_bytes=256,
                       long_min_bytes=2048, clock=clock, sleep=clock.sleep, long_mode="chunks")
    assert srv.run(reqs)["completed"] == len(reqs)
    assert not be.submits and be.lane_launches[1] > 0
    for r in reqs:
        msg = tr.data[r.src:r.src + r.length]
        assert r.result == tuple(oracle.hash_words(tr.keys[r.key_idx], msg, r.width)), r.rid
    with pytest.raises(ValueError):
        serve.Server(CpuBackend(tr.keys, tr.data, 1 << 17, 64, clock), budget_bytes=1 << 17,
                     long_mode="feed")


def test_stalled_loop_raises():
    # a feed whose results never appear: the loop gives up after stall_s of
    # virtual time instead of polling for ever
    from _serve_cpu import FeedCpuBackend

    class Stuck(FeedCpuBackend):
        def feed_submit(self, slots, offsets, lengths, widths, key_idx):
            t = self.next_ticket
            self.next_ticket += len(slots)
            return t

    tr = _trace(40, 1000.0, hi=9000, seed=61)
    clock = VirtualClock()
    be = Stuck(tr.keys, tr.data, 1 << 18, 64, clock)
    srv = serve.Server(be, budget_bytes=1 << 18, chunk_bytes=64, long_min_bytes=2048,
                       clock=clock, sleep=clock.sleep, stall_s=0.5)
    with pytest.raises(RuntimeError, match="no request finished"):
        srv.run(serve.requests_from_trace(tr))


def test_timer_slack_set_and_restored():
    # the loop sets a fine timer slack for real sleeps and puts the previous
    # one back (where prctl is available; else the call reports -1)
    prev = serve._timer_slack(1000)
    if prev < 0:
        pytest.skip("timer slack cannot be read here")
    try:
        assert serve._timer_slack(prev) == 1000
    finally:
        serve._timer_slack(prev)
