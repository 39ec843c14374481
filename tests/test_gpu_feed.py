"""The feed (hh_feed_*): a persistent kernel that hashes long messages as they
are submitted.  Every result equals the oracle's; a message submitted while a
much longer one is being hashed finishes first; a wave's 16 places are reused
as messages finish; slots are reused; a launch that has ended by its time
limit is relaunched while messages wait."""
import time

import numpy as np
import pytest
import torch

from _gpu import announce, dev, oracle_ref, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hh():
    return require_gpu()


def _buffer(rng, lengths):
    lengths = np.asarray(lengths, np.uint64)
    offsets = np.zeros(lengths.size, np.uint64)
    if lengths.size > 1:
        offsets[1:] = np.cumsum(lengths[:-1] + np.uint64(3))  # starts at every alignment
    total = int(offsets[-1] + lengths[-1]) if lengths.size else 0
    data = np.frombuffer(rng.bytes(max(total, 1)), np.uint8)
    return data, offsets, lengths


def _wait(feed, slots, tickets, limit_s=20.0):
    """Poll until every slot shows its ticket (bounded); returns the rows."""
    t_end = time.monotonic() + limit_s
    while True:
        if np.all(feed.rows[slots, 4] == tickets):
            return feed.rows[slots, :4].copy()
        assert time.monotonic() < t_end, "results did not arrive"
        feed.poll()
        time.sleep(1e-4)


def _submit_groups(feed, groups, offsets, lengths, key_idx, widths):
    """groups: index arrays submitted one call each; slot = message index.
    Returns the tickets."""
    tickets = np.zeros(lengths.size, np.uint64)
    for g in groups:
        while True:
            t = feed.submit(offsets[g], lengths[g], key_idx[g], widths[g], g)
            if t:
                break
            feed.poll()
            time.sleep(1e-4)
        tickets[g] = t + np.arange(len(g), dtype=np.uint64)
    return tickets


def _check(rows, want, widths):
    for j in range(want.shape[0]):
        w = int(widths[j])
        assert [int(x) for x in rows[j, :w]] == [int(x) for x in want[j, :w]], j


def test_messages_of_every_length_match_the_oracle(hh):
    rng = np.random.default_rng(71)
    lens = np.concatenate([np.arange(0, 70), rng.integers(70, 5000, 60),
                           rng.integers(5000, 400000, 30), [1 << 20, (1 << 20) + 31]])
    data, offsets, lengths = _buffer(rng, lens)
    n = lengths.size
    keys = rng.integers(0, 2**64, size=(5, 4), dtype=np.uint64)
    key_idx = rng.integers(0, 6, n).astype(np.uint32)  # 5 is clamped to 4
    widths = np.array([1, 2, 4], np.uint8)[rng.integers(0, 3, n)]
    perm = rng.permutation(n)
    groups, i = [], 0
    while i < n:
        k = int(rng.integers(1, 40))
        groups.append(perm[i:i + k])
        i += k
    k_t, d_t = dev(keys, torch.int64), dev(data)
    torch.cuda.synchronize()
    feed = hh.Feed(k_t, d_t, slots=n, waves=8, max_ms=2000,
                   stream=torch.cuda.Stream())
    try:
        announce("feed messages", n, len(groups))
        tickets = _submit_groups(feed, groups, offsets, lengths, key_idx, widths)
        rows = _wait(feed, np.arange(n), tickets)
    finally:
        feed.close()
    want = oracle_ref(4, keys, np.minimum(key_idx, 4), data, offsets, lengths)
    _check(rows, want, widths)


def test_short_message_overtakes_a_long_one(hh):
    # 32 MiB (about 36 ms of serial Updates), then 64 KiB a little later: the
    # second finishes while the first is still being hashed
    rng = np.random.default_rng(72)
    data, offsets, lengths = _buffer(rng, [32 << 20, 64 << 10])
    keys = rng.integers(0, 2**64, size=(1, 4), dtype=np.uint64)
    k_t, d_t = dev(keys, torch.int64), dev(data)
    torch.cuda.synchronize()
    feed = hh.Feed(k_t, d_t, slots=2, waves=4, max_ms=2000,
                   stream=torch.cuda.Stream())
    try:
        announce("feed overtake")
        z = np.zeros(1, np.uint32)
        t0 = feed.submit(offsets[:1], lengths[:1], z, np.ones(1, np.uint8), np.array([0]))
        time.sleep(2e-3)
        t1 = feed.submit(offsets[1:], lengths[1:], z, np.ones(1, np.uint8), np.array([1]))
        _wait(feed, np.array([1]), np.array([t1], np.uint64))
        long_done_first = feed.rows[0, 4] == t0
        rows = _wait(feed, np.array([0, 1]), np.array([t0, t1], np.uint64))
    finally:
        feed.close()
    assert not long_done_first
    want = oracle_ref(1, keys, None, data, offsets, lengths)
    assert [int(rows[0, 0]), int(rows[1, 0])] == [int(want[0, 0]), int(want[1, 0])]


def test_slots_reused_and_launches_renewed(hh):
    # each launch ends after 1 ms; rounds of groups 5 ms apart find it ended
    # and relaunch it; every round reuses the slots of the one before
    rng = np.random.default_rng(73)
    n = 24
    keys = rng.integers(0, 2**64, size=(3, 4), dtype=np.uint64)
    rounds = []
    for _ in range(4):
        rounds.append(_buffer(rng, rng.integers(0, 200000, n)))
    big = np.concatenate([r[0] for r in rounds])
    base = np.cumsum([0] + [r[0].size for r in rounds[:-1]])
    k_t, d_t = dev(keys, torch.int64), dev(big)
    torch.cuda.synchronize()
    feed = hh.Feed(k_t, d_t, slots=n, waves=6, max_ms=1,
                   stream=torch.cuda.Stream())
    try:
        for k, (data, offsets, lengths) in enumerate(rounds):
            announce("feed round", k)
            key_idx = rng.integers(0, 3, n).astype(np.uint32)
            widths = np.array([1, 2, 4], np.uint8)[rng.integers(0, 3, n)]
            groups = np.array_split(rng.permutation(n), 5)
            tickets = _submit_groups(feed, groups, offsets + np.uint64(base[k]), lengths,
                                     key_idx, widths)
            rows = _wait(feed, np.arange(n), tickets)
            want = oracle_ref(4, keys, key_idx, data, offsets, lengths)
            _check(rows, want, widths)
            time.sleep(5e-3)
    finally:
        feed.close()


def test_one_wave_reuses_its_places(hh):
    # one hashing wave (16 places) takes 60 messages of mixed lengths one by
    # one as its places free up
    rng = np.random.default_rng(75)
    data, offsets, lengths = _buffer(rng, rng.integers(0, 300000, 60))
    n = lengths.size
    keys = rng.integers(0, 2**64, size=(2, 4), dtype=np.uint64)
    key_idx = rng.integers(0, 2, n).astype(np.uint32)
    widths = np.array([1, 2, 4], np.uint8)[rng.integers(0, 3, n)]
    k_t, d_t = dev(keys, torch.int64), dev(data)
    torch.cuda.synchronize()
    feed = hh.Feed(k_t, d_t, slots=n, waves=2, max_ms=2000, stream=torch.cuda.Stream())
    try:
        announce("feed one wave", n)
        tickets = _submit_groups(feed, [np.arange(n)], offsets, lengths, key_idx, widths)
        rows = _wait(feed, np.arange(n), tickets)
    finally:
        feed.close()
    want = oracle_ref(4, keys, key_idx, data, offsets, lengths)
    _check(rows, want, widths)


def test_bad_arguments_rejected(hh):
    rng = np.random.default_rng(74)
    data, offsets, lengths = _buffer(rng, [100, 200])
    keys = rng.integers(0, 2**64, size=(1, 4), dtype=np.uint64)
    k_t, d_t = dev(keys, torch.int64), dev(data)
    torch.cuda.synchronize()
    feed = hh.Feed(k_t, d_t, slots=2, waves=2, max_ms=50,
                   stream=torch.cuda.Stream())
    try:
        z = np.zeros(1, np.uint32)
        with pytest.raises(hh.HHError):
            feed.submit(offsets[:1], lengths[:1], z, np.array([3], np.uint8), np.array([0]))
        with pytest.raises(hh.HHError):
            feed.submit(offsets[:1], lengths[:1], z, np.ones(1, np.uint8), np.array([2]))
        with pytest.raises(hh.HHError):   # more messages than slots
            feed.submit(np.zeros(3, np.uint64), np.zeros(3, np.uint64),
                        np.zeros(3, np.uint32), np.ones(3, np.uint8), np.zeros(3))
        assert feed.rows[:, 4].tolist() == [0, 0]   # nothing was queued
    finally:
        feed.close()


def test_ring_wraps_with_slots_recycled(hh):
    # 8 slots, so the 8-entry queue wraps around dozens of times; each slot
    # is submitted again as soon as its result is seen (one message per
    # call, or the queue is momentarily full and the call is repeated)
    rng = np.random.default_rng(76)
    n, slots = 300, 8
    data, offsets, lengths = _buffer(rng, rng.integers(0, 100000, n))
    keys = rng.integers(0, 2**64, size=(4, 4), dtype=np.uint64)
    key_idx = rng.integers(0, 4, n).astype(np.uint32)
    widths = np.array([1, 2, 4], np.uint8)[rng.integers(0, 3, n)]
    k_t, d_t = dev(keys, torch.int64), dev(data)
    torch.cuda.synchronize()
    feed = hh.Feed(k_t, d_t, slots=slots, waves=3, max_ms=2000, stream=torch.cuda.Stream())
    got = np.zeros((n, 4), np.uint64)
    owner = [-1] * slots          # message held by each slot
    ticket = np.zeros(slots, np.uint64)
    nxt, done, busy_calls = 0, 0, 0
    t_end = time.monotonic() + 30.0
    try:
        announce("feed ring wrap", n, slots)
        while done < n:
            assert time.monotonic() < t_end, "results did not arrive"
            for s in range(slots):
                j = owner[s]
                if j >= 0 and feed.rows[s, 4] == ticket[s]:
                    got[j] = feed.rows[s, :4]
                    owner[s] = -1
                    done += 1
                if owner[s] < 0 and nxt < n:
                    t = feed.submit(offsets[nxt:nxt + 1], lengths[nxt:nxt + 1],
                                    key_idx[nxt:nxt + 1], widths[nxt:nxt + 1], np.array([s]))
                    if t:
                        owner[s], ticket[s] = nxt, t
                        nxt += 1
                    else:
                        busy_calls += 1
            feed.poll()
    finally:
        feed.close()
    print("[gpu-case] queue-full retries", busy_calls, flush=True)
    want = oracle_ref(4, keys, key_idx, data, offsets, lengths)
    _check(got, want, widths)
