"""Serving loop: continuous batching of hash requests on one GPU.

A request is (key index, payload bytes, output width 1/2/4 words).  The loop
keeps every admitted request's payload on the device.  With device ingress,
requests up to 8 KiB take the whole lane: each pass hashes the ones that
arrived since the last in one launch on a stream of their own, with no state
and no admission kernel.  Other requests up to four chunks (256 KiB) advance
together in lane 0: each scheduler iteration gives
every active request one 64 KiB chunk (a multiple of 32 bytes, or its whole
remainder), launched as one kernel that mixes the updates and the
finalizations, with each request's 1024-bit state kept on the device between
iterations (only size mod 32 enters HighwayHash, Sec. 4.5 of the paper, so a
request resumes from its state and no length counter is kept).  Longer
requests go whole to the feed: a persistent kernel on a stream of its own
that takes them as they arrive and writes each hash into pinned host memory
(or, with long_mode="chunks", they advance 1 MiB per iteration in a second
lane of chunked iterations).

Requests that arrive while others are on the GPU are admitted as soon as a
state slot and device memory (the admission budget: payload bytes rounded to
256 plus 128 B of state and 32 B of output) are free, and join the next
iteration.  The host runs up to two iterations ahead of the GPU and harvests
completed iterations through events, so admission, chunk planning and
launches overlap the device work; the scheduler keeps its request state in
arrays and admits and retires requests in bulk.

    python -m paper_1612_06257_amd.serve [--requests N] [--loads 0.25,0.5,0.8]
        [--rates R1,R2,...] [--long-mode feed|chunks] [--whole-max BYTES]
        [--budget-gib G] [--source device|host]

prints one JSON line per load point: offered rate, GB/s, requests/s,
p50/p90/p99 latency.
"""
from __future__ import annotations

import argparse
import bisect
import collections
import concurrent.futures
import ctypes
import dataclasses
import gc
import json
import sys
import time
from typing import List, NamedTuple, Optional, Tuple

import numpy as np

STATE_BYTES = 128
OUT_BYTES = 32
GRANULE = 256


def _timer_slack(ns: int) -> int:
    """Set the calling thread's timer slack (Linux prctl) to ns nanoseconds;
    returns the previous value, or -1 where it cannot be read or set.  With
    the default slack of 50 us a sleep of a few microseconds lasted 55-100 us,
    which the serving loop's short sleeps added to every request in flight."""
    try:
        libc = ctypes.CDLL(None, use_errno=True)
        prev = libc.prctl(30, 0, 0, 0, 0)          # PR_GET_TIMERSLACK
        if prev < 0 or libc.prctl(29, ctypes.c_ulong(ns), 0, 0, 0) != 0:  # PR_SET_TIMERSLACK
            return -1
        return prev
    except (OSError, AttributeError):
        return -1


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    key_idx: int
    width: int              # output words: 1, 2 or 4
    length: int             # payload bytes
    src: int                # payload offset in the source buffer
    slot: int = -1          # state slot while admitted
    arena_off: int = -1     # payload offset in the device arena
    reserved: int = 0       # budget bytes held
    pos: int = 0            # bytes already launched
    final_launched: bool = False
    t_admit: float = -1.0
    t_done: float = -1.0
    result: Optional[Tuple[int, ...]] = None
    status: str = "queued"  # queued, active, done, rejected


class Arena:
    """Next-fit allocator over [0, capacity) in GRANULE units, coalescing.

    The search for a free range resumes where the previous allocation ended
    and wraps around, so with payloads that retire roughly in arrival order
    the arena behaves like a ring and an allocation rarely looks at more than
    one free range (a first-fit search from offset 0 walked past every small
    hole on each admission and dominated the scheduler's host time)."""

    def __init__(self, capacity: int):
        self.capacity = capacity // GRANULE * GRANULE
        self.free: List[Tuple[int, int]] = [(0, self.capacity)]  # (offset, size), sorted
        self.used = 0
        self.rover = 0  # the next search starts at the first range at or past this offset

    def alloc(self, nbytes: int) -> Optional[int]:
        n = max(GRANULE, (nbytes + GRANULE - 1) // GRANULE * GRANULE)
        k = len(self.free)
        start = bisect.bisect_left(self.free, (self.rover, 0))
        for j in range(k):
            i = start + j
            if i >= k:
                i -= k
            off, size = self.free[i]
            if size >= n:
                if size == n:
                    del self.free[i]
                else:
                    self.free[i] = (off + n, size - n)
                self.used += n
                self.rover = off + n
                return off
        return None

    def release(self, off: int, nbytes: int) -> None:
        self.release_many([(off, nbytes)])

    def release_many(self, spans) -> None:
        """Return (offset, nbytes) spans, coalescing with the free list (one
        sort-and-merge pass, so a harvest of thousands costs one pass)."""
        if not spans:
            return
        add = [(off, max(GRANULE, (n + GRANULE - 1) // GRANULE * GRANULE)) for off, n in spans]
        self.used -= sum(n for _, n in add)
        if len(add) == 1 and len(self.free) > 64:
            # a lone span: binary search and local merges
            off, n = add[0]
            lo = bisect.bisect_left(self.free, (off, 0))
            self.free.insert(lo, (off, n))
            if lo + 1 < len(self.free) and off + n == self.free[lo + 1][0]:
                self.free[lo] = (off, n + self.free[lo + 1][1])
                del self.free[lo + 1]
            if lo > 0 and self.free[lo - 1][0] + self.free[lo - 1][1] == self.free[lo][0]:
                self.free[lo - 1] = (self.free[lo - 1][0], self.free[lo - 1][1] + self.free[lo][1])
                del self.free[lo]
            return
        merged: List[Tuple[int, int]] = []
        for off, n in sorted(self.free + add):
            if merged and merged[-1][0] + merged[-1][1] == off:
                merged[-1] = (merged[-1][0], merged[-1][1] + n)
            else:
                merged.append((off, n))
        self.free = merged


class AdmitBatch(NamedTuple):
    """Newly admitted requests, as arrays in one order: payload source
    offset, arena offset, length, key index, state slot."""
    src: np.ndarray
    arena_off: np.ndarray
    length: np.ndarray
    key_idx: np.ndarray
    slot: np.ndarray

    @property
    def n(self) -> int:
        return int(self.slot.size)


class GpuBackend:
    """Device side of the loop: payload arena, states, outputs, launches.

    source="device": the trace's payloads sit in a device ingress buffer and
    the kernels read each request where it arrived (the arena is then only
    the budget's bookkeeping);
    source="host": they sit in pinned host memory and admission copies them
    into the arena on a copy stream that the compute stream waits for.
    Admission resets the new states in place.  Admission and iteration item
    lists go through rings of pinned staging sets that the kernels read
    where they are, and an iteration writes its finished hashes, compacted
    in launch order, straight into a pinned result set: no stream carries a
    copy for them, and a launch costs the host one kernel call and one event.

    Two lanes: lane 0 launches on the compute stream, lane 1 (the long
    requests' lane) on a stream of its own with its own staging and result
    sets, so that a long lane iteration never holds up the short requests'
    iterations.  Admission runs on the compute stream; the lane 1
    stream only ever receives that lane's iterations, or the feed's
    persistent kernel (feed_submit), which hashes a long request whole and
    writes its result into host memory.

    With device ingress the backend also has a whole lane (launch_whole): a
    stream of its own on which one launch hashes a batch of short requests
    whole, where they arrived, with no state and no admission, writing
    their 4-word hashes into a pinned result set."""

    RING = 6   # staging sets per lane; more than the scheduler's run-ahead + 1
    LANES = 2
    FEED = True

    def __init__(self, keys: np.ndarray, payload: np.ndarray, arena_bytes: int, max_slots: int,
                 source: str = "device", feed_waves: int = 64, feed_max_ms: int = 1000):
        import torch
        from . import hh
        self.torch, self.hh = torch, hh
        hh.lib()
        self.keys = torch.from_numpy(np.ascontiguousarray(keys)).view(torch.int64).cuda()
        self.max_slots = max_slots
        self.states = torch.zeros((max_slots, hh.STATE_WORDS), dtype=torch.int64, device="cuda")
        self.arena = torch.empty(max(arena_bytes, GRANULE), dtype=torch.uint8, device="cuda")
        self.source = source
        src = torch.from_numpy(np.ascontiguousarray(payload))
        if src.numel() == 0:
            src = torch.zeros(1, dtype=torch.uint8)
        if source == "device":
            self.ingress = src.cuda()
        else:
            self.ingress = torch.empty(src.numel(), dtype=torch.uint8, pin_memory=True)
            self.ingress.copy_(src)
        self.compute_stream = torch.cuda.current_stream()
        # the long lane (and the host-ingress copies) must not share a
        # hardware queue with the compute stream, or the short requests'
        # iterations would wait behind a long iteration: pick streams that are
        # measured to run concurrently with it
        extra = hh.independent_streams(2, avoid=[self.compute_stream])
        # the second extra stream carries the admission copies (host
        # ingress) or the whole lane's launches (device ingress)
        self.copy_stream = extra[1] if source == "host" else None
        self.whole_stream = extra[1] if source == "device" else None
        self.lane_streams = [self.compute_stream, extra[0]]
        # item metadata per staging set: offs u64, lens u64, out offs u64,
        # slots u32, widths u8 for at most max_slots items, each array 8-aligned
        self.meta_bytes = max_slots * (8 + 8 + 8 + 4 + 1) + 64
        self.h_meta = [[torch.empty(self.meta_bytes, dtype=torch.uint8, pin_memory=True)
                        for _ in range(self.RING)] for _ in range(self.LANES)]
        self.h_res = [[torch.empty((max_slots, 4), dtype=torch.int64, pin_memory=True)
                       for _ in range(self.RING)] for _ in range(self.LANES)]
        # admission metadata per staging set: src offs u64, arena offs u64,
        # lens u64, key index u32, slot u32
        self.adm_bytes = max_slots * 32
        self.h_adm = [torch.empty(self.adm_bytes, dtype=torch.uint8, pin_memory=True)
                      for _ in range(self.RING)]
        self.k = [0] * self.LANES
        self.ka = 0
        # the kernels read the staging sets and write the result sets where
        # they are, in pinned host memory (no copies on the streams, and less
        # host time per launch than torch copies and views): their device
        # addresses, and numpy views for the host's side
        self.meta_dev = [[hh.pinned_device_pointer(t) for t in ring] for ring in self.h_meta]
        self.res_dev = [[hh.pinned_device_pointer(t) for t in ring] for ring in self.h_res]
        self.adm_dev = [hh.pinned_device_pointer(t) for t in self.h_adm]
        # the whole lane (device ingress): message lists (offsets u64,
        # lengths u64, key index u32) and 4-word results per staging set
        self.whole = source == "device"
        self.kw = 0
        self.h_whole = [torch.empty(max_slots * 20 + 64, dtype=torch.uint8, pin_memory=True)
                        for _ in range(self.RING)] if self.whole else []
        self.h_wres = [torch.empty((max_slots, 4), dtype=torch.int64, pin_memory=True)
                       for _ in range(self.RING)] if self.whole else []
        self.whole_dev = [hh.pinned_device_pointer(t) for t in self.h_whole]
        self.wres_dev = [hh.pinned_device_pointer(t) for t in self.h_wres]
        self.whole_np = [t.numpy() for t in self.h_whole]
        self.wres_np = [t.numpy().view(np.uint64) for t in self.h_wres]
        self.meta_np = [[t.numpy() for t in ring] for ring in self.h_meta]
        self.res_np = [[t.numpy().view(np.uint64) for t in ring] for ring in self.h_res]
        self.adm_np = [t.numpy() for t in self.h_adm]
        self.launcher = concurrent.futures.ThreadPoolExecutor(max_workers=1)
        self.events = [[torch.cuda.Event() for _ in range(self.RING)] for _ in range(self.LANES)]
        self.whole_events = [torch.cuda.Event() for _ in range(self.RING)]
        self.adm_events = [torch.cuda.Event() for _ in range(self.RING)]
        # The first launch on a stream sets the stream up inside the runtime:
        # it took about 5 ms and held up every other launch of the process
        # meanwhile (the GPU idled and the requests in flight waited).  Pay it
        # here, from the thread that launches on each stream, before any
        # request arrives.
        self._warm = torch.zeros(1, dtype=torch.int64, device="cuda")
        self._warm_stream(self.compute_stream)
        self._warm_stream(extra[1])
        self.launcher.submit(self._warm_stream, self.lane_streams[1]).result()
        # With device ingress every kernel reads a request where it arrived
        # (reads_source: admission only resets states, there is no copy to
        # wait for; the budget still reserves the requests' bytes); with host
        # ingress they read the arena once admission has copied them there.
        self.reads_source = source == "device"
        self.data = self.ingress if self.reads_source else self.arena
        # the long requests' feed: a persistent kernel on the lane 1 stream
        # that hashes each long request whole; it launches on the first
        # submitted request, so a chunked long lane keeps that stream to
        # itself
        self.slot_key = np.zeros(max_slots, np.uint32)
        self._feed = hh.Feed(self.keys, self.data, max_slots, feed_waves, feed_max_ms,
                             self.lane_streams[1])

    def _warm_stream(self, stream) -> None:
        with self.torch.cuda.stream(stream):
            self._warm.add_(1)
        stream.synchronize()

    def admit(self, batch: AdmitBatch):
        """Copy the payloads of newly admitted requests into the arena and
        reset their states in place, on the compute stream.  Returns a ticket
        for done(): a request of the long lane joins that lane's launches only
        once its admission has completed, so the lane 1 stream needs no wait
        on another stream (host-side stream waits, and copies queued on a
        stream busy with a long iteration, stalled the loop for milliseconds
        now and then)."""
        if batch.n == 0:
            return None
        i = self.ka % self.RING
        self.ka += 1
        # that set's previous admission has finished reading it (normally long
        # ago; an event never recorded counts as complete)
        self.adm_events[i].synchronize()
        torch = self.torch
        n = batch.n
        h = self.adm_np[i]
        lens = batch.length
        h[:8 * n].view(np.int64)[:] = batch.src
        h[8 * n:16 * n].view(np.int64)[:] = batch.arena_off
        h[16 * n:24 * n].view(np.int64)[:] = lens
        h[24 * n:28 * n].view(np.int32)[:] = batch.key_idx
        h[28 * n:32 * n].view(np.int32)[:] = batch.slot
        self.slot_key[batch.slot] = batch.key_idx
        if not self.reads_source:
            # host ingress: the payloads go to the arena on the copy stream,
            # which the compute stream waits for
            with torch.cuda.stream(self.copy_stream):
                for so, do, ln in zip(batch.src.tolist(), batch.arena_off.tolist(),
                                      lens.tolist()):
                    if ln:
                        self.arena[do:do + ln].copy_(self.ingress[so:so + ln],
                                                     non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.copy_stream)
            self.compute_stream.wait_event(ev)
        d = self.adm_dev[i]
        self.hh.state_init_raw(self.keys, n, d + 24 * n, self.states, d + 28 * n,
                               self.compute_stream.cuda_stream)
        ev = self.adm_events[i]
        ev.record(self.compute_stream)
        return (ev, None)

    def launch(self, upd_slots, upd_offs, upd_lens, fin_slots, fin_offs, fin_lens, fin_widths,
               lane: int = 0):
        """One iteration of a lane: fold whole-packet chunks into the states of
        upd_slots, finish fin_slots, all in one kernel launch on the lane's
        stream (lane 0: the compute stream).  Arrays of equal length per
        group.  Returns a ticket for done()/wait()/results()."""
        if lane == 0:
            return self._launch(0, upd_slots, upd_offs, upd_lens, fin_slots, fin_offs, fin_lens,
                                fin_widths)
        # the long lane's launches go through a launcher thread: a launch now
        # and then holds the calling thread for milliseconds inside the
        # runtime, which must not stall the scheduling loop (the ctypes call
        # releases the interpreter lock)
        return self.launcher.submit(self._launch, lane, upd_slots, upd_offs, upd_lens, fin_slots,
                                    fin_offs, fin_lens, fin_widths)

    def _launch(self, lane, upd_slots, upd_offs, upd_lens, fin_slots, fin_offs, fin_lens,
                fin_widths):
        i = self.k[lane] % self.RING
        self.k[lane] += 1
        nu, nf = len(upd_slots), len(fin_slots)
        n = nu + nf
        res = None
        if n:
            # item lists in the pinned staging set: offsets, lengths, output
            # offsets (u64), state slots (u32), widths (u8); updates first,
            # then finals, whose words go to the result set at 4 * rank
            h = self.meta_np[lane][i]
            w64 = h[:24 * n].view(np.int64)
            w64[:nu] = upd_offs
            w64[nu:n] = fin_offs
            w64[n:n + nu] = upd_lens
            w64[n + nu:2 * n] = fin_lens
            w64[2 * n:2 * n + nu] = 0
            w64[2 * n + nu:3 * n] = np.arange(0, 4 * nf, 4)
            s32 = h[24 * n:28 * n].view(np.int32)
            s32[:nu] = upd_slots
            s32[nu:] = fin_slots
            h[28 * n:28 * n + nu] = 0
            h[28 * n + nu:29 * n] = fin_widths
            mb = self.meta_dev[lane][i]
            self.hh.state_step_raw(self.states, self.data, mb, mb + 8 * n, mb + 28 * n,
                                   self.res_dev[lane][i], self.max_slots * 4, mb + 16 * n,
                                   mb + 24 * n, n, self.lane_streams[lane].cuda_stream)
            if nf:
                res = self.res_np[lane][i][:nf]
        # events are reused round the staging ring (a set is re-recorded only
        # after the scheduler has harvested its previous launch)
        ev = self.events[lane][i]
        ev.record(self.lane_streams[lane])
        return (ev, res)

    def launch_whole(self, offsets, lengths, key_idx):
        """Hash requests whole in one launch on the whole lane's stream (device
        ingress: offsets into the ingress buffer; no state, no admission).
        Returns a ticket whose results() are the requests' 4-word hashes in
        this order.  At most RING - 1 of these may be in flight."""
        i = self.kw % self.RING
        self.kw += 1
        n = len(offsets)
        h = self.whole_np[i]
        w64 = h[:16 * n].view(np.int64)
        w64[:n] = offsets
        w64[n:] = lengths
        h[16 * n:20 * n].view(np.int32)[:] = key_idx
        d = self.whole_dev[i]
        self.hh.hash_raw(self.keys, self.data, d + 16 * n, d, d + 8 * n, n, self.wres_dev[i], 4,
                         "lane4", self.whole_stream.cuda_stream)
        ev = self.whole_events[i]
        ev.record(self.whole_stream)
        return (ev, self.wres_np[i][:n])

    @staticmethod
    def _resolve(ticket):
        return ticket.result() if isinstance(ticket, concurrent.futures.Future) else ticket

    def done(self, ticket) -> bool:
        if isinstance(ticket, concurrent.futures.Future) and not ticket.done():
            return False
        return self._resolve(ticket)[0].query()

    def wait(self, ticket) -> None:
        self._resolve(ticket)[0].synchronize()

    def results(self, ticket) -> Optional[np.ndarray]:
        """(n_fin, 4) uint64 hash words of the ticket's finished items, in the
        order they were launched."""
        return self._resolve(ticket)[1]

    def feed_submit(self, slots, offsets, lengths, widths, key_idx) -> int:
        """Hand admitted requests to the feed (taken in this order; offsets
        into self.data, the buffer the kernels read); returns the first
        request's ticket (request i: ticket + i), or 0 if the queue has no
        room for them yet.  A request's result appears in feed_rows()[slot]
        with its ticket."""
        return self._feed.submit(offsets, lengths, key_idx, widths, slots)

    def feed_rows(self) -> np.ndarray:
        """(max_slots, 5) uint64: hash words, then the ticket they belong to."""
        return self._feed.rows

    def feed_poll(self) -> None:
        self._feed.poll()

    def close(self) -> None:
        if self._feed is not None:
            self._feed.close()
            self._feed = None
        self.launcher.shutdown(wait=True)


class Server:
    """Scheduler: admission under the budget, continuous batching.

    Requests up to long_min_bytes advance chunk_bytes per iteration in lane
    0.  With a two-lane backend, longer requests take the long lane:

    long_mode="feed" (the default with a backend that has a feed): each long
    request goes whole to the backend's persistent kernel as soon as its
    admission is done (longest first), and is retired when its result row
    shows its ticket: it neither waits for an iteration to join nor for the
    longest chunk of one.  long_mode="chunks": long requests advance
    long_chunk_bytes per iteration on their own stream.  Every lane keeps its
    own work in flight, so long requests never stretch the short requests'
    iterations.

    With a backend that has a whole lane, requests up to whole_max_bytes
    (8 KiB by default) skip admission and lane 0: each pass hashes the ones
    admitted since the last in one launch on that lane's stream, so they
    wait neither for lane 0's queued iterations nor for the 64 KiB chunks in
    them."""

    def __init__(self, backend, budget_bytes: int, chunk_bytes: int = 1 << 16,
                 max_active: Optional[int] = None, clock=time.perf_counter,
                 sleep=time.sleep, run_ahead: int = 2, long_chunk_bytes: int = 1 << 20,
                 long_min_bytes: Optional[int] = None, poll_s: float = 5e-4,
                 long_mode: Optional[str] = None, feed_poll_s: float = 5e-5,
                 stall_s: float = 60.0, whole_max_bytes: Optional[int] = None):
        for c in (chunk_bytes, long_chunk_bytes):
            if c <= 0 or c % 32:
                raise ValueError("chunk sizes must be positive multiples of 32")
        if run_ahead + 1 >= getattr(backend, "RING", 1 << 30):
            raise ValueError("run_ahead too large for the backend's staging ring")
        self.backend = backend
        self.budget = budget_bytes
        self.chunk = chunk_bytes
        self.lanes = min(2, getattr(backend, "LANES", 1))
        self.chunks = [chunk_bytes, long_chunk_bytes]
        self.lane_run_ahead = [run_ahead, 1]
        self.poll_s = poll_s
        has_feed = getattr(backend, "FEED", False) and self.lanes > 1
        if long_mode is None:
            long_mode = "feed" if has_feed else "chunks"
        if long_mode not in ("feed", "chunks") or (long_mode == "feed" and not has_feed):
            raise ValueError("long_mode must be 'chunks', or 'feed' with a feed backend")
        self.long_mode = long_mode
        # requests longer than this take the long lane: in the feed, from
        # four chunks up (they are hashed whole there); chunked, from 16
        if long_min_bytes is None:
            long_min_bytes = (4 if long_mode == "feed" else 16) * chunk_bytes
        self.long_min = long_min_bytes
        # requests up to whole_max_bytes take the whole lane when the backend
        # has one (it hashes them where they arrived, in one launch on a
        # stream of their own, with no state and no admission)
        has_whole = bool(getattr(backend, "whole", False))
        if whole_max_bytes is None:
            whole_max_bytes = 8192 if has_whole else 0
        if whole_max_bytes and not has_whole:
            raise ValueError("whole_max_bytes needs a backend with a whole lane")
        if whole_max_bytes > long_min_bytes and self.lanes > 1:
            raise ValueError("whole_max_bytes must not exceed long_min_bytes")
        self.whole_max = whole_max_bytes
        self.whole_run_ahead = getattr(backend, "RING", 1 << 30) - 1
        self.feed_poll_s = feed_poll_s
        # the loop raises when admitted work makes no progress for this long
        self.stall_s = stall_s
        self.arena = Arena(budget_bytes)
        self.max_active = max_active or backend.max_slots
        # free state slots: a stack, slots[:n_free] (the top at the end)
        self.free_slots = np.arange(backend.max_slots, dtype=np.int64)[::-1].copy()
        self.n_free = backend.max_slots
        self.clock = clock
        self.sleep = sleep
        self.run_ahead = run_ahead
        self.max_bytes_in_flight = 0

    @staticmethod
    def reservation(length: int) -> int:
        return (max(length, 1) + GRANULE - 1) // GRANULE * GRANULE + STATE_BYTES + OUT_BYTES

    def run(self, requests: List[Request]) -> dict:
        """Serve `requests`.  Returns the run's metrics.

        The loop keeps every request attribute in arrays (arrival order) and
        does per-iteration work in bulk: the queue is a range of that order,
        admission takes the longest run of queued requests that the free
        slots, the budget and one contiguous arena range can hold, and a
        harvest retires a finished iteration's requests at once.  The Request
        objects are filled in after the run.

        Python's cyclic garbage collector is off while the loop runs (and
        back in its previous state after): a full pass over a process that
        holds a few hundred thousand objects stops the loop for about 40 ms,
        which held every request in flight that long in some runs.  The loop
        makes no reference cycles of its own.  With real sleeps, the thread's
        timer slack is 1 us while the loop runs (then restored)."""
        was_enabled = gc.isenabled()
        gc.disable()
        # real sleeps: a fine timer slack while the loop runs
        slack = _timer_slack(1000) if self.sleep is time.sleep else -1
        try:
            return self._run(requests)
        finally:
            if slack >= 0:
                _timer_slack(slack)
            if was_enabled:
                gc.enable()

    def _run(self, requests: List[Request]) -> dict:
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
        reqs = [requests[i] for i in order]
        n_total = len(reqs)
        arrival = np.fromiter((r.arrival for r in reqs), np.float64, n_total)
        r_len = np.fromiter((r.length for r in reqs), np.int64, n_total)
        r_width = np.fromiter((r.width for r in reqs), np.int64, n_total)
        r_key = np.fromiter((r.key_idx for r in reqs), np.int64, n_total)
        r_src = np.fromiter((r.src for r in reqs), np.int64, n_total)
        r_gran = (np.maximum(r_len, 1) + GRANULE - 1) // GRANULE * GRANULE
        r_need = r_gran + (STATE_BYTES + OUT_BYTES)
        status = np.zeros(n_total, np.int8)        # 0 waiting, 1 active, 2 done, 3 rejected
        r_slot = np.full(n_total, -1, np.int64)
        r_off = np.full(n_total, -1, np.int64)
        r_resv = np.zeros(n_total, np.int64)
        t_admit = np.full(n_total, -1.0)
        t_done = np.full(n_total, -1.0)
        results = np.zeros((n_total, 4), np.uint64)
        S = self.backend.max_slots
        # active set, indexed by state slot
        busy = np.zeros(S, bool)          # admitted, final not yet launched
        length = np.zeros(S, np.int64)
        pos = np.zeros(S, np.int64)
        base = np.zeros(S, np.int64)      # offset of the payload in the buffer the kernels read
        held = np.zeros(S, np.int64)      # arena offset of the reservation
        resv = np.zeros(S, np.int64)      # budget bytes held
        width = np.zeros(S, np.uint8)
        owner = np.full(S, -1, np.int64)  # request in the slot
        lane = np.zeros(S, np.int8)       # lane of the request in the slot
        ready = np.ones(S, bool)          # admission done (long lane: seen complete)
        gated: collections.deque = collections.deque()  # (admission ticket, slots)
        # per lane: (ticket, finishing slots) in launch order
        # (lane W: the whole lane)
        inflight = [collections.deque() for _ in range(self.lanes + 1)]
        W = self.lanes
        whole_wait = []                     # whole-lane slots not yet launched
        self.whole_launches = 0
        feed = self.long_mode == "feed"
        feed_wait = []                      # slots ready for the feed, not yet submitted
        fed_slots = np.zeros(0, np.int64)   # handed to the feed, result not yet seen
        key_of = np.zeros(S, np.int64)      # key index of the slot's request
        # with device ingress the kernels read a request where it arrived
        # (offsets into the ingress buffer), and a feed request needs no
        # admission at all: it is ready at once
        in_place = getattr(self.backend, "reads_source", False)
        direct = feed and in_place
        fticket = np.zeros(S, np.uint64)    # the feed ticket of that request
        n_fed = 0
        self.feed_submits = 0
        t0 = self.clock()
        arrived = 0   # requests [0, arrived) have arrived
        head = 0      # requests [head, arrived) are queued
        self.n_finished = 0
        iterations = 0
        self.reserved_bytes = 0
        n_busy = 0

        def harvest(ln: int, block: bool) -> None:
            ticket, fin = inflight[ln].popleft()
            if block:
                self.backend.wait(ticket)
            words = self.backend.results(ticket)
            if len(fin):
                retire(fin, words)

        def retire(fin: np.ndarray, words: np.ndarray) -> None:
            t = self.clock() - t0
            ridx = owner[fin]
            results[ridx] = words[:len(fin), :4]
            t_done[ridx] = t
            status[ridx] = 2
            owner[fin] = -1
            if not in_place:
                self.arena.release_many(list(zip(held[fin].tolist(),
                                                 np.maximum(length[fin], 1).tolist())))
            self.reserved_bytes -= int(resv[fin].sum())
            self.free_slots[self.n_free:self.n_free + fin.size] = fin
            self.n_free += fin.size
            self.n_finished += len(fin)

        last_progress, seen_finished = 0.0, 0
        while self.n_finished < n_total:
            now = self.clock() - t0
            if self.n_finished != seen_finished or not (n_busy or n_fed or any(inflight) or gated):
                last_progress, seen_finished = now, self.n_finished
            elif now - last_progress > self.stall_s:
                raise RuntimeError("serving loop: no request finished for %.1f s with %d in "
                                   "flight" % (now - last_progress,
                                               n_busy + n_fed + len(gated)))
            arrived = int(np.searchsorted(arrival, now, side="right"))
            # admission, in arrival order, while a slot and budget are free
            runs = []
            while head < arrived and self.n_free and n_busy < self.max_active:
                m = min(arrived - head, self.n_free, self.max_active - n_busy)
                need = r_need[head:head + m]
                over = np.flatnonzero(need > self.budget)
                if over.size and over[0] == 0:
                    # larger than the whole budget: refused
                    status[head], t_done[head] = 3, now
                    self.n_finished += 1
                    head += 1
                    continue
                if over.size:
                    m = int(over[0])
                k = int(np.searchsorted(np.cumsum(need[:m]), self.budget - self.reserved_bytes,
                                        side="right"))
                if k == 0:
                    break  # back-pressure: wait for completions
                gran = r_gran[head:head + k]
                if in_place:
                    # the kernels read the payloads where they arrived: the
                    # budget alone binds, no arena range is needed
                    offs = np.full(k, -1, np.int64)
                else:
                    off = self.arena.alloc(int(gran.sum()))
                    if off is None:
                        # no contiguous range for the run: the head request alone
                        k, gran = 1, gran[:1]
                        off = self.arena.alloc(int(gran[0]))
                        if off is None:
                            break  # fragmented: wait for completions
                    offs = off + np.cumsum(gran) - gran
                slots = self.free_slots[self.n_free - k:self.n_free][::-1].copy()
                self.n_free -= k
                # the run is requests head .. head+k-1 (slices of the
                # arrival-order arrays), in the slots just taken
                sl = slice(head, head + k)
                ridx = np.arange(head, head + k)
                rl = r_len[sl]
                status[sl], r_slot[sl], r_off[sl] = 1, slots, offs
                r_resv[sl], t_admit[sl] = need[:k], now
                busy[slots], length[slots], pos[slots] = True, rl, 0
                base[slots] = r_src[sl] if in_place else offs
                held[slots], resv[slots], width[slots] = offs, need[:k], r_width[sl]
                owner[slots] = ridx
                key_of[slots] = r_key[sl]
                ln = (rl > self.long_min).astype(np.int8) if self.lanes > 1 else np.zeros(k, np.int8)
                if self.whole_max:
                    ln[rl <= self.whole_max] = W
                lane[slots] = ln
                self.reserved_bytes += int(need[:k].sum())
                n_busy += k
                head += k
                runs.append(ridx)
            self.max_bytes_in_flight = max(self.max_bytes_in_flight, self.reserved_bytes)
            adm = None
            if runs:
                ridx = np.concatenate(runs)
                if self.whole_max:
                    # whole-lane requests skip admission altogether
                    is_whole = lane[r_slot[ridx]] == W
                    if is_whole.any():
                        whole_wait.append(r_slot[ridx[is_whole]])
                        ridx = ridx[~is_whole]
                is_long = ((lane[r_slot[ridx]] == 1) if self.lanes > 1
                           else np.zeros(ridx.size, bool))
                if direct:
                    # long requests skip admission: the feed reads their bytes
                    # where they arrived, so they are ready at once
                    if is_long.any():
                        feed_wait.append(r_slot[ridx[is_long]])
                    ridx = ridx[~is_long]
                    is_long = is_long[~is_long]
                if ridx.size:
                    adm = self.backend.admit(AdmitBatch(src=r_src[ridx], arena_off=r_off[ridx],
                                                        length=r_len[ridx], key_idx=r_key[ridx],
                                                        slot=r_slot[ridx]))
                    if is_long.any():
                        longs = r_slot[ridx][is_long]
                        ready[longs] = False
                        gated.append((adm, longs))
            # long-lane requests whose admission has completed may advance
            while gated and self.backend.done(gated[0][0]):
                longs = gated.popleft()[1]
                ready[longs] = True
                if feed:
                    feed_wait.append(longs)
            # feed mode: long requests whose admission is done go whole to the
            # feed, longest first
            if feed:
                if feed_wait:
                    g = feed_wait[0] if len(feed_wait) == 1 else np.concatenate(feed_wait)
                    g = g[np.argsort(-length[g], kind="stable")]
                    tk = self.backend.feed_submit(g, base[g],
                                                  length[g], width[g], key_of[g])
                    if tk:  # else the queue is full: they wait for the next pass
                        feed_wait = []
                        fticket[g] = tk + np.arange(g.size, dtype=np.uint64)
                        fed_slots = np.concatenate([fed_slots, g])
                        busy[g] = False
                        n_busy -= g.size
                        n_fed += g.size
                        self.feed_submits += 1
                    else:
                        feed_wait = [g]
                if n_fed:
                    rows = self.backend.feed_rows()
                    hit = rows[fed_slots, 4] == fticket[fed_slots]
                    if hit.any():
                        fin = fed_slots[hit]
                        fed_slots = fed_slots[~hit]
                        n_fed -= fin.size
                        retire(fin, rows[fin, :4].copy())
                    self.backend.feed_poll()
            # per lane, one chunk for every busy request of the lane (whole
            # packets, or its final rest), unless the lane is far enough ahead
            launched = False
            if whole_wait and len(inflight[W]) < self.whole_run_ahead:
                g = whole_wait[0] if len(whole_wait) == 1 else np.concatenate(whole_wait)
                whole_wait = []
                ticket = self.backend.launch_whole(base[g], length[g], key_of[g])
                busy[g] = False
                n_busy -= g.size
                inflight[W].append((ticket, g))
                self.whole_launches += 1
                launched = True
            for ln in range(self.lanes):
                if feed and ln == 1:
                    continue
                if len(inflight[ln]) > self.lane_run_ahead[ln]:
                    continue
                idx = (np.flatnonzero(busy & (lane == ln) & ready) if self.lanes > 1
                       else np.flatnonzero(busy & (lane == 0)))
                if not idx.size:
                    continue
                chunk = self.chunks[ln]
                rem = length[idx] - pos[idx]
                fin = rem <= chunk
                u, f = idx[~fin], idx[fin]
                args = (u, base[u] + pos[u], np.full(u.size, chunk), f, base[f] + pos[f],
                        rem[fin], width[f])
                ticket = (self.backend.launch(*args, lane=ln) if self.lanes > 1
                          else self.backend.launch(*args))
                pos[u] += chunk
                pos[f] = length[f]
                busy[f] = False
                n_busy -= f.size
                inflight[ln].append((ticket, f))
                iterations += 1
                launched = True
            # harvest what has finished; lane 0 blocks when too far ahead
            for ln in range(self.lanes + 1):
                while inflight[ln] and self.backend.done(inflight[ln][0][0]):
                    harvest(ln, False)
            while len(inflight[0]) > self.lane_run_ahead[0]:
                harvest(0, True)
            if not launched:
                if inflight[0] and not inflight[W]:
                    harvest(0, True)  # short iterations: wait for the oldest
                elif (any(inflight) or gated or n_fed) and head == arrived:
                    # only long work, whole-lane launches or admissions in
                    # flight: sleep until the next arrival (at most poll_s, or
                    # feed_poll_s while the feed or the whole lane holds
                    # requests)
                    nxt = (arrival[arrived] - (self.clock() - t0) if arrived < n_total
                           else self.poll_s)
                    cap = self.feed_poll_s if (n_fed or inflight[W]) else self.poll_s
                    self.sleep(max(0.0, min(cap, nxt)))
            if (not n_busy and not any(inflight) and not gated and not n_fed
                    and head == arrived and arrived < n_total):
                self.sleep(max(0.0, min(1e-3, arrival[arrived] - (self.clock() - t0))))
        t_end = self.clock() - t0
        # fill in the Request objects
        names = {0: "queued", 1: "active", 2: "done", 3: "rejected"}
        res_rows = results.tolist()
        for i, r in enumerate(reqs):
            r.status = names[int(status[i])]
            r.slot, r.arena_off, r.reserved = int(r_slot[i]), int(r_off[i]), int(r_resv[i])
            r.t_admit, r.t_done = float(t_admit[i]), float(t_done[i])
            if status[i] == 2:
                r.result = tuple(res_rows[i][:r.width])
        return self.metrics(requests, t_end, iterations)

    def metrics(self, requests: List[Request], t_end: float, iterations: int) -> dict:
        done = [r for r in requests if r.status == "done"]
        lat = np.array([r.t_done - r.arrival for r in done]) if done else np.zeros(1)
        # requests that fit one chunk: one iteration of work, so their latency
        # is queueing and scheduling
        one = np.array([r.length <= self.chunk for r in done], bool) if done else np.zeros(1, bool)
        lat_one = lat[one] if one.any() else np.zeros(1)
        nbytes = sum(r.length for r in done)
        first = min((r.arrival for r in requests), default=0.0)
        span = max(t_end - first, 1e-9)
        return {
            "requests": len(requests), "completed": len(done),
            "rejected": sum(r.status == "rejected" for r in requests),
            "bytes": nbytes, "seconds": span, "GBps": nbytes / span / 1e9,
            "requests_per_s": len(done) / span,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p90_ms": float(np.percentile(lat, 90) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "iterations": iterations,
            "one_chunk_requests": int(one.sum()),
            "one_chunk_p50_ms": float(np.percentile(lat_one, 50) * 1e3),
            "one_chunk_p99_ms": float(np.percentile(lat_one, 99) * 1e3),
            "chunk_bytes": self.chunk, "budget_bytes": self.budget,
            "max_bytes_in_flight": self.max_bytes_in_flight,
            "long_mode": self.long_mode, "long_min_bytes": self.long_min,
            "whole_max_bytes": self.whole_max, "whole_launches": self.whole_launches,
        }


def requests_from_trace(trace) -> List[Request]:
    return [Request(rid=i, arrival=float(trace.arrival_s[i]), key_idx=int(trace.key_idx[i]),
                    width=int(trace.width_words[i]), length=int(trace.lengths[i]),
                    src=int(trace.offsets[i])) for i in range(trace.n)]


def serve_trace(trace, budget_bytes: int = 32 << 30, chunk_bytes: int = 1 << 16,
                max_slots: int = 16384, source: str = "device", time_scale: float = 1.0,
                feed_waves: int = 64, **server_kw):
    """Run one trace on the GPU; returns (metrics, requests).  server_kw go to
    Server (long_mode, long_chunk_bytes, long_min_bytes, whole_max_bytes, poll_s,
    run_ahead);
    feed_waves sizes the backend's feed (one dispatcher wave, the others
    hashing up to 16 requests each)."""
    reqs = requests_from_trace(trace)
    for r in reqs:
        r.arrival *= time_scale
    arena = min(budget_bytes, max(GRANULE, sum(Server.reservation(r.length) for r in reqs)))
    backend = GpuBackend(trace.keys, trace.data, arena, max_slots, source, feed_waves)
    server = Server(backend, budget_bytes=arena if arena < budget_bytes else budget_bytes,
                    chunk_bytes=chunk_bytes, **server_kw)
    try:
        m = server.run(reqs)
    finally:
        backend.close()
    m["budget_bytes"] = budget_bytes
    m["source"] = source
    if server.long_mode == "feed":
        m["feed_waves"] = feed_waves
    return m, reqs


def results_array(reqs: List[Request], n: int) -> np.ndarray:
    """(n, 4) uint64 results by request id (words past a request's width and
    unfinished requests are 0)."""
    out = np.zeros((n, 4), np.uint64)
    for r in reqs:
        if r.result is not None:
            out[r.rid, :len(r.result)] = r.result
    return out


def load_sweep(n_requests: int = 10000, loads=(0.25, 0.5, 0.8), chunk_bytes: int = 1 << 16,
               budget_bytes: int = 32 << 30, source: str = "device", seed: Optional[int] = None,
               with_results: bool = False, rates=None, **server_kw):
    """Saturation run (every request arrives at t=0), then Poisson loads at
    the given fractions of the measured saturation request rate (or, with
    `rates`, at those offered requests/s, so that runs of different settings
    see the same arrivals).  Every point serves the same requests (lengths,
    payloads, keys, widths).  With with_results, returns (points, trace,
    per-point results_array)."""
    from . import workloads as W
    kw = {} if seed is None else {"seed": seed}
    base = W.serving_trace(n_requests, 1.0, **kw)
    base.arrival_s[:] = 0.0
    sat, reqs = serve_trace(base, budget_bytes, chunk_bytes, source=source, **server_kw)
    sat_rate = sat["requests_per_s"]
    out = [dict(sat, load="saturation", offered_requests_per_s=None)]
    results = [results_array(reqs, base.n)] if with_results else None
    points = ([(f, f * sat_rate) for f in loads] if rates is None
              else [(r / sat_rate, float(r)) for r in rates])
    for f, rate in points:
        tr = W.serving_trace(n_requests, rate, materialize=False, **kw)
        tr.data, tr.offsets, tr.lengths = base.data, base.offsets, base.lengths
        tr.key_idx, tr.width_words, tr.keys = base.key_idx, base.width_words, base.keys
        m, reqs = serve_trace(tr, budget_bytes, chunk_bytes, source=source, **server_kw)
        out.append(dict(m, load=f, offered_requests_per_s=rate))
        if with_results:
            results.append(results_array(reqs, base.n))
    return (out, base, results) if with_results else out


def bench_summary(n_requests: int = 10000, loads=(0.25, 0.5, 0.8),
                  chunk_bytes: int = 1 << 16):
    """The benchmark's serving run: a discarded warm-up pass (first-use
    allocations, clocks), then saturation and the Poisson loads, all with the
    same requests.  Returns (summary, trace, per-point results) so that the
    caller can check every result."""
    from . import workloads as W
    warm = W.serving_trace(400, 1.0, seed=W.SEED_BASE + 99)
    warm.arrival_s[:] = 0.0
    serve_trace(warm, chunk_bytes=chunk_bytes)
    pts, trace, results = load_sweep(n_requests, loads, chunk_bytes, with_results=True)
    summary = {"requests_per_point": n_requests, "saturation": pts[0],
               "loads": pts[1:]}
    return summary, trace, results


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=10000)
    ap.add_argument("--loads", default="0.25,0.5,0.8")
    ap.add_argument("--rates", default=None,
                    help="offered requests/s per point (comma list), instead of --loads")
    ap.add_argument("--chunk", type=int, default=1 << 16)
    ap.add_argument("--budget-gib", type=float, default=32.0)
    ap.add_argument("--source", default="device", choices=["device", "host"])
    ap.add_argument("--long-chunk", type=int, default=1 << 20)
    ap.add_argument("--long-mode", default=None, choices=["feed", "chunks"],
                    help="long requests whole in the feed's persistent kernel (default) or "
                         "in chunked iterations")
    ap.add_argument("--long-min", type=int, default=None,
                    help="requests longer than this take the long lane (default 4 chunks "
                         "with the feed, 16 chunked)")
    ap.add_argument("--feed-waves", type=int, default=64,
                    help="feed workgroups: one dispatcher, the others 16 requests each")
    ap.add_argument("--whole-max", type=int, default=None,
                    help="requests up to this many bytes take the whole lane (device "
                         "ingress; default 8192, 0 turns it off)")
    ap.add_argument("--poll-us", type=float, default=500.0)
    ap.add_argument("--max-slots", type=int, default=16384,
                    help="request states held on the device (128 B each)")
    args = ap.parse_args(argv)
    if args.max_slots < 1:
        ap.error("--max-slots must be at least 1")
    loads = tuple(float(x) for x in args.loads.split(",") if x)
    kw = dict(long_chunk_bytes=args.long_chunk, long_min_bytes=args.long_min,
              poll_s=args.poll_us * 1e-6, max_slots=args.max_slots, long_mode=args.long_mode,
              feed_waves=args.feed_waves, whole_max_bytes=args.whole_max)
    rates = [float(x) for x in args.rates.split(",") if x] if args.rates else None
    for p in load_sweep(args.requests, loads, args.chunk, int(args.budget_gib * 2**30), args.source,
                        rates=rates, **kw):
        p.update({k: v for k, v in kw.items() if v is not None})
        print(json.dumps(p), flush=True)


if __name__ == "__main__":
    sys.exit(main())
