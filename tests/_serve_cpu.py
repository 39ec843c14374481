"""A CPU stand-in for the serving loop's GPU backend (test infrastructure).

It keeps a byte arena exactly like the device backend, streams every request
through the oracle's incremental hasher, checks that admitted payload regions
never overlap, and advances a virtual clock by a simple cost model so that the
scheduler can be exercised without a GPU."""
import numpy as np

import oracle


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class CpuBackend:
    RING = 1 << 30
    LANES = 2

    def __init__(self, keys, payload, arena_bytes, max_slots, clock, ns_per_byte=0.05,
                 launch_s=20e-6, reads_source=False, whole=False):
        self.keys = np.asarray(keys, np.uint64).reshape(-1, 4)
        self.payload = payload
        self.arena = np.zeros(max(arena_bytes, 256), np.uint8)
        self.max_slots = max_slots
        self.clock = clock
        self.ns_per_byte = ns_per_byte
        self.launch_s = launch_s
        self.cats = {}
        self.live = {}   # slot -> (arena_off, length)
        self.launches = 0
        self.lane_launches = [0, 0]
        self.lane_of = {}  # slot -> lane of its first launch
        # reads_source: the kernels read requests where they arrived (offsets
        # into the payload), admission copies nothing
        self.reads_source = reads_source
        self.data = payload if reads_source else self.arena
        # whole: requests hashed whole from where they arrived, in one
        # launch, with no state (needs reads_source, as on the device)
        assert not whole or reads_source
        self.whole = whole
        self.whole_launched = []   # lengths per whole launch
        self.admitted = 0          # requests admitted (states reset)

    def _check_no_overlap(self):
        spans = sorted((o, o + max(n, 1)) for o, n in self.live.values())
        for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
            assert a1 <= b0, "arena regions overlap"

    def admit(self, batch):
        self.admitted += len(batch.slot)
        for src, off, n, key, slot in zip(batch.src.tolist(), batch.arena_off.tolist(),
                                          batch.length.tolist(), batch.key_idx.tolist(),
                                          batch.slot.tolist()):
            assert slot not in self.cats, "slot reused while live"
            if not self.reads_source:
                self.arena[off:off + n] = self.payload[src:src + n]
            self.cats[slot] = oracle.Cat(self.keys[key])
            if self.reads_source:
                assert off == -1   # no arena range: the budget alone binds
            else:
                self.live[slot] = (off, n)
        self._check_no_overlap()
        return ("admission",)

    def launch(self, upd_slots, upd_offs, upd_lens, fin_slots, fin_offs, fin_lens, fin_widths,
               lane=0):
        self.launches += 1
        self.lane_launches[lane] += 1
        for slot in list(upd_slots.tolist()) + list(fin_slots.tolist()):
            # a request stays in one lane for its whole life
            assert self.lane_of.setdefault(slot, lane) == lane
        for slot in fin_slots.tolist():
            del self.lane_of[slot]
        biggest = 0
        for slot, off, n in zip(upd_slots.tolist(), upd_offs.tolist(), upd_lens.tolist()):
            assert n % 32 == 0
            self.cats[slot].append(self.data[off:off + n])
            biggest = max(biggest, n)
        res = np.zeros((len(fin_slots), 4), np.uint64)
        for i, (slot, off, n) in enumerate(zip(fin_slots.tolist(), fin_offs.tolist(),
                                               fin_lens.tolist())):
            c = self.cats.pop(slot)
            c.append(self.data[off:off + n])
            res[i] = c.finish(4)
            self.live.pop(slot, None)
            biggest = max(biggest, n)
        self.clock.t += self.launch_s + biggest * self.ns_per_byte * 1e-9
        return res

    def launch_whole(self, offsets, lengths, key_idx):
        assert self.whole
        res = np.zeros((len(offsets), 4), np.uint64)
        for i, (off, n, k) in enumerate(zip(np.asarray(offsets).tolist(),
                                            np.asarray(lengths).tolist(),
                                            np.asarray(key_idx).tolist())):
            res[i] = oracle.hash_words(self.keys[k], self.payload[off:off + n], 4)
        self.whole_launched.append(np.asarray(lengths).copy())
        self.clock.t += self.launch_s + max([0] + np.asarray(lengths).tolist()) * \
            self.ns_per_byte * 1e-9
        return res

    def done(self, ticket):
        return True

    def wait(self, ticket):
        pass

    def results(self, ticket):
        return ticket


class FeedCpuBackend(CpuBackend):
    """CpuBackend with a feed: submitted requests are hashed whole at once
    (the longest one's cost advances the clock) and their rows show the
    results and tickets.  reads_source: the feed hashes a request from the
    payload where it arrived (the server then skips its admission); else
    from the arena after admission."""
    FEED = True

    def __init__(self, *args, **kw):
        super().__init__(*args, **kw)
        self.rows = np.zeros((self.max_slots, 5), np.uint64)
        self.next_ticket = 1
        self.submits = []   # (slots, lengths) per submit call

    def feed_submit(self, slots, offsets, lengths, widths, key_idx):
        assert len(slots) >= 1
        t = self.next_ticket
        self.next_ticket += len(slots)
        self.submits.append((np.asarray(slots).copy(), np.asarray(lengths).copy()))
        for i, (slot, off, n, k) in enumerate(zip(np.asarray(slots).tolist(),
                                                  np.asarray(offsets).tolist(),
                                                  np.asarray(lengths).tolist(),
                                                  np.asarray(key_idx).tolist())):
            if self.reads_source:
                assert slot not in self.cats  # the server skipped its admission
                c = oracle.Cat(self.keys[k])
            else:
                c = self.cats.pop(slot)
                self.live.pop(slot, None)
            c.append(self.data[off:off + n])
            self.rows[slot, :4] = c.finish(4)
            self.rows[slot, 4] = t + i
        self.clock.t += self.launch_s + max(np.asarray(lengths).tolist()) * self.ns_per_byte * 1e-9
        return t

    def feed_rows(self):
        return self.rows

    def feed_poll(self):
        pass
