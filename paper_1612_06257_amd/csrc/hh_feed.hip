// hh_feed.hip -- continuous hashing of long messages for a serving loop.
//
// A persistent kernel takes messages from a queue in host memory while it
// runs and hashes each one whole (Sec. 4.2-4.5, four threads per message as
// in the quad kernel), writing its result and then its ticket into host
// memory.  Each hashing wave is a 16-place engine: its quads take messages
// one by one as they become free, so messages that arrive at different times
// share a wave (a wave's chain of Updates runs no slower with 16 messages
// than with one, and every wave with a chain in it takes its SIMD's issue
// slots), and a message starts within one round (kRoundPackets packets) of a
// busy wave, or at once on an idle one.
//
// Shared memory (pinned host memory, fine-grained and mapped for the GPU):
//   shared.tail       messages submitted so far (host writes)
//   shared.exit       set by hh_feed_close (host writes)
//   ring[cap]         message descriptors, message i in ring[i % cap] (host writes)
//   consumed[cap]     i + 1 once a wave has read message i (GPU writes)
//   rows[slots][5]    four result words, then the ticket of the message whose
//                     result they are (GPU writes)
// Device memory:
//   head              messages claimed so far (compare-and-swap by the waves)
//   tail_seen         the dispatcher's latest copy of shared.tail
//   exit_gen          launch generation that has been told to stop
//   free_mask         bit w set while hashing wave w has a free place
//
// Packing: a wave that holds messages looks at the queue after every round;
// a wave that holds none takes a message only when no hashing wave with a
// lower index has a free place.  So new messages fill the busy waves and
// then the lowest idle ones, and as few waves (and CUs) as possible carry
// chains of Updates beside the other kernels on the GPU.
//
// Wave 0 of a launch is the dispatcher: it alone reads shared.tail and
// shared.exit over the host link and republishes them in device memory, so
// that the other waves poll the L2 and not the link.  Every launch stops
// taking messages after max_ms and ends when its waves have finished the
// messages they hold: the host relaunches it (hh_feed_submit, hh_feed_poll)
// while submitted messages wait.

#include <atomic>
#include <cstring>
#include <mutex>

#include "hh_device.hpp"
#include "hh_internal.hpp"
#include "hh_msg.hpp"

namespace hh {
namespace {

constexpr u64 kTicksPerMs = 100000;  // the real-time counter runs at 100 MHz
constexpr u64 kNone = ~0ull;
constexpr int kFeedRing = 48;            // packets in flight per thread
constexpr u32 kRoundPackets = 2048;      // packets per message between two looks at the queue
constexpr u32 kFullRoundPackets = 8192;  // at most this many in a round of a wave with no free place

struct FeedReq {
    u64 offset, length, ticket;
    u32 key_idx, slot, width, pad;
};

struct FeedShared {
    u64 tail;
    u64 pad0[15];
    u64 exit;
    u64 pad1[15];
};

struct FeedDev {
    u64 head;
    u64 pad0[15];
    u64 tail_seen;
    u64 pad1[15];
    u64 exit_gen;
    u64 pad2[15];
    u64 free_mask;  // bit w: hashing wave w has a free place
    u64 pad3[15];
};

struct FeedArgs {
    const u64* keys;
    u32 n_keys;
    u32 cap;
    const u8* data;
    u64 data_bytes;
    const FeedShared* shared;
    const FeedReq* ring;
    u64* consumed;
    u64* rows;
    u64 slots;
    FeedDev* dev;
    u64 gen;
    u64 max_ticks;
};

// Polls use relaxed atomic loads (coherent at their scope, so they see new
// values, but they do not invalidate caches); an acquire fence follows only
// once a poll has seen something new.
__device__ __forceinline__ u64 sys_load(const u64* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ u64 dev_load(const u64* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u32 sys_load32(const u32* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void sys_store(u64* p, u64 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ u64 ticks() { return __builtin_amdgcn_s_memrealtime(); }

__device__ __forceinline__ u64 wave_min(u64 v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const u64 o = __shfl_xor(v, d);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ u64 wave_broadcast(u64 v) {
    const u32 lo = (u32)__builtin_amdgcn_readfirstlane((int)(u32)v);
    const u32 hi = (u32)__builtin_amdgcn_readfirstlane((int)(u32)(v >> 32));
    return ((u64)hi << 32) | lo;
}

__global__ __launch_bounds__(64) void hh_feed_kernel(FeedArgs a) {
    const u32 lane = threadIdx.x;
    const u64 t0 = ticks();
    if (blockIdx.x == 0) {
        // dispatcher: republish the host's queue tail and stop request
        if (lane == 0) {
            u64 last = kNone;
            while (true) {
                const u64 t = sys_load(&a.shared->tail);
                if (t != last) {
                    // the messages below t were written before t: pass that on
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                    __hip_atomic_store(&a.dev->tail_seen, t, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    last = t;
                }
                if (sys_load(&a.shared->exit) != 0u || ticks() - t0 > a.max_ticks) {
                    __hip_atomic_store(&a.dev->exit_gen, a.gen, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(16);
            }
        }
        return;
    }
    const int q = (int)(lane & 3u);
    const u32 leader = lane & ~3u;  // lane 4r leads quad r
    const u32 w = blockIdx.x - 1u;   // hashing wave index (< 64)
    const u64 my_bit = 1ull << w, lower = my_bit - 1ull;
    bool bit_set = false;  // this wave's free_mask bit as last written
    // the message this quad holds (every lane of a quad agrees on all but s)
    bool active = false;
    State1 s;
    reset1(s, 0, q);
    const u8* msg = a.data;
    const u8* p = a.data;
    u64 len = 0, rem = 0, ticket = 0;
    u32 slot = 0, width = 0;
    while (true) {
        // take messages for the free quads, unless the launch is over
        const bool stop = dev_load(&a.dev->exit_gen) >= a.gen || ticks() - t0 > a.max_ticks;
        const u64 free_q = __ballot(q == 0 && !active);
        const bool busy = free_q != 0x1111111111111111ull;
        // an idle wave leaves new messages to busy waves and lower idle ones
        const bool may_take =
            !stop && free_q && (busy || (dev_load(&a.dev->free_mask) & lower) == 0u);
        u64 h = 0, m = 0;
        if (may_take) {
            if (lane == 0) {
                const u64 want = (u64)__popcll(free_q);
                while (true) {
                    const u64 t = dev_load(&a.dev->tail_seen);
                    u64 hh = dev_load(&a.dev->head);
                    if (hh >= t) break;
                    const u64 k = t - hh < want ? t - hh : want;
                    if (__hip_atomic_compare_exchange_strong(&a.dev->head, &hh, hh + k,
                                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) {
                        h = hh;
                        m = k;
                        break;
                    }
                }
            }
            h = wave_broadcast(h);
            m = wave_broadcast(m);
        }
        if (m) {
            // the claimed descriptors were written before the tail that
            // announced them
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            const u64 rank = (u64)__popcll(free_q & ((1ull << leader) - 1ull));
            const bool take = !active && rank < m;
            u64 idx = 0;
            if (take) {
                idx = h + rank;
                const FeedReq* rq = a.ring + (idx % a.cap);
                const u64 off = sys_load(&rq->offset), length = sys_load(&rq->length);
                ticket = sys_load(&rq->ticket);
                const u32 kidx = sys_load32(&rq->key_idx);
                slot = sys_load32(&rq->slot);
                width = sys_load32(&rq->width);
                const Msg mm = message(a.data, a.data_bytes, off, length);
                const u64 key_q =
                    a.keys[4u * (u64)(kidx < a.n_keys ? kidx : a.n_keys - 1u) + (u32)q];
                reset1(s, key_q, q);
                msg = mm.p;
                p = mm.p;
                len = mm.len;
                rem = mm.len >> 5;
                active = true;
            }
            // every taker holds its descriptor's fields: the entries may be reused
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
            if (take && q == 0) sys_store(&a.consumed[idx % a.cap], idx + 1u);
        }
        // publish whether this wave has a free place (after taking, and after
        // the round below has finished messages)
        const bool has_free = __ballot(q == 0 && !active) != 0u && !stop;
        if (has_free != bit_set) {
            if (lane == 0) {
                if (has_free)
                    __hip_atomic_fetch_or(&a.dev->free_mask, my_bit, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                else
                    __hip_atomic_fetch_and(&a.dev->free_mask, ~my_bit, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
            bit_set = has_free;
        }
        if (!__ballot(active)) {
            if (stop) return;
            __builtin_amdgcn_s_sleep(32);
            continue;
        }
        // one round: every quad with whole packets left absorbs up to `round`
        // of them.  A wave with a free place looks at the queue every
        // kRoundPackets; a full wave cannot take a message, so its round runs
        // on to the first of its messages to finish (at most
        // kFullRoundPackets): each round restarts the prefetch ring, and a
        // message's result is written at the end of the round that finishes it
        u64 round = kRoundPackets;
        if (!__ballot(q == 0 && !active)) {
            const u64 first_done = wave_min(active && rem ? rem : ~0ull);
            round = first_done < kRoundPackets ? kRoundPackets
                    : (first_done > kFullRoundPackets ? kFullRoundPackets : first_done);
        }
        if (active && rem) {
            const u32 npk = (u32)(rem < round ? rem : round);
            absorb_quad<kFeedRing>(s, p + 8u * (u32)q, npk);
            p += 32u * (u64)npk;
            rem -= npk;
        }
        // quads whose message has no whole packet left finish it
        const bool fin = active && rem == 0u;
        u64 sum = 0;
        if (fin) {
            const u32 r = (u32)(len & 31u);
            const u64 tail = r ? remainder_lane(msg + 32u * (len >> 5), r, len, q) : 0;
            if (r) remainder1(s, r, tail);
            sum = finalize1(s);
        }
        const bool valid_w = width == 1u || width == 2u || width == 4u;
        if (fin && slot < a.slots && valid_w && (u32)q < width) sys_store(&a.rows[5u * slot + q], sum);
        // the words are visible before the ticket that announces them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        if (fin && slot < a.slots && q == 0) sys_store(&a.rows[5u * slot + 4u], ticket);
        if (fin) active = false;
    }
}

}  // namespace
}  // namespace hh

using namespace hh;

struct hh_feed {
    int device = 0;
    hipStream_t stream = nullptr;
    const u64* keys = nullptr;
    u32 n_keys = 0;
    const u8* data = nullptr;
    u64 data_bytes = 0;
    u32 slots = 0, cap = 0, waves = 0;
    u64 max_ticks = 0;
    u8* host = nullptr;  // pinned, fine-grained: shared, ring, consumed, rows
    FeedShared* shared = nullptr;
    FeedReq* ring = nullptr;
    u64* consumed = nullptr;
    u64* rows = nullptr;
    u8* host_d = nullptr;  // the same memory as the GPU addresses it
    FeedDev* dev = nullptr;
    hipEvent_t done = nullptr;
    bool launched = false;
    u64 gen = 0, tail = 0, next_ticket = 1;
    std::mutex mu;
};

namespace {

u64 align64(u64 x) { return (x + 63u) & ~63ull; }

// Relaunch the kernel when the last launch has ended (it stops by itself
// after max_ms) and a submitted message is still unread.  Caller holds mu.
hh_status feed_keep_running(hh_feed* f) {
    if (f->tail == 0) return HH_OK;
    const u64 last = f->tail - 1u;
    const u64 seen = __atomic_load_n(&f->consumed[last % f->cap], __ATOMIC_ACQUIRE);
    if (seen == last + 1u) return HH_OK;  // every message has been taken
    if (f->launched) {
        const hipError_t q = hipEventQuery(f->done);
        if (q == hipErrorNotReady) return HH_OK;  // still running: it will take them
        if (q != hipSuccess) {
            (void)hipGetLastError();
            return HH_ERR_LAUNCH;
        }
    }
    FeedArgs a;
    a.keys = f->keys;
    a.n_keys = f->n_keys;
    a.cap = f->cap;
    a.data = f->data;
    a.data_bytes = f->data_bytes;
    const u64 ring_off = align64(sizeof(FeedShared));
    const u64 cons_off = ring_off + align64((u64)f->cap * sizeof(FeedReq));
    const u64 rows_off = cons_off + align64(8ull * f->cap);
    a.shared = (const FeedShared*)f->host_d;
    a.ring = (const FeedReq*)(f->host_d + ring_off);
    a.consumed = (u64*)(f->host_d + cons_off);
    a.rows = (u64*)(f->host_d + rows_off);
    a.slots = f->slots;
    a.dev = f->dev;
    a.gen = ++f->gen;
    a.max_ticks = f->max_ticks;
    hipLaunchKernelGGL(hh_feed_kernel, dim3(f->waves), dim3(64), 0, f->stream, a);
    if (hipGetLastError() != hipSuccess) return HH_ERR_LAUNCH;
    if (hipEventRecord(f->done, f->stream) != hipSuccess) {
        (void)hipGetLastError();
        return HH_ERR_LAUNCH;
    }
    f->launched = true;
    return HH_OK;
}

void feed_free(hh_feed* f) {
    if (f->done) (void)hipEventDestroy(f->done);
    if (f->dev) (void)hipFree(f->dev);
    if (f->host) (void)hipHostFree(f->host);
    (void)hipGetLastError();
    delete f;
}

}  // namespace

extern "C" {

hh_status hh_feed_open(const uint64_t* keys, uint32_t n_keys, const uint8_t* data,
                       uint64_t data_bytes, uint32_t slots, uint32_t waves, uint32_t max_ms,
                       void* stream, hh_feed** feed) {
    if (!feed) return HH_ERR_INVALID_ARG;
    *feed = nullptr;
    if (!keys || n_keys == 0 || !data || slots == 0 || slots > HH_FEED_MAX_SLOTS || waves < 2 ||
        waves > HH_FEED_MAX_WAVES || max_ms == 0 || max_ms > HH_FEED_MAX_MS)
        return HH_ERR_INVALID_ARG;
    int dev = 0;
    hh_status s = check_device(&dev);
    if (s != HH_OK) return s;
    hh_feed* f = new hh_feed();
    f->device = dev;
    f->stream = (hipStream_t)stream;
    f->keys = keys;
    f->n_keys = n_keys;
    f->data = data;
    f->data_bytes = data_bytes;
    f->slots = slots;
    f->cap = slots;  // every message in flight holds a slot
    f->waves = waves;
    f->max_ticks = (u64)max_ms * kTicksPerMs;
    const u64 bytes = align64(sizeof(FeedShared)) + align64((u64)f->cap * sizeof(FeedReq)) +
                      align64(8ull * f->cap) + 40ull * slots;
    void* host = nullptr;
    if (hipHostMalloc(&host, bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        feed_free(f);
        return HH_ERR_OUT_OF_MEMORY;
    }
    f->host = (u8*)host;
    memset(f->host, 0, bytes);
    void* host_d = nullptr;
    if (hipHostGetDevicePointer(&host_d, host, 0) != hipSuccess) {
        (void)hipGetLastError();
        feed_free(f);
        return HH_ERR_LAUNCH;
    }
    f->host_d = (u8*)host_d;
    const u64 ring_off = align64(sizeof(FeedShared));
    const u64 cons_off = ring_off + align64((u64)f->cap * sizeof(FeedReq));
    const u64 rows_off = cons_off + align64(8ull * f->cap);
    f->shared = (FeedShared*)f->host;
    f->ring = (FeedReq*)(f->host + ring_off);
    f->consumed = (u64*)(f->host + cons_off);
    f->rows = (u64*)(f->host + rows_off);
    if (hipMalloc(&f->dev, sizeof(FeedDev)) != hipSuccess) {
        (void)hipGetLastError();
        f->dev = nullptr;
        feed_free(f);
        return HH_ERR_OUT_OF_MEMORY;
    }
    // ordered on the feed's stream before its first launch
    if (hipMemsetAsync(f->dev, 0, sizeof(FeedDev), f->stream) != hipSuccess ||
        hipEventCreateWithFlags(&f->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        feed_free(f);
        return HH_ERR_LAUNCH;
    }
    *feed = f;
    return HH_OK;
}

hh_status hh_feed_submit(hh_feed* f, uint32_t n, const uint64_t* offsets, const uint64_t* lengths,
                         const uint32_t* key_idx, const uint8_t* width_words,
                         const uint32_t* slot, uint64_t* first_ticket) {
    if (!f || n == 0 || !offsets || !lengths || !width_words || !slot) return HH_ERR_INVALID_ARG;
    if (n > f->slots) return HH_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < n; ++i) {
        const uint8_t w = width_words[i];
        if ((w != 1 && w != 2 && w != 4) || slot[i] >= f->slots) return HH_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(f->mu);
    // every entry to be written must have been read by the wave that took
    // the message submitted cap places earlier
    for (uint32_t i = 0; i < n; ++i) {
        const u64 idx = f->tail + i;
        if (idx >= f->cap &&
            __atomic_load_n(&f->consumed[idx % f->cap], __ATOMIC_ACQUIRE) != idx - f->cap + 1u)
            return HH_ERR_BUSY;
    }
    for (uint32_t i = 0; i < n; ++i) {
        FeedReq& d = f->ring[(f->tail + i) % f->cap];
        d.offset = offsets[i];
        d.length = lengths[i];
        d.ticket = f->next_ticket + i;
        d.key_idx = key_idx ? key_idx[i] : 0u;
        d.slot = slot[i];
        d.width = width_words[i];
        d.pad = 0;
    }
    if (first_ticket) *first_ticket = f->next_ticket;
    f->next_ticket += n;
    f->tail += n;
    // the descriptors are complete before the GPU can see the new tail
    __atomic_store_n(&f->shared->tail, f->tail, __ATOMIC_RELEASE);
    return feed_keep_running(f);
}

hh_status hh_feed_poll(hh_feed* f) {
    if (!f) return HH_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(f->mu);
    return feed_keep_running(f);
}

const volatile uint64_t* hh_feed_results(const hh_feed* f) { return f ? f->rows : nullptr; }

hh_status hh_feed_close(hh_feed* f) {
    if (!f) return HH_ERR_INVALID_ARG;
    hh_status s = HH_OK;
    {
        std::lock_guard<std::mutex> lock(f->mu);
        __atomic_store_n(&f->shared->exit, 1ull, __ATOMIC_RELEASE);
        // the launch stops within microseconds of the flag (or at max_ms)
        if (f->launched && hipEventSynchronize(f->done) != hipSuccess) {
            (void)hipGetLastError();
            s = HH_ERR_LAUNCH;
        }
    }
    feed_free(f);
    return s;
}

}  // extern "C"
