// hh_feed.hip -- continuous hashing of long messages for a serving loop.
//
// A persistent kernel takes groups of up to 16 messages from a queue in host
// memory while it runs and hashes each message whole (Sec. 4.2-4.5, four
// threads per message as in the quad kernel), writing each result and then
// its ticket into host memory.  A message that is submitted while others are
// being hashed starts within microseconds on an idle wave, instead of waiting
// for the next launch of a chunked iteration.
//
// Shared memory (pinned host memory, fine-grained and mapped for the GPU):
//   shared.tail       groups submitted so far (host writes)
//   shared.exit       set by hh_feed_close (host writes)
//   ring[cap]         group descriptors, group g in ring[g % cap] (host writes)
//   consumed[cap]     g + 1 once a wave has read group g (GPU writes)
//   rows[slots][5]    four result words, then the ticket of the message whose
//                     result they are (GPU writes)
// Device memory:
//   head              groups claimed so far (compare-and-swap by the waves)
//   tail_seen         the dispatcher's latest copy of shared.tail
//   exit_gen          launch generation that has been told to stop
//
// Wave 0 of a launch is the dispatcher: it alone reads shared.tail and
// shared.exit over the host link and republishes them in device memory, so
// that idle waves poll the L2 and not the link.  Every launch ends by itself
// after max_ms (plus a grace period for the waves): the host relaunches it
// (hh_feed_submit, hh_feed_poll) while submitted groups wait.  A wave stops
// only between groups, so a running launch never leaves a claimed group
// unfinished.

#include <atomic>
#include <cstring>
#include <mutex>

#include "hh_device.hpp"
#include "hh_internal.hpp"
#include "hh_msg.hpp"

namespace hh {
namespace {

constexpr u32 kFeedGroup = 16;                 // messages per group: one wave, four threads each
constexpr u64 kTicksPerMs = 100000;            // the real-time counter runs at 100 MHz
constexpr u64 kGraceTicks = 50 * kTicksPerMs;  // waves outlive the dispatcher by at most this
constexpr u64 kNone = ~0ull;
constexpr int kFeedRing = 48;                  // packets in flight per thread

struct FeedReq {
    u64 offset, length, ticket;
    u32 key_idx, slot, width, pad;
};

struct FeedGroupDesc {
    u64 n;
    u64 pad[7];
    FeedReq req[kFeedGroup];
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
};

struct FeedArgs {
    const u64* keys;
    u32 n_keys;
    u32 cap;
    const u8* data;
    u64 data_bytes;
    const FeedShared* shared;
    const FeedGroupDesc* ring;
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
                    // the groups below t were written before t: pass that on
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
    const u32 r = lane >> 2;
    const int q = (int)(lane & 3u);
    while (true) {
        // lane 0 claims the next group, or learns that the launch is over
        u64 g = kNone;
        if (lane == 0) {
            while (true) {
                const u64 t = dev_load(&a.dev->tail_seen);
                u64 h = dev_load(&a.dev->head);
                if (h < t) {
                    if (__hip_atomic_compare_exchange_strong(&a.dev->head, &h, h + 1u,
                                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) {
                        g = h;
                        break;
                    }
                    continue;
                }
                if (dev_load(&a.dev->exit_gen) >= a.gen || ticks() - t0 > a.max_ticks + kGraceTicks)
                    break;
                __builtin_amdgcn_s_sleep(32);
            }
        }
        // the claimed group's descriptor was written before the tail that
        // announced it
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        g = wave_broadcast(g);
        if (g == kNone) return;
        const FeedGroupDesc* d = a.ring + (g % a.cap);
        const u64 n_raw = sys_load(&d->n);
        const u32 n = n_raw < kFeedGroup ? (u32)n_raw : kFeedGroup;
        const bool real = r < n;
        const FeedReq* rq = &d->req[real ? r : 0u];
        const u64 off = sys_load(&rq->offset), len = sys_load(&rq->length);
        const u64 ticket = sys_load(&rq->ticket);
        const u32 kidx = sys_load32(&rq->key_idx), slot = sys_load32(&rq->slot);
        const u32 width = sys_load32(&rq->width);
        // every lane holds its fields: the group's descriptor may be reused
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        if (lane == 0) sys_store(&a.consumed[g % a.cap], g + 1u);
        u64 sum = 0;
        if (real) {
            const Msg m = message(a.data, a.data_bytes, off, len);
            const u64 key_q = a.keys[4u * (u64)(kidx < a.n_keys ? kidx : a.n_keys - 1u) + (u32)q];
            sum = hash_quad<kFeedRing>(key_q, m.p, m.len, q);
        }
        const bool valid_w = width == 1u || width == 2u || width == 4u;
        if (real && slot < a.slots && valid_w && (u32)q < width) sys_store(&a.rows[5u * slot + q], sum);
        // the words are visible before the ticket that announces them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        if (real && slot < a.slots && q == 0) sys_store(&a.rows[5u * slot + 4u], ticket);
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
    FeedGroupDesc* ring = nullptr;
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
// after max_ms) and a submitted group is still unread.  Caller holds mu.
hh_status feed_keep_running(hh_feed* f) {
    if (f->tail == 0) return HH_OK;
    const u64 last = f->tail - 1u;
    const u64 seen = __atomic_load_n(&f->consumed[last % f->cap], __ATOMIC_ACQUIRE);
    if (seen == last + 1u) return HH_OK;  // every group has been taken
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
    const u64 cons_off = ring_off + align64((u64)f->cap * sizeof(FeedGroupDesc));
    const u64 rows_off = cons_off + align64(8ull * f->cap);
    a.shared = (const FeedShared*)f->host_d;
    a.ring = (const FeedGroupDesc*)(f->host_d + ring_off);
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
    f->cap = slots;  // every group in flight holds at least one slot
    f->waves = waves;
    f->max_ticks = (u64)max_ms * kTicksPerMs;
    const u64 bytes = align64(sizeof(FeedShared)) + align64((u64)f->cap * sizeof(FeedGroupDesc)) +
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
    const u64 cons_off = ring_off + align64((u64)f->cap * sizeof(FeedGroupDesc));
    const u64 rows_off = cons_off + align64(8ull * f->cap);
    f->shared = (FeedShared*)f->host;
    f->ring = (FeedGroupDesc*)(f->host + ring_off);
    f->consumed = (u64*)(f->host + cons_off);
    f->rows = (u64*)(f->host + rows_off);
    if (hipMalloc(&f->dev, sizeof(FeedDev)) != hipSuccess) {
        (void)hipGetLastError();
        f->dev = nullptr;
        feed_free(f);
        return HH_ERR_OUT_OF_MEMORY;
    }
    // synchronous: the counters are zero before any launch reads them
    if (hipMemset(f->dev, 0, sizeof(FeedDev)) != hipSuccess ||
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
    if (!f || n == 0 || n > HH_FEED_GROUP || !offsets || !lengths || !width_words || !slot)
        return HH_ERR_INVALID_ARG;
    for (uint32_t i = 0; i < n; ++i) {
        const uint8_t w = width_words[i];
        if ((w != 1 && w != 2 && w != 4) || slot[i] >= f->slots) return HH_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(f->mu);
    const u64 e = f->tail % f->cap;
    if (f->tail >= f->cap &&
        __atomic_load_n(&f->consumed[e], __ATOMIC_ACQUIRE) != f->tail - f->cap + 1u)
        return HH_ERR_BUSY;  // the group that used this entry has not been read yet
    FeedGroupDesc& d = f->ring[e];
    for (uint32_t i = 0; i < n; ++i) {
        d.req[i].offset = offsets[i];
        d.req[i].length = lengths[i];
        d.req[i].ticket = f->next_ticket + i;
        d.req[i].key_idx = key_idx ? key_idx[i] : 0u;
        d.req[i].slot = slot[i];
        d.req[i].width = width_words[i];
        d.req[i].pad = 0;
    }
    d.n = n;
    if (first_ticket) *first_ticket = f->next_ticket;
    f->next_ticket += n;
    ++f->tail;
    // the descriptor is complete before the GPU can see the new tail
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
