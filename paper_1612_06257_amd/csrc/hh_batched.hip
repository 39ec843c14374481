// hh_batched.hip -- the bucketed batch path: one call hashes messages of any
// mix of lengths.
//
// A message is one serial chain of ceil(L/32)+4 Updates (Sec. 4.2-4.5), so a
// batch of uneven lengths finishes no earlier than its longest message.  The
// path therefore (1) hashes short messages right away, one thread each, in a
// wide grid, (2) orders the long ones by length, longest first, and (3) hashes
// them four threads per message in a persistent grid of one wave per SIMD, so
// that every long chain owns its SIMD's issue slots and the longest chains
// start first (longest-processing-time-first list scheduling).
//
// Launch sequence on one stream (all device-side, no host synchronisation;
// optionally captured once per argument set into a hipGraph and replayed):
//   (hh_plan_reset_kernel  zero the plan: before a workspace's first sequence
//                          and after a sequence that failed part-way)
//   hh_split_kernel<W>     L < threshold: hash in-thread;  else: append the
//                          index to the long list and count it in its length
//                          bucket (8 buckets per octave of the packet count)
//   hh_scatter_kernel      bucket start offsets (longest bucket first, every
//                          block recomputes the 256-entry prefix), then long
//                          list -> bucket order; block 0 also decides how many
//                          leading (critical) items get a CU of their own,
//                          publishes the list length and clears the item
//                          counter for the persistent kernel
//   hh_long_kernel<W>      persistent: critical item b on wave 0 of workgroup
//                          b, the other waves of that workgroup idle; every
//                          other wave takes one item (16 messages, 4 threads
//                          each), then items from an atomic counter; one wave
//                          clears the split and scatter counters for the next
//                          sequence
// Every counter is cleared by a kernel that runs after its last reader and
// before its next writer, so no kernel counts its retiring waves: device-scope
// atomics on one address serialise, and a retire counter cost the persistent
// kernel about 13 us on an empty long list.
// A chain slows down by about 10% when other waves of its CU stream data
// alongside it (they share the CU's load path), which is why the few chains
// that set the batch's duration run alone on their CUs when the rest of the
// batch is light enough for the remaining CUs.
// Messages inside a bucket come out in any order; each message's result only
// depends on its own bytes, so outputs are deterministic.

#include <list>
#include <mutex>
#include <vector>

#include "hh_device.hpp"
#include "hh_internal.hpp"
#include "hh_msg.hpp"

namespace hh {

constexpr int kBuckets = 256;
constexpr u64 kPriorityBytes = 64u << 10;  // items this long run at wave priority 3

// Who writes and who clears each field (one sequence: split, scatter, long):
struct Plan {
    u32 n_long;     // split appends; scatter reads; long clears
    u32 item_next;  // long takes dynamic items; scatter clears
    u32 n_iso;      // scatter: leading items that get a CU each
    u32 n_order;    // scatter: entries of the ordered list (long reads)
    u32 hist[kBuckets];    // split counts; scatter reads; long clears
    u32 cursor[kBuckets];  // scatter reserves; long clears
};

// length bucket of a message with npk whole packets: 8 per octave,
// increasing with npk (messages without a whole packet share bucket 0)
__device__ __forceinline__ u32 bucket_of(u32 npk) {
    npk = npk ? npk : 1u;
    const u32 lz = 31u - (u32)__clz(npk);
    const u32 sub = lz >= 3u ? (npk >> (lz - 3u)) & 7u : (npk << (3u - lz)) & 7u;
    return lz * 8u + sub;
}

// smallest packet count of bucket b (inverse of bucket_of, at least 1)
__device__ __forceinline__ u64 bucket_floor(u32 b) {
    const u32 lz = b >> 3, sub = b & 7u;
    const u64 v = lz >= 3u ? (u64)(8u + sub) << (lz - 3u) : (u64)((8u + sub) >> (3u - lz));
    return v ? v : 1u;
}

// Isolation pays when the whole batch can stream from HBM in less than half
// the critical chain: packets * 32 B / 5.5 TB/s <= chain packets * 39 ns / 2,
// i.e. packets <= chain packets * 3350 (measured copy bandwidth and Update
// latency on MI355X).
constexpr u64 kIsoPacketsPerChainPacket = 3350;

__device__ __forceinline__ u32 packets_capped(u64 len) {
    const u64 npk = len >> 5;
    return npk > 0xffffffffull ? 0xffffffffu : (u32)npk;
}

__global__ __launch_bounds__(256) void hh_plan_reset_kernel(Plan* __restrict__ plan) {
    u32* w = (u32*)plan;
    for (u32 i = threadIdx.x; i < sizeof(Plan) / 4; i += blockDim.x) w[i] = 0u;
}

// Split threads per workgroup.  A workgroup reserves its long-list range with
// one global atomic per pass and flushes its histogram once: device-scope
// atomics on a few addresses serialise, and one per wave cost several
// microseconds on a 65,536-message batch.
constexpr u32 kSplitThreads = 1024;
constexpr u32 kSplitWaves = kSplitThreads / 64;

template <int W>
__global__ __launch_bounds__(kSplitThreads) void hh_split_kernel(
    const u64* __restrict__ keys, u32 n_keys, const u32* __restrict__ key_idx,
    const u8* __restrict__ data, u64 data_bytes, const u64* __restrict__ offsets,
    const u64* __restrict__ lengths, u64 n, u64* __restrict__ out, u64 long_min_bytes,
    Plan* __restrict__ plan, u32* __restrict__ long_list) {
    __shared__ u32 hist[kBuckets];
    __shared__ u32 wave_base[kSplitWaves];
    for (u32 i = threadIdx.x; i < kBuckets; i += kSplitThreads) hist[i] = 0u;
    const u32 lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const u64 stride = (u64)gridDim.x * kSplitThreads;
    // workgroup-uniform loop: every thread reaches the barriers
    for (u64 base = (u64)blockIdx.x * kSplitThreads; base < n; base += stride) {
        const u64 j = base + threadIdx.x;
        Msg m{nullptr, 0};
        bool is_long = false;
        if (j < n) {
            m = message(data, data_bytes, offsets[j], lengths[j]);
            is_long = m.len >= long_min_bytes;
        }
        const u64 mask = __ballot(is_long);
        __syncthreads();  // the previous pass has read wave_base
        if (lane == 0) wave_base[wave] = (u32)__popcll(mask);
        __syncthreads();
        if (threadIdx.x == 0) {
            u32 run = 0;
            for (u32 w = 0; w < kSplitWaves; ++w) {
                const u32 c = wave_base[w];
                wave_base[w] = run;
                run += c;
            }
            const u32 first = run ? atomicAdd(&plan->n_long, run) : 0u;
            for (u32 w = 0; w < kSplitWaves; ++w) wave_base[w] += first;
        }
        __syncthreads();
        if (is_long) {
            const u32 rank = __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
            const u32 at = wave_base[wave] + rank;
            if (at < n) long_list[at] = (u32)j;
            atomicAdd(&hist[bucket_of(packets_capped(m.len))], 1u);
        }
        if (j < n && !is_long) {
            const u64* kp = keys + 4 * key_index(key_idx, n_keys, j);
            const u64 key[4] = {kp[0], kp[1], kp[2], kp[3]};
            u64 sum[4];
            hash_thread<kThreadRing>(key, m.p, m.len, sum);
#pragma unroll
            for (int i = 0; i < W; ++i) out[(u64)W * j + i] = sum[i];
        }
    }
    __syncthreads();
    for (u32 i = threadIdx.x; i < kBuckets; i += kSplitThreads)
        if (hist[i]) atomicAdd(&plan->hist[i], hist[i]);
}

// Long list -> longest-first order.  Each block takes chunks of
// kScatterPer*256 entries, ranks them per bucket in LDS and reserves one range
// per bucket with a single global atomic.
constexpr int kScatterPer = 4;

__global__ __launch_bounds__(kBuckets) void hh_scatter_kernel(
    const u8* __restrict__ data, u64 data_bytes, const u64* __restrict__ offsets,
    const u64* __restrict__ lengths, Plan* __restrict__ plan, const u32* __restrict__ long_list,
    u32* __restrict__ order, u32 iso_cap, u32 n) {
    __shared__ u32 cnt[kBuckets];
    __shared__ u32 base[kBuckets];
    __shared__ u32 start[kBuckets];
    __shared__ unsigned long long total_packets;
    __shared__ u32 iso_s;
    // bucket starts: exclusive prefix over buckets, longest bucket first
    {
        const u32 t = threadIdx.x;
        const u32 b = kBuckets - 1u - t;
        const u32 c = plan->hist[b];
        cnt[t] = c;
        if (t == 0u) {
            total_packets = 0ull;
            iso_s = 0u;
        }
        __syncthreads();
        if (blockIdx.x == 0 && c)
            atomicAdd(&total_packets, (unsigned long long)c * bucket_floor(b));
        for (u32 d = 1; d < kBuckets; d <<= 1) {
            const u32 v = t >= d ? cnt[t - d] : 0u;
            __syncthreads();
            cnt[t] += v;
            __syncthreads();
        }
        start[b] = cnt[t] - c;
        // critical items: those holding the messages of the top octave of
        // lengths (8 buckets down from the longest non-empty one), when they
        // are few enough to give each a CU of its own and the rest of the
        // batch is light enough to run on the remaining CUs
        if (blockIdx.x == 0 && cnt[t] != 0u && (t == 0u || cnt[t - 1u] == 0u)) {
            const u32 top = cnt[t + 7u < kBuckets ? t + 7u : kBuckets - 1u];
            const u32 items = (top + 15u) >> 4;
            const bool light = total_packets <= bucket_floor(b) * kIsoPacketsPerChainPacket;
            iso_s = (items <= iso_cap && light) ? items : 0u;
        }
        __syncthreads();
        // for the persistent kernel, which runs after this one: the list
        // length, the critical items and a cleared item counter (the long
        // kernel of the previous sequence, its last user, has finished)
        if (blockIdx.x == 0 && t == 0u) {
            plan->n_order = min(plan->n_long, n);
            plan->n_iso = iso_s;
            plan->item_next = 0u;
        }
    }
    // the plan is this stream's own and zero before the split kernel ran, so
    // these bounds never bind; they keep every access inside the lists and
    // the caller's arrays whatever the plan holds
    const u32 n_long = min(plan->n_long, n);
    const u32 chunk = kScatterPer * 256u;
    for (u32 c0 = blockIdx.x * chunk; c0 < n_long; c0 += gridDim.x * chunk) {
        cnt[threadIdx.x] = 0u;
        __syncthreads();
        u32 jj[kScatterPer], bk[kScatterPer], rk[kScatterPer];
#pragma unroll
        for (int k = 0; k < kScatterPer; ++k) {
            const u32 i = c0 + (u32)k * 256u + threadIdx.x;
            bk[k] = kBuckets;
            if (i < n_long && long_list[i] < n) {
                jj[k] = long_list[i];
                const Msg m = message(data, data_bytes, offsets[jj[k]], lengths[jj[k]]);
                bk[k] = bucket_of(packets_capped(m.len));
                rk[k] = atomicAdd(&cnt[bk[k]], 1u);
            }
        }
        __syncthreads();
        {
            const u32 b = threadIdx.x;
            if (cnt[b]) base[b] = start[b] + atomicAdd(&plan->cursor[b], cnt[b]);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScatterPer; ++k)
            if (bk[k] < kBuckets && base[bk[k]] + rk[k] < n_long) order[base[bk[k]] + rk[k]] = jj[k];
        __syncthreads();
    }
}

// Run by one wave of hh_long_kernel: clear the split and scatter counters for
// the next sequence on this workspace (their last readers, the split and
// scatter kernels of this sequence, have finished; the calls of a workspace
// are ordered on its stream, and the end of this kernel makes the zeros
// visible to the next split kernel).  The persistent kernel reads none of
// these fields.
__device__ __forceinline__ void clear_split_counters(Plan* plan, u32 lane) {
    if (lane == 0) plan->n_long = 0u;
    for (u32 i = lane; i < kBuckets; i += 64u) {
        plan->hist[i] = 0u;
        plan->cursor[i] = 0u;
    }
}

// Persistent: 16 messages per item, 4 threads per message.  With n_iso
// critical items, wave 0 of workgroup b < n_iso takes item b and the other
// waves of that workgroup (one workgroup per CU) exit, so the critical chain
// has the CU to itself.  The remaining waves take items n_iso.. first,
// numbered so that consecutive items land on distinct workgroups, then items
// from plan->item_next (only when such dynamic items exist).
template <int W, int RING>
__global__ __launch_bounds__(256) void hh_long_kernel(
    const u64* __restrict__ keys, u32 n_keys, const u32* __restrict__ key_idx,
    const u8* __restrict__ data, u64 data_bytes, const u64* __restrict__ offsets,
    const u64* __restrict__ lengths, u64* __restrict__ out, Plan* __restrict__ plan,
    const u32* __restrict__ order, u32 n) {
    extern __shared__ u32 lds_reserve[];  // sized by the launch to set residency
    const u32 lane = threadIdx.x & 63u;
    const int q = (int)(lane & 3u);
    const u32 n_long = min(plan->n_order, n);  // never binds (see the scatter kernel)
    const u32 n_items = (n_long + 15u) >> 4;
    const u32 groups = gridDim.x, g = blockIdx.x, w = threadIdx.x >> 6;
    const u32 n_iso = min(plan->n_iso, groups);  // at most a quarter of the workgroups
    if (g == 0u && w == 3u) clear_split_counters(plan, lane);
    u32 item;
    if (g < n_iso) {
        if (w != 0u) return;
        item = g;
    } else {
        item = n_iso + w * (groups - n_iso) + (g - n_iso);
    }
    const u32 first_dynamic = n_iso + 4u * (groups - n_iso);
    const bool dynamic = first_dynamic < n_items;
    if (item >= n_items && threadIdx.x == 0) lds_reserve[0] = 0u;
    while (item < n_items) {
        const u32 k = 16u * item + (lane >> 2);
        // items come longest first: the item's first message decides whether
        // this wave's chain is long enough to claim its SIMD's issue slots
        const u32 first = min(__builtin_amdgcn_readfirstlane(order[16u * item]), n - 1u);
        const bool long_item = lengths[first] >= kPriorityBytes;
        if (long_item)
            __builtin_amdgcn_s_setprio(3);
        else
            __builtin_amdgcn_s_setprio(0);
        // a short item reserves the wave's next item now, so that the
        // atomic's round trip overlaps the item; a long one (its time dwarfs
        // the round trip) takes the next item only when it is done, so that
        // no item waits behind it
        u32 nxt = n_items;
        if (dynamic && !long_item && lane == 0)
            nxt = first_dynamic + atomicAdd(&plan->item_next, 1u);
        // the quads of a ragged last item repeat the item's first message
        // (same cache lines) and store nothing: the wave keeps all lanes on
        {
            const u32 jk = order[k < n_long ? k : 16u * item];
            const bool real = k < n_long && jk < n;
            const u32 j = real ? jk : first;
            const u64 key_q = keys[4 * key_index(key_idx, n_keys, j) + q];
            const Msg m = message(data, data_bytes, offsets[j], lengths[j]);
            const u64 sum = hash_quad<RING>(key_q, m.p, m.len, q);
            if (real && q < W) out[(u64)W * j + q] = sum;
        }
        if (dynamic && long_item && lane == 0)
            nxt = first_dynamic + atomicAdd(&plan->item_next, 1u);
        item = __builtin_amdgcn_readfirstlane(nxt);
    }
}

// ---------------------------------------------------------------------------
// host side: per (device, stream) workspace

namespace {

struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    u8* mem = nullptr;
    u64 cap_msgs = 0;
    Plan* plan = nullptr;
    u32* long_list = nullptr;
    u32* order = nullptr;
    bool dirty = false;  // plan not known to be zero (new, or a sequence failed part-way)
    // held from the lookup of the workspace through the last launch of a
    // sequence: host threads that share a stream enqueue whole sequences one
    // after another (interleaved launches would mix their plans), and none
    // regrows the buffers while another enqueues against them
    std::mutex mu;
};

std::mutex g_ws_mutex;
// a list: a workspace keeps its address while other threads add theirs
std::list<Workspace> g_ws;

// measurement hook: event pairs around hh_long_kernel launches
struct EventPair {
    hipEvent_t start, stop;
};
std::mutex g_timing_mutex;
bool g_timing_on = false;
std::vector<EventPair> g_timing_pool;     // created, reusable
std::vector<EventPair> g_timing_pending;  // recorded, not yet collected
constexpr size_t kMaxPendingPairs = 4096;

EventPair* timing_begin(hipStream_t st) {
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    if (!g_timing_on || g_timing_pending.size() >= kMaxPendingPairs) return nullptr;
    EventPair p;
    if (!g_timing_pool.empty()) {
        p = g_timing_pool.back();
        g_timing_pool.pop_back();
    } else if (hipEventCreate(&p.start) != hipSuccess || hipEventCreate(&p.stop) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    (void)st;
    g_timing_pending.push_back(p);
    return &g_timing_pending.back();
}

struct DeviceInfo {
    int cus;
    int lds_per_cu;
    int lds_per_block;
};

DeviceInfo device_info(int dev) {
    static std::mutex m;
    static DeviceInfo cache[64];
    static bool have[64];
    std::lock_guard<std::mutex> lock(m);
    if (dev >= 0 && dev < 64 && have[dev]) return cache[dev];
    DeviceInfo d{0, 0, 0};
    if (hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        d.cus <= 0)
        d.cus = 256;
    if (hipDeviceGetAttribute(&d.lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              dev) != hipSuccess)
        d.lds_per_cu = 0;
    if (hipDeviceGetAttribute(&d.lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
        hipSuccess)
        d.lds_per_block = 0;
    (void)hipGetLastError();
    if (dev >= 0 && dev < 64) {
        cache[dev] = d;
        have[dev] = true;
    }
    return d;
}

u64 align_up(u64 x, u64 a) { return (x + a - 1) / a * a; }

void drop_graphs_of(const u8* ws_mem);

// The workspace of (dev, st), grown to hold n messages, returned with its
// mutex held by `hold` (the caller keeps it until its launches are enqueued).
hh_status get_workspace(int dev, hipStream_t st, u64 n, Workspace** out,
                        std::unique_lock<std::mutex>* hold) {
    Workspace* ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_ws_mutex);
        for (auto& w : g_ws)
            if (w.device == dev && w.stream == st) ws = &w;
        if (!ws) {
            ws = &g_ws.emplace_back();
            ws->device = dev;
            ws->stream = st;
        }
    }
    *hold = std::unique_lock<std::mutex>(ws->mu);
    if (ws->cap_msgs < n || !ws->mem) {
        u64 cap = ws->cap_msgs ? ws->cap_msgs : 1024;
        while (cap < n) cap *= 2;
        const u64 plan_bytes = align_up(sizeof(Plan), 256);
        const u64 list_bytes = align_up(4 * cap, 256);
        u8* mem = nullptr;
        if (ws->mem) {
            // earlier work on this stream may still read the old buffers
            if (hipStreamSynchronize(st) != hipSuccess) return HH_ERR_LAUNCH;
            drop_graphs_of(ws->mem);
            (void)hipFree(ws->mem);
            ws->mem = nullptr;
            ws->cap_msgs = 0;
        }
        if (hipMalloc(&mem, plan_bytes + 2 * list_bytes) != hipSuccess) {
            (void)hipGetLastError();
            return HH_ERR_OUT_OF_MEMORY;
        }
        ws->mem = mem;
        ws->cap_msgs = cap;
        ws->plan = (Plan*)mem;
        ws->long_list = (u32*)(mem + plan_bytes);
        ws->order = (u32*)(mem + plan_bytes + list_bytes);
        // the first sequence zeroes the plan with a kernel on this stream: a
        // memset on the null stream is not ordered before work on a
        // non-blocking stream
        ws->dirty = true;
    }
    *out = ws;
    return HH_OK;
}

struct LaunchShape {
    u32 long_blocks;
    u32 lds;
    unsigned split_blocks;
    unsigned scatter_blocks;
    u32 iso_cap;  // most critical items given a CU each (0: isolation off)
};

LaunchShape launch_shape(const HashArgs& a, const DeviceInfo& di, const hh_tuning& tun) {
    LaunchShape ls;
    const u32 waves_per_cu = tun.waves_per_cu ? tun.waves_per_cu : 4u;
    const u32 blocks_per_cu = (waves_per_cu + 3u) / 4u;
    ls.long_blocks = (u32)di.cus * blocks_per_cu;
    // LDS per workgroup so that only blocks_per_cu workgroups fit on a CU
    ls.lds = 0;
    if (di.lds_per_cu > 0) {
        ls.lds = (u32)di.lds_per_cu / (blocks_per_cu + 1u) + 1024u;
        if (di.lds_per_block > 0 && ls.lds > (u32)di.lds_per_block) ls.lds = (u32)di.lds_per_block;
        ls.lds &= ~255u;
    }
    // a workgroup owns its CU only when one fits per CU
    ls.iso_cap = (tun.isolate_long && blocks_per_cu == 1u) ? ls.long_blocks / 4u : 0u;
    ls.split_blocks = (unsigned)std::min<u64>((a.n + kSplitThreads - 1) / kSplitThreads, 512);
    ls.scatter_blocks =
        (unsigned)std::min<u64>((a.n + kScatterPer * 256 - 1) / (kScatterPer * 256), 1024);
    return ls;
}

// The launches of one bucketed call: split, scatter, persistent kernel (whose
// last wave leaves the plan zeroed for the next call; launch_bucketed_w runs
// hh_plan_reset_kernel on the stream before a new workspace's first sequence
// and after a sequence that failed part-way).  `ev` (may be null) brackets the
// persistent kernel for the measurement hook.
template <int W>
void enqueue_sequence(const HashArgs& a, hipStream_t st, Workspace* ws, const LaunchShape& ls,
                      const hh_tuning& tun, EventPair* ev) {
    hipLaunchKernelGGL(hh_split_kernel<W>, dim3(ls.split_blocks), dim3(kSplitThreads), 0, st, a.keys,
                       a.n_keys, a.key_idx, a.data, a.data_bytes, a.offsets, a.lengths, a.n, a.out,
                       (u64)tun.lane4_min_bytes, ws->plan, ws->long_list);
    hipLaunchKernelGGL(hh_scatter_kernel, dim3(ls.scatter_blocks), dim3(kBuckets), 0, st, a.data,
                       a.data_bytes, a.offsets, a.lengths, ws->plan, ws->long_list, ws->order,
                       ls.iso_cap, (u32)a.n);
    if (ev && hipEventRecord(ev->start, st) != hipSuccess) (void)hipGetLastError();
#define HH_LONG(RING)                                                                        \
    hipLaunchKernelGGL((hh_long_kernel<W, RING>), dim3(ls.long_blocks), dim3(256), ls.lds, st, \
                       a.keys, a.n_keys, a.key_idx, a.data, a.data_bytes, a.offsets, a.lengths, \
                       a.out, ws->plan, ws->order, (u32)a.n)
    switch (tun.long_ring) {
        case 36: HH_LONG(36); break;
        case 48: HH_LONG(48); break;
        case 96: HH_LONG(96); break;
        default: HH_LONG(72); break;
    }
#undef HH_LONG
    if (ev && hipEventRecord(ev->stop, st) != hipSuccess) (void)hipGetLastError();
}

// ---------------------------------------------------------------------------
// hipGraph cache: one instantiated graph per (stream, arguments, tuning,
// workspace), least recently used evicted beyond kMaxGraphs.

struct GraphEntry {
    HashArgs a;
    hipStream_t st;
    hh_tuning tun;
    const u8* ws_mem;
    u64 ws_cap;
    hipGraphExec_t exec;
    u64 last_use;
};

constexpr size_t kMaxGraphs = 16;
std::mutex g_graph_mutex;
std::vector<GraphEntry> g_graphs;
u64 g_graph_clock = 0;

bool same_call(const GraphEntry& e, const HashArgs& a, hipStream_t st, const hh_tuning& t,
               const Workspace* ws) {
    return e.st == st && e.ws_mem == ws->mem && e.ws_cap == ws->cap_msgs && e.a.keys == a.keys &&
           e.a.n_keys == a.n_keys && e.a.key_idx == a.key_idx && e.a.data == a.data &&
           e.a.data_bytes == a.data_bytes && e.a.offsets == a.offsets &&
           e.a.lengths == a.lengths && e.a.n == a.n && e.a.out == a.out && e.a.width == a.width &&
           e.tun.lane4_min_bytes == t.lane4_min_bytes && e.tun.waves_per_cu == t.waves_per_cu &&
           e.tun.long_ring == t.long_ring && e.tun.isolate_long == t.isolate_long;
}

void drop_graphs_of(const u8* ws_mem) {
    std::lock_guard<std::mutex> lock(g_graph_mutex);
    for (size_t i = 0; i < g_graphs.size();) {
        if (g_graphs[i].ws_mem == ws_mem) {
            (void)hipGraphExecDestroy(g_graphs[i].exec);
            g_graphs.erase(g_graphs.begin() + i);
        } else {
            ++i;
        }
    }
}

template <int W>
hh_status launch_graph(const HashArgs& a, hipStream_t st, Workspace* ws, const LaunchShape& ls,
                       const hh_tuning& tun) {
    std::lock_guard<std::mutex> lock(g_graph_mutex);
    for (auto& e : g_graphs) {
        if (same_call(e, a, st, tun, ws)) {
            e.last_use = ++g_graph_clock;
            return hipGraphLaunch(e.exec, st) == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
        }
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return HH_ERR_LAUNCH;
    }
    enqueue_sequence<W>(a, st, ws, ls, tun, nullptr);
    const hipError_t launch_err = hipGetLastError();
    const hipError_t end_err = hipStreamEndCapture(st, &graph);
    if (launch_err != hipSuccess || end_err != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return HH_ERR_LAUNCH;
    }
    const hipError_t inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (inst != hipSuccess) {
        (void)hipGetLastError();
        return HH_ERR_LAUNCH;
    }
    if (g_graphs.size() >= kMaxGraphs) {
        size_t lru = 0;
        for (size_t i = 1; i < g_graphs.size(); ++i)
            if (g_graphs[i].last_use < g_graphs[lru].last_use) lru = i;
        (void)hipGraphExecDestroy(g_graphs[lru].exec);
        g_graphs.erase(g_graphs.begin() + lru);
    }
    g_graphs.push_back(GraphEntry{a, st, tun, ws->mem, ws->cap_msgs, exec, ++g_graph_clock});
    return hipGraphLaunch(exec, st) == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

template <int W>
hh_status launch_bucketed_w(const HashArgs& a, hipStream_t st, Workspace* ws, const DeviceInfo& di,
                            const hh_tuning& tun) {
    const LaunchShape ls = launch_shape(a, di, tun);
    // a plan that is not known to be zero (a new workspace, or a sequence that
    // failed part-way) is zeroed on this stream first, outside any graph
    if (ws->dirty) {
        hipLaunchKernelGGL(hh_plan_reset_kernel, dim3(1), dim3(256), 0, st, ws->plan);
        if (hipGetLastError() != hipSuccess) return HH_ERR_LAUNCH;
        ws->dirty = false;
    }
    EventPair* ev = timing_begin(st);
    hh_status s;
    // the null stream cannot be captured; timed calls launch directly
    if (tun.use_graph && st != nullptr && !ev) {
        s = launch_graph<W>(a, st, ws, ls, tun);
    } else {
        enqueue_sequence<W>(a, st, ws, ls, tun, ev);
        s = hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
    }
    if (s != HH_OK) ws->dirty = true;
    return s;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free variant (hh_hash_noalloc): the plan and the two index lists
// of at most HH_NOALLOC_MAX_MSGS messages live in `scratch`, a fixed array in
// the library's code object.  Every GPU holds its own copy at its own address;
// host code reaches it only through the address looked up per device below
// (the array's name on the host is a stand-in, not a device address).

constexpr u64 kNoallocPlanBytes = (sizeof(Plan) + 255) / 256 * 256;
constexpr u64 kNoallocListBytes = 4ull * HH_NOALLOC_MAX_MSGS;
constexpr u64 kNoallocScratchBytes = kNoallocPlanBytes + 2 * kNoallocListBytes;
static_assert(kNoallocScratchBytes == HH_NOALLOC_SCRATCH_BYTES, "hh.h states the array's size");

}  // namespace hh

static __device__ __align__(256) unsigned char scratch[hh::kNoallocScratchBytes];

namespace hh {

namespace {

constexpr int kNoallocDevices = 64;
std::mutex g_scratch_mutex;
u8* g_scratch_ptr[kNoallocDevices];  // device address of `scratch` per GPU

// device address of this GPU's `scratch` (dev must be the current device);
// looked up on the first call on each device, no allocation
hh_status scratch_address(int dev, u8** out) {
    if (dev < 0 || dev >= kNoallocDevices) return HH_ERR_UNSUPPORTED_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return HH_ERR_LAUNCH;
        }
        g_scratch_ptr[dev] = (u8*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return HH_OK;
}

}  // namespace

hh_status launch_bucketed_noalloc(const HashArgs& a, hipStream_t st) {
    if (a.n > HH_NOALLOC_MAX_MSGS) return HH_ERR_INVALID_ARG;
    int dev = 0;
    hh_status s = check_device(&dev);
    if (s != HH_OK) return s;
    u8* base = nullptr;
    if ((s = scratch_address(dev, &base)) != HH_OK) return s;
    Workspace ws;
    ws.device = dev;
    ws.stream = st;
    ws.mem = base;
    ws.cap_msgs = HH_NOALLOC_MAX_MSGS;
    ws.plan = (Plan*)base;
    ws.long_list = (u32*)(base + kNoallocPlanBytes);
    ws.order = (u32*)(base + kNoallocPlanBytes + kNoallocListBytes);
    const DeviceInfo di = device_info(dev);
    const hh_tuning tun = current_tuning();
    const LaunchShape ls = launch_shape(a, di, tun);
    // the array keeps whatever the last call on this GPU left: clear the plan
    // with a kernel (the lists are written before they are read)
    hipLaunchKernelGGL(hh_plan_reset_kernel, dim3(1), dim3(256), 0, st, ws.plan);
    switch (a.width) {
        case 1: enqueue_sequence<1>(a, st, &ws, ls, tun, nullptr); break;
        case 2: enqueue_sequence<2>(a, st, &ws, ls, tun, nullptr); break;
        default: enqueue_sequence<4>(a, st, &ws, ls, tun, nullptr); break;
    }
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

// Messages are processed in chunks of at most 2^30 so that indices fit 32 bits.
hh_status launch_bucketed(const HashArgs& a, hipStream_t st) {
    int dev = 0;
    hh_status s = check_device(&dev);
    if (s != HH_OK) return s;
    const DeviceInfo di = device_info(dev);
    const hh_tuning tun = current_tuning();
    const u64 chunk = 1ull << 30;
    for (u64 first = 0; first < a.n; first += chunk) {
        HashArgs c = a;
        c.n = std::min<u64>(chunk, a.n - first);
        c.offsets = a.offsets + first;
        c.lengths = a.lengths + first;
        c.key_idx = a.key_idx ? a.key_idx + first : nullptr;
        c.out = a.out + first * a.width;
        Workspace* ws = nullptr;
        std::unique_lock<std::mutex> hold;
        if ((s = get_workspace(dev, st, c.n, &ws, &hold)) != HH_OK) return s;
        switch (a.width) {
            case 1: s = launch_bucketed_w<1>(c, st, ws, di, tun); break;
            case 2: s = launch_bucketed_w<2>(c, st, ws, di, tun); break;
            default: s = launch_bucketed_w<4>(c, st, ws, di, tun); break;
        }
        if (s != HH_OK) return s;
    }
    return HH_OK;
}

hh_status timing_enable(bool on) {
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    g_timing_on = on;
    return HH_OK;
}

hh_status timing_collect(uint32_t* launches, double* total_ms) {
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    double sum = 0.0;
    uint32_t n = 0;
    hh_status s = HH_OK;
    for (auto& p : g_timing_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.stop) == hipSuccess &&
            hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            sum += ms;
            ++n;
        } else {
            (void)hipGetLastError();
            s = HH_ERR_LAUNCH;
        }
        g_timing_pool.push_back(p);
    }
    g_timing_pending.clear();
    if (launches) *launches = n;
    if (total_ms) *total_ms = sum;
    return s;
}

void release_bucketed() {
    {
        std::lock_guard<std::mutex> lock(g_graph_mutex);
        for (auto& e : g_graphs) (void)hipGraphExecDestroy(e.exec);
        g_graphs.clear();
    }
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    for (auto& w : g_ws) {
        if (w.mem) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(w.device);
            (void)hipStreamSynchronize(w.stream);
            (void)hipFree(w.mem);
            (void)hipSetDevice(cur);
        }
    }
    g_ws.clear();
}

}  // namespace hh
