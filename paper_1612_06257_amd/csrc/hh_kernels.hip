// hh_kernels.hip -- the single-launch HighwayHash kernels for gfx950 and
// their launchers (the C ABI of include/hh.h is in hh_api.hip).
//
// Kernels (all hash exactly the bytes named by offsets/lengths, clamped to the
// buffer):
//   hh_thread_kernel<W, RING>  one thread per message, the whole 1024-bit
//                        state in VGPRs; the plain one-launch kernel (RING
//                        packets in flight: 1 for mixed short batches, 8 for
//                        uniform lengths of 8 packets or more).
//   hh_quad_kernel<W>    four threads per message, one 64-bit lane each;
//                        shorter dependency chain per packet for long messages.
//   hh_prf_kernel<W>     counter-mode PRF: 8-byte counters built in registers.
// The bucketed planner and persistent kernel live in hh_batched.hip, the
// incremental-state and segment-copy kernels in hh_state.hip, the feed in
// hh_feed.hip, the avalanche statistics in hh_stats.hip.

#include <atomic>

#include "hh_device.hpp"
#include "hh_internal.hpp"
#include "hh_msg.hpp"

namespace hh {

template <int W, int RING>
__global__ __launch_bounds__(64) void hh_thread_kernel(
    const u64* __restrict__ keys, u32 n_keys, const u32* __restrict__ key_idx,
    const u8* __restrict__ data, u64 data_bytes, const u64* __restrict__ offsets,
    const u64* __restrict__ lengths, u64 uniform_length, u64 n, u64* __restrict__ out) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 j = (u64)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        const u64* kp = keys + 4 * key_index(key_idx, n_keys, j);
        const u64 key[4] = {kp[0], kp[1], kp[2], kp[3]};
        const Msg m = message(data, data_bytes, offsets[j], lengths ? lengths[j] : uniform_length);
        u64 sum[4];
        hash_thread<RING>(key, m.p, m.len, sum);
#pragma unroll
        for (int i = 0; i < W; ++i) out[(u64)W * j + i] = sum[i];
    }
}

template <int W>
__global__ __launch_bounds__(256) void hh_quad_kernel(
    const u64* __restrict__ keys, u32 n_keys, const u32* __restrict__ key_idx,
    const u8* __restrict__ data, u64 data_bytes, const u64* __restrict__ offsets,
    const u64* __restrict__ lengths, u64 n, u64* __restrict__ out) {
    const int q = threadIdx.x & 3;
    const u64 quad = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
    const u64 stride = ((u64)gridDim.x * blockDim.x) >> 2;  // a multiple of 16
    // wave-uniform loop: quads past n repeat the wave's first message and
    // store nothing, so the wave keeps every lane on (a partly masked wave
    // runs the chain about 10% slower)
    for (u64 base = quad & ~15ull; base < n; base += stride) {
        const u64 k = base + (quad & 15u);
        const bool real = k < n;
        const u64 j = real ? k : base;
        const u64 key_q = keys[4 * key_index(key_idx, n_keys, j) + q];
        const Msg m = message(data, data_bytes, offsets[j], lengths[j]);
        const u64 sum = hash_quad<kQuadRing>(key_q, m.p, m.len, q);
        if (real && q < W) out[(u64)W * j + q] = sum;
    }
}

// ---------------------------------------------------------------------------
// Counter-mode keyed PRF: message j is the 8-byte little-endian encoding of
// c = counter_base + j (mod 2^64), hashed under key c mod n_keys.  An 8-byte
// message has no whole packet; its remainder packet (Sec. 4.5, r = 8) is the
// counter in lane 0 and zeros, so nothing is read but the key.

// The part of an 8-byte message's hash that does not depend on the counter,
// for one key (Sec. 4.4, 4.5, 4.2): Reset; the size injection and v1
// rotation of the remainder step (r = 8); the absorb of the padded packet's
// zero words into lanes 1..3; the ZipperMerges of lane pair (2,3), whose
// inputs are then complete.  Lane 0 keeps v1 + mul0 (`a0`) and v0 as the
// absorb reads it (`v0_in`), and v0 + mul1 in the state, all independent of
// the counter.
struct PrfKey {
    State4 s;
    u64 a0, v0_in;
};

__device__ __forceinline__ void prf_prepare(const u64 key[4], PrfKey& k) {
    State4& s = k.s;
    reset4(s, key);
    const u64 inject = (8ull << 32) + 8ull;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        s.v0[i] += inject;
        s.v1[i] = rotl_halves(s.v1[i], 8u);
    }
#pragma unroll
    for (int i = 1; i < 4; ++i) {
        s.v1[i] += s.mul0[i];  // + the packet word, 0
        s.mul0[i] ^= mul_lo_hi(s.v1[i], s.v0[i]);
        s.v0[i] += s.mul1[i];
        s.mul1[i] ^= mul_lo_hi(s.v0[i], s.v1[i]);
    }
    k.a0 = s.v1[0] + s.mul0[0];
    k.v0_in = s.v0[0];
    s.v0[0] += s.mul1[0];
    u64 z2, z3;
    zipper_pair(s.v1[2], s.v1[3], z2, z3);
    s.v0[2] += z2;
    s.v0[3] += z3;
    zipper_pair(s.v0[2], s.v0[3], z2, z3);
    s.v1[2] += z2;
    s.v1[3] += z3;
}

// The rest of the remainder Update for counter c (lane 0 absorbs c, then the
// lane pair (0,1) is merged), then the finalization.
__device__ __forceinline__ void prf_finish(const PrfKey& k, u64 c, u64 sum[4]) {
    State4 s = k.s;
    s.v1[0] = k.a0 + c;
    s.mul0[0] ^= mul_lo_hi(s.v1[0], k.v0_in);
    s.mul1[0] ^= mul_lo_hi(s.v0[0], s.v1[0]);
    u64 z0, z1;
    zipper_pair(s.v1[0], s.v1[1], z0, z1);
    s.v0[0] += z0;
    s.v0[1] += z1;
    zipper_pair(s.v0[0], s.v0[1], z0, z1);
    s.v1[0] += z0;
    s.v1[1] += z1;
    finalize4(s, sum);
}

template <int W>
__global__ __launch_bounds__(256) void hh_prf_kernel(const u64* __restrict__ keys, u32 n_keys,
                                                     u64 counter_base, u64 n, u64 stride,
                                                     u64* __restrict__ out) {
    const u64 j0 = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (j0 >= stride) return;
    if (stride % n_keys == 0) {
        // every counter of this thread takes the same key: its
        // counter-independent part is computed once
        const u64* kp = keys + 4 * ((counter_base + j0) % n_keys);
        const u64 key[4] = {kp[0], kp[1], kp[2], kp[3]};
        PrfKey pk;
        prf_prepare(key, pk);
        for (u64 j = j0; j < n; j += stride) {
            u64 sum[4];
            prf_finish(pk, counter_base + j, sum);
#pragma unroll
            for (int i = 0; i < W; ++i) out[(u64)W * j + i] = sum[i];
        }
        return;
    }
    for (u64 j = j0; j < n; j += stride) {
        const u64 c = counter_base + j;
        const u64* kp = keys + 4 * (c % n_keys);
        const u64 key[4] = {kp[0], kp[1], kp[2], kp[3]};
        State4 s;
        reset4(s, key);
        const u64 pk[4] = {c, 0, 0, 0};
        remainder4(s, 8u, pk);
        u64 sum[4];
        finalize4(s, sum);
#pragma unroll
        for (int i = 0; i < W; ++i) out[(u64)W * j + i] = sum[i];
    }
}

// ---------------------------------------------------------------------------
// host-side launchers

namespace {

unsigned grid_for(u64 threads, unsigned block) {
    u64 g = (threads + block - 1) / block;
    const u64 cap = 1u << 20;  // grid-stride loops cover the rest
    if (g > cap) g = cap;
    return (unsigned)(g ? g : 1);
}

}  // namespace

template <int RING>
hh_status launch_thread_ring(const HashArgs& a, u64 uniform_length, hipStream_t st) {
    // one-wave workgroups: a retiring wave frees its slot for the next at once
    const unsigned block = 64;
    const unsigned grid = grid_for(a.n, block);
    const u64* lengths = a.lengths;
    switch (a.width) {
        case 1: hipLaunchKernelGGL((hh_thread_kernel<1, RING>), dim3(grid), dim3(block), 0, st,
                                   a.keys, a.n_keys, a.key_idx, a.data, a.data_bytes, a.offsets,
                                   lengths, uniform_length, a.n, a.out); break;
        case 2: hipLaunchKernelGGL((hh_thread_kernel<2, RING>), dim3(grid), dim3(block), 0, st,
                                   a.keys, a.n_keys, a.key_idx, a.data, a.data_bytes, a.offsets,
                                   lengths, uniform_length, a.n, a.out); break;
        default: hipLaunchKernelGGL((hh_thread_kernel<4, RING>), dim3(grid), dim3(block), 0, st,
                                    a.keys, a.n_keys, a.key_idx, a.data, a.data_bytes, a.offsets,
                                    lengths, uniform_length, a.n, a.out); break;
    }
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

// Uniform launches know their length: one of kThreadDeepMinPackets packets or
// more takes the deep-ring kernel (its few long chains are latency-bound, not
// occupancy-bound); mixed-length launches take the short-message kernel.
constexpr u64 kThreadDeepMinPackets = 8;

hh_status launch_thread(const HashArgs& a, u64 uniform_length, hipStream_t st) {
    if (!a.lengths && (uniform_length >> 5) >= kThreadDeepMinPackets)
        return launch_thread_ring<kThreadDeepRing>(a, uniform_length, st);
    return launch_thread_ring<kThreadRing>(a, uniform_length, st);
}

// Quad-layout launches use one-wave workgroups: the dispatcher spreads them
// over the CUs, so fewer long chains share a CU's load path (four waves of
// one workgroup on a CU ran each chain about 10% slower; serving saturation
// 179-182 -> 201-204 GB/s with the state kernels launched this way).
constexpr unsigned kQuadBlock = 64;

hh_status launch_quad(const HashArgs& a, hipStream_t st) {
    const unsigned block = kQuadBlock;
    const unsigned grid = grid_for(4 * a.n, block);
    switch (a.width) {
        case 1: hipLaunchKernelGGL(hh_quad_kernel<1>, dim3(grid), dim3(block), 0, st, a.keys,
                                   a.n_keys, a.key_idx, a.data, a.data_bytes, a.offsets,
                                   a.lengths, a.n, a.out); break;
        case 2: hipLaunchKernelGGL(hh_quad_kernel<2>, dim3(grid), dim3(block), 0, st, a.keys,
                                   a.n_keys, a.key_idx, a.data, a.data_bytes, a.offsets,
                                   a.lengths, a.n, a.out); break;
        default: hipLaunchKernelGGL(hh_quad_kernel<4>, dim3(grid), dim3(block), 0, st, a.keys,
                                    a.n_keys, a.key_idx, a.data, a.data_bytes, a.offsets,
                                    a.lengths, a.n, a.out); break;
    }
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

// Counter-mode PRF launch: a persistent grid whose thread count (the loop
// stride) is a multiple of n_keys when that fits, so that each thread keeps
// one key for all its counters.
template <int W>
u32 prf_resident_threads(unsigned block) {
    static std::atomic<u32> per_cu{0};
    u32 b = per_cu.load(std::memory_order_relaxed);
    if (!b) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, hh_prf_kernel<W>, (int)block, 0) !=
                hipSuccess ||
            nb < 1) {
            (void)hipGetLastError();
            nb = 1;
        }
        b = (u32)nb;
        per_cu.store(b, std::memory_order_relaxed);
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1) {
        (void)hipGetLastError();
        cus = 256;
    }
    return (u32)cus * b * block;
}

template <int W>
void launch_prf_w(const u64* keys, u32 n_keys, u64 counter_base, u64 n, u64* out,
                  hipStream_t st) {
    const unsigned block = 256;
    u64 stride = prf_resident_threads<W>(block);
    if (stride >= n_keys) stride = stride / n_keys * n_keys;
    if (stride > n) stride = n;
    const unsigned grid = grid_for(stride, block);
    hipLaunchKernelGGL(hh_prf_kernel<W>, dim3(grid), dim3(block), 0, st, keys, n_keys,
                       counter_base, n, stride, out);
}

hh_status launch_prf(u32 width, const u64* keys, u32 n_keys, u64 counter_base, u64 n, u64* out,
                     hipStream_t st) {
    switch (width) {
        case 1: launch_prf_w<1>(keys, n_keys, counter_base, n, out, st); break;
        case 2: launch_prf_w<2>(keys, n_keys, counter_base, n, out, st); break;
        default: launch_prf_w<4>(keys, n_keys, counter_base, n, out, st); break;
    }
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

}  // namespace hh
