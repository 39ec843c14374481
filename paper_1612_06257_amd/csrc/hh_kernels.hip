// hh_kernels.hip -- HighwayHash kernels for gfx950 and the C ABI of include/hh.h.
//
// Kernels (all hash exactly the bytes named by offsets/lengths, clamped to the
// buffer):
//   hh_thread_kernel<W>  one thread per message, the whole 1024-bit state in
//                        VGPRs; the plain one-launch kernel.
//   hh_quad_kernel<W>    four threads per message, one 64-bit lane each;
//                        shorter dependency chain per packet for long messages.
//   hh_state_*_kernel    incremental hashing over caller-owned device states.
// The bucketed planner and persistent kernel live in hh_batched.hip.

#include "hh_device.hpp"
#include "hh_internal.hpp"
#include "hh_msg.hpp"

namespace hh {

template <int W>
__global__ __launch_bounds__(256) void hh_thread_kernel(
    const u64* __restrict__ keys, u32 n_keys, const u32* __restrict__ key_idx,
    const u8* __restrict__ data, u64 data_bytes, const u64* __restrict__ offsets,
    const u64* __restrict__ lengths, u64 uniform_length, u64 n, u64* __restrict__ out) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 j = (u64)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        const u64* kp = keys + 4 * key_index(key_idx, n_keys, j);
        const u64 key[4] = {kp[0], kp[1], kp[2], kp[3]};
        const Msg m = message(data, data_bytes, offsets[j], lengths ? lengths[j] : uniform_length);
        u64 sum[4];
        hash_thread(key, m.p, m.len, sum);
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
    const u64 stride = ((u64)gridDim.x * blockDim.x) >> 2;
    for (u64 j = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 2; j < n; j += stride) {
        const u64 key_q = keys[4 * key_index(key_idx, n_keys, j) + q];
        const Msg m = message(data, data_bytes, offsets[j], lengths[j]);
        const u64 sum = hash_quad<kQuadRing>(key_q, m.p, m.len, q);
        if (q < W) out[(u64)W * j + q] = sum;
    }
}

// ---------------------------------------------------------------------------
// Counter-mode keyed PRF: message j is the 8-byte little-endian encoding of
// c = counter_base + j (mod 2^64), hashed under key c mod n_keys.  An 8-byte
// message has no whole packet; its remainder packet (Sec. 4.5, r = 8) is the
// counter in lane 0 and zeros, so nothing is read but the key.

template <int W>
__global__ __launch_bounds__(256) void hh_prf_kernel(const u64* __restrict__ keys, u32 n_keys,
                                                     u64 counter_base, u64 n,
                                                     u64* __restrict__ out) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 j = (u64)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
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
// incremental hashing: states[16*s + 4*v + q] = lane q of vector v
// (v0, v1, mul0, mul1).

__device__ __forceinline__ void load_state1(State1& s, const u64* st, int q) {
    s.v0 = st[q];
    s.v1 = st[4 + q];
    s.mul0 = st[8 + q];
    s.mul1 = st[12 + q];
    s.sel_hi = (q & 1) ? 0x07000601u : 0x00070106u;
}

__device__ __forceinline__ void store_state1(const State1& s, u64* st, int q) {
    st[q] = s.v0;
    st[4 + q] = s.v1;
    st[8 + q] = s.mul0;
    st[12 + q] = s.mul1;
}

__global__ __launch_bounds__(256) void hh_state_init_kernel(
    const u64* __restrict__ keys, u32 n_keys, const u32* __restrict__ key_idx,
    u64* __restrict__ states, u64 n) {
    const int q = threadIdx.x & 3;
    const u64 stride = ((u64)gridDim.x * blockDim.x) >> 2;
    for (u64 j = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 2; j < n; j += stride) {
        State1 s;
        reset1(s, keys[4 * key_index(key_idx, n_keys, j) + q], q);
        store_state1(s, states + 16 * j, q);
    }
}

template <bool FINAL>
__global__ __launch_bounds__(256) void hh_state_step_kernel(
    u64* __restrict__ states, const u32* __restrict__ state_idx, const u8* __restrict__ data,
    u64 data_bytes, const u64* __restrict__ offsets, const u64* __restrict__ lengths,
    const u8* __restrict__ width_words, u64* __restrict__ out,
    const u64* __restrict__ out_offsets, u64 n) {
    const int q = threadIdx.x & 3;
    const u64 stride = ((u64)gridDim.x * blockDim.x) >> 2;
    for (u64 k = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 2; k < n; k += stride) {
        u64* st = states + 16 * (state_idx ? (u64)state_idx[k] : k);
        const Msg m = message(data, data_bytes, offsets[k], lengths[k]);
        const u32 r = FINAL ? (u32)(m.len & 31u) : 0u;
        const u64 tail = r ? remainder_lane(m.p + 32 * (m.len >> 5), r, q) : 0;
        State1 s;
        load_state1(s, st, q);
        absorb_quad_all<kStateRing>(s, m.p, m.len >> 5, q);
        if (!FINAL) {
            store_state1(s, st, q);
        } else {
            if (r) remainder1(s, r, tail);
            const u64 sum = finalize1(s);
            const u32 w = width_words ? width_words[k] : 1u;
            const u64 o = out_offsets ? out_offsets[k] : 4 * k;
            if ((u32)q < w) out[o + q] = sum;
        }
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

hh_status launch_thread(const HashArgs& a, u64 uniform_length, hipStream_t st) {
    const unsigned block = 256;
    const unsigned grid = grid_for(a.n, block);
    const u64* lengths = a.lengths;
    switch (a.width) {
        case 1: hipLaunchKernelGGL(hh_thread_kernel<1>, dim3(grid), dim3(block), 0, st, a.keys,
                                   a.n_keys, a.key_idx, a.data, a.data_bytes, a.offsets, lengths,
                                   uniform_length, a.n, a.out); break;
        case 2: hipLaunchKernelGGL(hh_thread_kernel<2>, dim3(grid), dim3(block), 0, st, a.keys,
                                   a.n_keys, a.key_idx, a.data, a.data_bytes, a.offsets, lengths,
                                   uniform_length, a.n, a.out); break;
        default: hipLaunchKernelGGL(hh_thread_kernel<4>, dim3(grid), dim3(block), 0, st, a.keys,
                                    a.n_keys, a.key_idx, a.data, a.data_bytes, a.offsets, lengths,
                                    uniform_length, a.n, a.out); break;
    }
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

hh_status launch_quad(const HashArgs& a, hipStream_t st) {
    const unsigned block = 256;
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

hh_status launch_prf(u32 width, const u64* keys, u32 n_keys, u64 counter_base, u64 n, u64* out,
                     hipStream_t st) {
    const unsigned block = 256;
    const unsigned grid = grid_for(n, block);
    switch (width) {
        case 1: hipLaunchKernelGGL(hh_prf_kernel<1>, dim3(grid), dim3(block), 0, st, keys, n_keys,
                                   counter_base, n, out); break;
        case 2: hipLaunchKernelGGL(hh_prf_kernel<2>, dim3(grid), dim3(block), 0, st, keys, n_keys,
                                   counter_base, n, out); break;
        default: hipLaunchKernelGGL(hh_prf_kernel<4>, dim3(grid), dim3(block), 0, st, keys,
                                    n_keys, counter_base, n, out); break;
    }
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

hh_status launch_state_init(const u64* keys, u32 n_keys, const u32* key_idx, u64* states, u64 n,
                            hipStream_t st) {
    const unsigned block = 256;
    hipLaunchKernelGGL(hh_state_init_kernel, dim3(grid_for(4 * n, block)), dim3(block), 0, st,
                       keys, n_keys, key_idx, states, n);
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

hh_status launch_state_step(bool final_step, u64* states, const u32* state_idx, const u8* data,
                            u64 data_bytes, const u64* offsets, const u64* lengths,
                            const u8* width_words, u64* out, const u64* out_offsets, u64 n,
                            hipStream_t st) {
    const unsigned block = 256;
    const unsigned grid = grid_for(4 * n, block);
    if (final_step)
        hipLaunchKernelGGL(hh_state_step_kernel<true>, dim3(grid), dim3(block), 0, st, states,
                           state_idx, data, data_bytes, offsets, lengths, width_words, out,
                           out_offsets, n);
    else
        hipLaunchKernelGGL(hh_state_step_kernel<false>, dim3(grid), dim3(block), 0, st, states,
                           state_idx, data, data_bytes, offsets, lengths, width_words, out,
                           out_offsets, n);
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

}  // namespace hh
