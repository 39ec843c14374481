// hh_state.hip -- incremental hashing over caller-owned device states (the
// streaming API and the serving loop's iterations) and byte-segment copies.
//
//   hh_state_init_kernel     Reset (Sec. 4.4) into state slots
//   hh_state_step_kernel<M>  one launch of updates and/or finals: whole
//                            packets folded into a state, or the remainder
//                            step and finalization (Sec. 4.2, 4.5, 4.3)
//   hh_copy_segments_kernel  many byte-segment copies in one launch
// Four threads per state (one 64-bit lane each, as in the quad kernel).

#include "hh_device.hpp"
#include "hh_internal.hpp"
#include "hh_msg.hpp"

namespace hh {

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
    u64* __restrict__ states, u64 n_states, const u32* __restrict__ state_idx, u64 n) {
    const int q = threadIdx.x & 3;
    const u64 stride = ((u64)gridDim.x * blockDim.x) >> 2;
    for (u64 j = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 2; j < n; j += stride) {
        const u64 t = state_idx ? (u64)state_idx[j] : j;
        if (t >= n_states) continue;  // whole quad agrees
        State1 s;
        reset1(s, keys[4 * key_index(key_idx, n_keys, j) + q], q);
        store_state1(s, states + 16 * t, q);
    }
}

// Byte segments: dst[dst_offs[k] .. + lens[k]) = src[src_offs[k] .. + lens[k]),
// clamped to both buffers.  The blocks of one grid row (blockIdx.x) share a
// segment: whole 8-byte words with unaligned accesses, interleaved so that
// each wave moves 512 contiguous bytes, then block 0 moves the last bytes.
// Rows stride over the segments.
__global__ __launch_bounds__(256) void hh_copy_segments_kernel(
    u8* __restrict__ dst, u64 dst_bytes, const u8* __restrict__ src, u64 src_bytes,
    const u64* __restrict__ src_offs, const u64* __restrict__ dst_offs,
    const u64* __restrict__ lens, u64 n) {
    const u64 step = (u64)gridDim.x * blockDim.x;
    for (u64 k = blockIdx.y; k < n; k += gridDim.y) {
        u64 so = src_offs[k], d_o = dst_offs[k], len = lens[k];
        so = so < src_bytes ? so : src_bytes;
        d_o = d_o < dst_bytes ? d_o : dst_bytes;
        len = len < src_bytes - so ? len : src_bytes - so;
        len = len < dst_bytes - d_o ? len : dst_bytes - d_o;
        const u8* sp = src + so;
        u8* dp = dst + d_o;
        const u64 words = len >> 3;
        for (u64 w = (u64)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += step) {
            const u64 v = load_le64(sp + 8 * w);
            __builtin_memcpy(dp + 8 * w, &v, 8);
        }
        if (blockIdx.x == 0)
            for (u64 b = (words << 3) + threadIdx.x; b < len; b += blockDim.x) dp[b] = sp[b];
    }
}

// MODE 0: every item is an update; 1: every item finishes; 2: item k
// finishes when width_words[k] != 0 and is an update otherwise.
template <int MODE>
__global__ __launch_bounds__(256) void hh_state_step_kernel(
    u64* __restrict__ states, u64 n_states, const u32* __restrict__ state_idx,
    const u8* __restrict__ data, u64 data_bytes, const u64* __restrict__ offsets,
    const u64* __restrict__ lengths, const u8* __restrict__ width_words, u64* __restrict__ out,
    u64 out_words, const u64* __restrict__ out_offsets, u64 n) {
    // a serving iteration's short chunks: their waves take the issue slots
    // ahead of long chains (priority 0) that share their SIMD, so that a long
    // request never stretches a short one's iteration
    __builtin_amdgcn_s_setprio(1);
    const int q = threadIdx.x & 3;
    const u64 quad = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
    const u64 stride = ((u64)gridDim.x * blockDim.x) >> 2;  // a multiple of 16
    // wave-uniform loop: quads past n repeat the wave's first item without
    // storing anything (it reads what that item's quad reads, in the same
    // instructions, before any store), so the wave keeps every lane on
    for (u64 base = quad & ~15ull; base < n; base += stride) {
        const bool real = base + (quad & 15u) < n;
        const u64 k = real ? base + (quad & 15u) : base;
        const u64 t = state_idx ? (u64)state_idx[k] : k;
        if (t >= n_states) continue;  // whole quad agrees; the DPP exchange stays in step
        u64* st = states + 16 * t;
        const u32 w = MODE == 0 ? 0u : (width_words ? (u32)width_words[k] : 1u);
        const bool fin = MODE == 1 || (MODE == 2 && w != 0u);
        const Msg m = message(data, data_bytes, offsets[k], lengths[k]);
        const u32 r = fin ? (u32)(m.len & 31u) : 0u;
        const u64 tail = r ? remainder_lane(m.p + 32 * (m.len >> 5), r, m.len, q) : 0;
        State1 s;
        load_state1(s, st, q);
        absorb_quad_all<kStateRing>(s, m.p, m.len >> 5, q);
        if (!fin) {
            if (real) store_state1(s, st, q);
        } else {
            if (r) remainder1(s, r, tail);
            const u64 sum = finalize1(s);
            const u64 o = out_offsets ? out_offsets[k] : 4 * k;
            // widths other than 1, 2 and 4 write nothing
            const bool valid_w = w == 1u || w == 2u || w == 4u;
            if (real && valid_w && (u32)q < w && o < out_words && (u64)q < out_words - o)
                out[o + q] = sum;
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

// one-wave workgroups: the dispatcher spreads them over the CUs, so that
// fewer long chains share a CU's load path
constexpr unsigned kStateBlock = 64;

}  // namespace

hh_status launch_state_init(const u64* keys, u32 n_keys, const u32* key_idx, u64* states,
                            u64 n_states, const u32* state_idx, u64 n, hipStream_t st) {
    const unsigned block = 256;
    hipLaunchKernelGGL(hh_state_init_kernel, dim3(grid_for(4 * n, block)), dim3(block), 0, st,
                       keys, n_keys, key_idx, states, n_states, state_idx, n);
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

hh_status launch_copy_segments(u8* dst, u64 dst_bytes, const u8* src, u64 src_bytes,
                               const u64* src_offs, const u64* dst_offs, const u64* lens, u64 n,
                               u64 max_len, hipStream_t st) {
    // one block per 64 KiB of the longest segment, at most 64 per segment
    u64 gx = (max_len + 65535) >> 16;
    gx = gx < 1 ? 1 : (gx > 64 ? 64 : gx);
    const unsigned gy = (unsigned)(n < 65535 ? n : 65535);
    hipLaunchKernelGGL(hh_copy_segments_kernel, dim3((unsigned)gx, gy ? gy : 1), dim3(256), 0,
                       st, dst, dst_bytes, src, src_bytes, src_offs, dst_offs, lens, n);
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

hh_status launch_state_step(int mode, u64* states, u64 n_states, const u32* state_idx,
                            const u8* data, u64 data_bytes, const u64* offsets,
                            const u64* lengths, const u8* width_words, u64* out, u64 out_words,
                            const u64* out_offsets, u64 n, hipStream_t st) {
    const unsigned block = kStateBlock;
    const unsigned grid = grid_for(4 * n, block);
#define HH_STEP(M)                                                                          \
    hipLaunchKernelGGL(hh_state_step_kernel<M>, dim3(grid), dim3(block), 0, st, states,    \
                       n_states, state_idx, data, data_bytes, offsets, lengths, width_words, \
                       out, out_words, out_offsets, n)
    switch (mode) {
        case 0: HH_STEP(0); break;
        case 1: HH_STEP(1); break;
        default: HH_STEP(2); break;
    }
#undef HH_STEP
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

}  // namespace hh
