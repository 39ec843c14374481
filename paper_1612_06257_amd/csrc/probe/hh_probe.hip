// hh_probe.hip -- measurement kernels for the roofline figures (libhh_probe.so).
//
//   hh_probe_chain      cycles per Update of one wave running a long chain of
//                       Updates on register data (quad, pair or thread layout),
//                       with n_waves waves launched and an optional s_setprio
//                       for the first `prio_waves` of them.
//   hh_probe_op_rate    aggregate rate of one VALU instruction kind.
//   hh_probe_read       streaming HBM read (16-byte loads, grid-stride).
//   hh_probe_copy       plain device copy of known size (counter calibration).
// All loops have fixed trip counts and every access is in bounds.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../hh_device.hpp"

namespace hh {

// Pair layout (two threads per message, thread h holds lanes 2h and 2h+1):
// a lane pair is exactly a ZipperMerge pair, so the Update needs no
// exchange; only Permute (finalization) would take the other thread's v0.
// Here for the chain measurement only.
struct State2 {
    u64 v0[2], v1[2], mul0[2], mul1[2];
};

__device__ __forceinline__ void update2(State2& s, const u64 p[2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        s.v1[i] += p[i] + s.mul0[i];
        s.mul0[i] ^= mul_lo_hi(s.v1[i], s.v0[i]);
        s.v0[i] += s.mul1[i];
        s.mul1[i] ^= mul_lo_hi(s.v0[i], s.v1[i]);
    }
    u64 z[2];
    zipper_pair(s.v1[0], s.v1[1], z[0], z[1]);
    s.v0[0] += z[0];
    s.v0[1] += z[1];
    zipper_pair(s.v0[0], s.v0[1], z[0], z[1]);
    s.v1[0] += z[0];
    s.v1[1] += z[1];
}

// LAYOUT 0: thread (one thread per message), 1: quad, 2: pair.
template <int LAYOUT>
__global__ __launch_bounds__(64) void hh_probe_chain_kernel(u32 n_updates, u32 prio_waves,
                                                            u64* __restrict__ cycles,
                                                            u64* __restrict__ sink) {
    if (blockIdx.x < prio_waves) __builtin_amdgcn_s_setprio(3);
    const u32 lane = threadIdx.x;
    u64 x = 0x9e3779b97f4a7c15ull * (lane + 1) + blockIdx.x;
    u64 acc = 0;
    const u64 t0 = __builtin_amdgcn_s_memtime();
    if (LAYOUT == 2) {
        const int h = (int)(lane & 1u);
        State2 s;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int q = 2 * h + i;
            s.mul0[i] = init0(q);
            s.mul1[i] = init1(q);
            s.v0[i] = (x + i) ^ s.mul0[i];
            s.v1[i] = rot32(x + i) ^ s.mul1[i];
        }
        for (u32 t = 0; t < n_updates; ++t) {
            const u64 p[2] = {x + t, x ^ t};
            update2(s, p);
        }
        acc = s.v0[0] ^ s.v1[1] ^ s.mul0[0] ^ s.mul1[1];
    } else if (LAYOUT == 1) {
        State1 s;
        reset1(s, x, lane & 3);
        for (u32 t = 0; t < n_updates; ++t) update1(s, x + t);
        acc = s.v0 ^ s.v1 ^ s.mul0 ^ s.mul1;
    } else {
        State4 s;
        const u64 key[4] = {x, x + 1, x + 2, x + 3};
        reset4(s, key);
        for (u32 t = 0; t < n_updates; ++t) {
            const u64 p[4] = {x + t, x ^ t, x - t, x + 2 * t};
            update4(s, p);
        }
        acc = s.v0[0] ^ s.v1[1] ^ s.mul0[2] ^ s.mul1[3];
    }
    const u64 t1 = __builtin_amdgcn_s_memtime();
    sink[(u64)blockIdx.x * 64 + lane] = acc;
    if (lane == 0) cycles[blockIdx.x] = t1 - t0;
}

// One wave absorbs 16 messages of npk packets each (4 threads per message)
// straight from memory with the production packet loop.  Message m of wave w
// starts at data + (16*w + m) * msg_bytes + misalign.
template <int RING>
__global__ __launch_bounds__(64) void hh_probe_absorb_kernel(const u8* __restrict__ data,
                                                             u64 msg_bytes, u32 misalign, u32 npk,
                                                             u64* __restrict__ cycles,
                                                             u64* __restrict__ sink) {
    const u32 lane = threadIdx.x;
    const int q = (int)(lane & 3u);
    const u8* p = data + (16ull * blockIdx.x + (lane >> 2)) * msg_bytes + misalign;
    State1 s;
    reset1(s, 0x9e3779b97f4a7c15ull * (lane + 1), q);
    const u64 t0 = __builtin_amdgcn_s_memtime();
    absorb_quad<RING>(s, p + 8 * q, npk);
    const u64 t1 = __builtin_amdgcn_s_memtime();
    sink[(u64)blockIdx.x * 64 + lane] = s.v0 ^ s.v1 ^ s.mul0 ^ s.mul1;
    if (lane == 0) cycles[blockIdx.x] = t1 - t0;
}

// op kinds: 0 u64 add, 1 u32xu32->u64 multiply, 2 byte permute, 3 32-bit xor,
// 4 DPP move, 5 alignbyte
template <int OP>
__global__ __launch_bounds__(256) void hh_probe_op_kernel(u32 iters, u64* __restrict__ sink) {
    u64 a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] = 0x9e3779b97f4a7c15ull * (threadIdx.x + 8 * c + 1) + blockIdx.x;
    for (u32 i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                // each chain reads its neighbour so nothing folds algebraically
                const u64 b = a[(c + 1) & 7];
                if (OP == 0) a[c] = a[c] + b;
                if (OP == 1) a[c] = mul_lo_hi(a[c], b);
                if (OP == 2) a[c] = make64(perm(hi32(b), lo32(a[c]), 0x05020603u), hi32(a[c]));
                if (OP == 3) a[c] = make64(lo32(a[c]) ^ lo32(b), hi32(a[c]));
                if (OP == 4) a[c] = make64(quad_swap1(lo32(b)), hi32(a[c]));
                if (OP == 5) a[c] = make64(align_bytes(hi32(b), lo32(a[c]), 3u), hi32(a[c]));
            }
        }
    }
    u64 r = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) r ^= a[c];
    sink[(u64)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

typedef u32 u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void hh_probe_read_kernel(const u32x4* __restrict__ src, u64 n16,
                                                            u64* __restrict__ sink) {
    u32x4 acc = {0, 0, 0, 0};
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) acc ^= src[i];
    sink[(u64)blockIdx.x * blockDim.x + threadIdx.x] = make64(acc.x ^ acc.z, acc.y ^ acc.w);
}

__global__ __launch_bounds__(256) void hh_probe_copy_kernel(const u32x4* __restrict__ src,
                                                            u32x4* __restrict__ dst, u64 n16) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace hh

using namespace hh;

extern "C" {

// cycles[w] = s_memtime cycles of wave w for n_updates Updates; sink needs
// 64 * n_waves words.  layout: 0 thread, 1 quad, 2 pair.
int hh_probe_chain(int layout, u32 n_updates, u32 n_waves, u32 prio_waves, u64* cycles,
                   u64* sink, void* stream) {
    if (n_waves == 0 || !cycles || !sink || layout < 0 || layout > 2) return 1;
    hipStream_t st = (hipStream_t)stream;
    if (layout == 1)
        hipLaunchKernelGGL(hh_probe_chain_kernel<1>, dim3(n_waves), dim3(64), 0, st, n_updates,
                           prio_waves, cycles, sink);
    else if (layout == 2)
        hipLaunchKernelGGL(hh_probe_chain_kernel<2>, dim3(n_waves), dim3(64), 0, st, n_updates,
                           prio_waves, cycles, sink);
    else
        hipLaunchKernelGGL(hh_probe_chain_kernel<0>, dim3(n_waves), dim3(64), 0, st, n_updates,
                           prio_waves, cycles, sink);
    return hipGetLastError() == hipSuccess ? 0 : 4;
}

// data must hold 16 * n_waves * msg_bytes bytes; msg_bytes >= 32*npk + misalign + 12
int hh_probe_absorb(int ring, const void* data, u64 data_bytes, u64 msg_bytes, u32 misalign,
                    u32 npk, u32 n_waves, u64* cycles, u64* sink, void* stream) {
    if (!data || !cycles || !sink || n_waves == 0 || npk == 0 || misalign > 3) return 1;
    if (msg_bytes < 32ull * npk + misalign + 12 || 16ull * n_waves * msg_bytes > data_bytes) return 1;
    hipStream_t st = (hipStream_t)stream;
    const u8* d = (const u8*)data;
    switch (ring) {
        case 12: hipLaunchKernelGGL(hh_probe_absorb_kernel<12>, dim3(n_waves), dim3(64), 0, st, d, msg_bytes, misalign, npk, cycles, sink); break;
        case 24: hipLaunchKernelGGL(hh_probe_absorb_kernel<24>, dim3(n_waves), dim3(64), 0, st, d, msg_bytes, misalign, npk, cycles, sink); break;
        case 36: hipLaunchKernelGGL(hh_probe_absorb_kernel<36>, dim3(n_waves), dim3(64), 0, st, d, msg_bytes, misalign, npk, cycles, sink); break;
        case 48: hipLaunchKernelGGL(hh_probe_absorb_kernel<48>, dim3(n_waves), dim3(64), 0, st, d, msg_bytes, misalign, npk, cycles, sink); break;
        case 72: hipLaunchKernelGGL(hh_probe_absorb_kernel<72>, dim3(n_waves), dim3(64), 0, st, d, msg_bytes, misalign, npk, cycles, sink); break;
        case 96: hipLaunchKernelGGL(hh_probe_absorb_kernel<96>, dim3(n_waves), dim3(64), 0, st, d, msg_bytes, misalign, npk, cycles, sink); break;
        default: return 1;
    }
    return hipGetLastError() == hipSuccess ? 0 : 4;
}

// 256 threads x n_blocks, each 8 chains x 16 x iters operations; sink needs
// 256 * n_blocks words.
int hh_probe_op_rate(int op, u32 iters, u32 n_blocks, u64* sink, void* stream) {
    if (!sink || n_blocks == 0) return 1;
    hipStream_t st = (hipStream_t)stream;
    switch (op) {
        case 0: hipLaunchKernelGGL(hh_probe_op_kernel<0>, dim3(n_blocks), dim3(256), 0, st, iters, sink); break;
        case 1: hipLaunchKernelGGL(hh_probe_op_kernel<1>, dim3(n_blocks), dim3(256), 0, st, iters, sink); break;
        case 2: hipLaunchKernelGGL(hh_probe_op_kernel<2>, dim3(n_blocks), dim3(256), 0, st, iters, sink); break;
        case 3: hipLaunchKernelGGL(hh_probe_op_kernel<3>, dim3(n_blocks), dim3(256), 0, st, iters, sink); break;
        case 4: hipLaunchKernelGGL(hh_probe_op_kernel<4>, dim3(n_blocks), dim3(256), 0, st, iters, sink); break;
        case 5: hipLaunchKernelGGL(hh_probe_op_kernel<5>, dim3(n_blocks), dim3(256), 0, st, iters, sink); break;
        default: return 1;
    }
    return hipGetLastError() == hipSuccess ? 0 : 4;
}

// bytes must be a multiple of 16; sink needs 256 * n_blocks words
int hh_probe_read(const void* src, u64 bytes, u32 n_blocks, u64* sink, void* stream) {
    if (!src || !sink || (bytes & 15) || n_blocks == 0) return 1;
    hipLaunchKernelGGL(hh_probe_read_kernel, dim3(n_blocks), dim3(256), 0, (hipStream_t)stream,
                       (const u32x4*)src, bytes / 16, sink);
    return hipGetLastError() == hipSuccess ? 0 : 4;
}

int hh_probe_copy(const void* src, void* dst, u64 bytes, u32 n_blocks, void* stream) {
    if (!src || !dst || (bytes & 15) || n_blocks == 0) return 1;
    hipLaunchKernelGGL(hh_probe_copy_kernel, dim3(n_blocks), dim3(256), 0, (hipStream_t)stream,
                       (const u32x4*)src, (u32x4*)dst, bytes / 16);
    return hipGetLastError() == hipSuccess ? 0 : 4;
}

}  // extern "C"
