// hh_stats.hip -- avalanche statistics on the GPU (Sec. 6.1 test, Sec. 4.3
// finalization-round study).
//
// For every sample: a key and a message of msg_bytes (1..32) bytes in
// registers, the 64-bit hash with ROUNDS finalization rounds of the message
// and of the message with input bit b flipped, for each b of a group of at
// most 32 input bits.  The 64 lanes of a wave hold 64 samples; the wave
// transposes its 64x64 matrix of output-bit differences with lane shuffles so
// that lane k holds output bit k of all 64 samples, and a popcount adds them
// to that lane's counter for (b, k).
//
// Inputs: mode 0 draws key words and message words from SplitMix64 (Steele,
// Lea and Flood, 2014): word w (0..7) of sample s is output number 8s+w+1 of
// the generator seeded with `seed`, i.e. mix(seed + (8s+w+1)*0x9e3779b97f4a7c15)
// with mix(z): z ^= z>>30; z *= 0xbf58476d1ce4e5b9; z ^= z>>27;
// z *= 0x94d049bb133111eb; z ^= z>>31.  Words 0..3 are the key, words 4..7
// the message (bytes beyond msg_bytes cleared).  Mode 1 hashes the
// little-endian encoding of s itself under one fixed key, which enumerates
// every input when n_samples = 2^(8*msg_bytes).

#include "hh_device.hpp"
#include "hh_internal.hpp"
#include "hh_msg.hpp"

namespace hh {

__device__ __forceinline__ u64 splitmix_mix(u64 z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ u64 splitmix_output(u64 seed, u64 index) {
    return splitmix_mix(seed + index * 0x9e3779b97f4a7c15ull);
}

// 64-bit hash of a message of s (1..32) bytes held in four little-endian
// words (bytes beyond s zero), with R finalization rounds.
template <int R>
__device__ __forceinline__ u64 hash_small(const u64 key[4], const u64 m[4], u32 s) {
    State4 st;
    reset4(st, key);
    if (s == 32u) {
        update4(st, m);
    } else {
        // Sec. 4.5 padded packet: whole 4-byte groups stay in place, the
        // last s%4 bytes (the low bytes of dword q4, the rest of which is
        // zero) move to dword remainder_top_dword(s); here as dwords
        const u32 q4 = s >> 2, top = remainder_top_dword(s);
        u32 d[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            d[2 * i] = lo32(m[i]);
            d[2 * i + 1] = hi32(m[i]);
        }
        u32 tail = 0;
#pragma unroll
        for (u32 k = 0; k < 8; ++k) tail = (k == q4) ? d[k] : tail;
        u32 pd[8];
#pragma unroll
        for (u32 k = 0; k < 8; ++k) pd[k] = (k < q4) ? d[k] : (k == top ? tail : 0u);
        u64 pk[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) pk[i] = make64(pd[2 * i], pd[2 * i + 1]);
        remainder4(st, s, pk);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const u64 p[4] = {rot32(st.v0[2]), rot32(st.v0[3]), rot32(st.v0[0]), rot32(st.v0[1])};
        update4(st, p);
    }
    return st.v0[0] + st.v1[0] + st.mul0[0] + st.mul1[0];
}

__device__ __forceinline__ u64 shfl_xor64(u64 x, int mask) {
    const u32 l = (u32)__shfl_xor((int)lo32(x), mask, 64);
    const u32 h = (u32)__shfl_xor((int)hi32(x), mask, 64);
    return make64(l, h);
}

// 64x64 bit-matrix transpose across the wave: on return lane k holds, in bit
// l, bit k of lane l's input.  Six stages swap the off-diagonal blocks.
__device__ __forceinline__ u64 wave_transpose64(u64 x, u32 lane) {
    const u64 keep[6] = {0x00000000ffffffffull, 0x0000ffff0000ffffull, 0x00ff00ff00ff00ffull,
                         0x0f0f0f0f0f0f0f0full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const u32 w = 32u >> st;
        const u64 y = shfl_xor64(x, (int)w);
        const u64 m = keep[st];
        x = (lane & w) ? ((x & ~m) | ((y & ~m) >> w)) : ((x & m) | ((y & m) << w));
    }
    return x;
}

constexpr int kMaxBitsPerPass = 32;

template <int R>
__global__ __launch_bounds__(256) void hh_avalanche_kernel(int mode, u32 msg_bytes, u64 seed,
                                                           u64 k0, u64 k1, u64 k2, u64 k3, u64 n,
                                                           u32 bit_first, u32 bit_count,
                                                           u64* __restrict__ counts) {
    __shared__ u32 cnt[4][kMaxBitsPerPass][64];  // per wave: [bit][output bit]
    const u32 lane = threadIdx.x & 63u;
    const u32 wib = threadIdx.x >> 6;
    for (u32 i = 0; i < kMaxBitsPerPass; ++i) cnt[wib][i][lane] = 0u;
    const u64 n_batches = (n + 63) >> 6;
    const u64 first_wave = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const u64 n_waves = ((u64)gridDim.x * blockDim.x) >> 6;
    for (u64 batch = first_wave; batch < n_batches; batch += n_waves) {
        const u64 s = batch * 64 + lane;
        const bool valid = s < n;
        u64 key[4], m[4];
        if (mode == 0) {
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                key[w] = splitmix_output(seed, 8 * s + w + 1);
                m[w] = splitmix_output(seed, 8 * s + 4 + w + 1);
            }
        } else {
            key[0] = k0;
            key[1] = k1;
            key[2] = k2;
            key[3] = k3;
            m[0] = s;
            m[1] = m[2] = m[3] = 0;
        }
        // clear message bytes beyond msg_bytes
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const u32 lo = 8u * w;
            if (msg_bytes <= lo)
                m[w] = 0;
            else if (msg_bytes < lo + 8)
                m[w] &= (1ull << (8 * (msg_bytes - lo))) - 1;
        }
        const u64 h0 = hash_small<R>(key, m, msg_bytes);
        for (u32 i = 0; i < bit_count; ++i) {
            const u32 b = bit_first + i;
            u64 m2[4] = {m[0], m[1], m[2], m[3]};
            const u64 flip = 1ull << (b & 63u);
            m2[0] ^= (b >> 6) == 0 ? flip : 0;
            m2[1] ^= (b >> 6) == 1 ? flip : 0;
            m2[2] ^= (b >> 6) == 2 ? flip : 0;
            m2[3] ^= (b >> 6) == 3 ? flip : 0;
            const u64 hb = hash_small<R>(key, m2, msg_bytes);
            const u64 t = wave_transpose64(valid ? (h0 ^ hb) : 0ull, lane);
            cnt[wib][i][lane] += (u32)__popcll(t);
        }
    }
    for (u32 i = 0; i < bit_count; ++i) {
        const u32 c = cnt[wib][i][lane];
        if (c) atomicAdd((unsigned long long*)&counts[64ull * i + lane], (unsigned long long)c);
    }
}

hh_status launch_avalanche(int mode, u32 msg_bytes, u32 rounds, u64 seed, const u64 key[4], u64 n,
                           u32 bit_first, u32 bit_count, u64* counts, hipStream_t st) {
    // every sample costs ~bit_count hashes: enough waves to fill the chip,
    // each wave takes several batches of 64 samples
    u64 waves = (n + 63) / 64;
    if (waves > 16384) waves = 16384;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    const u64 k0 = key ? key[0] : 0, k1 = key ? key[1] : 0, k2 = key ? key[2] : 0,
              k3 = key ? key[3] : 0;
#define HH_AVAL(RR)                                                                          \
    hipLaunchKernelGGL(hh_avalanche_kernel<RR>, dim3(blocks), dim3(256), 0, st, mode,       \
                       msg_bytes, seed, k0, k1, k2, k3, n, bit_first, bit_count, counts)
    switch (rounds) {
        case 1: HH_AVAL(1); break;
        case 2: HH_AVAL(2); break;
        case 3: HH_AVAL(3); break;
        default: HH_AVAL(4); break;
    }
#undef HH_AVAL
    return hipGetLastError() == hipSuccess ? HH_OK : HH_ERR_LAUNCH;
}

}  // namespace hh
