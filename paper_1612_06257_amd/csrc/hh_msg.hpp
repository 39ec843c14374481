// hh_msg.hpp -- hashing one whole message (Sec. 4.2-4.5) on a thread or a
// quad, shared by the kernels of hh_kernels.hip and hh_batched.hip.
#pragma once

#include "hh_device.hpp"

namespace hh {

// per-message setup

struct Msg {
    const u8* p;
    u64 len;
};

__device__ __forceinline__ Msg message(const u8* data, u64 data_bytes, u64 off, u64 len) {
    off = off < data_bytes ? off : data_bytes;
    const u64 room = data_bytes - off;
    return Msg{data + off, len < room ? len : room};
}

__device__ __forceinline__ u64 key_index(const u32* key_idx, u32 n_keys, u64 j) {
    if (!key_idx) return 0;
    const u32 k = key_idx[j];
    return k < n_keys ? k : n_keys - 1u;
}

// Sec. 4.5 padded remainder packet for the r (1..31) tail bytes at t of a
// message of len bytes, as four lanes; loaded before the message's packets
// are absorbed so that its loads overlap them.
__device__ __forceinline__ void remainder_packet4(const u8* t, u32 r, u64 len, u64 pk[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
        pk[i] = make64(remainder_dword(t, r, 2 * i, len), remainder_dword(t, r, 2 * i + 1, len));
}

// Sec. 4.5 remainder step on a whole state held by one thread.
__device__ __forceinline__ void remainder4(State4& s, u32 r, const u64 pk[4]) {
    const u64 inject = ((u64)r << 32) + r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        s.v0[i] += inject;
        s.v1[i] = rotl_halves(s.v1[i], r);
    }
    update4(s, pk);
}

// Lane q of the Sec. 4.5 padded remainder packet (quad layout).
__device__ __forceinline__ u64 remainder_lane(const u8* t, u32 r, u64 len, int q) {
    return make64(remainder_dword(t, r, 2 * q, len), remainder_dword(t, r, 2 * q + 1, len));
}

// Sec. 4.5 remainder step, quad layout (thread holds lane q).
__device__ __forceinline__ void remainder1(State1& s, u32 r, u64 lane_word) {
    s.v0 += ((u64)r << 32) + r;
    s.v1 = rotl_halves(s.v1, r);
    update1(s, lane_word);
}

// Packets per absorb call.  Inside a call the loops form byte offsets as
// 32 * packet index in 32-bit arithmetic (one VALU op per address), so a call
// covers at most 4 GiB; longer messages take several calls, each starting
// from a 64-bit pointer.
constexpr u64 kMaxPacketsPerCall = 1ull << 27;

constexpr int kThreadHead = 2;  // packets loaded up front per thread (thread layout)
constexpr int kThreadRing = 1;  // packets in flight past those: short messages, many per launch
constexpr int kThreadDeepRing = 8;  // the same for long messages, few per launch
constexpr int kQuadRing = 12;   // packets in flight per thread (quad layout, wide grids)
constexpr int kStateRing = 48;  // packets in flight per thread (streaming-state kernels)

// The whole hash of one message in one thread; returns the final lane sums.
// The tail and the first kThreadHead packets are loaded together before the
// first Update, so a short message waits for memory once; longer messages
// continue through a ring of RING packets.  With RING = kThreadRing the small
// register footprint (under 80 VGPRs) lets six waves share a SIMD, which is
// what hides the latency of short messages; a long message alone in its wave
// needs the deeper ring instead, since every 128-byte line it reads from HBM
// would otherwise stall it for a full memory round trip.
template <int RING>
__device__ __forceinline__ void hash_thread(const u64* key, const u8* p, u64 len, u64 sum[4]) {
    const u32 r = (u32)(len & 31u);
    u64 nfull = len >> 5;
    u64 tail[4] = {0, 0, 0, 0};
    if (r) remainder_packet4(p + 32 * nfull, r, len, tail);
    Packet head[kThreadHead];
#pragma unroll
    for (int k = 0; k < kThreadHead; ++k)
        if ((u64)k < nfull) head[k] = load_packet(p + 32 * k);
    State4 s;
    reset4(s, key);
#pragma unroll
    for (int k = 0; k < kThreadHead; ++k)
        if ((u64)k < nfull) update4(s, head[k].w);
    if (nfull > (u64)kThreadHead) {
        const u8* cur = p + 32 * kThreadHead;
        nfull -= kThreadHead;
        while (nfull) {
            const u32 npk = (u32)(nfull < kMaxPacketsPerCall ? nfull : kMaxPacketsPerCall);
            absorb_thread<RING>(s, cur, npk);
            cur += 32 * (u64)npk;
            nfull -= npk;
        }
    }
    if (r) remainder4(s, r, tail);
    finalize4(s, sum);
}

// Whole packets of a message on a quad (thread q absorbs lane q), with RING
// packets in flight per thread.
template <int RING>
__device__ __forceinline__ const u8* absorb_quad_all(State1& s, const u8* p, u64 nfull, int q) {
    while (nfull) {
        const u32 npk = (u32)(nfull < kMaxPacketsPerCall ? nfull : kMaxPacketsPerCall);
        absorb_quad<RING>(s, p + 8 * q, npk);
        p += 32 * (u64)npk;
        nfull -= npk;
    }
    return p;
}

// The whole hash of one message on a quad; returns lane q of the sums.
template <int RING>
__device__ __forceinline__ u64 hash_quad(u64 key_q, const u8* p, u64 len, int q) {
    const u32 r = (u32)(len & 31u);
    const u64 nfull = len >> 5;
    const u64 tail = r ? remainder_lane(p + 32 * nfull, r, len, q) : 0;
    State1 s;
    reset1(s, key_q, q);
    absorb_quad_all<RING>(s, p, nfull, q);
    if (r) remainder1(s, r, tail);
    return finalize1(s);
}

}  // namespace hh
