// hh_device.hpp -- HighwayHash device primitives for gfx950 (CDNA4, wave64).
//
// Two register layouts of the 1024-bit state (Sec. 4.2: v0, v1, mul0, mul1,
// each four independent 64-bit lanes):
//
//   State4, the thread layout (one thread per message): a thread holds all 16
//     words.  ZipperMerge and Permute are register renaming plus v_perm_b32;
//     no exchange.
//   State1, the quad layout (four threads per message): thread q of a quad
//     (q = lane id mod 4) holds lane q of each vector, 4 words.  ZipperMerge of the pair
//     (0,1) / (2,3) needs only the partner's HIGH dword (one DPP move);
//     Permute needs lane q^2's v0 (two DPP moves).
//
// 64-bit adds compile to v_lshl_add_u64, the 32x32->64 products of
// _mm256_mul_epu32 to v_mad_u64_u32, byte permutes to v_perm_b32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hh {

typedef uint64_t u64;
typedef uint32_t u32;
typedef uint8_t u8;

// ---------------------------------------------------------------------------
// Sec. 4.4 initialization constants.  Lanes 3, 2, 1 of the first constant are
// the first three 64-bit words of the hexadecimal fraction of pi, lanes 3, 2,
// 1 of the second the fifth to seventh words; lane 0 of each is rebuilt so
// that a bit is set there exactly when zero or one of the other lanes set it.
constexpr u64 kPiWord0 = 0x243f6a8885a308d3ull;
constexpr u64 kPiWord1 = 0x13198a2e03707344ull;
constexpr u64 kPiWord2 = 0xa4093822299f31d0ull;
constexpr u64 kPiWord4 = 0x452821e638d01377ull;
constexpr u64 kPiWord5 = 0xbe5466cf34e90c6cull;
constexpr u64 kPiWord6 = 0xc0ac29b7c97c50ddull;

constexpr u64 rebuilt_lane(u64 a, u64 b, u64 c) { return ~((a & b) | (a & c) | (b & c)); }

constexpr u64 kInit0Lane0 = rebuilt_lane(kPiWord0, kPiWord1, kPiWord2);
constexpr u64 kInit1Lane0 = rebuilt_lane(kPiWord4, kPiWord5, kPiWord6);

__host__ __device__ constexpr u64 init0(int lane) {
    return lane == 0 ? kInit0Lane0 : lane == 1 ? kPiWord2 : lane == 2 ? kPiWord1 : kPiWord0;
}
__host__ __device__ constexpr u64 init1(int lane) {
    return lane == 0 ? kInit1Lane0 : lane == 1 ? kPiWord6 : lane == 2 ? kPiWord5 : kPiWord4;
}

// ---------------------------------------------------------------------------
// scalar helpers

__device__ __forceinline__ u32 lo32(u64 x) { return (u32)x; }
__device__ __forceinline__ u32 hi32(u64 x) { return (u32)(x >> 32); }
typedef u32 u32x2 __attribute__((ext_vector_type(2)));
// (hi:lo) as one 64-bit value; a vector bitcast rather than shift/or keeps
// the compiler from splitting later 64-bit adds of it into 32-bit pieces
__device__ __forceinline__ u64 make64(u32 lo, u32 hi) {
    const u32x2 v = {lo, hi};
    return __builtin_bit_cast(u64, v);
}
__device__ __forceinline__ u64 rot32(u64 x) { return make64(hi32(x), lo32(x)); }

// 32x32 -> 64 product of the low halves (_mm256_mul_epu32), v_mad_u64_u32
__device__ __forceinline__ u64 mul_lo_hi(u64 x, u64 y) { return (u64)lo32(x) * (u64)hi32(y); }

// v_perm_b32: result byte k = byte sel[k] of the 8-byte value (a:b), where
// selector values 0..3 name bytes of b and 4..7 bytes of a; 0x0c gives 0.
__device__ __forceinline__ u32 perm(u32 a, u32 b, u32 sel) {
    return __builtin_amdgcn_perm(a, b, sel);
}

// (hi:lo) >> 8*sh, low 32 bits (v_alignbyte_b32); sh in 0..3
__device__ __forceinline__ u32 align_bytes(u32 hi, u32 lo, u32 sh) {
    return __builtin_amdgcn_alignbyte(hi, lo, sh);
}

// rotate each 32-bit half of x left by r, 1 <= r <= 31 (v_alignbit_b32)
__device__ __forceinline__ u64 rotl_halves(u64 x, u32 r) {
    u32 l = lo32(x), h = hi32(x);
    return make64(__builtin_amdgcn_alignbit(l, l, 32u - r), __builtin_amdgcn_alignbit(h, h, 32u - r));
}

// ---------------------------------------------------------------------------
// Sec. 4.1 ZipperMerge of one 16-byte lane pair (a = lane 2k, b = lane 2k+1).
// Result bytes R_i = S_{P_i} with P (low byte first) =
//   3 12 2 5 | 14 1 15 0 | 11 4 10 13 | 9 6 8 7
// In dwords (a = al:ah, b = bl:bh):
//   R[0..3]   = al.3 bh.0 al.2 ah.1      R[4..7]   = bh.2 al.1 bh.3 al.0
//   R[8..11]  = bl.3 ah.0 bl.2 bh.1      R[12..15] = bl.1 ah.2 bl.0 ah.3
// Five v_perm_b32: m gathers the four bytes of ah/bh that the two
// three-source dwords need.
__device__ __forceinline__ void zipper_pair(u64 a, u64 b, u64& ra, u64& rb) {
    const u32 al = lo32(a), ah = hi32(a), bl = lo32(b), bh = hi32(b);
    const u32 m = perm(ah, bh, 0x05040100u);   // bh.0 bh.1 ah.0 ah.1
    const u32 r0 = perm(m, al, 0x07020403u);   // al.3 m.0 al.2 m.3
    const u32 r1 = perm(bh, al, 0x00070106u);  // bh.2 al.1 bh.3 al.0
    const u32 r2 = perm(m, bl, 0x05020603u);   // bl.3 m.2 bl.2 m.1
    const u32 r3 = perm(ah, bl, 0x07000601u);  // bl.1 ah.2 bl.0 ah.3
    ra = make64(r0, r1);
    rb = make64(r2, r3);
}

// ---------------------------------------------------------------------------
// Lanes4 layout: the whole state in one thread.

struct State4 {
    u64 v0[4], v1[4], mul0[4], mul1[4];
};

__device__ __forceinline__ void reset4(State4& s, const u64 key[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        s.mul0[i] = init0(i);
        s.mul1[i] = init1(i);
        s.v0[i] = key[i] ^ init0(i);
        s.v1[i] = rot32(key[i]) ^ init1(i);
    }
}

__device__ __forceinline__ void update4(State4& s, const u64 p[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        s.v1[i] += p[i] + s.mul0[i];
        s.mul0[i] ^= mul_lo_hi(s.v1[i], s.v0[i]);
        s.v0[i] += s.mul1[i];
        s.mul1[i] ^= mul_lo_hi(s.v0[i], s.v1[i]);
    }
    u64 z[4];
    zipper_pair(s.v1[0], s.v1[1], z[0], z[1]);
    zipper_pair(s.v1[2], s.v1[3], z[2], z[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) s.v0[i] += z[i];
    zipper_pair(s.v0[0], s.v0[1], z[0], z[1]);
    zipper_pair(s.v0[2], s.v0[3], z[2], z[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) s.v1[i] += z[i];
}

// x + rot32(y): the halves of y are added crosswise with a 32-bit add and an
// add-with-carry, so rot32(y) is never formed in a register pair (which costs
// two moves before a 64-bit add).
__device__ __forceinline__ u64 add_rot32(u64 x, u64 y) {
    unsigned int carry = 0;
    const u32 lo = __builtin_addc(lo32(x), hi32(y), 0u, &carry);
    const u32 hi = __builtin_addc(hi32(x), lo32(y), carry, &carry);
    return make64(lo, hi);
}

// Update(Permute(v0)) (Sec. 4.3): the packet is Permute(v0)[i] = rot32(v0[i^2]),
// taken before the Update changes v0; otherwise update4.
__device__ __forceinline__ void update4_permuted(State4& s) {
    const u64 q[4] = {s.v0[2], s.v0[3], s.v0[0], s.v0[1]};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        s.v1[i] = add_rot32(s.v1[i] + s.mul0[i], q[i]);
        s.mul0[i] ^= mul_lo_hi(s.v1[i], s.v0[i]);
        s.v0[i] += s.mul1[i];
        s.mul1[i] ^= mul_lo_hi(s.v0[i], s.v1[i]);
    }
    u64 z[4];
    zipper_pair(s.v1[0], s.v1[1], z[0], z[1]);
    zipper_pair(s.v1[2], s.v1[3], z[2], z[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) s.v0[i] += z[i];
    zipper_pair(s.v0[0], s.v0[1], z[0], z[1]);
    zipper_pair(s.v0[2], s.v0[3], z[2], z[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) s.v1[i] += z[i];
}

// Sec. 4.3: four rounds of Update(Permute(v0)); Permute(v0)[i] = rot32(v0[i^2]).
__device__ __forceinline__ void finalize4(State4& s, u64 sum[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) update4_permuted(s);
#pragma unroll
    for (int i = 0; i < 4; ++i) sum[i] = s.v0[i] + s.v1[i] + s.mul0[i] + s.mul1[i];
}

// ---------------------------------------------------------------------------
// Lane1 layout: thread q of a quad holds lane q.  All four threads of a quad
// must be active whenever these run.

// DPP quad_perm controls
constexpr int kQuadSwap1 = 0xB1;  // [1,0,3,2]: partner in the zipper pair
constexpr int kQuadSwap2 = 0x4E;  // [2,3,0,1]: lane q^2 (Permute)

__device__ __forceinline__ u32 quad_swap1(u32 x) {
    return (u32)__builtin_amdgcn_mov_dpp((int)x, kQuadSwap1, 0xF, 0xF, true);
}
__device__ __forceinline__ u32 quad_swap2(u32 x) {
    return (u32)__builtin_amdgcn_mov_dpp((int)x, kQuadSwap2, 0xF, 0xF, true);
}

struct State1 {
    u64 v0, v1, mul0, mul1;
    u32 sel_hi;  // v_perm selector of this lane's upper result dword
};

// Zipper result for this thread's lane: own dwords (L, H), partner's H = P.
//   even lane: lo = L.3 P.0 L.2 H.1   hi = P.2 L.1 P.3 L.0
//   odd lane:  lo = L.3 P.0 L.2 H.1   hi = L.1 P.2 L.0 P.3
// C gathers this lane's three bytes of the low result dword without waiting
// for the partner, so only one v_perm_b32 follows the DPP move on the
// critical path.
__device__ __forceinline__ u64 zipper1(u64 x, u32 sel_hi) {
    const u32 L = lo32(x), H = hi32(x);
    const u32 P = quad_swap1(H);
    const u32 C = perm(H, L, 0x05020c03u);    // L.3 0 L.2 H.1
    const u32 lo = perm(P, C, 0x03020400u);   // C.0 P.0 C.2 C.3
    const u32 hi = perm(P, L, sel_hi);
    return make64(lo, hi);
}

__device__ __forceinline__ void reset1(State1& s, u64 key, int q) {
    s.mul0 = init0(q);
    s.mul1 = init1(q);
    s.v0 = key ^ s.mul0;
    s.v1 = rot32(key) ^ s.mul1;
    s.sel_hi = (q & 1) ? 0x07000601u : 0x00070106u;
}

__device__ __forceinline__ void update1(State1& s, u64 p) {
    s.v1 += p + s.mul0;
    s.mul0 ^= mul_lo_hi(s.v1, s.v0);
    s.v0 += s.mul1;
    s.mul1 ^= mul_lo_hi(s.v0, s.v1);
    s.v0 += zipper1(s.v1, s.sel_hi);
    s.v1 += zipper1(s.v0, s.sel_hi);
}

__device__ __forceinline__ u64 finalize1(State1& s) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // Permute: lane q takes rot32 of lane q^2 of v0
        const u64 p = make64(quad_swap2(hi32(s.v0)), quad_swap2(lo32(s.v0)));
        update1(s, p);
    }
    return s.v0 + s.v1 + s.mul0 + s.mul1;
}

// ---------------------------------------------------------------------------
// Loads.  Messages start at any byte.  Packets and whole tail dwords are
// unaligned loads of exactly the message's bytes: the gfx950 memory path
// serves byte-aligned dword loads (the HSA unaligned access mode the compiler
// itself relies on), so a lane's 8 packet bytes are one global_load_dwordx2.
// The 1..3 bytes at the very end of a message come from the unaligned dword
// that ends at its last byte; a message shorter than 4 bytes is read byte by
// byte.  No load leaves the message's bytes.  Pointers keep their provenance
// (no integer round trip) so that the loads stay global_load.

typedef u64 u64_any_align __attribute__((aligned(1)));
typedef u32 u32_any_align __attribute__((aligned(1)));

__device__ __forceinline__ u64 load_le64(const u8* p) { return *(const u64_any_align*)p; }
__device__ __forceinline__ u32 load_le32(const u8* p) { return *(const u32_any_align*)p; }

// Little-endian word of the n (0..3) bytes at p, read one byte at a time
// (the bytes may end at the buffer's last byte); bytes past n read as 0.
__device__ __forceinline__ u32 load_partial_le32(const u8* p, u32 n) {
    u32 w = 0u;
    if (n > 0u) w = p[0];
    if (n > 1u) w |= (u32)p[1] << 8;
    if (n > 2u) w |= (u32)p[2] << 16;
    return w;
}

// Sec. 4.5 padded remainder packet: the dword that takes the last r%4 tail
// bytes.  The whole 4-byte groups are mask-loaded into the 16-byte half they
// end in, and the last bytes go to the low end of that half's most-significant
// dword: dword 3 when r < 16 (at most three groups precede it), dword 7
// otherwise (at most seven).
__device__ __forceinline__ u32 remainder_top_dword(u32 r) { return r < 16u ? 3u : 7u; }

// Sec. 4.5 padded remainder packet, dword k (0..7), for the r (1..31) tail
// bytes at t of a message (or final chunk) of len bytes, so that its first
// byte is t + r - len: the first q = r - r%4 bytes fill packet bytes 0..q-1,
// the last r%4 bytes fill, in order, the low bytes of dword
// remainder_top_dword(r) (packet bytes 12.. or 28..); all other bytes are
// zero.
__device__ __forceinline__ u32 remainder_dword(const u8* t, u32 r, u32 k, u64 len) {
    const u32 q4 = r >> 2;  // whole 4-byte groups
    if (k < q4) return load_le32(t + 4u * k);
    const u32 m = r & 3u;
    if (k != remainder_top_dword(r) || m == 0u) return 0u;
    // the dword ending at the last byte starts inside the message when len >= 4
    if (len >= 4u) return load_le32(t + r - 4u) >> (8u * (4u - m));
    return load_partial_le32(t + 4u * q4, m);
}

// An empty asm statement that reads v: the compiler has to wait for the load
// of v before it (one s_waitcnt).  Vector-memory loads retire in issue order,
// so that wait also covers every load issued before v, and the uses of those
// values that follow need no wait of their own.  (No instruction, no memory
// access inside the asm.)
__device__ __forceinline__ void wait_loaded(u64 v) { asm volatile("" ::"v"(v)); }

// Packets per explicit wait in the steady loop: the largest divisor of the
// ring third h up to 8.  Each wait (and the realignment after it) costs the
// wave an issue slot; with 8 packets per wait the single-wave packet loop
// takes 82.3 cycles per Update against 83.9 with 4, while one wait per whole
// third (24) issues its loads in one burst and slows the loop to 88.
constexpr u32 wait_group(u32 h) {
    u32 g = 1;
    for (u32 d = 1; d <= 8u; ++d)
        if (h % d == 0u) g = d;
    return g;
}

// Start the next instruction on an 8-byte boundary (the assembler pads with
// at most one s_nop).  A wave issues an 8-byte instruction that straddles an
// 8-byte boundary more slowly: a packet loop whose 8-byte instructions all
// straddle runs about 10% slower per Update (92.7 against 84.0 cycles) than
// the same loop placed 4 bytes further on.  The loop's 4-byte instructions
// (32-bit XORs, waits, scalar bookkeeping) decide that parity, so it is reset
// after each wait.
__device__ __forceinline__ void align_issue() { asm volatile(".p2align 3"); }

// One third of the ring in the steady loop: for each group of wait_group(H)
// packets of X, wait for the group, issue the loads of the same group of Y
// (consumed two thirds of a ring later), then Update over the group.  The
// scheduling barriers keep every group's loads and waits where they are
// written: loads spread one per Update keep the wave's load queue from
// filling (a burst of them stalls the issue of the rest), and one wait per
// group instead of one per packet saves instructions (a wave issues one per
// four cycles, so each one lengthens the chain).
template <u32 H>
__device__ __forceinline__ void ring_third(State1& s, u64 (&X)[H], u64 (&Y)[H], const u8* src) {
    constexpr u32 G = wait_group(H);
#pragma unroll
    for (u32 g0 = 0; g0 < H; g0 += G) {
        wait_loaded(X[g0 + G - 1]);
        __builtin_amdgcn_sched_barrier(0);
        align_issue();
#pragma unroll
        for (u32 k = g0; k < g0 + G; ++k) Y[k] = load_le64(src + 32u * k);
#pragma unroll
        for (u32 k = g0; k < g0 + G; ++k) update1(s, X[k]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Whole packets 0..npk-1 (npk >= 1) at lp + 32*t (this thread's lane: lp
// already offset by 8*q) through a quad's state.  RING packets are in flight
// per thread, in three register thirds A, B, C of H = RING/3: while the
// Updates run over one third, the third consumed after the next one is being
// loaded, so every load has about two thirds of the ring (2H Updates) to
// arrive.  All threads of a quad run with the same npk.
template <int RING>
__device__ __forceinline__ void absorb_quad(State1& s, const u8* lp, u32 npk) {
    constexpr u32 H = RING / 3;
    static_assert(RING % 3 == 0 && H >= 4, "ring: three thirds of at least four packets");
    const u32 last = npk - 1u;
    u64 A[H], B[H], C[H];
    // one load per barrier: the loop's waits are computed from the order of
    // the loads in flight, which must be the same here as in the loop
#pragma unroll
    for (u32 k = 0; k < H; ++k) {
        A[k] = load_le64(lp + 32u * min(k, last));
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (u32 k = 0; k < H; ++k) {
        B[k] = load_le64(lp + 32u * min(H + k, last));
        __builtin_amdgcn_sched_barrier(0);
    }
    u32 t0 = 0;
    for (; t0 + 5u * H <= npk; t0 += 3u * H) {
        const u8* nx = lp + 32u * (t0 + 2u * H);
        ring_third<H>(s, A, C, nx);
        ring_third<H>(s, B, A, nx + 32u * H);
        ring_third<H>(s, C, B, nx + 64u * H);
    }
    // drain: fewer than 5H packets remain; A and B hold the first 2H of them
    // (loads past the last packet repeat it and are not used)
#pragma unroll
    for (u32 k = 0; k < H; ++k) {
        C[k] = load_le64(lp + 32u * min(t0 + 2u * H + k, last));
        if (t0 + k < npk) update1(s, A[k]);
    }
#pragma unroll
    for (u32 k = 0; k < H; ++k) {
        A[k] = load_le64(lp + 32u * min(t0 + 3u * H + k, last));
        if (t0 + H + k < npk) update1(s, B[k]);
    }
#pragma unroll
    for (u32 k = 0; k < H; ++k) {
        B[k] = load_le64(lp + 32u * min(t0 + 4u * H + k, last));
        if (t0 + 2u * H + k < npk) update1(s, C[k]);
    }
#pragma unroll
    for (u32 k = 0; k < H; ++k)
        if (t0 + 3u * H + k < npk) update1(s, A[k]);
#pragma unroll
    for (u32 k = 0; k < H; ++k)
        if (t0 + 4u * H + k < npk) update1(s, B[k]);
}

// Thread layout: a packet is four unaligned 64-bit loads (two dwordx4).
struct Packet {
    u64 w[4];
};

__device__ __forceinline__ Packet load_packet(const u8* p) {
    Packet r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.w[i] = load_le64(p + 8 * i);
    return r;
}

// wait_loaded for a whole packet: the compiler may issue its two 16-byte loads
// in either order, so the asm reads all four words and one s_waitcnt before
// it covers both loads.
__device__ __forceinline__ void wait_packet(const Packet& q) {
    asm volatile("" ::"v"(q.w[0]), "v"(q.w[1]), "v"(q.w[2]), "v"(q.w[3]));
}

// Whole packets 0..npk-1 (npk >= 1) at p through a thread's state, D packets
// in flight.  With D = 1 the compiler itself issues the next packet's load
// ahead of the Update, into other registers.  Deeper rings are laid out by
// hand like the quad loop: the prologue issues its loads one per scheduling
// barrier in the loop's order, and each packet gets an explicit wait for its
// loads, a realignment (align_issue) and then its Update followed by the
// reload of its registers.  Left to itself the compiler sank a block's loads
// below its Updates and drained the whole ring at the loop head, so each
// packet had about one Update, not D, to arrive.
template <int D>
__device__ __forceinline__ void absorb_thread(State4& s, const u8* p, u32 npk) {
    const u32 last = npk - 1u;
    Packet ring[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        ring[k] = load_packet(p + 32u * min((u32)k, last));
        if constexpr (D > 1) __builtin_amdgcn_sched_barrier(0);
    }
    u32 t0 = 0;
    for (; t0 + 2u * D < npk; t0 += D) {
        const u8* blk = p + 32u * (t0 + D);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if constexpr (D > 1) {
                wait_packet(ring[k]);
                __builtin_amdgcn_sched_barrier(0);
                align_issue();
            }
            update4(s, ring[k].w);
            ring[k] = load_packet(blk + 32 * k);
            if constexpr (D > 1) __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (t0 + k < npk) {
            update4(s, ring[k].w);
            ring[k] = load_packet(p + 32u * min(t0 + D + k, last));
        }
    }
    t0 += D;
#pragma unroll
    for (int k = 0; k < D; ++k)
        if (t0 + k < npk) update4(s, ring[k].w);
}

}  // namespace hh
