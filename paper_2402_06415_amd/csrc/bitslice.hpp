// Bit-sliced Metropolis update of 32 spins of one colour at once (multi-spin
// coding, one bit per spin, bit 1 meaning s = -1), shared by the sweep
// kernels that keep lattices as colour bit planes.
//
// Draws follow the bit-plane layout: plane bit k of the 32-bit uniform r of
// the lanes of group g is word k&3 of the Philox block
// (g, lattice_id, 2t+c, 1 | (k>>2) << 8).  The comparison r < T is done
// most-significant bit first for all 32 lanes at once and stops as soon as
// every lane is decided, which leaves the outcome identical to a full
// 32-bit comparison.
#pragma once

#include "common.hpp"

namespace ising {

// Truth tables used by the bit-sliced update (a, b, c = operands 1..3).
constexpr uint32_t T_XOR3 = tt(kA ^ kB ^ kC);                     // a ^ b ^ c
constexpr uint32_t T_MAJ = tt((kA & kB) | (kA & kC) | (kB & kC));  // at least two set
constexpr uint32_t T_OR_AND = tt(kA | (kB & kC));                 // a | (b & c)
constexpr uint32_t T_NOR3 = tt(~(kA | kB | kC));                  // none set
constexpr uint32_t T_XOR_ANDN = tt((kA ^ kB) & ~kC);              // (a ^ b) & ~c
constexpr uint32_t T_AND_ANDN = tt(kA & kB & ~kC);                // a & b & ~c
constexpr uint32_t T_AND_XNOR = tt(kA & ~(kB ^ kC));              // a & (b == c)
constexpr uint32_t T_OR2 = tt(kA | kB);                           // a | b   (c unused)
constexpr uint32_t T_AND2 = tt(kA & kB);                          // a & b   (c unused)
constexpr uint32_t T_BITSEL = tt((kA & kB) | (~kA & kC));         // a ? b : c, bitwise
constexpr uint32_t T_OR3 = tt(kA | kB | kC);                      // a | b | c

// Bit-sliced state of one 32-spin word during its update (steps 2 and 3 of
// the single-spin-flip trial for 32 sites at once).
struct WordState {
    uint32_t W;     // spins before the update (bit 1: s = -1)
    uint32_t flip;  // lanes decided to flip so far
    uint32_t und;   // lanes whose comparison r < T is still undecided
    uint32_t m2;    // lanes with u = 2 (dE = 4); the other undecided lanes have u = 4
    uint32_t sm, a3, cy;  // A = sm + a3 + 2 cy anti-aligned neighbours (for dE)
};

// Classify the lanes of word W from its aligned, shifted, upper and lower
// neighbour words: u = s h = 4 - 2A with A the count of anti-aligned bonds.
__device__ __forceinline__ WordState classify(uint32_t W, uint32_t O, uint32_t S, uint32_t U,
                                              uint32_t D, const Accept& acc) {
    const uint32_t a0 = W ^ O, a1 = W ^ S, a2 = W ^ U, a3 = W ^ D;
    WordState st;
    st.W = W;
    st.a3 = a3;
    st.sm = bop3<T_XOR3>(a0, a1, a2);  // low bit of a0 + a1 + a2
    st.cy = bop3<T_MAJ>(a0, a1, a2);   // its carry
    st.flip = bop3<T_OR_AND>(st.cy, st.sm, a3);       // A >= 2: dE <= 0, always flips
    uint32_t m4 = bop3<T_NOR3>(st.sm, st.cy, a3);     // A == 0: u = 4
    uint32_t m2 = bop3<T_XOR_ANDN>(st.sm, a3, st.cy); // A == 1: u = 2
    if (acc.always2) {
        st.flip = bop3<T_OR2>(st.flip, m2, m2);
        m2 = 0;
    }
    if (acc.always4) {
        st.flip = bop3<T_OR2>(st.flip, m4, m4);
        m4 = 0;
    }
    st.m2 = m2;
    st.und = bop3<T_OR2>(m2, m4, m4);
    return st;
}

// Classification without the always-flip classes: for every beta whose
// thresholds are both below 2^32 (all beta > 1e-9 or so), u = 2 and u = 4
// always draw.  Branch-free; the caller picks it only in that case.  The
// anti-aligned counts are those of classify, formed with fewer operations:
// with a_i = W ^ N_i, a0 ^ a1 ^ a2 = W ^ O ^ S ^ U, and the majority of
// (a0, a1, a2) is W ^ MAJ(O, S, U) (complementing all three inputs of a
// majority complements it).
__device__ __forceinline__ WordState classify_draw(uint32_t W, uint32_t O, uint32_t S, uint32_t U,
                                                   uint32_t D) {
    WordState st;
    st.W = W;
    st.a3 = W ^ D;
    st.sm = bop3<T_XOR3>(W, O, S) ^ U;
    st.cy = W ^ bop3<T_MAJ>(O, S, U);
    st.flip = bop3<T_OR_AND>(st.cy, st.sm, st.a3);     // A >= 2: dE <= 0
    st.m2 = bop3<T_XOR_ANDN>(st.sm, st.a3, st.cy);     // A == 1: u = 2
    st.und = ~st.flip;                                  // A <= 1: u = 2 or 4, both draw
    return st;
}

// ---------------------------------------------------------------------------
// Plane-draw Philox blocks with the group-independent work hoisted.
//
// The blocks of one half-sweep have counters (g, lid, h, 1 | b << 8): only
// g varies between the lanes and only the tag between the blocks of one
// group.  Written out, Philox4x32-10's first three rounds then split into a
// part fixed for the half-sweep (PlaneHalf), a part fixed for the group
// (PlaneGroup: two products shared by its blocks) and 6 of the 12
// instructions of those rounds per block; rounds 4-10 are the plain ones.
// The result is bitwise Philox4x32-10 of that counter.
// ---------------------------------------------------------------------------
struct PlaneHalf {
    uint32_t a;  // lo(M1 h) ^ k0[1]      round 2: x = hi(M1 z1) ^ a
    uint32_t b;  // hi(M0 x1) ^ k1[1]     round 2: z = lo(M0 g) ^ b
    uint32_t c;  // lo(M0 x1) ^ k1[2]     round 3: z = hi(M0 x2) ^ c
};

// x1 = hi(M1 h) ^ lid ^ k0[0] is round 1's x; round keys k0[r] = rk.k[2r],
// k1[r] = rk.k[2r + 1].
__device__ __forceinline__ PlaneHalf plane_half(const RoundKeys& rk, uint32_t lid, uint32_t h) {
    const uint64_t ph = (uint64_t)kPhiloxM1 * h;
    const uint32_t x1 = xor3((uint32_t)(ph >> 32), lid, rk.k[0]);
    const uint64_t px = (uint64_t)kPhiloxM0 * x1;
    PlaneHalf r;
    r.a = (uint32_t)ph ^ rk.k[2];
    r.b = (uint32_t)(px >> 32) ^ rk.k[3];
    r.c = (uint32_t)px ^ rk.k[5];
    return r;
}

struct PlaneGroup {
    uint32_t h0;      // hi(M0 g): round 1's z is h0 ^ tag ^ k1[0]
    uint32_t hz, lz;  // M1 (lo(M0 g) ^ b): round 3's product of z
};

__device__ __forceinline__ PlaneGroup plane_group(uint32_t g, const PlaneHalf& ph) {
    const uint64_t pg = (uint64_t)kPhiloxM0 * g;
    const uint64_t pz = (uint64_t)kPhiloxM1 * ((uint32_t)pg ^ ph.b);
    PlaneGroup r;
    r.h0 = (uint32_t)(pg >> 32);
    r.hz = (uint32_t)(pz >> 32);
    r.lz = (uint32_t)pz;
    return r;
}

// The tag word of block b folded with round 1's key: (1 | b << 8) ^ k1[0].
__device__ __forceinline__ uint32_t plane_tag(uint32_t b, const RoundKeys& rk) {
    return (kTagPlane | (b << 8)) ^ rk.k[1];
}

__device__ __forceinline__ U4 plane_block(const PlaneGroup& pg, uint32_t tag, const PlaneHalf& ph,
                                          const RoundKeys& rk) {
    const uint64_t p1 = (uint64_t)kPhiloxM1 * (pg.h0 ^ tag);  // round 2
    const uint32_t x2 = (uint32_t)(p1 >> 32) ^ ph.a;
    const uint64_t p0 = (uint64_t)kPhiloxM0 * x2;             // round 3
    U4 c;
    c.x = xor3(pg.hz, (uint32_t)p1, rk.k[4]);
    c.y = pg.lz;
    c.z = (uint32_t)(p0 >> 32) ^ ph.c;
    c.w = (uint32_t)p0;
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        const uint64_t q0 = (uint64_t)kPhiloxM0 * c.x;
        const uint64_t q1 = (uint64_t)kPhiloxM1 * c.z;
        U4 n;
        n.x = xor3((uint32_t)(q1 >> 32), c.y, rk.k[2 * r]);
        n.y = (uint32_t)q1;
        n.z = xor3((uint32_t)(q0 >> 32), c.w, rk.k[2 * r + 1]);
        n.w = (uint32_t)q0;
        c = n;
    }
    return c;
}

// Per-thread constants of the comparison: the Philox round keys and, for
// the first eight planes, the threshold bits as all-ones/all-zero masks
// (t2m[k] for T2, t4m[k] for T4), both in vector registers.
// Per-thread constants of the draws: the Philox round keys and, for the
// kBlocks blocks drawn unconditionally, the threshold bit of each of their
// 4 kBlocks planes as a full mask.
template <int kBlocks>
struct DrawConstsT {
    RoundKeys rk;
    uint32_t t2m[4 * kBlocks], t4m[4 * kBlocks];
};
using DrawConsts = DrawConstsT<2>;

template <int kBlocks = 2>
__device__ __forceinline__ DrawConstsT<kBlocks> draw_consts(Key key, const Accept& acc) {
    DrawConstsT<kBlocks> dc;
    dc.rk = round_keys(key);
#pragma unroll
    for (int k = 0; k < 4 * kBlocks; ++k) {
        dc.t2m[k] = 0u - ((acc.T2 >> (31 - k)) & 1u);
        dc.t4m[k] = 0u - ((acc.T4 >> (31 - k)) & 1u);
        asm volatile("" : "+v"(dc.t2m[k]), "+v"(dc.t4m[k]));
    }
    return dc;
}

// Bit-select with the middle operand in a scalar register (a wave-uniform
// value; one scalar source is within the VALU's constant-bus limit).
template <uint32_t TT>
__device__ __forceinline__ uint32_t bop3_vsv(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:%4" : "=v"(r) : "v"(a), "s"(b), "v"(c), "i"(TT));
    return r;
}

// One plane of the most-significant-bit-first comparison r < T: P holds bit
// (31 - k) of r for the 32 lanes and tm the threshold bit of each lane (T2's
// for u = 2 lanes, T4's for u = 4 lanes).  Lanes that are already decided
// ignore tm, so tm = m2 ? t2 : t4 suffices.  A lane is decided at the first
// bit where r and its threshold differ: accepted when r has 0 there
// (r < T), rejected when r has 1.
__device__ __forceinline__ void compare_plane(WordState& st, uint32_t P, uint32_t tm) {
    st.flip = bop3<T_OR2>(st.flip, bop3<T_AND_ANDN>(st.und, tm, P), P);
    st.und = bop3<T_AND_XNOR>(st.und, P, tm);
}

// One plane of the comparison with the acceptance returned instead of
// merged into flip (the caller merges two planes' acceptances at once).
__device__ __forceinline__ uint32_t plane_accept(WordState& st, uint32_t P, uint32_t tm) {
    const uint32_t a = bop3<T_AND_ANDN>(st.und, tm, P);  // undecided, T bit 1, r bit 0
    st.und = bop3<T_AND_XNOR>(st.und, P, tm);
    return a;
}

// Compare the four planes of block b (planes 4b..4b+3) of one word, the
// threshold bits taken from the masks in vector registers (b < kBlocks).
template <int kBlocks>
__device__ __forceinline__ void compare_block(WordState& st, const U4& out, int b,
                                              const DrawConstsT<kBlocks>& dc) {
    const uint32_t m2 = st.m2;
    uint32_t a[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
        a[kk] = plane_accept(st, u4_get(out, kk),
                             bop3<T_BITSEL>(m2, dc.t2m[4 * b + kk], dc.t4m[4 * b + kk]));
    st.flip = bop3<T_OR3>(st.flip, a[0], a[1]);
    st.flip = bop3<T_OR3>(st.flip, a[2], a[3]);
}

// The same for any block, the threshold bits extracted from the
// wave-uniform thresholds (scalar work).
__device__ __forceinline__ void compare_block_uniform(WordState& st, const U4& out, uint32_t b,
                                                      const Accept& acc) {
    const uint32_t m2 = st.m2;
    uint32_t a[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const uint32_t sh = 31u - (4u * b + (uint32_t)kk);
        const uint32_t t2m = 0u - ((acc.T2 >> sh) & 1u), t4m = 0u - ((acc.T4 >> sh) & 1u);
        a[kk] = plane_accept(st, u4_get(out, kk), bop3_vsv<T_BITSEL>(m2, t2m, t4m));
    }
    st.flip = bop3<T_OR3>(st.flip, a[0], a[1]);
    st.flip = bop3<T_OR3>(st.flip, a[2], a[3]);
}

// Draw the Philox blocks of word group g and compare r < T plane by plane.
// kUniformAccept: the thresholds are the same in every lane of the wave
// (the tail's threshold bits then go in as scalar operands).
// The first kBlocks blocks (planes 0 .. 4 kBlocks - 1) are drawn
// unconditionally, straight-line: some lane of a wave needs them almost
// always (blocks 0 and 1; block 2 in about 98% of the waves at the critical
// point).  Further blocks are drawn while the lane still has undecided
// sites.  nblk counts the blocks the lane needed (those drawn while it still
// had an undecided site).
template <bool kUniformAccept = true, int kBlocks = 2>
__device__ __forceinline__ void draw_planes(WordState& st, uint32_t g, uint32_t h, uint32_t lid,
                                            const Accept& acc, const DrawConstsT<kBlocks>& dc,
                                            unsigned long long& nblk) {
    const uint32_t m2 = st.m2;
#pragma unroll
    for (uint32_t b = 0; b < (uint32_t)kBlocks; ++b) {
        nblk += st.und ? 1u : 0u;
        const U4 out = philox4x32_10({g, lid, h, kTagPlane | (b << 8)}, dc.rk);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = 4 * (int)b + kk;
            compare_plane(st, u4_get(out, kk), bop3<T_BITSEL>(m2, dc.t2m[k], dc.t4m[k]));
        }
    }
    for (uint32_t b = kBlocks; b < 8u && st.und; ++b) {
        ++nblk;
        const U4 out = philox4x32_10({g, lid, h, kTagPlane | (b << 8)}, dc.rk);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const uint32_t sh = 31u - (4u * b + (uint32_t)kk);
            if (kUniformAccept) {
                const uint32_t t2m = 0u - ((acc.T2 >> sh) & 1u), t4m = 0u - ((acc.T4 >> sh) & 1u);
                compare_plane(st, u4_get(out, kk), bop3_vsv<T_BITSEL>(m2, t2m, t4m));
            } else {
                // per-lane thresholds: one signed one-bit field extract each
                const uint32_t t2m = (uint32_t)__builtin_amdgcn_sbfe((int)acc.T2, (int)sh, 1);
                const uint32_t t4m = (uint32_t)__builtin_amdgcn_sbfe((int)acc.T4, (int)sh, 1);
                compare_plane(st, u4_get(out, kk), bop3<T_BITSEL>(m2, t2m, t4m));
            }
        }
    }
}

// New word after all draws (lanes still undecided have r == T: rejected);
// with kObs also the energy and magnetisation changes of the flips.
template <bool kObs>
__device__ __forceinline__ uint32_t finalize(const WordState& st, int& dE, int& dM) {
    if (kObs) {
        const uint32_t f = st.flip;
        const int nf = __popc(f);
        // dM = sum over flips of -2 s_old = 2 (#flipped down - #flipped up)
        dM += 2 * (2 * __popc(bop3<T_AND2>(f, st.W, st.W)) - nf);
        // dE = sum over flips of 2u = 8 - 4A;  A = sm + a3 + 2 cy
        dE += 8 * nf - 4 * (__popc(bop3<T_AND2>(f, st.sm, st.sm)) +
                            __popc(bop3<T_AND2>(f, st.a3, st.a3)) +
                            2 * __popc(bop3<T_AND2>(f, st.cy, st.cy)));
    }
    return st.W ^ st.flip;
}

// Complete Metropolis update of one word (all 32 planes available).
template <bool kObs, int kBlocks>
__device__ __forceinline__ uint32_t update_word(uint32_t W, uint32_t O, uint32_t S, uint32_t U,
                                                uint32_t D, uint32_t g, uint32_t h, uint32_t lid,
                                                const Accept& acc, const DrawConstsT<kBlocks>& dc,
                                                int& dE, int& dM, unsigned long long& nblk) {
    WordState st = classify(W, O, S, U, D, acc);
    draw_planes<true, kBlocks>(st, g, h, lid, acc, dc, nblk);
    return finalize<kObs>(st, dE, dM);
}

__device__ __forceinline__ uint32_t side_word(uint32_t O, uint32_t Oprev, uint32_t Onext, int p) {
    // p == 0: left neighbour (compact column i-1); p == 1: right (i+1)
    return p == 0 ? (O << 1) | (Oprev >> 31) : (O >> 1) | (Onext << 31);
}

}  // namespace ising
