// Four-site update of an INT8 lattice with per-site draws (internal to
// libising.so), shared by the batch sweep (lattice in LDS) and the
// single-lattice global half-sweep.
//
// A thread updates the four colour-c sites of an 8-byte span of one row
// (L % 8 == 0): three 8-byte reads (the row and the rows above and below)
// plus one byte across the span's edge give all sixteen neighbours, the
// anti-aligned neighbour counts of the four sites are formed byte-parallel
// in one register, and the four sites share one Philox4x32-10 block (they
// are q = 4g..4g+3 of their colour).
#pragma once

#include "common.hpp"

namespace ising {

constexpr uint32_t T_XOR_AND = tt((kA ^ kB) & kC);    // (a ^ b) & c
constexpr uint32_t T_OR_AND2 = tt((kA | kB) & kC);    // (a | b) & c
constexpr uint32_t T_ANDN_AND = tt(kA & ~kB & kC);    // a & ~b & c
constexpr uint32_t T_NOR_AND = tt(~(kA | kB) & kC);   // ~(a | b) & c
constexpr uint32_t T_AND_OR = tt((kA & kB) | kC);     // (a & b) | c

// Bytes 0, 2, 4, 6 and 1, 3, 5, 7 of the 8-byte value {hi:lo}.
constexpr uint32_t kSelEven = 0x06040200u;
constexpr uint32_t kSelOdd = 0x07050301u;
constexpr uint32_t kOnes = 0x01010101u;

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// Acceptance data of one lattice in the form the four-site update uses.
// A site with u = 2 flips iff r < T2, with u = 4 iff r < T4, and T4 <= T2
// (exp(-8 beta) <= exp(-4 beta)).  So with lvl = (r < T2) + (r < T4) a site
// flips iff lvl >= need, where need = 1 for u = 2, 2 for u = 4 and 0 when
// no draw is needed (u <= 0, or the class always flips).  When u = 2
// always flips, T2 is replaced by 2^32 - 1: that keeps lvl = 2 exactly
// when r < T4 and need(u = 2) is then 0.
struct QuadAccept {
    uint32_t T2, T4;  // thresholds as compared
    uint32_t M2, M0;  // need of u = 2 (0 or 1) and of u = 4 (0 or 2), in every byte
};

__device__ __forceinline__ QuadAccept quad_accept(uint32_t T2, uint32_t T4, bool always2,
                                                 bool always4) {
    return QuadAccept{always2 ? 0xFFFFFFFFu : T2, T4, always2 ? 0u : kOnes,
                      always4 ? 0u : 2u * kOnes};
}

// Per-thread counts from which a half-sweep's dE and dM follow:
// dE = 8 nflip - 2 sum_a2 (dE = 2u = 8 - 4 na per flip, a2 = 2 na), and
// dM = 2 (2 ndown - nflip) (-2 s_old per flip).
struct QuadCounts {
    uint32_t nflip = 0, ndown = 0, sum_a2 = 0;
};

// Update the four colour-c sites of the span x0..x0+7 of row y of the
// lattice (LDS or global memory).  g is their Philox group (compact indices 4g..4g+3), h = 2t+c.
// Spins are bytes 0x01 (+1) and 0xFF (-1): two spins differ exactly when
// bit 1 of their XOR is set, and a flip is an XOR with 0xFE.  All four
// sites are handled byte-parallel in one register, without branches.
// Returns the four sites' new bytes packed (byte j = site j).
__device__ __forceinline__ uint32_t update_quad(int8_t* lat, int L, int N, int y, int row, int x0,
                                                int c, uint32_t g, uint32_t h, const RoundKeys& rk,
                                                uint32_t lid, const QuadAccept& qa,
                                                QuadCounts& cnt, unsigned long long& nblk) {
    const int p = (y + c) & 1;  // colour-c sites sit at x0 + p + 2j
    // row = y L; the rows above and below, periodic
    const int rup = (row == 0 ? N : row) - L;
    const int rdn = (row + L == N ? 0 : row + L);
    const uint2 R = *reinterpret_cast<const uint2*>(lat + row + x0);
    const uint2 U = *reinterpret_cast<const uint2*>(lat + rup + x0);
    const uint2 D = *reinterpret_cast<const uint2*>(lat + rdn + x0);
    // the one neighbour outside the span: left of x0 (p = 0) or right of x0 + 7 (p = 1)
    const int xl = x0 == 0 ? L - 1 : x0 - 1;
    const int xr = x0 + 8 == L ? 0 : x0 + 8;
    const uint32_t X = (uint8_t)lat[row + (p ? xr : xl)];
    const uint32_t ev = perm(R.y, R.x, kSelEven), od = perm(R.y, R.x, kSelOdd);
    const uint32_t sel = p ? kSelOdd : kSelEven;
    const uint32_t S = p ? od : ev;                        // the four sites, byte j = site j
    const uint32_t Lf = p ? ev : ((od << 8) | X);          // their left neighbours
    const uint32_t Rt = p ? ((ev >> 8) | (X << 24)) : od;  // right neighbours
    const uint32_t Up = perm(U.y, U.x, sel), Dn = perm(D.y, D.x, sel);
    const uint32_t bit1 = 2u * kOnes;
    // byte j: a2 = twice the number of anti-aligned neighbours of site j (0..8)
    const uint32_t a2 = bop3<T_XOR_AND>(S, Lf, bit1) + bop3<T_XOR_AND>(S, Rt, bit1) +
                        bop3<T_XOR_AND>(S, Up, bit1) + bop3<T_XOR_AND>(S, Dn, bit1);
    // classes per byte (bit 0): two or more anti-aligned (u <= 0), exactly
    // one (u = 2), none (u = 4)
    const uint32_t h1 = a2 >> 1;
    const uint32_t ge2 = bop3<T_OR_AND2>(a2 >> 2, a2 >> 3, kOnes);
    const uint32_t is2 = bop3<T_ANDN_AND>(h1, ge2, kOnes);
    const uint32_t is0 = bop3<T_NOR_AND>(h1, ge2, kOnes);
    const uint32_t need = bop3<T_AND_OR>(is0 << 1, qa.M0, is2 & qa.M2);
    U4 r = {0u, 0u, 0u, 0u};
    if (need) {
        r = philox4x32_10({g, lid, h, kTagSite}, rk);
        ++nblk;
    }
    uint32_t lvl = 4u * kOnes;  // 4 + lvl_j - need_j stays in 2..6: no borrow between bytes
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t rj = u4_get(r, j);
        lvl |= ((uint32_t)(rj < qa.T2) + (uint32_t)(rj < qa.T4)) << (8 * j);
    }
    const uint32_t fb = ((lvl - need) >> 2) & kOnes;  // bit 0 of byte j: site j flips
    // 0xFE in flipped bytes: fb * 254 as a shift and a subtraction (the
    // empty asm keeps the compiler from forming a quarter-rate multiply)
    uint32_t fb8 = fb << 8;
    asm volatile("" : "+v"(fb8));
    const uint32_t F = fb8 - (fb << 1);
    cnt.nflip += __popc(fb);
    cnt.ndown += __popc(fb & (S >> 7));
    cnt.sum_a2 = __builtin_amdgcn_udot4(a2, fb, cnt.sum_a2, false);  // sum of a2_j over flips
    // spread F's bytes 0..3 to span bytes p, p + 2, p + 4, p + 6 (zeros from lo)
    const uint32_t Fx = perm(F, 0u, p ? 0x05000400u : 0x00050004u);
    const uint32_t Fy = perm(F, 0u, p ? 0x07000600u : 0x00070006u);
    *reinterpret_cast<uint2*>(lat + row + x0) = make_uint2(R.x ^ Fx, R.y ^ Fy);
    return S ^ F;
}

}  // namespace ising
