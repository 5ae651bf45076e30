// Device helpers shared by the sweep kernels of libising.so.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): per round the two
// 32x32->64 products M0*c0 and M1*c2 (one v_mad_u64_u32 each on gfx950)
// and two three-input XORs with the round key (one v_bitop3_b32 each);
// the key schedule is wave-uniform and stays in scalar registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Fourth counter word: which stream a draw belongs to.
constexpr uint32_t kTagSite = 0u;   // one uint32 per site (INT8 layout)
constexpr uint32_t kTagPlane = 1u;  // bit planes, block index in bits 8.. (BIT1)
constexpr uint32_t kTagInit = 2u;   // random start
constexpr uint32_t kTagSwap = 5u;      // replica-exchange draws
constexpr uint32_t kTagNNSample = 6u;  // site draws of the learned proposal
constexpr uint32_t kTagMH = 7u;        // acceptance draws of whole-lattice moves
constexpr uint32_t kTagXy = 8u;        // XY trials: new angle and decision
constexpr uint32_t kTagXyInit = 9u;    // XY random start

struct Key {
    uint32_t k0, k1;
};

struct U4 {
    uint32_t x, y, z, w;
};

// v_bitop3_b32 evaluates any three-input boolean function given as an 8-bit
// truth table: result bit = table[(a << 2) | (b << 1) | c].  A table is the
// function applied to the canonical operand patterns A, B, C below.
constexpr uint32_t kA = 0xF0u, kB = 0xCCu, kC = 0xAAu;
constexpr uint32_t tt(uint32_t v) { return v & 0xFFu; }

// One v_bitop3_b32 with an explicit table.  It is issued through inline
// assembly on purpose: the compiler's own fusion of and/or/xor chains into
// v_bitop3_b32 produced wrong tables for the bit-sliced comparison in this
// toolchain (ROCm 7.2, gfx950), so every multi-input bit operation of the
// sweep goes through this helper and the compiler never sees a chain to fuse.
template <uint32_t TT>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:%4" : "=v"(r) : "v"(a), "v"(b), "v"(c), "i"(TT));
    return r;
}

constexpr uint32_t kTableXor3 = (kA ^ kB ^ kC) & 0xFFu;

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, kTableXor3);
}

// The ten round keys (k + r W), computed once per thread.  They are held in
// vector registers on purpose: recomputing them in every call costs twenty
// scalar instructions per block, and keeping twenty in scalar registers
// across the sweep loops spills; as VGPR operands of v_bitop3_b32 they cost
// nothing per call.
struct RoundKeys {
    uint32_t k[20];
};

__device__ __forceinline__ RoundKeys round_keys(Key key) {
    RoundKeys rk;
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        rk.k[2 * r] = k0;
        rk.k[2 * r + 1] = k1;
        asm volatile("" : "+v"(rk.k[2 * r]), "+v"(rk.k[2 * r + 1]));
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return rk;
}

__device__ __forceinline__ U4 philox4x32_10(U4 c, const RoundKeys& rk) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
        uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
        U4 n;
        n.x = xor3((uint32_t)(p1 >> 32), c.y, rk.k[2 * r]);
        n.y = (uint32_t)p1;
        n.z = xor3((uint32_t)(p0 >> 32), c.w, rk.k[2 * r + 1]);
        n.w = (uint32_t)p0;
        c = n;
    }
    return c;
}

// Convenience form for kernels that draw only a few blocks per thread.
__device__ __forceinline__ U4 philox4x32_10(U4 c, Key key) {
    return philox4x32_10(c, round_keys(key));
}

__device__ __forceinline__ uint32_t u4_get(const U4& v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// Acceptance data passed by value to every sweep kernel.  Index k = (u+4)/2
// for u = s_i h_i in {-4,-2,0,2,4}.  Only u = 2 and u = 4 ever need a draw.
struct Accept {
    uint32_t T2, T4;         // thresholds for u = 2 (dE = 4) and u = 4 (dE = 8)
    uint32_t always2, always4;  // 1 if that class flips without a draw
};

// Wave-level sum of a 64-bit integer over the 64 lanes.
__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace ising
