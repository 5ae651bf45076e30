// BIT1 layout kernels: multi-spin coding, one bit per spin, colour planes.
//
// Plane c holds the colour-c sites; word w of row y holds compact columns
// 32w..32w+31 (bit b <-> x = 2(32w+b) + ((y+c)&1)), bit 1 meaning s = -1.
// A word of colour c has its four neighbours in plane 1-c: the aligned word
// of the same row, the words of rows y-1 and y+1 at the same index, and the
// same-row word shifted by one compact column (left when (y+c) is even,
// right when odd), so one lane updates 32 spins with bitwise logic.
//
// Draws follow the bit-plane layout: plane bit k of the 32-bit uniform r of
// the lanes of group g (= word y*L/64 + w) is word k&3 of the Philox block
// (g, lattice_id, 2t+c, 1 | (k>>2) << 8).  The comparison r < T is done
// most-significant bit first for all 32 lanes at once and stops as soon as
// every lane is decided, which leaves the outcome identical to a full
// 32-bit comparison.
#include "kernels.hpp"

namespace ising {

namespace {

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

// Per-thread constants of the comparison: the Philox round keys and, for
// the first eight planes, the threshold bits as all-ones/all-zero masks
// (t2m[k] for T2, t4m[k] for T4), both in vector registers.
struct DrawConsts {
    RoundKeys rk;
    uint32_t t2m[8], t4m[8];
};

__device__ __forceinline__ DrawConsts draw_consts(Key key, const Accept& acc) {
    DrawConsts dc;
    dc.rk = round_keys(key);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
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

// Draw the Philox blocks of word group g and compare r < T plane by plane.
// Blocks 0 and 1 (planes 0-7) are drawn unconditionally: some lane of a
// wave needs them almost always.  Further blocks are drawn while the lane
// still has undecided sites.  nblk counts the blocks the lane needed (those
// drawn while it still had an undecided site).
__device__ __forceinline__ void draw_planes(WordState& st, uint32_t g, uint32_t h, uint32_t lid,
                                            const Accept& acc, const DrawConsts& dc,
                                            unsigned long long& nblk) {
    const uint32_t m2 = st.m2;
#pragma unroll
    for (uint32_t b = 0; b < 2; ++b) {
        nblk += st.und ? 1u : 0u;
        const U4 out = philox4x32_10({g, lid, h, kTagPlane | (b << 8)}, dc.rk);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = 4 * (int)b + kk;
            compare_plane(st, u4_get(out, kk), bop3<T_BITSEL>(m2, dc.t2m[k], dc.t4m[k]));
        }
    }
    for (uint32_t b = 2; b < 8u && st.und; ++b) {
        ++nblk;
        const U4 out = philox4x32_10({g, lid, h, kTagPlane | (b << 8)}, dc.rk);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const uint32_t sh = 31u - (4u * b + (uint32_t)kk);
            const uint32_t t2m = 0u - ((acc.T2 >> sh) & 1u), t4m = 0u - ((acc.T4 >> sh) & 1u);
            compare_plane(st, u4_get(out, kk), bop3_vsv<T_BITSEL>(m2, t2m, t4m));
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
template <bool kObs>
__device__ __forceinline__ uint32_t update_word(uint32_t W, uint32_t O, uint32_t S, uint32_t U,
                                                uint32_t D, uint32_t g, uint32_t h, uint32_t lid,
                                                const Accept& acc, const DrawConsts& dc, int& dE,
                                                int& dM, unsigned long long& nblk) {
    WordState st = classify(W, O, S, U, D, acc);
    draw_planes(st, g, h, lid, acc, dc, nblk);
    return finalize<kObs>(st, dE, dM);
}

__device__ __forceinline__ uint32_t side_word(uint32_t O, uint32_t Oprev, uint32_t Onext, int p) {
    // p == 0: left neighbour (compact column i-1); p == 1: right (i+1)
    return p == 0 ? (O << 1) | (Oprev >> 31) : (O >> 1) | (Onext << 31);
}

__global__ void k_init_bit1(uint32_t* planes, int L, int start, Key key, uint32_t lid) {
    const int nw = L >> 6;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)L * nw)
        return;
    const int y = (int)(idx / nw), w = (int)(idx % nw);
    const int64_t plane = (int64_t)L * nw;
    uint32_t word[2] = {0u, 0u};
    if (start != 0) {
        // sites n = y*L + 64w + 4j + jj, j = 0..15: Philox block n >> 2
        const int64_t base = ((int64_t)y * L + 64 * w) >> 2;
        for (int j = 0; j < 16; ++j) {
            U4 o = philox4x32_10({(uint32_t)(base + j), lid, 0u, kTagInit}, key);
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int x = 64 * w + 4 * j + jj;
                const int col = (x + y) & 1;
                const uint32_t bit = u4_get(o, jj) >> 31;
                word[col] |= bit << (2 * j + (jj >> 1));
            }
        }
    }
    planes[idx] = word[0];
    planes[plane + idx] = word[1];
}

__device__ __forceinline__ void block_add_i64(long long a, long long b, long long* outA,
                                              long long* outB) {
    __shared__ long long red[2][16];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwaves = (blockDim.x + 63) >> 6;
    a = wave_sum_i64(a);
    b = wave_sum_i64(b);
    if (lane == 0) {
        red[0][wave] = a;
        red[1][wave] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long A = 0, B = 0;
        for (int w = 0; w < nwaves; ++w) {
            A += red[0][w];
            B += red[1][w];
        }
        if (outA && A)
            atomicAdd(reinterpret_cast<unsigned long long*>(outA), (unsigned long long)A);
        if (outB && B)
            atomicAdd(reinterpret_cast<unsigned long long*>(outB), (unsigned long long)B);
    }
}

// Adds per-lane counts into the device total: a wave and workgroup
// reduction, then one atomic into slot blockIdx % kRngSlots so that atomics
// to one address stay few.  Every thread of the workgroup must reach it.
__device__ __forceinline__ void add_count(unsigned long long v, unsigned long long* slots) {
    __shared__ unsigned long long part[16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w)
            t += part[w];
        if (t)
            atomicAdd(slots + (blockIdx.x % WsLayout::kRngSlots), t);
    }
}

// One half-sweep over the whole lattice, one word per thread, from global
// memory (any L % 64 == 0).
__global__ void __launch_bounds__(256) k_halfsweep_bit1(uint32_t* planes, int L, int c,
                                                        uint32_t h, Key key, uint32_t lid,
                                                        Accept acc, long long* dEo,
                                                        long long* dMo,
                                                        unsigned long long* nblk_out) {
    const int nw = L >> 6;
    const int64_t plane = (int64_t)L * nw;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int dE = 0, dM = 0;
    unsigned long long nblk = 0;
    if (idx < plane) {
        const int y = (int)(idx / nw), w = (int)(idx % nw);
        uint32_t* P = planes + (int64_t)c * plane;
        const uint32_t* Q = planes + (int64_t)(1 - c) * plane;
        const int64_t row = (int64_t)y * nw;
        const int wm = (w == 0) ? nw - 1 : w - 1;
        const int wp = (w + 1 == nw) ? 0 : w + 1;
        const int ym = (y == 0) ? L - 1 : y - 1;
        const int yp = (y + 1 == L) ? 0 : y + 1;
        const uint32_t W = P[row + w];
        const uint32_t O = Q[row + w];
        const int p = (y + c) & 1;
        const uint32_t S = side_word(O, Q[row + wm], Q[row + wp], p);
        const uint32_t U = Q[(int64_t)ym * nw + w];
        const uint32_t D = Q[(int64_t)yp * nw + w];
        const DrawConsts dc = draw_consts(key, acc);
        P[row + w] = update_word<true>(W, O, S, U, D, (uint32_t)(row + w), h, lid, acc, dc, dE, dM,
                                       nblk);
    }
    add_count(nblk, nblk_out);
    if (dEo || dMo)
        block_add_i64(dE, dM, dEo, dMo);
}

// Anti-aligned bonds (each bond joins a colour-0 and a colour-1 site, so the
// four bonds of every colour-0 site count each bond once) and set bits.
__global__ void __launch_bounds__(256) k_measure_bit1(const uint32_t* planes, int L,
                                                      long long* acc) {
    const int nw = L >> 6;
    const int64_t plane = (int64_t)L * nw;
    long long anti = 0, ones = 0;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < plane;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(idx / nw), w = (int)(idx % nw);
        const uint32_t* P = planes;
        const uint32_t* Q = planes + plane;
        const int64_t row = (int64_t)y * nw;
        const int wm = (w == 0) ? nw - 1 : w - 1;
        const int wp = (w + 1 == nw) ? 0 : w + 1;
        const int ym = (y == 0) ? L - 1 : y - 1;
        const int yp = (y + 1 == L) ? 0 : y + 1;
        const uint32_t W = P[row + w];
        const uint32_t O = Q[row + w];
        const uint32_t S = side_word(O, Q[row + wm], Q[row + wp], y & 1);
        anti += __popc(W ^ O) + __popc(W ^ S) + __popc(W ^ Q[(int64_t)ym * nw + w]) +
                __popc(W ^ Q[(int64_t)yp * nw + w]);
        ones += __popc(W) + __popc(O);
    }
    block_add_i64(anti, ones, acc, acc + 1);
}

__global__ void k_to_int8_bit1(const uint32_t* planes, int L, int8_t* out) {
    const int nw = L >> 6;
    const int64_t plane = (int64_t)L * nw;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= plane)
        return;
    const int y = (int)(idx / nw), w = (int)(idx % nw);
    const uint32_t wd[2] = {planes[idx], planes[plane + idx]};
    uint32_t* o = reinterpret_cast<uint32_t*>(out + (int64_t)y * L + 64 * w);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        uint32_t v = 0;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int xo = 4 * q + jj;  // x - 64w
            const int col = (xo + y) & 1;
            const uint32_t bit = (wd[col] >> (xo >> 1)) & 1u;
            v |= (bit ? 0xFFu : 0x01u) << (8 * jj);
        }
        o[q] = v;
    }
}

__global__ void k_from_int8_bit1(uint32_t* planes, int L, const int8_t* in) {
    const int nw = L >> 6;
    const int64_t plane = (int64_t)L * nw;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= plane)
        return;
    const int y = (int)(idx / nw), w = (int)(idx % nw);
    const int8_t* src = in + (int64_t)y * L + 64 * w;
    uint32_t wd[2] = {0u, 0u};
    for (int xo = 0; xo < 64; ++xo) {
        const int col = (xo + y) & 1;
        wd[col] |= (src[xo] < 0 ? 1u : 0u) << (xo >> 1);
    }
    planes[idx] = wd[0];
    planes[plane + idx] = wd[1];
}

// ---------------------------------------------------------------------------
// Persistent tile-resident sweep.
//
// Each workgroup owns `rows` consecutive full-width rows (both colours) in
// LDS for the whole call, the GPU analogue of the paper's supercell with a
// dedicated update block per group of spins.  Per half-sweep the waves
// holding the first and last row need the facing row of the neighbouring
// tile, of the other colour, from the previous half-sweep; they run first,
// at raised priority, and the interior rows, which depend only on the
// tile itself, are updated behind them.
//
// Rows are handed over through halo slots of 64-bit words, each carrying
// the 32-bit spin word and, in the high half, the number of the half-sweep
// that produced it plus one.  A reader polls its own word until the tag is
// the one it expects, so each hand-off involves a single memory location
// (relaxed agent-scope atomics: no cache write-back or invalidation, no
// grid-wide barrier).  A slot of colour c is rewritten two half-sweeps
// later, only after its writer has read the neighbour's next row, which
// the neighbour publishes after reading the slot.  Slots are zeroed before
// every call, so no tag from an earlier call can match.  Waits are bounded:
// on time-out the device error word is set and the kernel runs to
// completion.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t wait_slot(const unsigned long long* slot, uint32_t tag,
                                              uint32_t limit, uint32_t* err) {
    uint32_t spins = 0;
    unsigned long long v;
    for (;;) {
        v = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == tag)
            break;
        if (++spins > limit) {
            atomicOr(err, 1u);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return (uint32_t)v;
}

__device__ __forceinline__ void publish_slot(unsigned long long* slot, uint32_t tag,
                                             uint32_t word) {
    __hip_atomic_store(slot, ((unsigned long long)tag << 32) | word, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Tile geometry shared by the two tile-resident kernels.
struct TileGeom {
    int nw, tr, ntiles, me, up, down, y0;
    int64_t plane;
};

__device__ __forceinline__ TileGeom tile_geom(int L, int rows) {
    TileGeom t;
    t.nw = L >> 6;
    t.plane = (int64_t)L * t.nw;
    t.tr = rows + 2;
    t.ntiles = gridDim.x;
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous band of tiles so most hand-offs stay within one XCD.
    t.me = blockIdx.x;
    if ((t.ntiles & 7) == 0)
        t.me = (blockIdx.x & 7) * (t.ntiles >> 3) + (blockIdx.x >> 3);
    t.up = (t.me == 0) ? t.ntiles - 1 : t.me - 1;
    t.down = (t.me + 1 == t.ntiles) ? 0 : t.me + 1;
    t.y0 = t.me * rows;
    return t;
}

// halo[tile][colour][0 = first row, 1 = last row][nw] of (tag << 32 | word)
__device__ __forceinline__ unsigned long long* halo_row(unsigned long long* halo, int nw, int t,
                                                        int col, int which) {
    return halo + (((int64_t)t * 2 + col) * 2 + which) * (int64_t)nw;
}

__device__ __forceinline__ void load_tile(uint32_t* tile, const uint32_t* planes, int L, int rows,
                                          const TileGeom& t) {
    for (int i = threadIdx.x; i < 2 * t.tr * t.nw; i += blockDim.x) {
        const int col = i / (t.tr * t.nw);
        const int rem = i - col * t.tr * t.nw;
        const int r = rem / t.nw - 1, w = rem % t.nw;
        int y = t.y0 + r;
        y = (y < 0) ? y + L : (y >= L ? y - L : y);
        tile[i] = planes[(int64_t)col * t.plane + (int64_t)y * t.nw + w];
    }
}

__device__ __forceinline__ void store_tile(uint32_t* planes, const uint32_t* tile, int rows,
                                           const TileGeom& t, int first_row, int row_step) {
    for (int r = first_row; r < rows; r += row_step)
        for (int col = 0; col < 2; ++col)
            for (int w = (int)(threadIdx.x & 63); w < t.nw; w += 64)
                planes[(int64_t)col * t.plane + (int64_t)(t.y0 + r) * t.nw + w] =
                    tile[(col * t.tr + r + 1) * t.nw + w];
}

// Update row r of colour c of the tile (both neighbours of every word are
// available): one word per lane, 64-word chunks.  Rows 0 and rows-1 read
// the facing row of the neighbouring tile from its halo slot (after the
// first half-sweep) and publish their own.
template <bool kObs>
__device__ __forceinline__ void update_row(uint32_t* tile, const TileGeom& t, int rows, int r,
                                           int64_t hs, uint32_t t0, uint32_t lid,
                                           const Accept& acc, const DrawConsts& dc,
                                           unsigned long long* halo,
                                           uint32_t* err, uint32_t spin_limit, int& dE, int& dM,
                                           unsigned long long& nblk) {
    const int c = (int)(hs & 1), o = c ^ 1;
    const int nw = t.nw;
    const uint32_t h = 2u * t0 + (uint32_t)hs;
    const uint32_t tag_in = (uint32_t)hs;        // written at half-sweep hs - 1
    const uint32_t tag_out = (uint32_t)hs + 1u;  // written now
    uint32_t* Tc = tile + c * t.tr * nw;
    const uint32_t* To = tile + o * t.tr * nw;
    const bool first = (r == 0), last = (r == rows - 1);
    const int y = t.y0 + r;
    for (int w = (int)(threadIdx.x & 63); w < nw; w += 64) {
        const int wm = (w == 0) ? nw - 1 : w - 1;
        const int wp = (w + 1 == nw) ? 0 : w + 1;
        const uint32_t* Orow = To + (r + 1) * nw;
        const uint32_t W = Tc[(r + 1) * nw + w];
        const uint32_t O = Orow[w];
        const uint32_t S = side_word(O, Orow[wm], Orow[wp], (y + c) & 1);
        const uint32_t U = (hs > 0 && first)
                               ? wait_slot(halo_row(halo, nw, t.up, o, 1) + w, tag_in, spin_limit, err)
                               : To[r * nw + w];
        const uint32_t D = (hs > 0 && last)
                               ? wait_slot(halo_row(halo, nw, t.down, o, 0) + w, tag_in, spin_limit, err)
                               : To[(r + 2) * nw + w];
        WordState st = classify(W, O, S, U, D, acc);
        draw_planes(st, (uint32_t)((int64_t)y * nw + w), h, lid, acc, dc, nblk);
        const uint32_t nwd = finalize<kObs>(st, dE, dM);
        Tc[(r + 1) * nw + w] = nwd;
        if (first)
            publish_slot(halo_row(halo, nw, t.me, c, 0) + w, tag_out, nwd);
        if (last)
            publish_slot(halo_row(halo, nw, t.me, c, 1) + w, tag_out, nwd);
    }
}

// Row order within a half-sweep: the first and last rows, which the
// neighbouring tiles wait for, come first; interior rows after them.
__device__ __forceinline__ int row_of(int k, int rows) {
    return (rows <= 2 || k == 0) ? k : (k == 1 ? rows - 1 : k - 1);
}

// All rows of a half-sweep complete before the next starts (one workgroup
// barrier per half-sweep); with kObs the workgroup also sums the energy and
// magnetisation changes of each sweep into the traces.
template <bool kObs>
__global__ void __launch_bounds__(1024) k_sweep_bit1_tiles(
    uint32_t* planes, int L, int rows, int64_t n, uint32_t t0, Key key, uint32_t lid, Accept acc,
    long long* dEtr, long long* dMtr, unsigned long long* halo, uint32_t* err,
    unsigned long long* nblk_out, uint32_t spin_limit) {
    extern __shared__ uint32_t tile[];  // [2][rows + 2][nw]
    __shared__ long long red[2][16];
    const TileGeom t = tile_geom(L, rows);
    const int nwaves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const DrawConsts dc = draw_consts(key, acc);
    load_tile(tile, planes, L, rows, t);
    __syncthreads();
    long long sE = 0, sM = 0;
    unsigned long long nblk = 0;
    for (int64_t hs = 0; hs < 2 * n; ++hs) {
        int dE = 0, dM = 0;
        for (int k = wave; k < rows; k += nwaves) {
            const int r = row_of(k, rows);
            const bool edge = (r == 0) || (r == rows - 1);
            if (edge)
                __builtin_amdgcn_s_setprio(3);
            update_row<kObs>(tile, t, rows, r, hs, t0, lid, acc, dc, halo, err, spin_limit, dE, dM,
                             nblk);
            if (edge)
                __builtin_amdgcn_s_setprio(0);
        }
        sE += dE;
        sM += dM;
        if (kObs && (hs & 1)) {
            long long e = wave_sum_i64(sE), m = wave_sum_i64(sM);
            if (lane == 0) {
                red[0][wave] = e;
                red[1][wave] = m;
            }
            sE = 0;
            sM = 0;
        }
        __syncthreads();
        if (kObs && (hs & 1) && threadIdx.x == 0) {
            long long e = 0, m = 0;
            for (int v = 0; v < nwaves; ++v) {
                e += red[0][v];
                m += red[1][v];
            }
            const int64_t j = hs >> 1;
            if (dEtr && e)
                atomicAdd(reinterpret_cast<unsigned long long*>(dEtr + j), (unsigned long long)e);
            if (dMtr && m)
                atomicAdd(reinterpret_cast<unsigned long long*>(dMtr + j), (unsigned long long)m);
        }
    }
    add_count(nblk, nblk_out);
    store_tile(planes, tile, rows, t, wave, nwaves);
}

inline unsigned blocks_for(int64_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

hipError_t launch_init_bit1(uint32_t* planes, int L, int start, Key key, uint32_t lid,
                            hipStream_t st) {
    int64_t words = (int64_t)L * (L >> 6);
    hipLaunchKernelGGL(k_init_bit1, dim3(blocks_for(words, 256)), dim3(256), 0, st, planes, L,
                       start, key, lid);
    return hipGetLastError();
}

hipError_t launch_halfsweep_bit1(uint32_t* planes, int L, int c, uint32_t h, Key key,
                                 uint32_t lid, Accept acc, long long* dE, long long* dM,
                                 unsigned long long* nblk, hipStream_t st) {
    int64_t words = (int64_t)L * (L >> 6);
    hipLaunchKernelGGL(k_halfsweep_bit1, dim3(blocks_for(words, 256)), dim3(256), 0, st, planes, L,
                       c, h, key, lid, acc, dE, dM, nblk);
    return hipGetLastError();
}

hipError_t launch_measure_bit1(const uint32_t* planes, int L, long long* acc, hipStream_t st) {
    int64_t words = (int64_t)L * (L >> 6);
    unsigned blocks = blocks_for(words, 256);
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(k_measure_bit1, dim3(blocks), dim3(256), 0, st, planes, L, acc);
    return hipGetLastError();
}

hipError_t launch_to_int8_bit1(const uint32_t* planes, int L, int8_t* out, hipStream_t st) {
    int64_t words = (int64_t)L * (L >> 6);
    hipLaunchKernelGGL(k_to_int8_bit1, dim3(blocks_for(words, 256)), dim3(256), 0, st, planes, L,
                       out);
    return hipGetLastError();
}

hipError_t launch_from_int8_bit1(uint32_t* planes, int L, const int8_t* in, hipStream_t st) {
    int64_t words = (int64_t)L * (L >> 6);
    hipLaunchKernelGGL(k_from_int8_bit1, dim3(blocks_for(words, 256)), dim3(256), 0, st, planes, L,
                       in);
    return hipGetLastError();
}

size_t tile_lds_bytes(int L, int rows) {
    // tile of both colours with one halo row each side
    return (size_t)2 * (rows + 2) * (L >> 6) * sizeof(uint32_t);
}

bool plan_bit1_tiles(int L, int device_cus, int tiles_per_cu, Bit1TilePlan* plan) {
    const int nw = L >> 6;
    if (nw < 1 || nw > 0xFFFF || tiles_per_cu < 1)
        return false;
    int maxt = device_cus * tiles_per_cu;
    if (maxt > WsLayout::kMaxTiles)
        maxt = WsLayout::kMaxTiles;
    if (maxt > L)
        maxt = L;
    // Largest tile count that divides L and whose tiles fit their share of
    // the CU's LDS (at most 64 KiB each); a multiple of 8 (one band of tiles
    // per XCD) is preferred when it is at least half as large.
    const size_t lds_cap = (size_t)(160 * 1024) / (size_t)tiles_per_cu < (size_t)(64 * 1024)
                               ? (size_t)(160 * 1024) / (size_t)tiles_per_cu
                               : (size_t)(64 * 1024);
    int best = 0, best8 = 0;
    for (int t = maxt; t >= 2; --t) {
        if (L % t)
            continue;
        if (tile_lds_bytes(L, L / t) > lds_cap)
            continue;
        if (!best)
            best = t;
        if ((t & 7) == 0 && !best8)
            best8 = t;
    }
    if (best8 && 2 * best8 >= best)
        best = best8;
    if (best < 2)
        return false;
    plan->ntiles = best;
    plan->rows = L / best;
    plan->threads = 64 * (plan->rows < 16 ? plan->rows : 16);
    plan->lds = tile_lds_bytes(L, plan->rows);
    return true;
}

hipError_t launch_sweep_bit1_tiles(uint32_t* planes, int L, const Bit1TilePlan& plan, int64_t n,
                                   uint32_t t0, Key key, uint32_t lid, Accept acc, long long* dE,
                                   long long* dM, unsigned char* ws, uint32_t spin_limit,
                                   hipStream_t st) {
    unsigned long long* halo = reinterpret_cast<unsigned long long*>(ws + WsLayout::kHalo);
    uint32_t* err = reinterpret_cast<uint32_t*>(ws + WsLayout::kErr);
    unsigned long long* nblk = reinterpret_cast<unsigned long long*>(ws + WsLayout::kRngBlocks);
    // zero every tag so that nothing left by an earlier call can match
    hipError_t e = launch_fill_i64(reinterpret_cast<long long*>(halo),
                                   (int64_t)plan.ntiles * 2 * 2 * (L >> 6), 0, st);
    if (e != hipSuccess)
        return e;
    int rows = plan.rows;
    void* args[] = {&planes, (void*)&L, &rows, &n, &t0, &key, &lid, &acc, &dE, &dM,
                    &halo, &err, &nblk, &spin_limit};
    const void* kern = (dE || dM) ? reinterpret_cast<const void*>(k_sweep_bit1_tiles<true>)
                                  : reinterpret_cast<const void*>(k_sweep_bit1_tiles<false>);
    return hipLaunchCooperativeKernel(kern, dim3(plan.ntiles), dim3(plan.threads), args, plan.lds,
                                      st);
}

}  // namespace ising
