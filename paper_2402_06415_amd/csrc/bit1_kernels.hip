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
#include "bitslice.hpp"
#include "handoff.hpp"
#include "kernels.hpp"

namespace ising {

namespace {

// Philox blocks drawn straight-line before the conditional tail: three for
// the single lattice (block 2 is needed by some lane of nearly every wave at
// the critical point; 3958 against 3759 attempts/ns at L = 4096).
constexpr int kStraightBlocks = 3;

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

// One half-sweep over the whole lattice from global memory (any
// L % 64 == 0): a grid-stride loop over the words of colour c, so that the
// Philox round keys and threshold masks are set up once per thread; the
// five loads of a word are issued together and its straight-line Philox
// blocks computed while they are in flight.  L <= 65536 keeps every word
// index within 32 bits.
template <bool kGeneral, bool kCount>
__global__ void __launch_bounds__(256) k_halfsweep_bit1(uint32_t* planes, int L, int c,
                                                        uint32_t h, Key key, uint32_t lid,
                                                        Accept acc, long long* dEo,
                                                        long long* dMo,
                                                        unsigned long long* nblk_out) {
    const int nw = L >> 6;
    const uint32_t plane = (uint32_t)L * (uint32_t)nw;
    const uint32_t stride = gridDim.x * blockDim.x;
    // Workgroups are dealt to the 8 XCDs in turn: give each XCD a contiguous
    // band of the words of every pass, so that the rows above and below a
    // word, which the neighbouring workgroups also read, are in its own L2.
    uint32_t wg = blockIdx.x;
    if ((gridDim.x & 7) == 0)
        wg = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    uint32_t i = wg * blockDim.x + threadIdx.x;
    int dE = 0, dM = 0;
    unsigned long long nblk = 0;
    if (i < plane) {
        const DrawConstsT<kStraightBlocks> dc = draw_consts<kStraightBlocks>(key, acc);
        uint32_t tag[kStraightBlocks];
#pragma unroll
        for (int b = 0; b < kStraightBlocks; ++b)
            tag[b] = plane_tag((uint32_t)b, dc.rk);
        const PlaneHalf ph = plane_half(dc.rk, lid, h);
        uint32_t* P = planes + (size_t)c * plane;
        const uint32_t* Q = planes + (size_t)(1 - c) * plane;
        int y = (int)(i / (uint32_t)nw), w = (int)(i - (uint32_t)y * (uint32_t)nw);
        const int sy = (int)(stride / (uint32_t)nw), sx = (int)(stride - (uint32_t)sy * (uint32_t)nw);
        for (; i < plane; i += stride) {
            const uint32_t row = (uint32_t)y * (uint32_t)nw;
            const int wm = (w == 0) ? nw - 1 : w - 1;
            const int wp = (w + 1 == nw) ? 0 : w + 1;
            const int ym = (y == 0) ? L - 1 : y - 1;
            const int yp = (y + 1 == L) ? 0 : y + 1;
            const int p = (y + c) & 1;  // 0: the side word is the left one
            const uint32_t W = P[row + w];
            const uint32_t O = Q[row + w];
            const uint32_t X = Q[row + (p == 0 ? wm : wp)];
            const uint32_t U = Q[(uint32_t)ym * (uint32_t)nw + w];
            const uint32_t D = Q[(uint32_t)yp * (uint32_t)nw + w];
            const PlaneGroup pg = plane_group(row + (uint32_t)w, ph);
            U4 blk[kStraightBlocks];
#pragma unroll
            for (int b = 0; b < kStraightBlocks; ++b)
                blk[b] = plane_block(pg, tag[b], ph, dc.rk);
            const uint32_t S = p ? __builtin_amdgcn_alignbit(X, O, 1)
                                 : __builtin_amdgcn_alignbit(O, X, 31);
            WordState st = kGeneral ? classify(W, O, S, U, D, acc) : classify_draw(W, O, S, U, D);
#pragma unroll
            for (int b = 0; b < kStraightBlocks; ++b) {
                if (kCount)
                    nblk += st.und ? 1u : 0u;
                compare_block<kStraightBlocks>(st, blk[b], b, dc);
            }
            for (uint32_t b = kStraightBlocks; b < 8u && st.und; ++b) {
                if (kCount)
                    ++nblk;
                compare_block_uniform(st, plane_block(pg, plane_tag(b, dc.rk), ph, dc.rk), b,
                                      acc);
            }
            P[row + w] = finalize<true>(st, dE, dM);
            w += sx;
            y += sy;
            if (w >= nw) {
                w -= nw;
                ++y;
            }
        }
    }
    if (kCount)
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
// dedicated update block per group of spins.  The tile also keeps one halo
// row above and below it, per colour: the facing rows of the neighbouring
// tiles.  In each half-sweep the waves holding the first and last row
// update them first, at raised priority, and publish them.  When a wave
// holds several rows, the edge waves, once done with all their rows, wait
// for the neighbours' facing rows of the colour just updated and store them
// as the tile's halo rows while the interior rows are still being updated
// (the next half-sweep then reads LDS only).  With one row per wave that
// wait would hold up the half-sweep's barrier, so the edge waves instead
// wait for the neighbours' rows at the start of the next half-sweep, while
// the interior rows proceed.
//
// Rows are handed over through halo slots of 64-bit words, each carrying
// the 32-bit spin word and, in the high half, the number of the half-sweep
// that produced it plus one.  A reader polls its own word until the tag is
// the one it expects, so each hand-off involves a single memory location
// (relaxed agent-scope atomics: no cache write-back or invalidation, no
// grid-wide barrier).  A slot of colour c is rewritten two half-sweeps
// later, only after its writer has received the neighbour's next row,
// which the neighbour publishes only after it has received the slot (both
// receipts precede a workgroup barrier).  Slots are zeroed before every
// call, so no tag from an earlier call can match.  Waits are bounded: on
// time-out the device error word is set and the kernel runs to completion.
// ---------------------------------------------------------------------------

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

// Keeps a block's words where they are computed: the compiler may not sink
// the Philox rounds below this point (towards their first use, past the
// waits for the loads they are meant to hide).
__device__ __forceinline__ void pin(U4& v) {
    asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w));
}

// Per-thread constants of the tile sweep's draws: round keys and threshold
// masks of the straight-line blocks, and the tag words of those blocks.
struct TileDraws {
    DrawConstsT<kStraightBlocks> dc;
    uint32_t tag[kStraightBlocks];
};

// One row of one colour in a half-sweep, as the word loop sees it; every
// field is uniform in the wave.
struct RowCtx {
    uint32_t* Wr;                    // the row being updated (colour c)
    const uint32_t *Or, *Ur, *Dr;    // colour 1-c: same row, rows above and below
    const unsigned long long *su, *sd;  // halo slots of the rows above / below
    unsigned long long *pub_first, *pub_last;  // slots this row publishes (or NULL)
    uint32_t g0;                     // draw group of word 0: y * nw
    uint32_t tag_in, tag_out;        // hs (slots written by hs - 1), hs + 1
    int p;                           // 0: side neighbour left, 1: right
    bool wait_u, wait_d;             // rows above / below from the slots
};

// The decision for one word whose straight-line Philox blocks are drawn:
// classification from the word and its neighbours (X: the same-row word on
// the side given by p), the plane-by-plane comparison, further blocks while
// some site is undecided; returns the new word.
template <bool kObs, bool kGeneral, bool kCount>
__device__ __forceinline__ uint32_t decide_word(uint32_t W, uint32_t O, uint32_t X, uint32_t U,
                                                uint32_t D, int p,
                                                const U4 (&blk)[kStraightBlocks],
                                                const PlaneGroup& pg, const PlaneHalf& ph,
                                                const Accept& acc, const TileDraws& td, int& dE,
                                                int& dM, unsigned long long& nblk) {
    // side neighbour: compact column i - 1 (p == 0: the funnel shift
    // O:X >> 31) or i + 1 (p == 1: X:O >> 1)
    const uint32_t S = __builtin_amdgcn_alignbit(p ? X : O, p ? O : X, p ? 1u : 31u);
    WordState st = kGeneral ? classify(W, O, S, U, D, acc) : classify_draw(W, O, S, U, D);
#pragma unroll
    for (int b = 0; b < kStraightBlocks; ++b) {
        if (kCount)
            nblk += st.und ? 1u : 0u;
        compare_block<kStraightBlocks>(st, blk[b], b, td.dc);
    }
    for (uint32_t b = kStraightBlocks; b < 8u && st.und; ++b) {
        if (kCount)
            ++nblk;
        compare_block_uniform(st, plane_block(pg, plane_tag(b, td.dc.rk), ph, td.dc.rk), b, acc);
    }
    return finalize<kObs>(st, dE, dM);
}

// Update the words of one row: one word per lane, 64-word chunks.  The
// Philox blocks of a word do not depend on the spins, so they are computed
// between issuing the word's loads and using them: the LDS and halo-slot
// latencies hide behind them.  kGeneral: the thresholds may have
// always-flip classes (beta near 0); kCount: count the blocks drawn.
template <bool kObs, bool kGeneral, bool kCount>
__device__ __forceinline__ void update_row(const RowCtx& rc, int nw, const PlaneHalf& ph,
                                           const Accept& acc, const TileDraws& td, uint32_t* err,
                                           uint32_t spin_limit, int& dE, int& dM,
                                           unsigned long long& nblk) {
    for (int w = (int)(threadIdx.x & 63); w < nw; w += 64) {
        const int wx = rc.p ? ((w + 1 == nw) ? 0 : w + 1) : ((w == 0) ? nw - 1 : w - 1);
        // the five LDS loads are unconditional (a waiting edge row reads its
        // stale halo row and replaces it): a load issued on one side of a
        // branch only would make the compiler wait for every load at the join
        const uint32_t W = rc.Wr[w];
        const uint32_t O = rc.Or[w];
        const uint32_t X = rc.Or[wx];
        uint32_t U = rc.Ur[w];
        uint32_t D = rc.Dr[w];
        unsigned long long su, sd;
        asm("" : "=v"(su));  // defined below when used, no instruction here
        asm("" : "=v"(sd));
        if (rc.wait_u)
            su = __hip_atomic_load(rc.su + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (rc.wait_d)
            sd = __hip_atomic_load(rc.sd + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const PlaneGroup pg = plane_group(rc.g0 + (uint32_t)w, ph);
        U4 blk[kStraightBlocks];
#pragma unroll
        for (int b = 0; b < kStraightBlocks; ++b) {
            blk[b] = plane_block(pg, td.tag[b], ph, td.dc.rk);
            pin(blk[b]);
        }
        // nothing that waits on the loads moves above the draws
        __builtin_amdgcn_sched_barrier(0);
        if (rc.wait_u)
            U = finish_wait(su, rc.su + w, rc.tag_in, spin_limit, err);
        if (rc.wait_d)
            D = finish_wait(sd, rc.sd + w, rc.tag_in, spin_limit, err);
        const uint32_t nwd = decide_word<kObs, kGeneral, kCount>(W, O, X, U, D, rc.p, blk, pg, ph,
                                                                 acc, td, dE, dM, nblk);
        rc.Wr[w] = nwd;
        if (rc.pub_first)
            publish_slot(rc.pub_first + w, rc.tag_out, nwd);
        if (rc.pub_last)
            publish_slot(rc.pub_last + w, rc.tag_out, nwd);
    }
}

// The context of row r (0 <= r < rows) of the tile in half-sweep hs.  late:
// the first and last rows take the neighbour rows from the slots (after the
// first half-sweep) instead of the tile's halo rows.
__device__ __forceinline__ RowCtx row_ctx(uint32_t* tile, const TileGeom& t, int rows, int r,
                                          int64_t hs, bool late, unsigned long long* halo) {
    const int c = (int)(hs & 1), o = c ^ 1;
    const int nw = t.nw;
    uint32_t* Tc = tile + c * t.tr * nw;
    const uint32_t* To = tile + o * t.tr * nw;
    const bool first = (r == 0), last = (r == rows - 1);
    const int y = t.y0 + r;
    RowCtx rc;
    rc.Wr = Tc + (r + 1) * nw;
    rc.Or = To + (r + 1) * nw;
    rc.Ur = To + r * nw;
    rc.Dr = To + (r + 2) * nw;
    rc.su = halo_row(halo, nw, t.up, o, 1);
    rc.sd = halo_row(halo, nw, t.down, o, 0);
    rc.pub_first = first ? halo_row(halo, nw, t.me, c, 0) : nullptr;
    rc.pub_last = last ? halo_row(halo, nw, t.me, c, 1) : nullptr;
    rc.g0 = (uint32_t)y * (uint32_t)nw;
    rc.tag_in = (uint32_t)hs;
    rc.tag_out = (uint32_t)hs + 1u;
    rc.p = (y + c) & 1;
    rc.wait_u = late && hs > 0 && first;
    rc.wait_d = late && hs > 0 && last;
    if (late && hs == 0) {  // the one-row-per-wave kernel masks hs > 0 itself
        rc.wait_u = first;
        rc.wait_d = last;
    }
    return rc;
}

// Receive the facing row of colour c that a neighbouring tile published in
// half-sweep hs (tag hs + 1) into halo row `dst` (0 above the tile, rows + 1
// below it) of the tile's colour-c plane.
__device__ __forceinline__ void receive_row(uint32_t* tile, const TileGeom& t, int c, int dst,
                                            const unsigned long long* slots, uint32_t tag,
                                            uint32_t spin_limit, uint32_t* err) {
    uint32_t* row = tile + (c * t.tr + dst) * t.nw;
    for (int w = (int)(threadIdx.x & 63); w < t.nw; w += 64)
        row[w] = wait_slot(slots + w, tag, spin_limit, err);
}

// Row order within a half-sweep: the first and last rows, which the
// neighbouring tiles wait for, come first; interior rows after them.
__device__ __forceinline__ int row_of(int k, int rows) {
    return (rows <= 2 || k == 0) ? k : (k == 1 ? rows - 1 : k - 1);
}

// Sums the per-sweep energy and magnetisation changes of the workgroup
// into the traces; every thread of the workgroup takes part, after the
// half-sweep's barrier (red is free again by then).
__device__ __forceinline__ void trace_add(long long sE, long long sM, long long (*red)[16],
                                          int wave, int lane, int nwaves, int64_t j,
                                          long long* dEtr, long long* dMtr) {
    const long long e = wave_sum_i64(sE), m = wave_sum_i64(sM);
    if (lane == 0) {
        red[0][wave] = e;
        red[1][wave] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long E = 0, M = 0;
        for (int v = 0; v < nwaves; ++v) {
            E += red[0][v];
            M += red[1][v];
        }
        if (dEtr && E)
            atomicAdd(reinterpret_cast<unsigned long long*>(dEtr + j), (unsigned long long)E);
        if (dMtr && M)
            atomicAdd(reinterpret_cast<unsigned long long*>(dMtr + j), (unsigned long long)M);
    }
}

// One wave per row (rows == waves of the workgroup): wave v owns row
// row_of(v) for the whole call, so the edge rows (waves 0 and 1) keep a
// raised priority throughout, and the row's geometry is set up once.  The
// edge waves take the neighbours' facing rows from the slots when they next
// need them (late receipt), the interior rows proceed meanwhile; one
// workgroup barrier per half-sweep.
template <bool kObs, bool kGeneral, bool kCount>
__global__ void __launch_bounds__(1024) k_sweep_bit1_rows(
    uint32_t* planes, int L, int rows, int64_t n, uint32_t t0, Key key, uint32_t lid, Accept acc,
    long long* dEtr, long long* dMtr, unsigned long long* halo, uint32_t* err,
    unsigned long long* nblk_out, uint32_t spin_limit) {
    extern __shared__ uint32_t tile[];  // [2][rows + 2][nw]
    __shared__ long long red[2][16];
    const TileGeom t = tile_geom(L, rows);
    const int nwaves = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    // rows to waves rotated by the workgroup index, so that the edge rows of
    // the tiles sharing a compute unit fall on different SIMDs
    const int r = row_of((wave + (int)blockIdx.x) % rows, rows);
    TileDraws td;
    td.dc = draw_consts<kStraightBlocks>(key, acc);
#pragma unroll
    for (int b = 0; b < kStraightBlocks; ++b)
        td.tag[b] = plane_tag((uint32_t)b, td.dc.rk);
    load_tile(tile, planes, L, rows, t);
    __syncthreads();
    if (r == 0 || r == rows - 1)
        __builtin_amdgcn_s_setprio(3);  // the neighbouring tiles wait for these rows
    long long sE = 0, sM = 0;
    unsigned long long nblk = 0;
    // the row's context in the two colours, set up once
    const RowCtx rc0 = row_ctx(tile, t, rows, r, 0, true, halo);
    const RowCtx rc1 = row_ctx(tile, t, rows, r, 1, true, halo);
    for (int64_t hs = 0; hs < 2 * n; ++hs) {
        int dE = 0, dM = 0;
        const PlaneHalf ph = plane_half(td.dc.rk, lid, 2u * t0 + (uint32_t)hs);
        RowCtx rc = (hs & 1) ? rc1 : rc0;
        rc.tag_in = (uint32_t)hs;
        rc.tag_out = (uint32_t)hs + 1u;
        rc.wait_u = rc.wait_u && hs > 0;
        rc.wait_d = rc.wait_d && hs > 0;
        update_row<kObs, kGeneral, kCount>(rc, t.nw, ph, acc, td, err, spin_limit, dE, dM, nblk);
        __syncthreads();
        if (kObs) {
            sE += dE;
            sM += dM;
            if (hs & 1) {
                trace_add(sE, sM, red, wave, lane, nwaves, hs >> 1, dEtr, dMtr);
                sE = sM = 0;
            }
        }
    }
    __builtin_amdgcn_s_setprio(0);
    if (kCount)
        add_count(nblk, nblk_out);
    store_tile(planes, tile, rows, t, wave, nwaves);
}

// The one-wave-per-row kernel for rows of at most 64 words (one word per
// lane), with the draws pipelined across half-sweeps: a wave draws the
// Philox blocks of its word for half-sweep hs + 1 right after publishing
// its word of half-sweep hs, before the barrier, so that the draws fill the
// barrier's wait and after the barrier only the loads, the wait for the
// neighbours' rows, the decision and the publication remain: the chain of
// hand-offs between neighbouring tiles (each edge row needs the
// neighbour's edge row of the previous half-sweep) gets that much shorter.
template <bool kObs, bool kGeneral, bool kCount>
__global__ void __launch_bounds__(1024) k_sweep_bit1_rows_pipe(
    uint32_t* planes, int L, int rows, int64_t n, uint32_t t0, Key key, uint32_t lid, Accept acc,
    long long* dEtr, long long* dMtr, unsigned long long* halo, uint32_t* err,
    unsigned long long* nblk_out, uint32_t spin_limit) {
    extern __shared__ uint32_t tile[];  // [2][rows + 2][nw]
    __shared__ long long red[2][16];
    const TileGeom t = tile_geom(L, rows);
    const int nw = t.nw;
    const int nwaves = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int r = row_of((wave + (int)blockIdx.x) % rows, rows);
    TileDraws td;
    td.dc = draw_consts<kStraightBlocks>(key, acc);
#pragma unroll
    for (int b = 0; b < kStraightBlocks; ++b)
        td.tag[b] = plane_tag((uint32_t)b, td.dc.rk);
    load_tile(tile, planes, L, rows, t);
    __syncthreads();
    if (r == 0 || r == rows - 1)
        __builtin_amdgcn_s_setprio(3);  // the neighbouring tiles wait for these rows
    const RowCtx rc0 = row_ctx(tile, t, rows, r, 0, true, halo);
    const RowCtx rc1 = row_ctx(tile, t, rows, r, 1, true, halo);
    const int w = lane;
    const bool active = w < nw;
    // the side-neighbour word for p = 0 (left) and p = 1 (right)
    const int wl = (w == 0) ? nw - 1 : w - 1, wr = (w + 1 >= nw) ? 0 : w + 1;
    PlaneHalf ph = plane_half(td.dc.rk, lid, 2u * t0);
    PlaneGroup pg = plane_group(rc0.g0 + (uint32_t)w, ph);
    U4 blk[kStraightBlocks];
#pragma unroll
    for (int b = 0; b < kStraightBlocks; ++b)
        blk[b] = plane_block(pg, td.tag[b], ph, td.dc.rk);
    long long sE = 0, sM = 0;
    unsigned long long nblk = 0;
    for (int64_t hs = 0; hs < 2 * n; ++hs) {
        int dE = 0, dM = 0;
        RowCtx rc = (hs & 1) ? rc1 : rc0;
        rc.tag_in = (uint32_t)hs;
        rc.tag_out = (uint32_t)hs + 1u;
        rc.wait_u = rc.wait_u && hs > 0;
        rc.wait_d = rc.wait_d && hs > 0;
        if (active) {
            const uint32_t W = rc.Wr[w];
            const uint32_t O = rc.Or[w];
            const uint32_t X = rc.Or[rc.p ? wr : wl];
            uint32_t U = rc.Ur[w];
            uint32_t D = rc.Dr[w];
            if (rc.wait_u)
                U = finish_wait(
                    __hip_atomic_load(rc.su + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                    rc.su + w, rc.tag_in, spin_limit, err);
            if (rc.wait_d)
                D = finish_wait(
                    __hip_atomic_load(rc.sd + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                    rc.sd + w, rc.tag_in, spin_limit, err);
            const uint32_t nwd = decide_word<kObs, kGeneral, kCount>(W, O, X, U, D, rc.p, blk, pg,
                                                                     ph, acc, td, dE, dM, nblk);
            rc.Wr[w] = nwd;
            if (rc.pub_first)
                publish_slot(rc.pub_first + w, rc.tag_out, nwd);
            if (rc.pub_last)
                publish_slot(rc.pub_last + w, rc.tag_out, nwd);
        }
        // the publication goes out before the next half-sweep's draws
        __builtin_amdgcn_sched_barrier(0);
        if (hs + 1 < 2 * n) {
            ph = plane_half(td.dc.rk, lid, 2u * t0 + (uint32_t)hs + 1u);
            pg = plane_group(rc0.g0 + (uint32_t)w, ph);
#pragma unroll
            for (int b = 0; b < kStraightBlocks; ++b)
                blk[b] = plane_block(pg, td.tag[b], ph, td.dc.rk);
        }
        __syncthreads();
        if (kObs) {
            sE += dE;
            sM += dM;
            if (hs & 1) {
                trace_add(sE, sM, red, wave, lane, nwaves, hs >> 1, dEtr, dMtr);
                sE = sM = 0;
            }
        }
    }
    __builtin_amdgcn_s_setprio(0);
    if (kCount)
        add_count(nblk, nblk_out);
    store_tile(planes, tile, rows, t, wave, nwaves);
}

// Several rows per wave: all rows of a half-sweep complete before the next
// starts (one workgroup barrier per half-sweep); the edge rows come first
// in each half-sweep at raised priority, and the waves holding them take in
// the neighbours' facing rows into the tile's halo rows before the barrier,
// behind the interior rows.
template <bool kObs, bool kGeneral, bool kCount>
__global__ void __launch_bounds__(1024) k_sweep_bit1_tiles(
    uint32_t* planes, int L, int rows, int64_t n, uint32_t t0, Key key, uint32_t lid, Accept acc,
    long long* dEtr, long long* dMtr, unsigned long long* halo, uint32_t* err,
    unsigned long long* nblk_out, uint32_t spin_limit) {
    extern __shared__ uint32_t tile[];  // [2][rows + 2][nw]
    __shared__ long long red[2][16];
    const TileGeom t = tile_geom(L, rows);
    const int nwaves = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    TileDraws td;
    td.dc = draw_consts<kStraightBlocks>(key, acc);
#pragma unroll
    for (int b = 0; b < kStraightBlocks; ++b)
        td.tag[b] = plane_tag((uint32_t)b, td.dc.rk);
    load_tile(tile, planes, L, rows, t);
    __syncthreads();
    long long sE = 0, sM = 0;
    unsigned long long nblk = 0;
    for (int64_t hs = 0; hs < 2 * n; ++hs) {
        int dE = 0, dM = 0;
        const PlaneHalf ph = plane_half(td.dc.rk, lid, 2u * t0 + (uint32_t)hs);
        for (int k = wave; k < rows; k += nwaves) {
            const int r = row_of(k, rows);
            const bool edge = (r == 0) || (r == rows - 1);
            if (edge)
                __builtin_amdgcn_s_setprio(3);
            const RowCtx rc = row_ctx(tile, t, rows, r, hs, false, halo);
            update_row<kObs, kGeneral, kCount>(rc, t.nw, ph, acc, td, err, spin_limit, dE, dM,
                                               nblk);
            if (edge)
                __builtin_amdgcn_s_setprio(0);
        }
        // the waves of the first and last row take in the neighbours' rows
        // of this colour for the next half-sweep (row_of: k = 0 is the
        // first row, k = 1 the last)
        if (hs + 1 < 2 * n) {
            const int c = (int)(hs & 1);
            const uint32_t tag = (uint32_t)hs + 1u;
            if (wave == 0)
                receive_row(tile, t, c, 0, halo_row(halo, t.nw, t.up, c, 1), tag, spin_limit, err);
            if (wave == (rows == 1 ? 0 : 1 % nwaves))
                receive_row(tile, t, c, rows + 1, halo_row(halo, t.nw, t.down, c, 0), tag,
                            spin_limit, err);
        }
        __syncthreads();
        if (kObs) {
            sE += dE;
            sM += dM;
            if (hs & 1) {
                trace_add(sE, sM, red, wave, lane, nwaves, hs >> 1, dEtr, dMtr);
                sE = sM = 0;
            }
        }
    }
    if (kCount)
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
                                 unsigned long long* nblk, bool count, hipStream_t st) {
    // at most 4096 workgroups: a thread takes up to 64 words at L = 65536
    int64_t words = (int64_t)L * (L >> 6);
    unsigned blocks = blocks_for(words, 256);
    if (blocks > 4096)
        blocks = 4096;
    const bool general = acc.always2 || acc.always4;
    auto kern = general ? (count ? k_halfsweep_bit1<true, true> : k_halfsweep_bit1<true, false>)
                        : (count ? k_halfsweep_bit1<false, true> : k_halfsweep_bit1<false, false>);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, st, planes, L, c, h, key, lid, acc, dE,
                       dM, nblk);
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

// Tiles (workgroups) per CU: four when each still holds at least four rows,
// so that a half-sweep barrier spans a quarter of the CU's waves and the
// other tiles keep its SIMDs busy meanwhile; one for smaller lattices, whose
// tiles would be all edge rows waiting on their neighbours.
bool plan_bit1_tiles(int L, int device_cus, Bit1TilePlan* plan) {
    const int nw = L >> 6;
    if (nw < 1 || nw > 0xFFFF || device_cus < 1)
        return false;
    if (nw <= 64) {
        // Rows of at most 64 words: one tile per CU and one wave per row, with
        // the draws pipelined across half-sweeps; the tallest tile (up to
        // 16 rows, the CU's 16 waves) that still gives every CU a tile, so
        // that the fewest rows are edge rows.  A multiple of 8 tiles keeps
        // one band of tiles per XCD.
        int rows = 0;
        for (int r = 16; r >= 1 && !rows; --r) {
            const int t = L / r;
            if (L % r || t > WsLayout::kMaxTiles || t < 2)
                continue;
            if (t >= device_cus || r == 1)
                rows = r;
        }
        if (!rows)
            return false;
        plan->ntiles = L / rows;
        plan->rows = rows;
        plan->threads = 64 * rows;
        plan->lds = tile_lds_bytes(L, rows);
        return true;
    }
    const int tiles_per_cu = (int64_t)L >= (int64_t)16 * device_cus ? 4 : 1;
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
    // at most 16 waves per CU in all: the tiles sharing a CU split them
    const int wmax = 16 / tiles_per_cu > 1 ? 16 / tiles_per_cu : 1;
    plan->threads = 64 * (plan->rows < wmax ? plan->rows : wmax);
    plan->lds = tile_lds_bytes(L, plan->rows);
    return true;
}

namespace {

template <bool kObs>
const void* tiles_kernel_of(bool rows_kernel, bool pipe, bool general, bool count) {
#define ISING_TK(K, G, C) reinterpret_cast<const void*>(K<kObs, G, C>)
    if (rows_kernel && pipe)
        return general ? (count ? ISING_TK(k_sweep_bit1_rows_pipe, true, true)
                                : ISING_TK(k_sweep_bit1_rows_pipe, true, false))
                       : (count ? ISING_TK(k_sweep_bit1_rows_pipe, false, true)
                                : ISING_TK(k_sweep_bit1_rows_pipe, false, false));
    if (rows_kernel)
        return general ? (count ? ISING_TK(k_sweep_bit1_rows, true, true)
                                : ISING_TK(k_sweep_bit1_rows, true, false))
                       : (count ? ISING_TK(k_sweep_bit1_rows, false, true)
                                : ISING_TK(k_sweep_bit1_rows, false, false));
    return general ? (count ? ISING_TK(k_sweep_bit1_tiles, true, true)
                            : ISING_TK(k_sweep_bit1_tiles, true, false))
                   : (count ? ISING_TK(k_sweep_bit1_tiles, false, true)
                            : ISING_TK(k_sweep_bit1_tiles, false, false));
#undef ISING_TK
}

// The tile kernel variant a call launches: one wave per row (with the
// draws pipelined when a row is at most 64 words) or several rows per wave;
// with or without traces; thresholds with or without always-flip classes;
// counting the draws or not.
const void* tiles_kernel(int L, const Bit1TilePlan& plan, bool obs, bool general, bool count) {
    const bool rows_kernel = plan.rows * 64 == plan.threads;
    const bool pipe = (L >> 6) <= 64;
    return obs ? tiles_kernel_of<true>(rows_kernel, pipe, general, count)
               : tiles_kernel_of<false>(rows_kernel, pipe, general, count);
}

}  // namespace

int bit1_tiles_resident(int L, const Bit1TilePlan& plan, bool obs, bool general, bool count) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, tiles_kernel(L, plan, obs, general, count), plan.threads, plan.lds) !=
        hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_sweep_bit1_tiles(uint32_t* planes, int L, const Bit1TilePlan& plan, int64_t n,
                                   uint32_t t0, Key key, uint32_t lid, Accept acc, long long* dE,
                                   long long* dM, unsigned char* ws, uint32_t spin_limit,
                                   bool count, hipStream_t st) {
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
    const bool general = acc.always2 || acc.always4;
    return hipLaunchCooperativeKernel(tiles_kernel(L, plan, dE || dM, general, count),
                                      dim3(plan.ntiles), dim3(plan.threads), args, plan.lds, st);
}

}  // namespace ising
