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
constexpr uint32_t T_XOR3 = tt(kA ^ kB ^ kC);              // a ^ b ^ c
constexpr uint32_t T_MAJ = tt((kA & kB) | (kA & kC) | (kB & kC));  // at least two set
constexpr uint32_t T_OR_AND = tt(kA | (kB & kC));          // a | (b & c)
constexpr uint32_t T_NOR3 = tt(~(kA | kB | kC));           // none set
constexpr uint32_t T_XOR_ANDN = tt((kA ^ kB) & ~kC);       // (a ^ b) & ~c
constexpr uint32_t T_AND_XNOR = tt(kA & ~(kB ^ kC));       // a & (b == c)
constexpr uint32_t T_AND_ANDN = tt(kA & kB & ~kC);         // a & b & ~c
constexpr uint32_t T_OR3 = tt(kA | kB | kC);               // a | b | c
constexpr uint32_t T_AND = tt(kA & kB);                    // a & b (c ignored)

// Metropolis update of one 32-spin word W of colour c (steps 2 and 3 of the
// single-spin-flip trial, for 32 sites at once).  O, S, U, D are the aligned,
// shifted, upper and lower neighbour words.  Returns the new word; with
// kObs it also adds the energy and magnetisation changes of the flips.
template <bool kObs>
__device__ __forceinline__ uint32_t update_word(uint32_t W, uint32_t O, uint32_t S, uint32_t U,
                                                uint32_t D, uint32_t g, uint32_t h, Key key,
                                                uint32_t lid, const Accept& acc, int& dE,
                                                int& dM, unsigned long long& nblk) {
    // anti-aligned bonds a_k; A = a0 + a1 + a2 + a3 per lane and u = 4 - 2A.
    const uint32_t a0 = W ^ O, a1 = W ^ S, a2 = W ^ U, a3 = W ^ D;
    const uint32_t sm = bop3<T_XOR3>(a0, a1, a2);  // low bit of a0 + a1 + a2
    const uint32_t cy = bop3<T_MAJ>(a0, a1, a2);   // its carry
    const uint32_t ge2 = bop3<T_OR_AND>(cy, sm, a3);    // A >= 2: dE <= 0, flip
    uint32_t m4 = bop3<T_NOR3>(sm, cy, a3);             // A == 0: u = 4, dE = 8
    uint32_t m2 = bop3<T_XOR_ANDN>(sm, a3, cy);         // A == 1: u = 2, dE = 4
    uint32_t flip = ge2;
    if (acc.always2) {
        flip = bop3<T_OR3>(flip, m2, 0u);
        m2 = 0;
    }
    if (acc.always4) {
        flip = bop3<T_OR3>(flip, m4, 0u);
        m4 = 0;
    }
    const uint32_t m24 = bop3<T_OR3>(m2, m4, 0u);
    uint32_t und = m24;  // lanes whose r < T is still undecided
    uint32_t yes = 0;
    for (uint32_t b = 0; b < 8u && und; ++b) {
        U4 out = philox4x32_10({g, lid, h, kTagPlane | (b << 8)}, key);
        ++nblk;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const uint32_t sh = 31u - (4u * b + (uint32_t)kk);
            const bool t2 = (acc.T2 >> sh) & 1u, t4 = (acc.T4 >> sh) & 1u;
            const uint32_t tm = t2 ? (t4 ? m24 : m2) : (t4 ? m4 : 0u);  // T bit per lane
            const uint32_t P = u4_get(out, kk);                          // r bit per lane
            yes = bop3<T_OR3>(yes, bop3<T_AND_ANDN>(und, tm, P), 0u);    // r bit 0 < T bit 1
            und = bop3<T_AND_XNOR>(und, P, tm);                          // equal bits: undecided
        }
    }
    flip = bop3<T_OR3>(flip, yes, 0u);  // lanes still undecided have r == T: rejected
    if (kObs) {
        // dM = sum over flips of -2 s_old = 2 (#flipped down - #flipped up)
        const int nf = __popc(flip);
        dM += 2 * (2 * __popc(bop3<T_AND>(flip, W, 0u)) - nf);
        // dE = sum over flips of 2u = 8 - 4A;  A = sm + a3 + 2 cy
        dE += 8 * nf - 4 * (__popc(bop3<T_AND>(flip, sm, 0u)) + __popc(bop3<T_AND>(flip, a3, 0u)) +
                            2 * __popc(bop3<T_AND>(flip, cy, 0u)));
    }
    return W ^ flip;
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

// Adds a per-lane count into a device total (one atomic per wave).
__device__ __forceinline__ void add_count(unsigned long long v, unsigned long long* out) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0 && v)
        atomicAdd(out, v);
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
        P[row + w] = update_word<true>(W, O, S, U, D, (uint32_t)(row + w), h, key, lid, acc, dE, dM,
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
// dedicated update block per spin group.  Per half-sweep a workgroup first
// updates its interior rows, which depend only on its own tile; the waves
// holding the first and last row then wait until the neighbouring tile has
// published the facing row of the other colour from the previous half-sweep
// (a per-tile counter released at agent scope), read that row from the
// neighbour's halo slot, update, and publish their own row.  No grid-wide
// barrier is used.  Waits are bounded: on time-out the device error word is
// set and the kernel runs to completion.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void wait_counter(const uint32_t* flag, uint32_t target,
                                             uint32_t limit, uint32_t* err) {
    uint32_t spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > limit) {
            atomicOr(err, 1u);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

__global__ void __launch_bounds__(1024) k_sweep_bit1_tiles(
    uint32_t* planes, int L, int rows, int64_t n, uint32_t t0, Key key, uint32_t lid, Accept acc,
    long long* dEtr, long long* dMtr, uint32_t* flags, uint32_t* halo, uint32_t* err,
    unsigned long long* nblk_out, uint32_t spin_limit) {
    extern __shared__ uint32_t tile[];  // [2][rows + 2][nw]
    __shared__ long long red[2][16];
    const int nw = L >> 6;
    const int64_t plane = (int64_t)L * nw;
    const int ntiles = gridDim.x;
    const int nwaves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous band of tiles so most halo traffic stays in one L2.
    int me = blockIdx.x;
    if ((ntiles & 7) == 0)
        me = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
    const int up = (me == 0) ? ntiles - 1 : me - 1;
    const int down = (me + 1 == ntiles) ? 0 : me + 1;
    const int y0 = me * rows;
    const int tr = rows + 2;
    const uint32_t fstride = 32;  // 128 B between counters
    const int64_t hslot = (int64_t)nw;  // one row
    // halo[tile][colour][0 = first row, 1 = last row][nw]
    auto halo_row = [&](int t, int col, int which) -> uint32_t* {
        return halo + (((int64_t)t * 2 + col) * 2 + which) * hslot;
    };

    for (int i = threadIdx.x; i < 2 * tr * nw; i += blockDim.x) {
        const int col = i / (tr * nw);
        const int rem = i - col * tr * nw;
        const int r = rem / nw - 1, w = rem % nw;
        int y = y0 + r;
        y = (y < 0) ? y + L : (y >= L ? y - L : y);
        tile[i] = planes[(int64_t)col * plane + (int64_t)y * nw + w];
    }
    __syncthreads();

    const int nchunks = (nw + 63) >> 6;
    const int nitems = rows * nchunks;
    long long sE = 0, sM = 0;
    unsigned long long nblk = 0;
    for (int64_t hs = 0; hs < 2 * n; ++hs) {
        const int c = (int)(hs & 1), o = c ^ 1;
        const uint32_t h = 2u * t0 + (uint32_t)hs;
        uint32_t* Tc = tile + c * tr * nw;
        const uint32_t* To = tile + o * tr * nw;
        int dE = 0, dM = 0;
        bool published = false;
        for (int it = wave; it < nitems; it += nwaves) {
            // interior rows first, then the first row, then the last row
            int r;
            const int chunk = it % nchunks;
            const int k = it / nchunks;
            if (rows <= 2)
                r = k;
            else
                r = (k < rows - 2) ? k + 1 : (k == rows - 2 ? 0 : rows - 1);
            const bool first = (r == 0), last = (r == rows - 1);
            if (hs > 0 && first)
                wait_counter(flags + (int64_t)up * fstride, (uint32_t)hs, spin_limit, err);
            if (hs > 0 && last)
                wait_counter(flags + (int64_t)down * fstride, (uint32_t)hs, spin_limit, err);
            const int w = chunk * 64 + lane;
            if (w < nw) {
                const int y = y0 + r;
                const int wm = (w == 0) ? nw - 1 : w - 1;
                const int wp = (w + 1 == nw) ? 0 : w + 1;
                const uint32_t* Orow = To + (r + 1) * nw;
                const uint32_t W = Tc[(r + 1) * nw + w];
                const uint32_t O = Orow[w];
                const uint32_t S = side_word(O, Orow[wm], Orow[wp], (y + c) & 1);
                uint32_t U, D;
                if (hs > 0 && first)
                    U = __builtin_nontemporal_load(halo_row(up, o, 1) + w);
                else
                    U = To[r * nw + w];
                if (hs > 0 && last)
                    D = __builtin_nontemporal_load(halo_row(down, o, 0) + w);
                else
                    D = To[(r + 2) * nw + w];
                const uint32_t nwd = update_word<true>(W, O, S, U, D, (uint32_t)((int64_t)y * nw + w),
                                                 h, key, lid, acc, dE, dM, nblk);
                Tc[(r + 1) * nw + w] = nwd;
                if (first)
                    halo_row(me, c, 0)[w] = nwd;
                if (last)
                    halo_row(me, c, 1)[w] = nwd;
            }
            if (first || last)
                published = true;
        }
        if (published)
            __threadfence();  // halo rows visible at agent scope before the counter
        sE += dE;
        sM += dM;
        if (hs & 1) {
            long long e = wave_sum_i64(sE), m = wave_sum_i64(sM);
            if (lane == 0) {
                red[0][wave] = e;
                red[1][wave] = m;
            }
            sE = 0;
            sM = 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_store(flags + (int64_t)me * fstride, (uint32_t)(hs + 1), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
            if ((hs & 1) && (dEtr || dMtr)) {
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
    }
    add_count(nblk, nblk_out);
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * rows * nw; i += blockDim.x) {
        const int col = i / (rows * nw);
        const int rem = i - col * rows * nw;
        const int r = rem / nw, w = rem % nw;
        planes[(int64_t)col * plane + (int64_t)(y0 + r) * nw + w] = tile[(col * tr + r + 1) * nw + w];
    }
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

bool plan_bit1_tiles(int L, int device_cus, Bit1TilePlan* plan) {
    const int nw = L >> 6;
    if (nw < 1)
        return false;
    int maxt = device_cus < WsLayout::kMaxTiles ? device_cus : WsLayout::kMaxTiles;
    if (maxt > L)
        maxt = L;
    // Largest tile count that divides L and fits 64 KiB of LDS; a multiple of
    // 8 (one band of tiles per XCD) is preferred when it is at least half
    // as large.
    int best = 0, best8 = 0;
    for (int t = maxt; t >= 2; --t) {
        if (L % t)
            continue;
        const size_t lds = (size_t)2 * (L / t + 2) * nw * sizeof(uint32_t);
        if (lds > 64 * 1024)
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
    plan->lds = (size_t)2 * (plan->rows + 2) * nw * sizeof(uint32_t);
    return true;
}

hipError_t launch_sweep_bit1_tiles(uint32_t* planes, int L, const Bit1TilePlan& plan, int64_t n,
                                   uint32_t t0, Key key, uint32_t lid, Accept acc, long long* dE,
                                   long long* dM, unsigned char* ws, uint32_t spin_limit,
                                   hipStream_t st) {
    uint32_t* flags = reinterpret_cast<uint32_t*>(ws + WsLayout::kFlags);
    uint32_t* halo = reinterpret_cast<uint32_t*>(ws + WsLayout::halo_offset());
    uint32_t* err = reinterpret_cast<uint32_t*>(ws + WsLayout::kErr);
    unsigned long long* nblk = reinterpret_cast<unsigned long long*>(ws + WsLayout::kRngBlocks);
    hipError_t e = launch_fill_i64(reinterpret_cast<long long*>(flags),
                                   (int64_t)plan.ntiles * WsLayout::kFlagStride / 8, 0, st);
    if (e != hipSuccess)
        return e;
    int rows = plan.rows;
    void* args[] = {&planes, (void*)&L, &rows, &n, &t0, &key, &lid, &acc, &dE, &dM,
                    &flags, &halo, &err, &nblk, &spin_limit};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_sweep_bit1_tiles),
                                      dim3(plan.ntiles), dim3(1024), args, plan.lds, st);
}

}  // namespace ising
