// INT8 layout kernels: one byte per spin, row-major, draws in per-site mode.
//
// A half-sweep updates every site of one colour (sublattice A or B of the
// paper's bipartition, Fig. 2a-b); sites of one colour are never neighbours,
// so all of them are independent and updated in parallel.  Each thread owns
// four consecutive compact indices q = 4g..4g+3 of the colour, which share
// one Philox4x32-10 block (counter (g, lattice_id, 2t+c, 0)).
#include "handoff.hpp"
#include "kernels.hpp"
#include "quad.hpp"

namespace ising {

namespace {

__device__ __forceinline__ bool accept_u(int u, uint32_t r, const Accept& a) {
    if (u <= 0)
        return true;
    if (u == 2)
        return a.always2 || r < a.T2;
    return a.always4 || r < a.T4;
}

__device__ __forceinline__ bool needs_draw(int u, const Accept& a) {
    return (u == 2 && !a.always2) || (u == 4 && !a.always4);
}

// Site of colour c with compact index q on an L x L lattice (L even).
__device__ __forceinline__ void site_of(int64_t q, int halfL, int c, int& x, int& y) {
    y = (int)(q / halfL);
    int i = (int)(q - (int64_t)y * halfL);
    x = 2 * i + ((y + c) & 1);
}

__global__ void k_init_int8(int8_t* s, int64_t N, int start, Key key, uint32_t lid) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * g >= N)
        return;
    uint32_t word;
    if (start == 0) {
        word = 0x01010101u;
    } else {
        U4 o = philox4x32_10({(uint32_t)g, lid, 0u, kTagInit}, key);
        uint32_t b0 = (o.x >> 31) ? 0xFFu : 0x01u;
        uint32_t b1 = (o.y >> 31) ? 0xFFu : 0x01u;
        uint32_t b2 = (o.z >> 31) ? 0xFFu : 0x01u;
        uint32_t b3 = (o.w >> 31) ? 0xFFu : 0x01u;
        word = b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
    }
    reinterpret_cast<uint32_t*>(s)[g] = word;  // N % 4 == 0 for even L
}

// Update the four sites of group g (colour c) of lattice `s` (global or
// LDS); returns the energy and magnetisation change of the accepted flips.
template <typename Ptr>
__device__ __forceinline__ void update_group(Ptr s, int L, int c, int64_t g, uint32_t h,
                                             const RoundKeys& rk, uint32_t lid, const Accept& acc,
                                             int& dE, int& dM, unsigned long long& nblk) {
    const int halfL = L >> 1;
    const int64_t nhalf = (int64_t)L * halfL;  // sites per colour
    int u[4];
    int64_t idx[4];
    bool live[4];
    bool draw = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        // when L % 4 == 2 the last group of a colour holds two sites only
        live[j] = 4 * g + j < nhalf;
        if (!live[j]) {
            u[j] = 0;
            idx[j] = 0;
            continue;
        }
        int x, y;
        site_of(4 * g + j, halfL, c, x, y);
        int xp = (x + 1 == L) ? 0 : x + 1;
        int xm = (x == 0) ? L - 1 : x - 1;
        int yp = (y + 1 == L) ? 0 : y + 1;
        int ym = (y == 0) ? L - 1 : y - 1;
        int64_t row = (int64_t)y * L;
        int64_t n = row + x;
        int hsum = s[row + xp] + s[row + xm] + s[(int64_t)yp * L + x] + s[(int64_t)ym * L + x];
        idx[j] = n;
        u[j] = s[n] * hsum;
        draw |= needs_draw(u[j], acc);
    }
    U4 r = {0u, 0u, 0u, 0u};
    if (draw) {
        r = philox4x32_10({(uint32_t)g, lid, h, kTagSite}, rk);
        ++nblk;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (live[j] && accept_u(u[j], u4_get(r, j), acc)) {
            int8_t old = s[idx[j]];
            s[idx[j]] = (int8_t)-old;
            dE += 2 * u[j];
            dM -= 2 * old;
        }
    }
}

// Adds a per-lane count into the device total: a workgroup reduction, then
// one atomic into slot blockIdx % kRngSlots so that atomics to one address
// stay few.  Must be reached by every thread of the workgroup.
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

// Whole-lattice-in-LDS kernel: one workgroup runs all n sweeps of a small
// lattice and writes E and M after every sweep.
__global__ void __launch_bounds__(1024) k_sweep_int8_resident(int8_t* s_glob, int L, int64_t n,
                                                              uint32_t t0, Key key, uint32_t lid,
                                                              Accept acc, int64_t* Etr,
                                                              int64_t* Mtr,
                                                              unsigned long long* nblk_out) {
    extern __shared__ __align__(16) int8_t sh[];  // 8-byte span loads
    __shared__ long long red[2][16];
    const int N = L * L;
    const int tid = threadIdx.x;
    const int nwaves = (blockDim.x + 63) >> 6;
    const int wave = tid >> 6, lane = tid & 63;
    for (int i = tid; i < N; i += blockDim.x)
        sh[i] = s_glob[i];
    __syncthreads();
    // starting E and M
    long long e = 0, m = 0;
    for (int i = tid; i < N; i += blockDim.x) {
        int x = i % L, y = i / L;
        int right = sh[y * L + ((x + 1 == L) ? 0 : x + 1)];
        int down = sh[((y + 1 == L) ? 0 : y + 1) * L + x];
        e -= sh[i] * (right + down);
        m += sh[i];
    }
    e = wave_sum_i64(e);
    m = wave_sum_i64(m);
    if (lane == 0) {
        red[0][wave] = e;
        red[1][wave] = m;
    }
    __syncthreads();
    long long E = 0, M = 0;
    for (int w = 0; w < nwaves; ++w) {
        E += red[0][w];
        M += red[1][w];
    }
    __syncthreads();
    const int64_t groups = ((N >> 1) + 3) >> 2;  // N/2 sites per colour, 4 per group
    const RoundKeys rk = round_keys(key);
    // L % 8 == 0: the byte-parallel span update (quad.hpp); span gi = y L/8 + k
    // is Philox group gi, and a thread's spans advance without divisions
    const bool span = (L & 7) == 0;
    const QuadAccept qa = quad_accept(acc.T2, acc.T4, acc.always2 != 0, acc.always4 != 0);
    const int gpr = L >> 3;
    const int y0 = span ? tid / gpr : 0, k0 = span ? tid - y0 * gpr : 0;
    const int dy = span ? (int)blockDim.x / gpr : 0, dk = span ? (int)blockDim.x - dy * gpr : 0;
    unsigned long long nblk = 0;
    for (int64_t j = 0; j < n; ++j) {
        int dE = 0, dM = 0;
        for (int c = 0; c < 2; ++c) {
            uint32_t h = 2u * (t0 + (uint32_t)j) + (uint32_t)c;
            if (span) {
                QuadCounts cnt;
                int y = y0, k = k0;
                for (int gi = tid; gi < (int)groups; gi += blockDim.x) {
                    update_quad(sh, L, N, y, y * L, 8 * k, c, (uint32_t)gi, h, rk, lid, qa, cnt,
                                nblk);
                    k += dk;
                    y += dy;
                    if (k >= gpr) {
                        k -= gpr;
                        ++y;
                    }
                }
                dE += 8 * (int)cnt.nflip - 2 * (int)cnt.sum_a2;
                dM += 2 * (2 * (int)cnt.ndown - (int)cnt.nflip);
            } else {
                for (int64_t g = tid; g < groups; g += blockDim.x)
                    update_group(sh, L, c, g, h, rk, lid, acc, dE, dM, nblk);
            }
            __syncthreads();
        }
        dE = wave_sum_i32(dE);
        dM = wave_sum_i32(dM);
        if (lane == 0) {
            red[0][wave] = dE;
            red[1][wave] = dM;
        }
        __syncthreads();
        for (int w = 0; w < nwaves; ++w) {
            E += red[0][w];
            M += red[1][w];
        }
        if (tid == 0) {
            if (Etr)
                Etr[j] = E;
            if (Mtr)
                Mtr[j] = M;
        }
        __syncthreads();
    }
    for (int i = tid; i < N; i += blockDim.x)
        s_glob[i] = sh[i];
    add_count(nblk, nblk_out);
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

// Half-sweep of colour c from global memory for L % 8 == 0 and L^2 < 2^31:
// the byte-parallel update of the four colour-c sites of an 8-byte span
// (quad.hpp), in a grid-stride loop over the spans so that the Philox round
// keys are set up once per thread.  Span gi = y L/8 + k (columns 8k..8k+7 of
// row y) is Philox group gi; its row and column advance incrementally.
__global__ void __launch_bounds__(256) k_halfsweep_int8_quad(int8_t* s, int L, int c, uint32_t h,
                                                             Key key, uint32_t lid, Accept acc,
                                                             long long* dEo, long long* dMo,
                                                             unsigned long long* nblk_out) {
    const int gpr = L >> 3, N = L * L;
    const uint32_t ngroups = (uint32_t)L * (uint32_t)gpr;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
    QuadCounts cnt;
    unsigned long long nblk = 0;
    if (gi < ngroups) {
        const RoundKeys rk = round_keys(key);
        const QuadAccept qa = quad_accept(acc.T2, acc.T4, acc.always2 != 0, acc.always4 != 0);
        int y = (int)(gi / (uint32_t)gpr), k = (int)(gi - (uint32_t)y * (uint32_t)gpr);
        const int dy = (int)(stride / (uint32_t)gpr), dk = (int)(stride - (uint32_t)dy * (uint32_t)gpr);
        int row = y * L;
        for (; gi < ngroups; gi += stride) {
            update_quad(s, L, N, y, row, 8 * k, c, gi, h, rk, lid, qa, cnt, nblk);
            k += dk;
            y += dy;
            row += dy * L;
            if (k >= gpr) {
                k -= gpr;
                ++y;
                row += L;
            }
        }
    }
    add_count(nblk, nblk_out);
    if (dEo || dMo) {
        const long long dE = 8ll * cnt.nflip - 2ll * cnt.sum_a2;
        const long long dM = 2ll * (2ll * cnt.ndown - (long long)cnt.nflip);
        block_add_i64(dE, dM, dEo, dMo);
    }
}

// ---------------------------------------------------------------------------
// Persistent tile-resident INT8 sweep (L % 8 == 0).
//
// Each workgroup owns `rows` consecutive full-width rows as bytes in LDS for
// the whole call, with one halo row above and one below: the facing rows of
// the neighbouring tiles.  A half-sweep updates the colour-c sites of the
// tile span by span (four sites of an 8-byte span share one Philox block,
// quad.hpp), the first and last rows first; those rows publish their spans'
// new colour-c bytes (four bytes, one tagged slot per span) for the
// neighbouring tiles.  After its spans, every thread takes part in receiving
// the neighbours' facing rows of this half-sweep into the halo rows, merging
// their colour-c bytes; then one workgroup barrier.  No reader of this
// half-sweep is disturbed by that merge: the spans being updated read only
// the other colour's bytes of the halo rows, and the merge rewrites those
// with the values they already hold.  Slots come in two sets, by the parity
// of the half-sweep: a slot is rewritten two half-sweeps later, only after
// its writer has received the neighbour's next row, which the neighbour
// publishes only after it has received the slot.
// ---------------------------------------------------------------------------

// halo[tile][parity of hs][first, last row][L/8 spans] of (tag << 32 | bytes)
__device__ __forceinline__ unsigned long long* quad_slots(unsigned long long* halo, int gpr, int t,
                                                          int par, int which) {
    return halo + (((int64_t)t * 2 + par) * 2 + which) * gpr;
}

// Row order within a half-sweep: the first and last rows come first.
__device__ __forceinline__ int int8_row_of(int k, int rows) {
    return (rows <= 2 || k == 0) ? k : (k == 1 ? rows - 1 : k - 1);
}

template <bool kObs>
__global__ void __launch_bounds__(1024) k_sweep_int8_tiles(
    int8_t* s, int L, int rows, int64_t n, uint32_t t0, Key key, uint32_t lid, Accept acc,
    long long* dEtr, long long* dMtr, unsigned long long* halo, uint32_t* err,
    unsigned long long* nblk_out, uint32_t spin_limit) {
    extern __shared__ uint2 tile8[];  // [rows + 2][L] bytes, 8-byte aligned
    int8_t* tile = reinterpret_cast<int8_t*>(tile8);
    __shared__ long long red[2][16];
    const int gpr = L >> 3;
    const int ntiles = gridDim.x;
    // workgroups are dealt to the 8 XCDs in turn: a contiguous band of
    // tiles per XCD keeps most hand-offs within one XCD
    int me = blockIdx.x;
    if ((ntiles & 7) == 0)
        me = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
    const int up = (me == 0) ? ntiles - 1 : me - 1;
    const int down = (me + 1 == ntiles) ? 0 : me + 1;
    const int y0 = me * rows;
    const int yu = (y0 == 0) ? L - 1 : y0 - 1;          // the row above the tile
    const int yd = (y0 + rows == L) ? 0 : y0 + rows;     // the row below it
    const int nwaves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < (rows + 2) * gpr; i += blockDim.x) {
        const int r = i / gpr - 1, k = i - (r + 1) * gpr;
        const int y = (r < 0) ? yu : (r == rows ? yd : y0 + r);
        tile8[i] = *reinterpret_cast<const uint2*>(s + (int64_t)y * L + 8 * k);
    }
    __syncthreads();
    const RoundKeys rk = round_keys(key);
    const QuadAccept qa = quad_accept(acc.T2, acc.T4, acc.always2 != 0, acc.always4 != 0);
    const int N = (rows + 2) * L;  // the tile's rows: update_quad never wraps inside it
    const int tasks = rows * gpr;
    const int k_first = (int)threadIdx.x / gpr, xk_first = (int)threadIdx.x - k_first * gpr;
    const int dk = (int)blockDim.x / gpr, dxk = (int)blockDim.x - dk * gpr;
    long long sE = 0, sM = 0;
    unsigned long long nblk = 0;
    for (int64_t hs = 0; hs < 2 * n; ++hs) {
        const int c = (int)(hs & 1), par = (int)(hs & 1);
        const uint32_t h = 2u * t0 + (uint32_t)hs, tag = (uint32_t)hs + 1u;
        QuadCounts cnt;
        // task = k gpr + xk (k-th row in edge-first order, span xk), advanced
        // incrementally: no division per span
        int k = k_first, xk = xk_first;
        for (int task = threadIdx.x; task < tasks; task += blockDim.x) {
            const int r = int8_row_of(k, rows);
            const int y = y0 + r;
            const uint32_t g = (uint32_t)(y * L + 8 * xk) >> 3;  // L^2 < 2^31
            const uint32_t nb = update_quad(tile, L, N, y, (r + 1) * L, 8 * xk, c, g, h, rk, lid,
                                            qa, cnt, nblk);
            if (r == 0)
                publish_slot(quad_slots(halo, gpr, me, par, 0) + xk, tag, nb);
            if (r == rows - 1)
                publish_slot(quad_slots(halo, gpr, me, par, 1) + xk, tag, nb);
            xk += dxk;
            k += dk;
            if (xk >= gpr) {
                xk -= gpr;
                ++k;
            }
        }
        // the neighbours' facing rows of this half-sweep: merge their new
        // colour-c bytes (positions p + 2j of each span, p the row's parity)
        for (int i = threadIdx.x; i < 2 * gpr; i += blockDim.x) {
            const int which = i >= gpr, xk = i - which * gpr;
            const unsigned long long* slot = which ? quad_slots(halo, gpr, down, par, 0) + xk
                                                   : quad_slots(halo, gpr, up, par, 1) + xk;
            const uint32_t v = wait_slot(slot, tag, spin_limit, err);
            const int pn = ((which ? yd : yu) + c) & 1;
            uint2* dst = tile8 + (which ? (rows + 1) : 0) * gpr + xk;
            const uint2 old = *dst;
            uint2 nv;
            nv.x = __builtin_amdgcn_perm(v, old.x, pn ? 0x05020400u : 0x03050104u);
            nv.y = __builtin_amdgcn_perm(v, old.y, pn ? 0x07020600u : 0x03070106u);
            *dst = nv;
        }
        __syncthreads();
        if (kObs) {
            sE += 8ll * cnt.nflip - 2ll * cnt.sum_a2;
            sM += 2ll * (2ll * cnt.ndown - (long long)cnt.nflip);
            if (hs & 1) {
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
                    const int64_t j = hs >> 1;
                    if (dEtr && E)
                        atomicAdd(reinterpret_cast<unsigned long long*>(dEtr + j),
                                  (unsigned long long)E);
                    if (dMtr && M)
                        atomicAdd(reinterpret_cast<unsigned long long*>(dMtr + j),
                                  (unsigned long long)M);
                }
                sE = sM = 0;
            }
        }
    }
    add_count(nblk, nblk_out);
    for (int i = threadIdx.x; i < rows * gpr; i += blockDim.x)
        *reinterpret_cast<uint2*>(s + (int64_t)(y0 + i / gpr) * L + 8 * (i % gpr)) = tile8[gpr + i];
}

__global__ void __launch_bounds__(256) k_halfsweep_int8(int8_t* s, int L, int c, uint32_t h,
                                                        Key key, uint32_t lid, Accept acc,
                                                        long long* dEo, long long* dMo,
                                                        unsigned long long* nblk_out) {
    const int64_t groups = ((((int64_t)L * L) >> 1) + 3) >> 2;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int dE = 0, dM = 0;
    unsigned long long nblk = 0;
    if (g < groups)
        update_group(s, L, c, g, h, round_keys(key), lid, acc, dE, dM, nblk);
    add_count(nblk, nblk_out);
    if (dEo || dMo)
        block_add_i64(dE, dM, dEo, dMo);
}

__global__ void __launch_bounds__(256) k_measure_int8(const int8_t* s, int L, long long* acc) {
    const int64_t N = (int64_t)L * L;
    long long e = 0, m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        int x = (int)(i % L), y = (int)(i / L);
        int right = s[(int64_t)y * L + ((x + 1 == L) ? 0 : x + 1)];
        int down = s[(int64_t)((y + 1 == L) ? 0 : y + 1) * L + x];
        e -= s[i] * (right + down);
        m += s[i];
    }
    block_add_i64(e, m, acc, acc + 1);
}

__global__ void k_convert_int8(const int8_t* in, int8_t* out, int64_t N) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N)
        out[i] = in[i] < 0 ? (int8_t)-1 : (int8_t)1;
}

__global__ void k_fill_i64(long long* p, int64_t n, long long v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

__global__ void k_copy_u32(const uint32_t* src, uint32_t* dst) {
    if (threadIdx.x == 0)
        *dst = *src;
}

// Single-workgroup inclusive scan: out[j] = base + sum_{i<=j} d[i].
__global__ void __launch_bounds__(1024) k_prefix_i64(long long* d, int64_t n,
                                                     const long long* base) {
    __shared__ long long part[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (n + blockDim.x - 1) / blockDim.x;
    const int64_t lo = tid * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    long long sum = 0;
    for (int64_t i = lo; i < hi; ++i)
        sum += d[i];
    part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        long long run = *base;
        for (int i = 0; i < (int)blockDim.x; ++i) {
            long long v = part[i];
            part[i] = run;
            run += v;
        }
    }
    __syncthreads();
    long long run = part[tid];
    for (int64_t i = lo; i < hi; ++i) {
        run += d[i];
        d[i] = run;
    }
}

__global__ void k_finish_measure(const long long* acc, long long aE, long long bE, long long aM,
                                 long long bM, long long* E_out, long long* M_out,
                                 long long* E_copy, long long* M_copy) {
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    long long E = aE * acc[0] + bE;
    long long M = aM * acc[1] + bM;
    if (E_out)
        *E_out = E;
    if (M_out)
        *M_out = M;
    if (E_copy)
        *E_copy = E;
    if (M_copy)
        *M_copy = M;
}

inline unsigned blocks_for(int64_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

hipError_t launch_init_int8(int8_t* s, int L, int start, Key key, uint32_t lid,
                            hipStream_t st) {
    int64_t N = (int64_t)L * L;
    hipLaunchKernelGGL(k_init_int8, dim3(blocks_for(N / 4, 256)), dim3(256), 0, st, s, N, start,
                       key, lid);
    return hipGetLastError();
}

bool int8_resident_fits(int L) { return L <= 128; }

hipError_t launch_sweep_int8_resident(int8_t* s, int L, int64_t n, uint32_t t0, Key key,
                                      uint32_t lid, Accept acc, int64_t* Etr, int64_t* Mtr,
                                      unsigned long long* nblk, hipStream_t st) {
    int64_t groups = ((((int64_t)L * L) >> 1) + 3) >> 2;
    int threads = (int)((groups + 63) / 64 * 64);
    if (threads > 1024)
        threads = 1024;
    if (threads < 64)
        threads = 64;
    size_t lds = (size_t)L * L;
    hipLaunchKernelGGL(k_sweep_int8_resident, dim3(1), dim3(threads), lds, st, s, L, n, t0, key,
                       lid, acc, Etr, Mtr, nblk);
    return hipGetLastError();
}

hipError_t launch_halfsweep_int8(int8_t* s, int L, int c, uint32_t h, Key key, uint32_t lid,
                                 Accept acc, long long* dE, long long* dM,
                                 unsigned long long* nblk, hipStream_t st) {
    int64_t groups = ((((int64_t)L * L) >> 1) + 3) >> 2;
    if ((L & 7) == 0 && (int64_t)L * L < (int64_t)1 << 31) {
        // one 8-byte span per group; at most 4096 workgroups (a thread takes
        // up to 128 spans at L = 32768)
        unsigned blocks = blocks_for(groups, 256);
        if (blocks > 4096)
            blocks = 4096;
        hipLaunchKernelGGL(k_halfsweep_int8_quad, dim3(blocks), dim3(256), 0, st, s, L, c, h, key,
                           lid, acc, dE, dM, nblk);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_halfsweep_int8, dim3(blocks_for(groups, 256)), dim3(256), 0, st, s, L, c,
                       h, key, lid, acc, dE, dM, nblk);
    return hipGetLastError();
}

bool plan_int8_tiles(int L, int device_cus, int max_lds, Int8TilePlan* plan) {
    if ((L & 7) != 0 || L > kInt8TilesMaxL || device_cus < 1)
        return false;
    // the tallest tile (one per CU, at most 16 rows) that still gives every
    // CU a tile and fits the LDS a workgroup may use
    int rows = 0;
    for (int r = 16; r >= 1 && !rows; --r) {
        const int t = L / r;
        if (L % r || t > WsLayout::kMaxTiles || t < 2)
            continue;
        if ((int64_t)(r + 2) * L > (int64_t)max_lds)
            continue;
        if (t >= device_cus || r == 1)
            rows = r;
    }
    if (!rows)
        return false;
    const int ntiles = L / rows;
    // tiles sharing a CU split its 16 waves
    const int per_cu = (ntiles + device_cus - 1) / device_cus;
    int waves = 16 / (per_cu > 0 ? per_cu : 1);
    const int spans = rows * (L >> 3);
    const int need = (spans + 63) / 64;
    if (waves > need)
        waves = need;
    if (waves < 1)
        waves = 1;
    plan->ntiles = ntiles;
    plan->rows = rows;
    plan->threads = 64 * waves;
    plan->lds = (size_t)(rows + 2) * (size_t)L;
    return true;
}

size_t int8_halo_bytes(int L, int ntiles) {
    return (size_t)ntiles * 2 * 2 * (size_t)(L >> 3) * 8;
}

int int8_tiles_resident(const Int8TilePlan& plan, bool obs) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const void* k = obs ? reinterpret_cast<const void*>(k_sweep_int8_tiles<true>)
                        : reinterpret_cast<const void*>(k_sweep_int8_tiles<false>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, plan.threads, plan.lds) !=
        hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_sweep_int8_tiles(int8_t* s, int L, const Int8TilePlan& plan, int64_t n,
                                   uint32_t t0, Key key, uint32_t lid, Accept acc, long long* dE,
                                   long long* dM, unsigned char* ws, uint32_t spin_limit,
                                   hipStream_t st) {
    unsigned long long* halo = reinterpret_cast<unsigned long long*>(ws + WsLayout::kHalo);
    uint32_t* err = reinterpret_cast<uint32_t*>(ws + WsLayout::kErr);
    unsigned long long* nblk = reinterpret_cast<unsigned long long*>(ws + WsLayout::kRngBlocks);
    // zero every tag so that nothing left by an earlier call can match
    hipError_t e = launch_fill_i64(reinterpret_cast<long long*>(halo),
                                   (int64_t)int8_halo_bytes(L, plan.ntiles) / 8, 0, st);
    if (e != hipSuccess)
        return e;
    int rows = plan.rows;
    void* args[] = {&s, (void*)&L, &rows, &n, &t0, &key, &lid, &acc, &dE, &dM,
                    &halo, &err, &nblk, &spin_limit};
    const void* k = (dE || dM) ? reinterpret_cast<const void*>(k_sweep_int8_tiles<true>)
                               : reinterpret_cast<const void*>(k_sweep_int8_tiles<false>);
    return hipLaunchCooperativeKernel(k, dim3(plan.ntiles), dim3(plan.threads), args, plan.lds,
                                      st);
}

hipError_t launch_measure_int8(const int8_t* s, int L, long long* acc, hipStream_t st) {
    int64_t N = (int64_t)L * L;
    unsigned blocks = blocks_for(N, 256);
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(k_measure_int8, dim3(blocks), dim3(256), 0, st, s, L, acc);
    return hipGetLastError();
}

hipError_t launch_convert_int8(const int8_t* in, int8_t* out, int64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_convert_int8, dim3(blocks_for(N, 256)), dim3(256), 0, st, in, out, N);
    return hipGetLastError();
}

hipError_t launch_fill_i64(long long* p, int64_t n, long long v, hipStream_t st) {
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_i64, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy_u32(const uint32_t* src, uint32_t* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(64), 0, st, src, dst);
    return hipGetLastError();
}

hipError_t launch_prefix_i64(long long* d, int64_t n, const long long* base, hipStream_t st) {
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_prefix_i64, dim3(1), dim3(1024), 0, st, d, n, base);
    return hipGetLastError();
}

hipError_t launch_finish_measure(const long long* acc, long long aE, long long bE, long long aM,
                                 long long bM, long long* E_out, long long* M_out,
                                 long long* E_copy, long long* M_copy, hipStream_t st) {
    hipLaunchKernelGGL(k_finish_measure, dim3(1), dim3(64), 0, st, acc, aE, bE, aM, bM, E_out,
                       M_out, E_copy, M_copy);
    return hipGetLastError();
}

}  // namespace ising
