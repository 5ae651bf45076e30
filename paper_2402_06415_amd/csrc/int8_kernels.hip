// INT8 layout kernels: one byte per spin, row-major, draws in per-site mode.
//
// A half-sweep updates every site of one colour (sublattice A or B of the
// paper's bipartition, Fig. 2a-b); sites of one colour are never neighbours,
// so all of them are independent and updated in parallel.  Each thread owns
// four consecutive compact indices q = 4g..4g+3 of the colour, which share
// one Philox4x32-10 block (counter (g, lattice_id, 2t+c, 0)).
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
