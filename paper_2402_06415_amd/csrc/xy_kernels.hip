// Metropolis Monte Carlo of the 2D classical XY model in double precision.
//
// Up to L = 80 one workgroup owns one lattice: its L*L angles, with the
// cosine and sine of each (24 bytes per site), sit in LDS for all n sweeps
// of a call.  Within a half-sweep the threads take the sites of one colour
// in turn; a site's trial reads its four neighbours (the other colour) and
// writes its own angle, so the update is in place and race-free.
//
// A lattice on one CU leaves the rest of the GPU idle when lattices are
// fewer than CUs, and above L = 80 it no longer fits one workgroup's LDS.
// Then (L > 32) the lattice is cut into bands of rows, one resident
// workgroup each for the whole call, that hand the edge rows' cosines and
// sines to each other through tagged slots (k_xy_sweep_bands).  Where the
// bands of all lattices cannot be resident together (L > 80 and many
// lattices), the lattices are swept by one launch per half-sweep over many
// workgroups instead: angles, cosines and sines stay in global memory (the
// latter two in the workspace, filled at the start of each call), each
// thread makes one trial, and the energy trace is carried by per-lattice
// sums in the workspace that alternate between two slots from sweep to
// sweep, so that each sweep's total is read only after a kernel boundary.
//
// All forms take the energy change of a trial from the cached cosines and
// sines by the angle-difference identity, cos(a - b) = cos a cos b +
// sin a sin b: one sincos of the proposed angle per trial instead of eight
// cosines, and an accepted angle stores the pair just computed.  The result
// equals the direct sum up to rounding, so a trial can be decided
// differently from the direct form only when the uniform draw lies within a
// few units in the last place of the acceptance probability.  For the
// energy trace H is summed over
// the lattice once per call and then carried from sweep to sweep by adding
// the energy changes of the accepted trials (each wave sums its own, and
// thread 0 adds the per-wave partials in a fixed order behind the next
// half-sweep barrier).  Every floating-point operation is rounded on its
// own (no fused multiply-add), as the trial is defined operation by
// operation.
#include "handoff.hpp"
#include "xy.hpp"

namespace ising {

namespace {

constexpr double kTwoPi = 6.283185307179586;  // nearest double to 2 pi
// dynamic LDS up to which the sweep also keeps cos and sin of every angle
constexpr size_t kXyCacheLds = 156 * 1024;
// most bands of the band-tiled sweep (bounds its hand-off slots), and the
// smallest side it serves
constexpr int kXyBandsMax = 2048;
constexpr int kXyBandsMinL = 34;

struct XyHeader {
    uint32_t magic, count;
    uint64_t t, t0;
    uint32_t ok, err;
};

__device__ __forceinline__ XyHeader* xy_header(unsigned char* ws) {
    return reinterpret_cast<XyHeader*>(ws);
}

__device__ __forceinline__ double unit53(uint32_t hi, uint32_t lo) {
    return (double)((((uint64_t)hi << 32) | lo) >> 11) * 0x1.0p-53;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// H of an L x L lattice (angles `th`, LDS or global), summed into thread 0;
// `red` holds one slot per wave (at most 16).
__device__ __forceinline__ double energy_to0(const double* th, int L, double* red) {
#pragma clang fp contract(off)
    double e = 0.0;
    const int N = L * L;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const int y = n / L, x = n - y * L;
        const double t = th[n];
        e -= cos(t - th[y * L + (x + 1 == L ? 0 : x + 1)]) +
             cos(t - th[(y + 1 == L ? 0 : y + 1) * L + x]);
    }
    e = wave_sum_f64(e);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = e;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
            s += red[w];
    return s;
}

__global__ void k_xy_init(unsigned char* ws, double* theta, int L, int count, int start, Key key,
                          uint32_t lid0) {
    const int j = blockIdx.y;
    const int N = L * L;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        reinterpret_cast<unsigned long long*>(ws + kXyAccepted)[j] = 0;
        if (j == 0) {
            XyHeader* hd = xy_header(ws);
            hd->magic = kXyMagic;
            hd->count = (uint32_t)count;
            hd->t = 0;
            hd->ok = 0;
        }
    }
    if (n >= N)
        return;
    double v = 0.0;
    if (start != 0) {
        const U4 o = philox4x32_10({(uint32_t)n, lid0 + (uint32_t)j, 0u, kTagXyInit}, key);
        v = unit53(o.x, o.y) * kTwoPi;
    }
    theta[(int64_t)j * N + n] = v;
}

__global__ void k_xy_prepare(unsigned char* ws, int count, int64_t n) {
    XyHeader* hd = xy_header(ws);
    uint32_t e = (hd->magic == kXyMagic && hd->count == (uint32_t)count) ? 0u : kXyErrNotInit;
    if (e == 0 && hd->t + (uint64_t)n > (1ull << 31))
        e = kXyErrSweepIndex;
    if (e) {
        hd->err |= e;
        hd->ok = 0;
    } else {
        hd->ok = 1;
        hd->t0 = hd->t;
    }
}

__global__ void k_xy_advance(unsigned char* ws, int64_t n) {
    XyHeader* hd = xy_header(ws);
    if (hd->ok)
        hd->t += (uint64_t)n;
}

__global__ void __launch_bounds__(512) k_xy_sweep(unsigned char* ws, double* theta, int L,
                                                  int count, int64_t n, double beta, Key key,
                                                  uint32_t lid0, double* E_trace) {
#pragma clang fp contract(off)
    extern __shared__ double th[];  // [N] angles, [N] cos, [N] sin
    __shared__ double red[16];
    XyHeader* hd = xy_header(ws);
    if (hd->ok == 0)
        return;
    const int j = blockIdx.x;
    const uint32_t lid = lid0 + (uint32_t)j;
    const int N = L * L, half = L >> 1;
    const uint32_t t0 = (uint32_t)hd->t;
    double* g = theta + (int64_t)j * N;
    double* const cs = th + N;
    double* const sn = th + 2 * N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        th[i] = g[i];
        sincos(th[i], &sn[i], &cs[i]);
    }
    __syncthreads();
    const RoundKeys rk = round_keys(key);
    unsigned long long acc = 0;
    // per-wave sums of the accepted energy changes, by sweep parity
    __shared__ double part[2][16];
    const int nwaves = (int)(blockDim.x >> 6), wave = (int)(threadIdx.x >> 6);
    double E = 0.0;  // thread 0: H after the sweeps so far
    if (E_trace)
        E = energy_to0(th, L, red);
    double dEs = 0.0;  // this thread's accepted changes in the current sweep
    for (int64_t sw = 0; sw < n; ++sw) {
        for (int c = 0; c < 2; ++c) {
            const uint32_t h = 2u * (t0 + (uint32_t)sw) + (uint32_t)c;
            for (int q = threadIdx.x; q < (N >> 1); q += blockDim.x) {
                const int y = q / half, x = 2 * (q - y * half) + ((y + c) & 1);
                const int row = y * L;
                const U4 o = philox4x32_10({(uint32_t)q, lid, h, kTagXy}, rk);
                const double th_new = unit53(o.x, o.y) * kTwoPi;
                const double p = unit53(o.z, o.w);
                const int i = row + x;
                const int nbi[4] = {row + (x + 1 == L ? 0 : x + 1), row + (x == 0 ? L - 1 : x - 1),
                                    (y + 1 == L ? 0 : y + 1) * L + x,
                                    (y == 0 ? L - 1 : y - 1) * L + x};
                // sum_k cos(a - b_k) = cos a sum_k cos b_k + sin a sum_k sin b_k
                double c_new, s_new;
                sincos(th_new, &s_new, &c_new);
                double sc = 0.0, ss = 0.0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    sc += cs[nbi[k]];
                    ss += sn[nbi[k]];
                }
                const double d = (c_new - cs[i]) * sc + (s_new - sn[i]) * ss;
                const double dE = -d;
                const double P = exp(-beta * dE);
                if (p < P) {
                    th[i] = th_new;
                    cs[i] = c_new;
                    sn[i] = s_new;
                    ++acc;
                    dEs += dE;
                }
            }
            if (E_trace && c == 1) {
                const double w = wave_sum_f64(dEs);
                dEs = 0.0;
                if ((threadIdx.x & 63) == 0)
                    part[sw & 1][wave] = w;
            }
            __syncthreads();
            // the previous sweep's partials are complete behind this barrier
            // and are rewritten only after the next one
            if (E_trace && c == 0 && sw > 0 && threadIdx.x == 0) {
                for (int v = 0; v < nwaves; ++v)
                    E += part[(sw - 1) & 1][v];
                E_trace[(sw - 1) * count + j] = E;
            }
        }
    }
    if (E_trace && n > 0 && threadIdx.x == 0) {
        for (int v = 0; v < nwaves; ++v)
            E += part[(n - 1) & 1][v];
        E_trace[(n - 1) * count + j] = E;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x)
        g[i] = th[i];
    // accepted rotations of this lattice
    __shared__ unsigned long long racc[16];
    unsigned long long a = acc;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        a += __shfl_xor(a, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        racc[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
            t += racc[w];
        reinterpret_cast<unsigned long long*>(ws + kXyAccepted)[j] += t;
    }
}

__global__ void k_xy_energy(const double* theta, int L, double* E_out) {
    __shared__ double red[16];
    const double E = energy_to0(theta + (int64_t)blockIdx.x * L * L, L, red);
    if (threadIdx.x == 0)
        E_out[blockIdx.x] = E;
}

// One half-sweep (colour c, sweep sw of the call) of every lattice from
// global memory, one trial per thread: grid (trials / blockDim, count).
// The trial is k_xy_sweep's, the cached cosines and sines taken from trig
// (double[count][2][L*L], filled by k_xy_trig_fill).  Energy sums S (two
// slots of count doubles): sweep sw adds into slot sw & 1; the colour-0
// launch of sweep sw >= 1 first carries the previous slot's total in (and
// writes it to the trace), and the colour-1 launch clears the other slot for
// the next sweep.
__global__ void __launch_bounds__(256) k_xy_halfsweep_g(unsigned char* ws, double* theta, int L,
                                                        int count, int c, int64_t sw, int64_t n,
                                                        double beta, Key key, uint32_t lid0,
                                                        double* S, double* trig, double* E_trace) {
#pragma clang fp contract(off)
    __shared__ double red[4];
    __shared__ unsigned long long racc[4];
    XyHeader* hd = xy_header(ws);
    if (hd->ok == 0)
        return;
    const int j = blockIdx.y;
    const uint32_t lid = lid0 + (uint32_t)j;
    const int N = L * L, half = L >> 1;
    const uint32_t h = 2u * ((uint32_t)hd->t0 + (uint32_t)sw) + (uint32_t)c;
    double* th = theta + (int64_t)j * N;
    double* cur = S + (size_t)(sw & 1) * count;
    double* other = S + (size_t)((sw + 1) & 1) * count;
    if (E_trace && blockIdx.x == 0 && threadIdx.x == 0) {
        if (c == 0 && sw > 0) {
            E_trace[(sw - 1) * count + j] = other[j];
            atomicAdd(cur + j, other[j]);
        }
        if (c == 1)
            other[j] = 0.0;  // read by this sweep's colour-0 launch, free now
    }
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    double dE_acc = 0.0;
    unsigned long long acc = 0;
    if (q < (N >> 1)) {
        const RoundKeys rk = round_keys(key);
        const int y = q / half, x = 2 * (q - y * half) + ((y + c) & 1);
        const int row = y * L;
        const U4 o = philox4x32_10({(uint32_t)q, lid, h, kTagXy}, rk);
        const double th_new = unit53(o.x, o.y) * kTwoPi;
        const double p = unit53(o.z, o.w);
        const int i = row + x;
        const int nbi[4] = {row + (x + 1 == L ? 0 : x + 1), row + (x == 0 ? L - 1 : x - 1),
                            (y + 1 == L ? 0 : y + 1) * L + x, (y == 0 ? L - 1 : y - 1) * L + x};
        // the angle-difference identity over cached cosines and sines, the
        // same arithmetic as the workgroup-resident form
        double* cs = trig + (size_t)j * 2 * N;
        double* sn = cs + N;
        double sc = 0.0, ss = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sc += cs[nbi[k]];
            ss += sn[nbi[k]];
        }
        double s_new, c_new;
        sincos(th_new, &s_new, &c_new);
        const double d = (c_new - cs[i]) * sc + (s_new - sn[i]) * ss;
        const double dE = -d;
        const double P = exp(-beta * dE);
        if (p < P) {
            th[i] = th_new;
            cs[i] = c_new;
            sn[i] = s_new;
            acc = 1;
            dE_acc = dE;
        }
    }
    // per-workgroup sums: one atomic each into the lattice's counters
    const double w = wave_sum_f64(dE_acc);
    unsigned long long a = acc;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        a += __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = w;
        racc[threadIdx.x >> 6] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double e = 0.0;
        unsigned long long t = 0;
        for (int v = 0; v < (int)(blockDim.x >> 6); ++v) {
            e += red[v];
            t += racc[v];
        }
        if (E_trace && e != 0.0)
            atomicAdd(cur + j, e);
        if (t)
            atomicAdd(reinterpret_cast<unsigned long long*>(ws + kXyAccepted) + j, t);
    }
}

// Energy sums before the first sweep of a call: slot 0 = H, slot 1 = 0.
__global__ void k_xy_sums_start(unsigned char* ws, const double* theta, int L, int count,
                                double* S) {
    __shared__ double red[16];
    if (xy_header(ws)->ok == 0)
        return;
    const double E = energy_to0(theta + (int64_t)blockIdx.x * L * L, L, red);
    if (threadIdx.x == 0) {
        S[blockIdx.x] = E;
        S[count + blockIdx.x] = 0.0;
    }
}

// Cosine and sine of every angle, for the global-memory sweep of a call.
__global__ void k_xy_trig_fill(unsigned char* ws, const double* theta, int N, double* trig) {
    if (xy_header(ws)->ok == 0)
        return;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N)
        return;
    const int j = blockIdx.y;
    double* cs = trig + (size_t)j * 2 * N;
    sincos(theta[(int64_t)j * N + n], &cs[N + n], &cs[n]);
}

// The last sweep's energies into the trace.
__global__ void k_xy_sums_finish(unsigned char* ws, int count, int64_t n, const double* S,
                                 double* E_trace) {
    if (xy_header(ws)->ok == 0)
        return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count)
        E_trace[(n - 1) * count + j] = S[(size_t)((n - 1) & 1) * count + j];
}

// Persistent band-tiled sweep: lattice j is cut into P = L / rb bands of rb
// rows, one workgroup each, resident for all n sweeps of the call.  A band
// keeps its angles and the cosine and sine of its rows in LDS; thread q
// makes trial q of the band in each half-sweep.  The rows just above and
// below the band (the halo) are read from LDS only in the first half-sweep
// of the call (filled from the angles in global memory); after that, the
// halo site (y0 - 1, x) is needed only by the trial at (y0, x), and
// (y0 + rb, x) only by the one at (y0 + rb - 1, x).  So each edge-row trial
// of half-sweep h (colour c) hands its own site's cosine and sine to the
// neighbouring band as soon as it is made: four 32-bit halves in tagged
// slots (tag h + 1) by band, edge, colour and site; and the edge-row trial
// that needs a neighbour's site waits for exactly those four words.  A slot
// is written again two half-sweeps later, by the same trial position, after
// the one thread that reads it has read it (its own publication in between
// is what the writer waits for).  The trial is k_xy_sweep's, operation for
// operation.  Energy trace: each band adds its running sum of accepted
// energy changes to the lattice's entry of every sweep, which holds H at
// the start of the call.
__global__ void __launch_bounds__(512) k_xy_sweep_bands(unsigned char* ws, double* theta, int L,
                                                        int count, int rb, int64_t n, double beta,
                                                        Key key, uint32_t lid0,
                                                        unsigned long long* slots,
                                                        uint32_t spin_limit, double* E_trace) {
#pragma clang fp contract(off)
    // th[rb][L] angles of the band; cs, sn [rb + 2][L]: row r is lattice row y0 - 1 + r
    extern __shared__ double sh[];
    __shared__ double part[16];
    XyHeader* hd = xy_header(ws);
    if (hd->ok == 0)
        return;
    const int P = L / rb, half = L >> 1;
    const int j = blockIdx.x / P, p = blockIdx.x - j * P;
    const int y0 = p * rb, N = L * L;
    const uint32_t lid = lid0 + (uint32_t)j;
    const uint32_t t0 = (uint32_t)hd->t0;
    double* const th = sh;
    double* const cs = sh + rb * L;
    double* const sn = cs + (rb + 2) * L;
    double* g = theta + (int64_t)j * N;
    for (int i = threadIdx.x; i < (rb + 2) * L; i += blockDim.x) {
        const int r = i / L, x = i - r * L;
        int y = y0 - 1 + r;
        y = y < 0 ? y + L : (y >= L ? y - L : y);
        const double a = g[y * L + x];
        if (r >= 1 && r <= rb)
            th[(r - 1) * L + x] = a;
        sincos(a, &sn[i], &cs[i]);
    }
    __syncthreads();
    const RoundKeys rk = round_keys(key);
    const int nwaves = (int)(blockDim.x >> 6), wave = (int)(threadIdx.x >> 6);
    const int q = (int)threadIdx.x;
    const int yl = q / half, kq = q - yl * half;  // local row and index of this thread's trial
    const bool trial = q < rb * half;
    const bool top = trial && yl == 0, bot = trial && yl == rb - 1;
    // slots [band][edge][colour][site][4 words]; this trial's own (edge rows),
    // and the neighbour's it reads: above, the last row of band p - 1; below,
    // the first row of band p + 1
    const size_t per_colour = (size_t)half * 4, per_band = 4 * per_colour;
    const int pu = p == 0 ? P - 1 : p - 1, pd = p == P - 1 ? 0 : p + 1;
    unsigned long long* mine =
        slots + (size_t)blockIdx.x * per_band + (bot ? 2 * per_colour : 0) + 4 * kq;
    const unsigned long long* from_up =
        slots + (size_t)(j * P + pu) * per_band + 2 * per_colour + 4 * kq;
    const unsigned long long* from_dn = slots + (size_t)(j * P + pd) * per_band + 4 * kq;
    uint32_t* const err = &hd->err;
    unsigned long long acc = 0;
    double dEs = 0.0, cum = 0.0;  // thread: this sweep's changes; thread 0: the band's since the start
    for (int64_t sw = 0; sw < n; ++sw) {
        for (int c = 0; c < 2; ++c) {
            const uint32_t h = 2u * (t0 + (uint32_t)sw) + (uint32_t)c;
            const bool first = sw == 0 && c == 0, last = sw == n - 1 && c == 1;
            if (trial) {
                const int y = y0 + yl, x = 2 * kq + ((y + c) & 1);
                const U4 o = philox4x32_10({(uint32_t)(y * half + kq), lid, h, kTagXy}, rk);
                const double th_new = unit53(o.x, o.y) * kTwoPi;
                const double pr = unit53(o.z, o.w);
                const int i = (yl + 1) * L + x;
                double cd = cs[i + L], sd = sn[i + L], cu = cs[i - L], su = sn[i - L];
                // the neighbours' sites (colour c ^ 1) from their half-sweep h - 1
                if (!first && (top || bot)) {
                    const unsigned long long* src = (top ? from_up : from_dn) + (c ^ 1) * per_colour;
                    uint32_t wd[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        wd[k] = wait_slot(src + k, h, spin_limit, err, kXyErrHandoff);
                    const double cv = __hiloint2double((int)wd[1], (int)wd[0]);
                    const double sv = __hiloint2double((int)wd[3], (int)wd[2]);
                    if (top) {
                        cu = cv;
                        su = sv;
                    } else {
                        cd = cv;
                        sd = sv;
                    }
                }
                const int ir = (yl + 1) * L + (x + 1 == L ? 0 : x + 1);
                const int il = (yl + 1) * L + (x == 0 ? L - 1 : x - 1);
                double c_new, s_new;
                sincos(th_new, &s_new, &c_new);
                // right, left, down, up: the order of the other forms
                double sc = 0.0, ss = 0.0;
                sc += cs[ir];
                ss += sn[ir];
                sc += cs[il];
                ss += sn[il];
                sc += cd;
                ss += sd;
                sc += cu;
                ss += su;
                const double d = (c_new - cs[i]) * sc + (s_new - sn[i]) * ss;
                const double dE = -d;
                const double Pa = exp(-beta * dE);
                double cv = cs[i], sv = sn[i];
                if (pr < Pa) {
                    th[yl * L + x] = th_new;
                    cs[i] = c_new;
                    sn[i] = s_new;
                    cv = c_new;
                    sv = s_new;
                    ++acc;
                    dEs += dE;
                }
                if (!last && (top || bot)) {
                    unsigned long long* dst = mine + c * per_colour;
                    const uint64_t cb = (uint64_t)__double_as_longlong(cv);
                    const uint64_t sb = (uint64_t)__double_as_longlong(sv);
                    publish_slot(dst + 0, h + 1u, (uint32_t)cb);
                    publish_slot(dst + 1, h + 1u, (uint32_t)(cb >> 32));
                    publish_slot(dst + 2, h + 1u, (uint32_t)sb);
                    publish_slot(dst + 3, h + 1u, (uint32_t)(sb >> 32));
                }
            }
            if (E_trace && c == 1) {
                const double w = wave_sum_f64(dEs);
                dEs = 0.0;
                if ((threadIdx.x & 63) == 0)
                    part[wave] = w;
            }
            __syncthreads();
            if (E_trace && c == 1 && threadIdx.x == 0) {
                double e = 0.0;
                for (int v = 0; v < nwaves; ++v)
                    e += part[v];
                cum += e;
                atomicAdd(E_trace + sw * count + j, cum);
            }
        }
    }
    for (int i = threadIdx.x; i < rb * L; i += blockDim.x)
        g[y0 * L + i] = th[i];
    __shared__ unsigned long long racc[16];
    unsigned long long a = acc;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        a += __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0)
        racc[wave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int v = 0; v < nwaves; ++v)
            t += racc[v];
        if (t)
            atomicAdd(reinterpret_cast<unsigned long long*>(ws + kXyAccepted) + j, t);
    }
}

// E_trace[sw][j] = H of lattice j at the start of the call (slot 0 of S), for
// the bands to add their accepted changes to.
__global__ void k_xy_trace_fill(unsigned char* ws, const double* S, int count, int64_t n,
                                double* E_trace) {
    if (xy_header(ws)->ok == 0)
        return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n * count)
        E_trace[i] = S[i % count];
}

}  // namespace

bool xy_global_path(int L) { return 3 * (size_t)L * L * sizeof(double) > kXyCacheLds; }

size_t xy_trig_offset(int count) {
    return xy_energy_sums_offset(count) + (((size_t)count * 16 + 255) & ~(size_t)255);
}

namespace {

// Hand-off slots of the band-tiled sweep: per band, 2 edges x 2 colours x
// L/2 sites x 4 words.
size_t xy_slot_words_per_band(int L) { return (size_t)2 * 2 * (L / 2) * 4; }

int xy_max_bands(int L, int count) {
    const int64_t most = (int64_t)count * (L / 2);
    return (int)(most < kXyBandsMax ? most : kXyBandsMax);
}

size_t xy_slots_offset(int L, int count) {
    return xy_trig_offset(count) +
           (xy_global_path(L) ? (((size_t)count * L * L * 16 + 255) & ~(size_t)255) : 0);
}

constexpr uint32_t kXySpinLimit = 1u << 24;  // ~64 clocks a spin

size_t xy_bands_lds(int L, int rb) { return (size_t)(3 * rb + 4) * L * sizeof(double); }

// Whether the band-tiled sweep serves lattices of side L, and if so its
// band height rb (L/rb >= 2 bands of rb >= 2 rows, at most 512 trials a
// band: the double-precision trial needs more registers than a lane has at
// 1024 threads): the smallest with at least 256 trials a band, else the
// largest below that, such that all count * L/rb bands are resident
// together.  It serves L > 80 whenever that fits, and 32 < L <= 80 (where a
// lattice fits one workgroup's LDS, but would leave the trials of a
// half-sweep to 512 threads) when fewer lattices than compute units leave
// most of the chip idle otherwise.
bool xy_bands_plan(int L, int count, int& rb, int& threads, size_t& lds) {
    int dev = 0, cus = 0;
    if (L < kXyBandsMinL || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return false;
    if (!xy_global_path(L) && count >= cus)
        return false;
    const int half = L / 2;
    int cand[64], nc = 0;
    for (int d = 2; d <= L / 2 && nc < 64; ++d)
        if (L % d == 0 && d * half <= 512 && d * half >= 256)
            cand[nc++] = d;
    for (int d = L / 2; d >= 2 && nc < 64; --d)
        if (L % d == 0 && d * half < 256)
            cand[nc++] = d;
    for (int i = 0; i < nc; ++i) {
        const int d = cand[i], bands = count * (L / d);
        const int thr = ((d * half + 63) / 64) * 64;
        const size_t sh = xy_bands_lds(L, d);
        int per_cu = 0;
        if (bands > xy_max_bands(L, count) ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_xy_sweep_bands, thr, sh) !=
                hipSuccess)
            continue;
        if ((int64_t)per_cu * cus >= bands) {
            rb = d;
            threads = thr;
            lds = sh;
            return true;
        }
    }
    return false;
}

}  // namespace

size_t xy_workspace_bytes(int L, int count) {
    // accepted counters, the two slots of per-lattice energy sums, then for
    // L > 80 the cosines and sines of every angle (per-half-sweep sweep) and
    // for L > 32 the hand-off slots of the band-tiled sweep
    if (L < kXyBandsMinL)
        return xy_trig_offset(count);
    return xy_slots_offset(L, count) +
           (size_t)xy_max_bands(L, count) * xy_slot_words_per_band(L) * 8;
}

hipError_t launch_xy_init(unsigned char* ws, double* theta, int L, int count, int start, Key key,
                          uint32_t lid0, hipStream_t st) {
    const int N = L * L;
    hipLaunchKernelGGL(k_xy_init, dim3((N + 255) / 256, count), dim3(256), 0, st, ws, theta, L,
                       count, start, key, lid0);
    return hipGetLastError();
}

hipError_t launch_xy_sweep(unsigned char* ws, double* theta, int L, int count, int64_t n,
                           double beta, Key key, uint32_t lid0, double* E_trace, hipStream_t st) {
    hipLaunchKernelGGL(k_xy_prepare, dim3(1), dim3(1), 0, st, ws, count, n);
    int rb = 0, threads = 0;
    size_t lds = 0;
    if (n > 0 && xy_bands_plan(L, count, rb, threads, lds)) {
        // one persistent launch of resident bands
        double* S = reinterpret_cast<double*>(ws + xy_energy_sums_offset(count));
        unsigned long long* slots =
            reinterpret_cast<unsigned long long*>(ws + xy_slots_offset(L, count));
        const int bands = count * (L / rb);
        // zero every tag so that nothing left by an earlier call can match
        hipError_t e = launch_fill_i64(reinterpret_cast<long long*>(slots),
                                       (int64_t)bands * (int64_t)xy_slot_words_per_band(L), 0, st);
        if (e != hipSuccess)
            return e;
        if (E_trace) {
            hipLaunchKernelGGL(k_xy_sums_start, dim3(count), dim3(256), 0, st, ws, theta, L, count,
                               S);
            hipLaunchKernelGGL(k_xy_trace_fill, dim3((unsigned)((n * count + 255) / 256)),
                               dim3(256), 0, st, ws, S, count, n, E_trace);
        }
        uint32_t spin_limit = kXySpinLimit;
        void* args[] = {&ws, &theta, &L, &count, &rb, &n, &beta, &key, &lid0, &slots,
                        &spin_limit, &E_trace};
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_xy_sweep_bands),
                                       dim3(bands), dim3(threads), args, lds, st);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_xy_advance, dim3(1), dim3(1), 0, st, ws, n);
        return hipGetLastError();
    }
    if (xy_global_path(L)) {
        // one launch per half-sweep over many workgroups
        double* S = reinterpret_cast<double*>(ws + xy_energy_sums_offset(count));
        double* trig = reinterpret_cast<double*>(ws + xy_trig_offset(count));
        const int trials = L * L / 2;
        const dim3 grid((unsigned)((trials + 255) / 256), (unsigned)count);
        hipLaunchKernelGGL(k_xy_trig_fill, dim3((unsigned)((L * L + 255) / 256), (unsigned)count),
                           dim3(256), 0, st, ws, theta, L * L, trig);
        if (E_trace)
            hipLaunchKernelGGL(k_xy_sums_start, dim3(count), dim3(256), 0, st, ws, theta, L, count,
                               S);
        for (int64_t sw = 0; sw < n; ++sw)
            for (int c = 0; c < 2; ++c)
                hipLaunchKernelGGL(k_xy_halfsweep_g, grid, dim3(256), 0, st, ws, theta, L, count,
                                   c, sw, n, beta, key, lid0, S, trig, E_trace);
        if (E_trace && n > 0)
            hipLaunchKernelGGL(k_xy_sums_finish, dim3((count + 255) / 256), dim3(256), 0, st, ws,
                               count, n, S, E_trace);
        hipLaunchKernelGGL(k_xy_advance, dim3(1), dim3(1), 0, st, ws, n);
        return hipGetLastError();
    }
    // one trial per thread per half-sweep where the lattice allows (up to 512:
    // the double-precision trial needs more than the 128 registers a lane
    // has at 1024 threads)
    int thr = ((L * L / 2 + 63) / 64) * 64;
    thr = thr < 64 ? 64 : (thr > 512 ? 512 : thr);
    const size_t plane = (size_t)L * L * sizeof(double);
    hipLaunchKernelGGL(k_xy_sweep, dim3(count), dim3(thr), 3 * plane, st, ws, theta, L, count,
                       n, beta, key, lid0, E_trace);
    hipLaunchKernelGGL(k_xy_advance, dim3(1), dim3(1), 0, st, ws, n);
    return hipGetLastError();
}

hipError_t launch_xy_energy(const double* theta, int L, int count, double* E_out, hipStream_t st) {
    hipLaunchKernelGGL(k_xy_energy, dim3(count), dim3(256), 0, st, theta, L, E_out);
    return hipGetLastError();
}

}  // namespace ising
