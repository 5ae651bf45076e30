// Batches of small INT8 lattices, each resident in LDS for a whole call.
//
// Every lattice of the batch runs the same checkerboard Metropolis chain
// as a single INT8 lattice (Fig. 2a-c; SITE draws with the lattice's own
// id), at its own beta.  One workgroup owns one lattice at a time: it
// copies the lattice into LDS, runs all n sweeps there with one barrier
// per half-sweep, reduces E and M after each sweep into the moments, and
// writes the lattice back.  Workgroups take lattices from a device work
// queue ordered largest first, so uneven sides balance over the CUs.
//
// Within a half-sweep a thread updates the four colour-c sites of an
// 8-byte span of one row (L % 8 == 0): three 8-byte LDS reads (the row and
// the rows above and below) plus one byte across the span's edge give all
// sixteen neighbours, the anti-aligned neighbour counts of the four sites
// are formed byte-parallel in one register, and the four sites share one
// Philox4x32-10 block (they are q = 4g..4g+3 of their colour).
#include "batch.hpp"
#include "quad.hpp"

namespace ising {

namespace {

struct Header {
    uint32_t magic, count;
    uint64_t t, t_scratch;
    uint32_t ok, pad0;
    uint32_t queue, pad1;
    uint32_t err;
};

__device__ __forceinline__ Header* header(unsigned char* ws) {
    return reinterpret_cast<Header*>(ws);
}

__device__ __forceinline__ QuadAccept quad_accept(const BatchDesc& d) {
    const bool a2 = d.always & 1u, a4 = (d.always >> 1) & 1u;
    return QuadAccept{a2 ? 0xFFFFFFFFu : d.T2, d.T4, a2 ? 0u : kOnes, a4 ? 0u : 2u * kOnes};
}

// One half-sweep (colour c) of an LDS lattice of side L (L % 8 == 0) by
// the whole workgroup.  Group gi (Philox counter word g = gi) is the span
// of columns 8k..8k+7 of row y, gi = y L/8 + k.
// Thread tid takes gi = tid, tid + blockDim, ...; its row and span advance
// incrementally, without divisions or 32-bit multiplies.
__device__ __forceinline__ void halfsweep_lds(int8_t* lat, int L, int c, uint32_t h,
                                              const RoundKeys& rk, uint32_t lid,
                                              const QuadAccept& qa, QuadCounts& cnt,
                                              unsigned long long& nblk) {
    const int tid = threadIdx.x, bd = blockDim.x;
    const int gpr = L >> 3, ngroups = L * gpr, N = L * L;
    const int y0 = tid / gpr, k0 = tid - y0 * gpr;
    const int dy = bd / gpr, dk = bd - dy * gpr;
    const int dyL = dy * L;
    int y = y0, k = k0, row = y0 * L;
    for (int gi = tid; gi < ngroups; gi += bd) {
        update_quad(lat, L, N, y, row, 8 * k, c, (uint32_t)gi, h, rk, lid, qa, cnt, nblk);
        k += dk;
        y += dy;
        row += dyL;
        if (k >= gpr) {
            k -= gpr;
            ++y;
            row += L;
        }
    }
}

// Sum of a per-thread value over the workgroup, valid in thread 0.  Must
// be reached by every thread; `red` holds one slot per wave.
__device__ __forceinline__ long long block_sum_to0(long long v, long long* red) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwaves = (blockDim.x + 63) >> 6;
    v = wave_sum_i64(v);
    __syncthreads();
    if (lane == 0)
        red[wave] = v;
    __syncthreads();
    long long t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nwaves; ++w)
            t += red[w];
    return t;
}

// E and M of an L x L lattice (row-major bytes), summed into thread 0.
__device__ __forceinline__ void count_em(const int8_t* s, int L, long long* red, long long& E,
                                         long long& M) {
    long long e = 0, m = 0;
    const int N = L * L;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int y = i / L, x = i - y * L;
        const int right = s[y * L + (x + 1 == L ? 0 : x + 1)];
        const int down = s[(y + 1 == L ? 0 : y + 1) * L + x];
        e -= s[i] * (right + down);
        m += s[i];
    }
    E = block_sum_to0(e, red);
    M = block_sum_to0(m, red);
}

__global__ void k_batch_prepare(unsigned char* ws, int scratch_t, int count, uint64_t spins_bytes,
                                int max_L, int64_t n, int mode, int draws) {
    Header* hd = header(ws);
    const BatchDesc* desc = reinterpret_cast<const BatchDesc*>(ws + BatchWs::desc_offset(count));
    const int32_t* order = reinterpret_cast<const int32_t*>(ws + BatchWs::kOrder);
    __shared__ uint32_t bad;
    if (threadIdx.x == 0)
        bad = (hd->magic == kBatchMagic && hd->count == (uint32_t)count) ? 0u : kBatchErrNotSetUp;
    __syncthreads();
    if (bad == 0) {
        uint32_t mine = 0;
        for (int j = threadIdx.x; j < count; j += blockDim.x) {
            const BatchDesc d = desc[j];
            const bool ok_L = d.L >= 8 && d.L <= max_L && (d.L & 7) == 0;
            const bool ok_off = (d.off & 255u) == 0 &&
                                d.off + (uint64_t)d.L * (uint64_t)d.L <= spins_bytes;
            const bool ok_order = order[j] >= 0 && order[j] < count;
            if (!(ok_L && ok_off && ok_order))
                mine = kBatchErrDescriptor;
        }
        if (mine)
            atomicOr(&bad, mine);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t e = bad;
        if (e == 0 && mode == kPrepareSweep) {
            const uint64_t t = scratch_t ? hd->t_scratch : hd->t;
            if (t + (uint64_t)n > (1ull << 31))
                e = kBatchErrSweepIndex;
            if (*reinterpret_cast<const uint32_t*>(ws + BatchWs::kDraws) != (uint32_t)draws)
                e |= kBatchErrDraws;
        }
        if (e) {
            hd->err |= e;
            hd->ok = 0;
        } else {
            hd->ok = 1;
            hd->queue = 0;
            if (mode == kPrepareInit)
                hd->t = 0;
        }
    }
    if (mode == kPrepareInit && bad == 0) {
        unsigned long long* slots = reinterpret_cast<unsigned long long*>(ws + BatchWs::kRngBlocks);
        for (int i = threadIdx.x; i < 64; i += blockDim.x)
            slots[i] = 0;
    }
}

// One workgroup per lattice: random or cold start (same draws as a single
// INT8 lattice with this lattice id).
__global__ void k_batch_init(unsigned char* ws, int count, int8_t* spins, int start, Key key) {
    if (header(ws)->ok == 0)
        return;
    const BatchDesc d =
        reinterpret_cast<const BatchDesc*>(ws + BatchWs::desc_offset(count))[blockIdx.x];
    uint32_t* s = reinterpret_cast<uint32_t*>(spins + d.off);
    const int nw = d.L * d.L / 4;
    const RoundKeys rk = round_keys(key);
    for (int g = threadIdx.x; g < nw; g += blockDim.x) {
        uint32_t word = 0x01010101u;
        if (start != 0) {
            const U4 o = philox4x32_10({(uint32_t)g, d.lid, 0u, kTagInit}, rk);
            word = ((o.x >> 31) ? 0xFFu : 0x01u) | (((o.y >> 31) ? 0xFFu : 0x01u) << 8) |
                   (((o.z >> 31) ? 0xFFu : 0x01u) << 16) | (((o.w >> 31) ? 0xFFu : 0x01u) << 24);
        }
        s[g] = word;
    }
}

__global__ void k_batch_measure(unsigned char* ws, int count, const int8_t* spins, int64_t* E_out,
                                int64_t* M_out) {
    __shared__ long long red[16];
    if (header(ws)->ok == 0)
        return;
    const BatchDesc d =
        reinterpret_cast<const BatchDesc*>(ws + BatchWs::desc_offset(count))[blockIdx.x];
    long long E, M;
    count_em(spins + d.off, d.L, red, E, M);
    if (threadIdx.x == 0) {
        if (E_out)
            E_out[blockIdx.x] = E;
        if (M_out)
            M_out[blockIdx.x] = M;
    }
}

// Adds a per-lane count into slot blockIdx % 64 of `slots`.  Must be
// reached by every thread of the workgroup.
__device__ __forceinline__ void add_count(unsigned long long v, unsigned long long* slots,
                                          long long* red) {
    const long long t = block_sum_to0((long long)v, red);
    if (threadIdx.x == 0 && t)
        atomicAdd(slots + (blockIdx.x % 64), (unsigned long long)t);
}

// Persistent sweep: workgroups take lattices off the queue until it is
// empty.  No workgroup waits on another, so any grid size is safe.
__global__ void __launch_bounds__(1024) k_batch_sweep(unsigned char* ws, int scratch_t, int count,
                                                      int8_t* spins, int64_t n, Key key,
                                                      int64_t* moments, int64_t* trace) {
    extern __shared__ uint2 lds2[];
    int8_t* lat = reinterpret_cast<int8_t*>(lds2);
    __shared__ int s_item;
    __shared__ long long red[16];
    __shared__ int redi[2][2][16];
    Header* hd = header(ws);
    if (hd->ok == 0)
        return;  // uniform: every workgroup reads the same word
    const BatchDesc* desc = reinterpret_cast<const BatchDesc*>(ws + BatchWs::desc_offset(count));
    const int32_t* order = reinterpret_cast<const int32_t*>(ws + BatchWs::kOrder);
    unsigned long long* slots =
        reinterpret_cast<unsigned long long*>(ws + (scratch_t ? BatchWs::kRngScratch : BatchWs::kRngBlocks));
    const uint32_t t0 = (uint32_t)(scratch_t ? hd->t_scratch : hd->t);
    const RoundKeys rk = round_keys(key);
    const int tid = threadIdx.x, bd = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nwaves = (bd + 63) >> 6;
    unsigned long long nblk = 0;
    for (;;) {
        if (tid == 0)
            s_item = (int)atomicAdd(&hd->queue, 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= count)
            break;
        const int j = order[item];
        const BatchDesc d = desc[j];
        const QuadAccept qa = quad_accept(d);
        const int L = d.L;
        const int n8 = L * L / 8;
        const uint2* src = reinterpret_cast<const uint2*>(spins + d.off);
        for (int i = tid; i < n8; i += bd)
            lds2[i] = src[i];
        __syncthreads();
        long long E, M;
        count_em(lat, L, red, E, M);
        long long sE = 0, sE2 = 0, sAM = 0, sM2 = 0;
        unsigned long long m4lo = 0, m4hi = 0;
        for (int64_t sw = 0; sw < n; ++sw) {
            QuadCounts cnt;
            for (int c = 0; c < 2; ++c) {
                const uint32_t h = 2u * (t0 + (uint32_t)sw) + (uint32_t)c;
                halfsweep_lds(lat, L, c, h, rk, d.lid, qa, cnt, nblk);
                if (c == 0)
                    __syncthreads();
            }
            const int dE = wave_sum_i32(8 * (int)cnt.nflip - 2 * (int)cnt.sum_a2);
            const int dM = wave_sum_i32(2 * (2 * (int)cnt.ndown - (int)cnt.nflip));
            const int par = (int)(sw & 1);
            if (lane == 0) {
                redi[par][0][wave] = dE;
                redi[par][1][wave] = dM;
            }
            __syncthreads();
            if (tid == 0) {
                for (int w = 0; w < nwaves; ++w) {
                    E += redi[par][0][w];
                    M += redi[par][1][w];
                }
                sE += E;
                sE2 += E * E;
                sAM += M < 0 ? -M : M;
                const unsigned long long m2 = (unsigned long long)(M * M);
                sM2 += (long long)m2;
                const unsigned long long lo = m2 * m2, hi = __umul64hi(m2, m2);
                m4lo += lo;
                m4hi += hi + (m4lo < lo ? 1u : 0u);
                if (trace) {
                    int64_t* tr = trace + (sw * count + j) * 2;
                    tr[0] = E;
                    tr[1] = M;
                }
            }
        }
        uint2* dst = reinterpret_cast<uint2*>(spins + d.off);
        for (int i = tid; i < n8; i += bd)
            dst[i] = lds2[i];
        if (tid == 0 && moments) {
            int64_t* mo = moments + (int64_t)j * 8;
            mo[0] = E;
            mo[1] = M;
            mo[2] = sE;
            mo[3] = sE2;
            mo[4] = sAM;
            mo[5] = sM2;
            mo[6] = (int64_t)m4lo;
            mo[7] = (int64_t)m4hi;
        }
    }
    add_count(nblk, slots, red);
}

__global__ void k_batch_advance(unsigned char* ws, int64_t n) {
    Header* hd = header(ws);
    if (hd->ok)
        hd->t += (uint64_t)n;
}

}  // namespace

size_t batch_lds_bytes(int max_L) { return (size_t)max_L * (size_t)max_L; }

hipError_t launch_batch_prepare(unsigned char* ws, bool scratch_t, int count, uint64_t spins_bytes,
                                int max_L, int64_t n, int mode, int draws, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_prepare, dim3(1), dim3(256), 0, st, ws, scratch_t ? 1 : 0, count,
                       spins_bytes, max_L, n, mode, draws);
    return hipGetLastError();
}

hipError_t launch_batch_init(unsigned char* ws, int count, int8_t* spins, int start, Key key,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_batch_init, dim3(count), dim3(256), 0, st, ws, count, spins, start, key);
    return hipGetLastError();
}

hipError_t launch_batch_sweep(unsigned char* ws, bool scratch_t, int count, int8_t* spins,
                              int max_L, int64_t n, Key key, int64_t* moments, int64_t* trace,
                              int threads, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_sweep, dim3(blocks), dim3(threads), batch_lds_bytes(max_L), st, ws,
                       scratch_t ? 1 : 0, count, spins, n, key, moments, trace);
    return hipGetLastError();
}

hipError_t launch_batch_advance(unsigned char* ws, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(1), 0, st, ws, n);
    return hipGetLastError();
}

hipError_t launch_batch_measure(unsigned char* ws, int count, const int8_t* spins, int64_t* E,
                                int64_t* M, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_measure, dim3(count), dim3(256), 0, st, ws, count, spins, E, M);
    return hipGetLastError();
}

}  // namespace ising
