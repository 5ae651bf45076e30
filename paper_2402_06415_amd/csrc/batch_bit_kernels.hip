// Batches with bit-plane draws: every lattice (side 32 or a multiple of 64)
// runs the checkerboard Metropolis chain of the BIT1 layout (Fig. 2a-c,
// PLANE draws with the lattice's own id) at its own beta, 32 sites per
// lane.  The lattice is INT8 in global memory; a workgroup packs it into
// two colour bit planes in LDS, runs all n sweeps there and unpacks it.
//
// Plane c of a lattice holds its colour-c sites by compact index
// q = (y L + x) >> 1 = y L/2 + i (x = 2i + ((y + c) & 1)): word g is
// q = 32g .. 32g + 31, bit q & 31, bit 1 meaning s = -1.  For L % 64 == 0 a
// word lies in one row (L/64 words per row); for L = 32 word g holds rows
// 2g (bits 0-15) and 2g + 1 (bits 16-31).  Word g draws the Philox blocks
// (g, lattice id, 2t + c, 1 | b << 8), as the oracle's plane mode.
//
// Work is dealt out statically: the queue order is sorted by side, largest
// first, and workgroup g of G takes positions g, 2G - 1 - g, 2G + g, ...
// (a snake over the workgroups), so every workgroup gets lattices of every
// side and a near-equal share of words.  A workgroup runs its lattices
// together, one team of lanes per lattice with the same number of words
// per lane, in lockstep: one barrier per half-sweep, none at all when every
// team sits inside one wave.
#include "batch.hpp"
#include "bitslice.hpp"

namespace ising {

namespace {

// Header words of the batch workspace (offsets in BatchWs).
__device__ __forceinline__ uint32_t& ws_u32(unsigned char* ws, size_t off) {
    return *reinterpret_cast<uint32_t*>(ws + off);
}

// Order within a wave: LDS traffic of one wave is processed in issue order;
// the fences keep the compiler from moving loads and stores across.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr uint32_t T_SEL = tt((kA & kB) | (~kA & kC));  // a ? b : c, bitwise

// Geometry of a lattice in plane form.
struct BitGeom {
    int L;
    int nw;          // words per row (L / 64), 0 for L = 32 (two rows per word)
    int nwc;         // words per colour
    uint32_t magic;  // floor(g / nw) = umulhi(g, magic) for nw = 2, 3, 4
};

__device__ __forceinline__ BitGeom bit_geom(int L) {
    BitGeom b;
    b.L = L;
    b.nw = L >> 6;
    b.nwc = L * L / 64;
    b.magic = b.nw > 1 ? 0xFFFFFFFFu / (uint32_t)b.nw + 1u : 0u;
    return b;
}

// Where the neighbour words of word g come from, fixed for a lattice: the
// side words (left, for rows of parity (y + c) & 1 == 0, and right), the
// rows above and below (word indices < 2^15), and the parity of y, packed
// in two registers.  Computed once per word and bundle, used in every
// half-sweep.
struct WordNb {
    uint32_t lr;  // left | right << 16 | (y & 1) << 31
    uint32_t ud;  // up | down << 16
};

__device__ __forceinline__ WordNb word_nb(const BitGeom& b, int g) {
    uint32_t iL, iR, iU, iD, py;
    if (b.nw > 0) {
        // exact for g < 2^31: the words of a lattice are at most 1024
        const int y = b.nw == 1 ? g : (int)__umulhi((uint32_t)g, b.magic), w = g - y * b.nw;
        const int row = y * b.nw;
        iL = (uint32_t)(row + (w == 0 ? b.nw - 1 : w - 1));
        iR = (uint32_t)(row + (w + 1 == b.nw ? 0 : w + 1));
        iU = (uint32_t)((y == 0 ? b.L - 1 : y - 1) * b.nw + w);
        iD = (uint32_t)((y + 1 == b.L ? 0 : y + 1) * b.nw + w);
        py = (uint32_t)y & 1u;
    } else {
        iL = iR = (uint32_t)g;
        iU = (uint32_t)(g + 15) & 15u;  // L = 32: 16 words of two rows
        iD = (uint32_t)(g + 1) & 15u;
        py = 0u;
    }
    return WordNb{iL | iR << 16 | py << 31, iU | iD << 16};
}

// The four neighbour words of word g of colour c, from the other plane Po:
// O aligned (same compact index, same row), S the same row shifted by one
// compact column (left when the row's parity (y + c) & 1 is 0, right when
// 1), U and D the rows above and below, periodic.
__device__ __forceinline__ void neighbours(const uint32_t* Po, const BitGeom& b, int g,
                                           const WordNb& n, int c, uint32_t& O, uint32_t& S,
                                           uint32_t& U, uint32_t& D) {
    O = Po[g];
    if (b.nw > 0) {
        // left: bit i <- compact i - 1 (bit 0 from the previous word's bit 31);
        // right: bit i <- compact i + 1
        const bool left = (((n.lr >> 31) + (uint32_t)c) & 1u) == 0u;
        const uint32_t X = Po[left ? (n.lr & 0xFFFFu) : ((n.lr >> 16) & 0x7FFFu)];
        S = left ? __builtin_amdgcn_alignbit(O, X, 31) : __builtin_amdgcn_alignbit(X, O, 1);
        U = Po[n.ud & 0xFFFFu];
        D = Po[n.ud >> 16];
    } else {
        // L = 32: the halves are rows 2g (parity c) and 2g + 1 (parity 1 - c),
        // sixteen compact columns each, periodic within the half
        const uint32_t left = bop3<T_SEL>(0xFFFEFFFEu, O << 1, O >> 15);
        const uint32_t right = bop3<T_SEL>(0x7FFF7FFFu, O >> 1, O << 15);
        S = c == 0 ? bop3<T_SEL>(0x0000FFFFu, left, right) : bop3<T_SEL>(0x0000FFFFu, right, left);
        U = __builtin_amdgcn_alignbit(O, Po[n.ud & 0xFFFFu], 16);  // rows 2g - 1 | 2g
        D = __builtin_amdgcn_alignbit(Po[n.ud >> 16], O, 16);     // rows 2g + 1 | 2g + 2
    }
}

// Pack rows of the INT8 lattice (global) into the two planes (LDS): each
// step takes one 32-byte row segment, sixteen compact columns of each
// colour, i.e. one 16-bit half of a word of each plane.
__device__ __forceinline__ void pack_lattice(uint32_t* P, const int8_t* lat, const BitGeom& b,
                                             int tl, int tt) {
    uint16_t* P0 = reinterpret_cast<uint16_t*>(P);
    uint16_t* P1 = reinterpret_cast<uint16_t*>(P + b.nwc);
    const int segs_per_row = b.L >> 5, nseg = b.L * segs_per_row;
    for (int k = tl; k < nseg; k += tt) {
        const int y = k / segs_per_row, sgm = k - y * segs_per_row;
        const uint4* src = reinterpret_cast<const uint4*>(lat + y * b.L + 32 * sgm);
        uint32_t even = 0, odd = 0;  // bit j: site at x = 32 sgm + 2j (+1), s = -1
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const uint4 u = src[v];
            const uint32_t wd[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = 8 * v + 2 * e;  // compact column of byte 0 of this word
                even |= ((wd[e] >> 7) & 1u) << j | ((wd[e] >> 23) & 1u) << (j + 1);
                odd |= ((wd[e] >> 15) & 1u) << j | ((wd[e] >> 31) & 1u) << (j + 1);
            }
        }
        // colour of the even columns is y & 1; half index of the segment
        const int half = y * segs_per_row + sgm;
        const bool c0_even = (y & 1) == 0;
        P0[half] = (uint16_t)(c0_even ? even : odd);
        P1[half] = (uint16_t)(c0_even ? odd : even);
    }
}

__device__ __forceinline__ void unpack_lattice(int8_t* lat, const uint32_t* P, const BitGeom& b,
                                               int tl, int tt) {
    const uint16_t* P0 = reinterpret_cast<const uint16_t*>(P);
    const uint16_t* P1 = reinterpret_cast<const uint16_t*>(P + b.nwc);
    const int segs_per_row = b.L >> 5, nseg = b.L * segs_per_row;
    for (int k = tl; k < nseg; k += tt) {
        const int y = k / segs_per_row, sgm = k - y * segs_per_row;
        const int half = y * segs_per_row + sgm;
        const bool c0_even = (y & 1) == 0;
        const uint32_t even = c0_even ? P0[half] : P1[half];
        const uint32_t odd = c0_even ? P1[half] : P0[half];
        uint32_t out[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            // bytes x = 4q .. 4q + 3: columns 2q (even, odd), 2q + 1 (even, odd)
            const uint32_t b0 = (even >> (2 * q)) & 1u, b1 = (odd >> (2 * q)) & 1u;
            const uint32_t b2 = (even >> (2 * q + 1)) & 1u, b3 = (odd >> (2 * q + 1)) & 1u;
            out[q] = (b0 ? 0xFFu : 0x01u) | (b1 ? 0xFF00u : 0x0100u) |
                     (b2 ? 0xFF0000u : 0x010000u) | (b3 ? 0xFF000000u : 0x01000000u);
        }
        uint4* dst = reinterpret_cast<uint4*>(lat + y * b.L + 32 * sgm);
        dst[0] = make_uint4(out[0], out[1], out[2], out[3]);
        dst[1] = make_uint4(out[4], out[5], out[6], out[7]);
    }
}

// Per-lane anti-aligned bonds and down spins of the colour-0 words of this
// lane (each bond joins a colour-0 and a colour-1 site).
__device__ __forceinline__ void count_bits(const uint32_t* P, const BitGeom& b, int tl, int tt,
                                           int& anti, int& ones) {
    anti = 0;
    ones = 0;
    for (int g = tl; g < b.nwc; g += tt) {
        uint32_t O, S, U, D;
        neighbours(P + b.nwc, b, g, word_nb(b, g), 0, O, S, U, D);
        const uint32_t W = P[g];
        anti += __popc(W ^ O) + __popc(W ^ S) + __popc(W ^ U) + __popc(W ^ D);
        ones += __popc(W) + __popc(O);
    }
}

// Lanes of a team for nwc words at k words per lane: whole waves from 64
// lanes up, a power of two below (so that teams sorted by size stay aligned).
__device__ __forceinline__ int team_lanes(int nwc, int k) {
    const int x = (nwc + k - 1) / k;
    if (x >= 64)
        return (x + 63) & ~63;
    int p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

// Sum over an aligned team of tt lanes (tt a power of two up to 64; a team
// of more lanes gets the sum over its part of this wave).  Every lane takes
// part in every shuffle.
__device__ __forceinline__ int team_sum(int v, int tt) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(v, off, 64);
        if (off < tt)
            v += o;
    }
    return v;
}

// Most lattices a workgroup runs at once, one team of lanes each.
constexpr int kMaxTeams = 64;

// Persistent sweep with bit-plane draws.  Workgroup g of G owns the
// lattices at queue positions r G + g for even r and r G + G - 1 - g for
// odd r (the queue is sorted by side, largest first, so each workgroup gets
// a near-equal share of words).  It runs as many of them at once as fit its
// LDS (lds_words) and kMaxTeams: with k words per lane, the smallest k for
// which every lattice gets a team of ceil(words / k) lanes, all lattices of
// the pass sweep in lockstep with one barrier per half-sweep.  No workgroup
// waits on another.
__global__ void __launch_bounds__(1024) k_batch_sweep_bit(unsigned char* ws, int scratch_t,
                                                          int count, int8_t* spins, int64_t n,
                                                          Key key, int64_t* moments,
                                                          int64_t* trace, int lds_words) {
    extern __shared__ uint32_t planes[];
    __shared__ int s_team[kMaxTeams][4];  // lattice, first lane, lanes, LDS word offset
    __shared__ int s_nteam, s_next, s_small;
    __shared__ int redi[2][2][16];
    __shared__ long long red[16];
    if (ws_u32(ws, BatchWs::kOk) == 0)
        return;  // uniform: every workgroup reads the same word
    const BatchDesc* desc = reinterpret_cast<const BatchDesc*>(ws + BatchWs::desc_offset(count));
    const int32_t* order = reinterpret_cast<const int32_t*>(ws + BatchWs::kOrder);
    unsigned long long* slots = reinterpret_cast<unsigned long long*>(
        ws + (scratch_t ? BatchWs::kRngScratch : BatchWs::kRngBlocks));
    const uint32_t t0 = (uint32_t)*reinterpret_cast<const uint64_t*>(
        ws + (scratch_t ? BatchWs::kTScratch : BatchWs::kT));
    const int tid = threadIdx.x, bd = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int G = (int)gridDim.x, gid = (int)blockIdx.x;
    unsigned long long nblk = 0;
    int r = 0;  // next round of this workgroup's queue positions
    for (;;) {
        if (tid == 0) {
            // the next lattices of this workgroup while they fit
            int nt = 0, words = 0, lds = 0, rr = r;
            for (; nt < kMaxTeams; ++rr) {
                const int64_t pos = (int64_t)rr * G + ((rr & 1) ? G - 1 - gid : gid);
                if (pos >= count)
                    break;
                const int j = order[pos];
                const int nwc = desc[j].L * desc[j].L / 64;
                if (nt > 0 && lds + 2 * nwc > lds_words)
                    break;
                s_team[nt][0] = j;
                s_team[nt][3] = lds;
                lds += 2 * nwc;
                words += nwc;
                ++nt;
            }
            int k = words > bd ? (words + bd - 1) / bd : 1;
            for (;; ++k) {
                int lanes = 0;
                for (int q = 0; q < nt; ++q) {
                    const int L = desc[s_team[q][0]].L;
                    lanes += team_lanes(L * L / 64, k);
                }
                if (lanes <= bd)
                    break;
            }
            int lane0 = 0, small = 1;
            for (int q = 0; q < nt; ++q) {
                const int L = desc[s_team[q][0]].L;
                const int tt = team_lanes(L * L / 64, k);
                s_team[q][1] = lane0;
                s_team[q][2] = tt;
                lane0 += tt;
                small &= tt <= 64 ? 1 : 0;
            }
            s_nteam = nt;
            s_next = rr;
            s_small = small;
        }
        __syncthreads();
        const int nt = s_nteam;
        if (nt == 0)
            break;  // uniform
        const bool small = s_small != 0;  // every team within one wave: no workgroup barriers
        int team = -1;
        for (int q = 0; q < nt; ++q)
            if (tid >= s_team[q][1] && tid < s_team[q][1] + s_team[q][2])
                team = q;
        const int j = team >= 0 ? s_team[team][0] : 0;
        const int tt = team >= 0 ? s_team[team][2] : 1;
        const int tl = team >= 0 ? tid - s_team[team][1] : 0;
        const bool big = tt > 64;  // the team spans waves
        const BatchDesc d = desc[j];
        const BitGeom b = bit_geom(d.L);
        bool active = team >= 0;
        if (active && !(b.L == 32 || (b.L % 64) == 0)) {
            if (tl == 0)
                atomicOr(&ws_u32(ws, BatchWs::kErr), kBatchErrDraws);
            active = false;
        }
        const Accept acc{d.T2, d.T4, d.always & 1u, (d.always >> 1) & 1u};
        const DrawConsts dc = draw_consts(key, acc);
        uint32_t* P = planes + (team >= 0 ? s_team[team][3] : 0);
        if (active)
            pack_lattice(P, spins + d.off, b, tl, tt);
        __syncthreads();
        // E and M of the lattice before the sweeps (team leader)
        int anti = 0, ones = 0;
        if (active)
            count_bits(P, b, tl, tt, anti, ones);
        long long E = 0, M = 0;
        {
            const int a = team_sum(anti, tt), o = team_sum(ones, tt);
            if (big && lane == 0) {
                redi[0][0][wave] = a;
                redi[0][1][wave] = o;
            }
            __syncthreads();
            long long A = a, Oc = o;
            if (big && tl == 0) {
                A = 0;
                Oc = 0;
                for (int w = (tid >> 6); w < (tid >> 6) + (tt >> 6); ++w) {
                    A += redi[0][0][w];
                    Oc += redi[0][1][w];
                }
            }
            E = 2 * A - 2 * (long long)b.L * b.L;
            M = (long long)b.L * b.L - 2 * Oc;
            __syncthreads();
        }
        long long sE = 0, sE2 = 0, sAM = 0, sM2 = 0;
        unsigned long long m4lo = 0, m4hi = 0;
        // neighbour sources of this lane's first two words
        const WordNb nb0 = word_nb(b, tl < b.nwc ? tl : 0);
        const WordNb nb1 = word_nb(b, tl + tt < b.nwc ? tl + tt : 0);
        for (int64_t sw = 0; sw < n; ++sw) {
            int dE = 0, dM = 0;
            for (int c = 0; c < 2; ++c) {
                const uint32_t h = 2u * (t0 + (uint32_t)sw) + (uint32_t)c;
                if (active) {
                    uint32_t* Pc = P + c * b.nwc;
                    const uint32_t* Po = P + (c ^ 1) * b.nwc;
                    for (int g = tl, q = 0; g < b.nwc; g += tt, ++q) {
                        uint32_t O, S, U, D;
                        neighbours(Po, b, g, q == 0 ? nb0 : (q == 1 ? nb1 : word_nb(b, g)), c, O,
                                   S, U, D);
                        WordState st = classify(Pc[g], O, S, U, D, acc);
                        draw_planes<false>(st, (uint32_t)g, h, d.lid, acc, dc, nblk);
                        Pc[g] = finalize<true>(st, dE, dM);
                    }
                }
                if (small) {
                    wave_sync();
                } else if (c == 0) {
                    __syncthreads();
                }
            }
            const int e = team_sum(dE, tt), m = team_sum(dM, tt);
            if (small) {
                E += e;
                M += m;
            } else {
                const int par = (int)(sw & 1);
                if (big && lane == 0) {
                    redi[par][0][wave] = e;
                    redi[par][1][wave] = m;
                }
                __syncthreads();
                if (!big) {
                    E += e;
                    M += m;
                } else if (tl == 0) {
                    for (int w = (tid >> 6); w < (tid >> 6) + (tt >> 6); ++w) {
                        E += redi[par][0][w];
                        M += redi[par][1][w];
                    }
                }
            }
            if (tl == 0 && active) {
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
        __syncthreads();
        if (active)
            unpack_lattice(spins + d.off, P, b, tl, tt);
        if (tl == 0 && active && moments) {
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
        r = s_next;
        __syncthreads();  // s_team and the planes are rewritten by the next pass
    }
    // draw counters: one atomic per workgroup
    long long v = wave_sum_i64((long long)nblk);
    __syncthreads();
    if (lane == 0)
        red[wave] = v;
    __syncthreads();
    if (tid == 0) {
        long long t = 0;
        for (int w = 0; w < ((bd + 63) >> 6); ++w)
            t += red[w];
        if (t)
            atomicAdd(slots + (blockIdx.x % 64), (unsigned long long)t);
    }
}

}  // namespace

size_t batch_bit_lds_bytes(int threads, int max_L) {
    // the least a workgroup needs: both planes of one lattice of side max_L
    (void)threads;
    return (size_t)max_L * max_L / 64 * 2 * 4;
}

hipError_t launch_batch_sweep_bit(unsigned char* ws, bool scratch_t, int count, int8_t* spins,
                                  int64_t n, Key key, int64_t* moments, int64_t* trace,
                                  int threads, int blocks, size_t lds_bytes, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_sweep_bit, dim3(blocks), dim3(threads), lds_bytes, st, ws,
                       scratch_t ? 1 : 0, count, spins, n, key, moments, trace,
                       (int)(lds_bytes / 4));
    return hipGetLastError();
}

}  // namespace ising
