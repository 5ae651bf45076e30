// 3D Edwards-Anderson +-J spin glass with replica exchange.
//
// All replicas are swept together: one launch per half-sweep covers every
// replica, one thread per 8-byte span of a row (the four colour-c sites of
// the span share one Philox4x32-10 block, SITE draws).  The six neighbours
// of the four sites come from the span's row (plus one byte across its
// edge), the rows above and below and the planes in front and behind; the
// couplings from the same places of the three bond arrays.  A bond is
// unsatisfied when J s_i s_j = -1: for +-1 bytes (0x01 / 0xFF) that is bit 1
// of s_i ^ s_j ^ J, so the unsatisfied counts of the four sites are summed
// byte-parallel.  With n_u unsatisfied bonds, u = 6 - 2 n_u: n_u >= 3 flips
// without a draw, n_u = 2, 1, 0 need r < T2, T4, T6 (T6 <= T4 <= T2), i.e.
// lvl = (r < T2) + (r < T4) + (r < T6) >= 1, 2, 3.
//
// Per-block energy changes go to a partials array; a per-sweep kernel sums
// them in a fixed order, then the exchange kernel (a no-op between
// exchanges) swaps temperatures and advances the device sweep index.
#include "bitslice.hpp"
#include "ea.hpp"

namespace ising {

namespace {

constexpr uint32_t T_AND_OR = tt((kA & kB) | kC);       // (a & b) | c
constexpr uint32_t T_OR_AND = tt((kA | kB) & kC);       // (a | b) & c
constexpr uint32_t T_NOR_AND = tt(~(kA | kB) & kC);     // ~(a | b) & c
constexpr uint32_t T_ANDN_AND = tt(kA & ~kB & kC);      // a & ~b & c
constexpr uint32_t T_AND2 = tt(kA & kB);                // a & b
constexpr uint32_t kOnes = 0x01010101u;
constexpr uint32_t kSelEven = 0x06040200u;  // bytes 0, 2, 4, 6 of {hi:lo}
constexpr uint32_t kSelOdd = 0x07050301u;   // bytes 1, 3, 5, 7

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

struct EaHeader {
    uint32_t magic, R;
    uint64_t t, t0;
    uint32_t ok, err;
};

__device__ __forceinline__ EaHeader* ea_header(unsigned char* ws) {
    return reinterpret_cast<EaHeader*>(ws);
}

// Thresholds of one temperature as the update compares them (written by
// ising_ea_setup).
struct EaAccept {
    uint32_t T2, T4, T6;   // 0xFFFFFFFF where the class always flips
    uint32_t M2, M4, M6;   // need of u = 2, 4, 6 in every byte (0 when always)
};

// The four sites' bytes of a span (p: parity of their x) and the byte
// across the span's edge.
struct Span {
    uint32_t S, Lf, Rt;
};
__device__ __forceinline__ Span split_row(uint2 R, uint32_t X, int p) {
    const uint32_t ev = perm(R.y, R.x, kSelEven), od = perm(R.y, R.x, kSelOdd);
    Span s;
    s.S = p ? od : ev;
    s.Lf = p ? ev : ((od << 8) | X);
    s.Rt = p ? ((ev >> 8) | (X << 24)) : od;
    return s;
}

// bit 1 of each byte set where J s_i s_j = -1
__device__ __forceinline__ uint32_t unsat(uint32_t a, uint32_t b, uint32_t j) {
    return xor3(a, b, j) & 0x02020202u;
}

// Fourth word of a raw buffer resource on gfx950 (32-bit data, no swizzle).
constexpr int kBufferWord3 = 0x00020000;

// Philox round keys left to the scalar unit: a thread of the half-sweep
// draws at most one block, so a key schedule in vector registers would cost
// as much as the block itself.
__device__ __forceinline__ RoundKeys scalar_round_keys(Key key) {
    RoundKeys rk;
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        rk.k[2 * i] = k0;
        rk.k[2 * i + 1] = k1;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return rk;
}

__global__ void k_ea_halfsweep(unsigned char* ws, const EaLayout lay, int8_t* spins,
                               const int8_t* bonds, int lgL, int R, int c, Key key) {
    EaHeader* hd = ea_header(ws);
    if (hd->ok == 0)
        return;
    // grid (spans of a plane / 256, z, replica); L = 2^lgL, 32-bit index math
    const int L = 1 << lgL, lgG = lgL - 3;          // spans per row: 2^lgG
    const uint32_t N = 1u << (3 * lgL);
    const uint32_t LL = 1u << (2 * lgL);
    const int r = blockIdx.z, z = blockIdx.y;
    const uint32_t gp = blockIdx.x * 256u + threadIdx.x;  // span within the plane
    const int bpr = (int)(gridDim.x * gridDim.y);
    const int bi = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    int dE = 0, nblk = 0;
    if (gp < (LL >> 3)) {
        const int y = (int)(gp >> lgG), k = (int)(gp & ((1u << lgG) - 1));
        const int p = (y + z + c) & 1;
        const int x0 = 8 * k;
        const uint32_t row = ((uint32_t)z << (2 * lgL)) | ((uint32_t)y << lgL);
        const uint32_t rup = (y == 0 ? row + LL - L : row - L);      // y - 1
        const uint32_t rdn = (y + 1 == L ? row - LL + L : row + L);  // y + 1
        const uint32_t rbk = (z == 0 ? row + N - LL : row - LL);     // z - 1
        const uint32_t rft = (z + 1 == L ? row - N + LL : row + LL); // z + 1
        const int xe = p ? (x0 + 8 == L ? 0 : x0 + 8) : (x0 == 0 ? L - 1 : x0 - 1);
        // Buffer loads: the replica's spins and the couplings are addressed by
        // 32-bit offsets from a wave-uniform base (no 64-bit address math per
        // load); Jy and Jz are the coupling buffer at scalar offsets N and 2N.
        const __amdgpu_buffer_rsrc_t bs = __builtin_amdgcn_make_buffer_rsrc(
            spins + (size_t)r * N, (short)0, (int)N, kBufferWord3);
        const __amdgpu_buffer_rsrc_t bj = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<int8_t*>(bonds), (short)0, (int)(3 * N), kBufferWord3);
        auto ld = [&](__amdgpu_buffer_rsrc_t b, uint32_t off, uint32_t soff) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(b, off, soff, 0);
            return make_uint2(v[0], v[1]);
        };
        const uint2 Rw = ld(bs, row + x0, 0u);
        const Span sp = split_row(Rw, __builtin_amdgcn_raw_buffer_load_b8(bs, row + xe, 0u, 0), p);
        const uint32_t sel = p ? kSelOdd : kSelEven;
        auto at = [&](__amdgpu_buffer_rsrc_t b, uint32_t rb, uint32_t soff) {
            const uint2 w = ld(b, rb + x0, soff);
            return perm(w.y, w.x, sel);
        };
        // couplings: right bond J_x(n) at the sites; left bond J_x(n - e_x)
        const uint2 Jxw = ld(bj, row + x0, 0u);
        const uint32_t jev = perm(Jxw.y, Jxw.x, kSelEven), jod = perm(Jxw.y, Jxw.x, kSelOdd);
        const uint32_t JR = p ? jod : jev;
        const uint32_t JL =
            p ? jev
              : ((jod << 8) |
                 __builtin_amdgcn_raw_buffer_load_b8(bj, row + (x0 == 0 ? L - 1 : x0 - 1), 0u, 0));
        const uint32_t a2 = unsat(sp.S, sp.Lf, JL) + unsat(sp.S, sp.Rt, JR) +
                            unsat(sp.S, at(bs, rup, 0u), at(bj, rup, N)) +
                            unsat(sp.S, at(bs, rdn, 0u), at(bj, row, N)) +
                            unsat(sp.S, at(bs, rbk, 0u), at(bj, rbk, 2 * N)) +
                            unsat(sp.S, at(bs, rft, 0u), at(bj, row, 2 * N));
        // a2 = 2 n_u per byte (0..12); classes on n_u = 0, 1, 2 (bits 0..2 of n_u)
        // (multi-input logic through bop3 with explicit tables, as elsewhere)
        const uint32_t nu = (a2 >> 1) & 0x07070707u;
        const uint32_t b1s = nu >> 1, b2s = nu >> 2;              // bits 1, 2 at bit 0
        const uint32_t hi = bop3<T_OR_AND>(b1s, b2s, kOnes);      // n_u >= 2
        const uint32_t is0 = bop3<T_NOR_AND>(nu, hi, kOnes);      // n_u == 0: u = 6
        const uint32_t is1 = bop3<T_ANDN_AND>(nu, hi, kOnes);     // n_u == 1: u = 4
        const uint32_t lo2 = bop3<T_NOR_AND>(nu, b2s, kOnes);     // bits 0 and 2 clear
        const uint32_t is2 = bop3<T_AND2>(b1s, lo2, lo2);         // n_u == 2: u = 2
        const EaAccept a = reinterpret_cast<const EaAccept*>(ws + lay.thr)[
            reinterpret_cast<const int32_t*>(ws + lay.tidx)[r]];
        const uint32_t n6 = bop3<T_OR_AND>(is0, is0 << 1, a.M6);  // 3 where u = 6
        const uint32_t need = n6 | bop3<T_AND_OR>(is1 << 1, a.M4, is2 & a.M2);
        U4 rr = {0u, 0u, 0u, 0u};
        if (need) {
            rr = philox4x32_10({(row + (uint32_t)x0) >> 3, (uint32_t)r,
                                2u * (uint32_t)hd->t + (uint32_t)c, kTagSite},
                               scalar_round_keys(key));
            nblk = 1;
        }
        uint32_t lvl = 4u * kOnes;  // 4 + lvl_j - need_j stays in 1..7
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t rj = u4_get(rr, j);
            lvl |= ((uint32_t)(rj < a.T2) + (uint32_t)(rj < a.T4) + (uint32_t)(rj < a.T6))
                   << (8 * j);
        }
        const uint32_t fb = ((lvl - need) >> 2) & kOnes;
        uint32_t fb8 = fb << 8;
        asm volatile("" : "+v"(fb8));
        const uint32_t F = fb8 - (fb << 1);  // 0xFE in flipped bytes
        // dE = 2u = 12 - 4 n_u = 12 - 2 a2 per flip
        dE = 12 * (int)__popc(fb) - 2 * (int)__builtin_amdgcn_udot4(a2, fb, 0u, false);
        const uint32_t Fx = perm(F, 0u, p ? 0x05000400u : 0x00050004u);
        const uint32_t Fy = perm(F, 0u, p ? 0x07000600u : 0x00070006u);
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(u32x2{Rw.x ^ Fx, Rw.y ^ Fy}, bs, row + x0, 0u, 0);
    }
    // block sums of dE and of the Philox blocks drawn -> partials[c][r][bi]
    __shared__ int red[2][4];
    dE = wave_sum_i32(dE);
    nblk = wave_sum_i32(nblk);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = dE;
        red[1][threadIdx.x >> 6] = nblk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t at = ((int64_t)c * R + r) * bpr + bi;
        reinterpret_cast<int32_t*>(ws + lay.partial)[at] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        reinterpret_cast<int32_t*>(ws + lay.partial_blk)[at] =
            red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// ---------------------------------------------------------------------------
// Plane draws (L >= 64, a power of two): the colour-c spins of a replica are
// bit planes, word g holding compact indices q = 32g .. 32g + 31 (q = n >> 1,
// all in one row (z, y): g = (z L + y) L/64 + w), bit 1 meaning s = -1; the
// couplings J_d(n) likewise by the colour of n.  One lane updates the 32
// sites of a word with bitwise logic: a bond is unsatisfied where the XOR of
// the two spin bits and the coupling bit is 1, the six unsatisfied bits are
// summed bit-sliced into n_u (0..6), and the draws of group g (Philox blocks
// (g, replica, 2t + c, 1 | b << 8), most significant plane first) are
// compared with the class's threshold plane by plane until every site is
// decided.
// ---------------------------------------------------------------------------

constexpr uint32_t T_NOR_OR = tt(~(kA | kB | kC));       // none set
constexpr uint32_t T_A_NOT_BC = tt(kA & ~(kB | kC));     // a and neither b nor c
constexpr uint32_t T_MAJ3 = tt((kA & kB) | (kA & kC) | (kB & kC));
constexpr uint32_t T_OR_AND3 = tt(kA | (kB & kC));       // a | (b & c)
constexpr uint32_t T_SEL3 = tt((kA & kB) | (~kA & kC));  // a ? b : c, bitwise
constexpr uint32_t T_X3 = tt(kA ^ kB ^ kC);

// Pack 64 bytes (x = 64w .. 64w + 63 of one row) into the word of the even
// columns and the word of the odd ones (bit j <-> column 2j or 2j + 1).
__device__ __forceinline__ void pack64(const int8_t* src, uint32_t& even, uint32_t& odd) {
    const uint4* s4 = reinterpret_cast<const uint4*>(src);
    even = 0;
    odd = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const uint4 u = s4[v];
        const uint32_t wd[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 8 * v + 2 * e;  // compact column of byte 0 of this word
            even |= ((wd[e] >> 7) & 1u) << j | ((wd[e] >> 23) & 1u) << (j + 1);
            odd |= ((wd[e] >> 15) & 1u) << j | ((wd[e] >> 31) & 1u) << (j + 1);
        }
    }
}

// Spins: one thread per (replica, row, 64-column span) -> word w of both colours.
__global__ void k_ea_pack_spins(uint32_t* sbits, const int8_t* spins, int lgL, int R) {
    const int L = 1 << lgL, lgnw = lgL - 6;
    const uint32_t wpc = 1u << (3 * lgL - 6);
    const uint32_t g = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (g >= wpc)
        return;
    const uint32_t row = g >> lgnw, w = g & ((1u << lgnw) - 1);
    const uint32_t y = row & (uint32_t)(L - 1), z = row >> lgL;
    uint32_t even, odd;
    pack64(spins + (size_t)r * ((size_t)wpc << 6) + ((size_t)row << lgL) + 64 * w, even, odd);
    const int c_even = (int)((y + z) & 1u);  // colour of the even columns
    sbits[((size_t)r * 2 + c_even) * wpc + g] = even;
    sbits[((size_t)r * 2 + (c_even ^ 1)) * wpc + g] = odd;
}

__global__ void k_ea_unpack_spins(int8_t* spins, const uint32_t* sbits, int lgL, int R) {
    const int L = 1 << lgL, lgnw = lgL - 6;
    const uint32_t wpc = 1u << (3 * lgL - 6);
    const uint32_t g = blockIdx.x * 256u + threadIdx.x;
    const int r = blockIdx.y;
    if (g >= wpc)
        return;
    const uint32_t row = g >> lgnw, w = g & ((1u << lgnw) - 1);
    const uint32_t y = row & (uint32_t)(L - 1), z = row >> lgL;
    const int c_even = (int)((y + z) & 1u);
    const uint32_t even = sbits[((size_t)r * 2 + c_even) * wpc + g];
    const uint32_t odd = sbits[((size_t)r * 2 + (c_even ^ 1)) * wpc + g];
    uint4* dst = reinterpret_cast<uint4*>(spins + (size_t)r * ((size_t)wpc << 6) +
                                          ((size_t)row << lgL) + 64 * w);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        uint32_t out[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 8 * v + 2 * e;
            const uint32_t b0 = (even >> j) & 1u, b1 = (odd >> j) & 1u;
            const uint32_t b2 = (even >> (j + 1)) & 1u, b3 = (odd >> (j + 1)) & 1u;
            out[e] = (b0 ? 0xFFu : 0x01u) | (b1 ? 0xFF00u : 0x0100u) |
                     (b2 ? 0xFF0000u : 0x010000u) | (b3 ? 0xFF000000u : 0x01000000u);
        }
        dst[v] = make_uint4(out[0], out[1], out[2], out[3]);
    }
}

// Couplings: bonds[d N + n] -> jbits[d][colour of n][word].
__global__ void k_ea_pack_bonds(uint32_t* jbits, const int8_t* bonds, int lgL) {
    const int L = 1 << lgL, lgnw = lgL - 6;
    const uint32_t wpc = 1u << (3 * lgL - 6);
    const uint32_t g = blockIdx.x * 256u + threadIdx.x;
    const int d = blockIdx.y;
    if (g >= wpc)
        return;
    const uint32_t row = g >> lgnw, w = g & ((1u << lgnw) - 1);
    const uint32_t y = row & (uint32_t)(L - 1), z = row >> lgL;
    uint32_t even, odd;
    pack64(bonds + (size_t)d * ((size_t)wpc << 6) + ((size_t)row << lgL) + 64 * w, even, odd);
    const int c_even = (int)((y + z) & 1u);
    jbits[((size_t)d * 2 + c_even) * wpc + g] = even;
    jbits[((size_t)d * 2 + (c_even ^ 1)) * wpc + g] = odd;
}

// Words per thread of the plane half-sweep: the round keys and the
// threshold masks of the first eight planes are set up once per thread and
// reused for each of its words.
constexpr int kEaWordsPerThread = 4;

// One half-sweep (colour c) of every replica with plane draws: kEaWordsPerThread
// words per thread (256 words apart), bpr_bit / kEaWordsPerThread workgroups
// per replica.  Workgroups are dealt to the eight XCDs in turn; when R is a
// multiple of 8 the blocks of replica r all go to XCD r mod 8, so a replica's
// planes stay in one XCD's L2.
__global__ void __launch_bounds__(256) k_ea_halfsweep_bit(unsigned char* ws, const EaLayout lay,
                                                          int lgL, int R, int c, Key key) {
    EaHeader* hd = ea_header(ws);
    if (hd->ok == 0)
        return;
    const int L = 1 << lgL, lgnw = lgL - 6;
    const uint32_t wpc = 1u << (3 * lgL - 6);
    const uint32_t nwm = (1u << lgnw) - 1, Lm = (uint32_t)L - 1;
    const uint32_t bpr = (uint32_t)lay.bpr_bit / kEaWordsPerThread, i = blockIdx.x;
    uint32_t r, bx;
    if ((R & 7) == 0) {
        const uint32_t j = i >> 3;
        r = (i & 7u) + 8u * (j / bpr);
        bx = j % bpr;
    } else {
        r = i / bpr;
        bx = i % bpr;
    }
    const uint32_t* sb = reinterpret_cast<const uint32_t*>(ws + lay.sbits);
    const uint32_t* jb = reinterpret_cast<const uint32_t*>(ws + lay.jbits);
    uint32_t* Pc = const_cast<uint32_t*>(sb) + ((size_t)r * 2 + c) * wpc;
    const uint32_t* Po = sb + ((size_t)r * 2 + (c ^ 1)) * wpc;
    const uint32_t* J0c = jb + (size_t)c * wpc;
    const uint32_t* J0o = jb + (size_t)(c ^ 1) * wpc;
    const uint32_t* J1c = jb + (size_t)(2 + c) * wpc;
    const uint32_t* J1o = jb + (size_t)(2 + (c ^ 1)) * wpc;
    const uint32_t* J2c = jb + (size_t)(4 + c) * wpc;
    const uint32_t* J2o = jb + (size_t)(4 + (c ^ 1)) * wpc;
    const EaAccept a = reinterpret_cast<const EaAccept*>(ws + lay.thr)[
        reinterpret_cast<const int32_t*>(ws + lay.tidx)[r]];
    const bool al2 = a.M2 == 0, al4 = a.M4 == 0, al6 = a.M6 == 0;  // always flips
    // per-thread constants: Philox round keys, threshold masks of planes 0-11
    const RoundKeys rk = round_keys(key);
    uint32_t t2m[12], t4m[12], t6m[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        t2m[k] = 0u - ((a.T2 >> (31 - k)) & 1u);
        t4m[k] = 0u - ((a.T4 >> (31 - k)) & 1u);
        t6m[k] = 0u - ((a.T6 >> (31 - k)) & 1u);
        asm volatile("" : "+v"(t2m[k]), "+v"(t4m[k]), "+v"(t6m[k]));
    }
    const uint32_t h = 2u * (uint32_t)hd->t + (uint32_t)c;
    int dE = 0;
    unsigned long long nblk = 0;
    for (int k = 0; k < kEaWordsPerThread; ++k) {
        const uint32_t g = (bx * kEaWordsPerThread + (uint32_t)k) * 256u + threadIdx.x;
        if (g >= wpc)
            break;
        const uint32_t row = g >> lgnw, w = g & nwm;
        const uint32_t y = row & Lm, z = row >> lgL;
        const uint32_t p = (y + z + (uint32_t)c) & 1u;
        const uint32_t rowb = g - w;
        const uint32_t wm = rowb + ((w - 1) & nwm), wp = rowb + ((w + 1) & nwm);
        const uint32_t gU = ((((z << lgL) | ((y - 1) & Lm)) << lgnw) | w);
        const uint32_t gD = ((((z << lgL) | ((y + 1) & Lm)) << lgnw) | w);
        const uint32_t gB = ((((((z - 1) & Lm) << lgL) | y) << lgnw) | w);
        const uint32_t gF = ((((((z + 1) & Lm) << lgL) | y) << lgnw) | w);
        // every load of the word first, so that they are in flight together
        // (the bit operations below are inline assembly, which the compiler
        // does not move loads across)
        const uint32_t W = Pc[g], O = Po[g];
        const uint32_t X = Po[p ? wp : wm];
        const uint32_t jc = J0c[g], jo = J0o[g], jom = J0o[wm];
        const uint32_t sU = Po[gU], jU = J1o[gU];  // y - 1: J_y at (x, y - 1, z)
        const uint32_t sD = Po[gD], jD = J1c[g];   // y + 1: J_y at n
        const uint32_t sB = Po[gB], jB = J2o[gB];  // z - 1: J_z at (x, y, z - 1)
        const uint32_t sF = Po[gF], jF = J2c[g];   // z + 1: J_z at n
        // p = 0: O is the right neighbour (x + 1), the side word the left one;
        // p = 1: O is the left neighbour, the side word the right one.
        const uint32_t S = p ? __builtin_amdgcn_alignbit(X, O, 1) : __builtin_amdgcn_alignbit(O, X, 31);
        const uint32_t bO = p ? jo : jc;  // J_x at the left site (p = 1) or at n (p = 0)
        const uint32_t bS = p ? jc : __builtin_amdgcn_alignbit(jo, jom, 31);
        const uint32_t u0 = bop3<T_X3>(W, O, bO);
        const uint32_t u1 = bop3<T_X3>(W, S, bS);
        const uint32_t u2 = bop3<T_X3>(W, sU, jU);
        const uint32_t u3 = bop3<T_X3>(W, sD, jD);
        const uint32_t u4 = bop3<T_X3>(W, sB, jB);
        const uint32_t u5 = bop3<T_X3>(W, sF, jF);
        // n_u = b0 + 2 b1 + 4 b2, bit-sliced
        const uint32_t s1 = bop3<T_X3>(u0, u1, u2), c1 = bop3<T_MAJ3>(u0, u1, u2);
        const uint32_t s2 = bop3<T_X3>(u3, u4, u5), c2 = bop3<T_MAJ3>(u3, u4, u5);
        const uint32_t b0 = s1 ^ s2, k0 = s1 & s2;
        const uint32_t b1 = bop3<T_X3>(c1, c2, k0), b2 = bop3<T_MAJ3>(c1, c2, k0);
        // n_u >= 3 (u <= 0) flips without a draw; n_u = 2, 1, 0 are u = 2, 4, 6
        const uint32_t ge3 = bop3<T_OR_AND3>(b2, b1, b0);
        const uint32_t is0 = bop3<T_NOR_OR>(b0, b1, b2);
        const uint32_t is1 = bop3<T_A_NOT_BC>(b0, b1, b2);
        const uint32_t is2 = bop3<T_A_NOT_BC>(b1, b0, b2);
        WordState st;
        st.W = W;
        st.flip = ge3 | (al2 ? is2 : 0u) | (al4 ? is1 : 0u) | (al6 ? is0 : 0u);
        st.und = (al2 ? 0u : is2) | (al4 ? 0u : is1) | (al6 ? 0u : is0);
        // blocks 0 to 2 straight-line with the masks in registers (some lane
        // of nearly every wave needs block 2)
#pragma unroll
        for (uint32_t blk = 0; blk < 3; ++blk) {
            nblk += st.und ? 1u : 0u;
            const U4 out = philox4x32_10({g, r, h, kTagPlane | (blk << 8)}, rk);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int q = 4 * (int)blk + kk;
                const uint32_t tm = bop3<T_SEL3>(is2, t2m[q], bop3<T_SEL3>(is1, t4m[q], t6m[q]));
                compare_plane(st, u4_get(out, kk), tm);
            }
        }
        // further blocks while the lane has undecided sites
        for (uint32_t blk = 3; blk < 8u && st.und; ++blk) {
            ++nblk;
            const U4 out = philox4x32_10({g, r, h, kTagPlane | (blk << 8)}, rk);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const uint32_t sh = 31u - (4u * blk + (uint32_t)kk);
                // uniform values: these stay on the scalar unit
                const uint32_t t2 = 0u - ((a.T2 >> sh) & 1u), t4 = 0u - ((a.T4 >> sh) & 1u);
                const uint32_t t6 = 0u - ((a.T6 >> sh) & 1u);
                const uint32_t tm = bop3_vsv<T_SEL3>(is2, t2, bop3_vsv<T_SEL3>(is1, t4, t6));
                compare_plane(st, u4_get(out, kk), tm);
            }
        }
        const uint32_t f = st.flip;
        // dE = 2u = 12 - 4 n_u per flip
        dE += 12 * __popc(f) - 4 * (__popc(f & b0) + 2 * __popc(f & b1) + 4 * __popc(f & b2));
        Pc[g] = W ^ f;
    }
    // block sums of dE and of the Philox blocks drawn -> partials[c][r][bx],
    // bpr entries per replica
    __shared__ int red[2][4];
    dE = wave_sum_i32(dE);
    const int nb = wave_sum_i32((int)nblk);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = dE;
        red[1][threadIdx.x >> 6] = nb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t at = ((int64_t)c * R + r) * bpr + bx;
        reinterpret_cast<int32_t*>(ws + lay.partial)[at] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        reinterpret_cast<int32_t*>(ws + lay.partial_blk)[at] =
            red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// Per replica: E += sum of both half-sweeps' partials (fixed order); trace.
__global__ void k_ea_reduce(unsigned char* ws, const EaLayout lay, int R, int bpr, int64_t* trace) {
    EaHeader* hd = ea_header(ws);
    if (hd->ok == 0)
        return;
    const int r = blockIdx.x;
    const int32_t* part = reinterpret_cast<const int32_t*>(ws + lay.partial);
    const int32_t* pblk = reinterpret_cast<const int32_t*>(ws + lay.partial_blk);
    long long v = 0, nb = 0;
    for (int i = threadIdx.x; i < bpr; i += blockDim.x) {
        v += (long long)part[(int64_t)r * bpr + i] + part[((int64_t)R + r) * bpr + i];
        nb += (long long)pblk[(int64_t)r * bpr + i] + pblk[((int64_t)R + r) * bpr + i];
    }
    __shared__ long long red[2][4];
    v = wave_sum_i64(v);
    nb = wave_sum_i64(nb);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = v;
        red[1][threadIdx.x >> 6] = nb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long* E = reinterpret_cast<long long*>(ws + lay.E);
        E[r] += red[0][0] + red[0][1] + red[0][2] + red[0][3];
        atomicAdd(reinterpret_cast<unsigned long long*>(ws + lay.rng_blocks),
                  (unsigned long long)(red[1][0] + red[1][1] + red[1][2] + red[1][3]));
        if (trace)
            trace[(int64_t)(hd->t - hd->t0) * R + r] = E[r];
    }
}

// Exchange step after sweep t if due, then t += 1.  One thread per pair.
__global__ void k_ea_exchange(unsigned char* ws, const EaLayout lay, int R, int every, Key key) {
    EaHeader* hd = ea_header(ws);
    if (hd->ok == 0)
        return;
    const uint64_t t = hd->t;
    if (every > 0 && (t + 1) % (uint64_t)every == 0) {
        const uint64_t m = (t + 1) / (uint64_t)every - 1;
        const int k = (int)(m & 1) + 2 * (int)threadIdx.x;
        if (k + 1 < R) {
            int32_t* perm_ = reinterpret_cast<int32_t*>(ws + lay.perm);
            int32_t* tidx = reinterpret_cast<int32_t*>(ws + lay.tidx);
            const long long* E = reinterpret_cast<const long long*>(ws + lay.E);
            const int32_t a = perm_[k], b = perm_[k + 1];
            const long long D = E[a] - E[b];
            bool swap = D <= 0;
            if (!swap) {
                if (D & 3) {
                    atomicOr(&hd->err, kEaErrEnergy);
                } else {
                    const EaSwapMeta meta = reinterpret_cast<const EaSwapMeta*>(ws + lay.swap_meta)[k];
                    const uint64_t q = (uint64_t)(D >> 2);
                    uint32_t T;
                    if (q < meta.len)
                        T = reinterpret_cast<const uint32_t*>(ws + lay.swap_tab)[(int64_t)k * kEaSwapTable + q];
                    else
                        T = q < meta.zero_from ? 1u : 0u;
                    const U4 o = philox4x32_10({(uint32_t)k, (uint32_t)m, 0u, kTagSwap}, key);
                    swap = o.x < T;
                }
            }
            if (swap) {
                perm_[k] = b;
                perm_[k + 1] = a;
                tidx[b] = k;
                tidx[a] = k + 1;
                reinterpret_cast<unsigned long long*>(ws + lay.accepts)[k] += 1;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0)
        hd->t = t + 1;
}

__global__ void k_ea_prepare(unsigned char* ws, const EaLayout lay, int R, int64_t n, int mode) {
    EaHeader* hd = ea_header(ws);
    __shared__ uint32_t bad;
    if (threadIdx.x == 0) {
        uint32_t e = (hd->magic == kEaMagic && hd->R == (uint32_t)R) ? 0u : kEaErrNotSetUp;
        if (e == 0 && mode == kEaPrepareSweep && hd->t + (uint64_t)n > (1ull << 31))
            e = kEaErrSweepIndex;
        bad = e;
        if (e) {
            hd->err |= e;
            hd->ok = 0;
        } else {
            hd->ok = 1;
            if (mode == kEaPrepareSweep)
                hd->t0 = hd->t;
            if (mode == kEaPrepareInit)
                hd->t = 0;
        }
    }
    __syncthreads();
    if (bad == 0 && mode == kEaPrepareInit)
        for (int i = threadIdx.x; i < R; i += blockDim.x) {
            reinterpret_cast<int32_t*>(ws + lay.perm)[i] = i;
            reinterpret_cast<int32_t*>(ws + lay.tidx)[i] = i;
            reinterpret_cast<long long*>(ws + lay.E)[i] = 0;
            reinterpret_cast<unsigned long long*>(ws + lay.accepts)[i] = 0;
        }
    if (bad == 0 && mode == kEaPrepareInit && threadIdx.x == 0)
        *reinterpret_cast<unsigned long long*>(ws + lay.rng_blocks) = 0;
}

__global__ void k_ea_init(unsigned char* ws, int8_t* spins, int L, int R, int start, Key key) {
    if (ea_header(ws)->ok == 0)
        return;
    const int64_t N = (int64_t)L * L * L, words = N >> 2;
    const int64_t bpr = (words + 255) >> 8;
    const int r = (int)(blockIdx.x / bpr);
    const int64_t g = (int64_t)(blockIdx.x - r * bpr) * 256 + threadIdx.x;
    if (g >= words)
        return;
    uint32_t word = 0x01010101u;
    if (start != 0) {
        const U4 o = philox4x32_10({(uint32_t)g, (uint32_t)r, 0u, kTagInit}, key);
        word = ((o.x >> 31) ? 0xFFu : 0x01u) | (((o.y >> 31) ? 0xFFu : 0x01u) << 8) |
               (((o.z >> 31) ? 0xFFu : 0x01u) << 16) | (((o.w >> 31) ? 0xFFu : 0x01u) << 24);
    }
    reinterpret_cast<uint32_t*>(spins + (int64_t)r * N)[g] = word;
}

// E of every replica (atomic sums of block totals into out[r], zeroed first).
__global__ void k_ea_energy(unsigned char* ws, const int8_t* spins, const int8_t* bonds, int L,
                            int R, long long* out) {
    if (ea_header(ws)->ok == 0)
        return;
    const int64_t N = (int64_t)L * L * L;
    const int64_t bpr = (N + 255) >> 8;
    const int r = (int)(blockIdx.x / bpr);
    const int64_t n = (int64_t)(blockIdx.x - r * bpr) * 256 + threadIdx.x;
    long long e = 0;
    if (n < N) {
        const int8_t* s = spins + (int64_t)r * N;
        const int x = (int)(n % L), y = (int)((n / L) % L), z = (int)(n / ((int64_t)L * L));
        const int64_t nx = n - x + (x + 1 == L ? 0 : x + 1);
        const int64_t ny = n + (y + 1 == L ? -(int64_t)(L - 1) * L : L);
        const int64_t nz = n + (z + 1 == L ? -(int64_t)(L - 1) * L * L : (int64_t)L * L);
        e = -(long long)s[n] * (bonds[n] * s[nx] + bonds[N + n] * s[ny] + bonds[2 * N + n] * s[nz]);
    }
    __shared__ long long red[4];
    e = wave_sum_i64(e);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long t = red[0] + red[1] + red[2] + red[3];
        if (t)
            atomicAdd(reinterpret_cast<unsigned long long*>(out + r), (unsigned long long)t);
    }
}

__global__ void k_ea_fill(long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0;
}

}  // namespace

EaLayout ea_ws_layout(int L, int R) {
    EaLayout l;
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    l.plane_blocks = (int)((((size_t)L * L / 8) + 255) / 256);
    size_t o = 256;
    l.perm = o;
    o += up((size_t)R * 4);
    l.tidx = o;
    o += up((size_t)R * 4);
    l.E = o;
    o += up((size_t)R * 8);
    l.accepts = o;
    o += up((size_t)R * 8);
    l.thr = o;
    o += up((size_t)R * sizeof(uint32_t) * 6);
    l.swap_meta = o;
    o += up((size_t)R * sizeof(EaSwapMeta));
    l.swap_tab = o;
    o += up((size_t)R * kEaSwapTable * 4);
    l.bpr = l.plane_blocks * L;
    l.partial = o;
    o += up((size_t)2 * R * l.bpr * 4);
    l.partial_blk = o;
    o += up((size_t)2 * R * l.bpr * 4);
    l.rng_blocks = o;
    o += 256;
    const size_t wpc = (size_t)L * L * L / 64;  // words per colour
    l.bpr_bit = (int)((wpc + 255) / 256);
    l.sbits = o;
    o += up((size_t)R * 2 * wpc * 4);
    l.jbits = o;
    o += up((size_t)3 * 2 * wpc * 4);
    l.bytes = o;
    return l;
}

hipError_t launch_ea_prepare(unsigned char* ws, const EaLayout& lay, int R, int64_t n, int mode,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_ea_prepare, dim3(1), dim3(256), 0, st, ws, lay, R, n, mode);
    return hipGetLastError();
}

hipError_t launch_ea_init(unsigned char* ws, int8_t* spins, int L, int R, int start, Key key,
                          hipStream_t st) {
    const int64_t words = (int64_t)L * L * L / 4;
    hipLaunchKernelGGL(k_ea_init, dim3((unsigned)(R * ((words + 255) / 256))), dim3(256), 0, st, ws,
                       spins, L, R, start, key);
    return hipGetLastError();
}

hipError_t launch_ea_energy(unsigned char* ws, const int8_t* spins, const int8_t* bonds, int L,
                            int R, long long* out, hipStream_t st) {
    const int64_t N = (int64_t)L * L * L;
    hipLaunchKernelGGL(k_ea_fill, dim3((R + 255) / 256), dim3(256), 0, st, out, R);
    hipLaunchKernelGGL(k_ea_energy, dim3((unsigned)(R * ((N + 255) / 256))), dim3(256), 0, st, ws,
                       spins, bonds, L, R, out);
    return hipGetLastError();
}

hipError_t launch_ea_sweep(unsigned char* ws, const EaLayout& lay, int8_t* spins,
                           const int8_t* bonds, int L, int R, int every, Key key, int64_t* trace,
                           hipStream_t st) {
    int lgL = 0;
    while ((1 << lgL) < L)
        ++lgL;
    for (int c = 0; c < 2; ++c)
        hipLaunchKernelGGL(k_ea_halfsweep, dim3((unsigned)lay.plane_blocks, (unsigned)L, (unsigned)R),
                           dim3(256), 0, st, ws, lay, spins, bonds, lgL, R, c, key);
    hipLaunchKernelGGL(k_ea_reduce, dim3(R), dim3(256), 0, st, ws, lay, R, lay.bpr, trace);
    hipLaunchKernelGGL(k_ea_exchange, dim3(1), dim3(512), 0, st, ws, lay, R, every, key);
    return hipGetLastError();
}

namespace {
int log2_of(int L) {
    int lg = 0;
    while ((1 << lg) < L)
        ++lg;
    return lg;
}
}  // namespace

hipError_t launch_ea_pack_bonds(unsigned char* ws, const EaLayout& lay, const int8_t* bonds, int L,
                                hipStream_t st) {
    const unsigned blocks = (unsigned)((((size_t)L * L * L / 64) + 255) / 256);
    hipLaunchKernelGGL(k_ea_pack_bonds, dim3(blocks, 3), dim3(256), 0, st,
                       reinterpret_cast<uint32_t*>(ws + lay.jbits), bonds, log2_of(L));
    return hipGetLastError();
}

hipError_t launch_ea_pack_spins(unsigned char* ws, const EaLayout& lay, const int8_t* spins, int L,
                                int R, hipStream_t st) {
    hipLaunchKernelGGL(k_ea_pack_spins, dim3((unsigned)lay.bpr_bit, (unsigned)R), dim3(256), 0, st,
                       reinterpret_cast<uint32_t*>(ws + lay.sbits), spins, log2_of(L), R);
    return hipGetLastError();
}

hipError_t launch_ea_unpack_spins(unsigned char* ws, const EaLayout& lay, int8_t* spins, int L,
                                  int R, hipStream_t st) {
    hipLaunchKernelGGL(k_ea_unpack_spins, dim3((unsigned)lay.bpr_bit, (unsigned)R), dim3(256), 0,
                       st, spins, reinterpret_cast<const uint32_t*>(ws + lay.sbits), log2_of(L), R);
    return hipGetLastError();
}

hipError_t launch_ea_sweep_bit(unsigned char* ws, const EaLayout& lay, int L, int R, int every,
                               Key key, int64_t* trace, hipStream_t st) {
    const int lgL = log2_of(L);
    for (int c = 0; c < 2; ++c)
        hipLaunchKernelGGL(k_ea_halfsweep_bit, dim3((unsigned)(lay.bpr_bit / kEaWordsPerThread * R)),
                           dim3(256), 0, st, ws, lay, lgL, R, c, key);
    hipLaunchKernelGGL(k_ea_reduce, dim3(R), dim3(256), 0, st, ws, lay, R,
                       lay.bpr_bit / kEaWordsPerThread, trace);
    hipLaunchKernelGGL(k_ea_exchange, dim3(1), dim3(512), 0, st, ws, lay, R, every, key);
    return hipGetLastError();
}

}  // namespace ising
