// Kernels of the learned whole-lattice proposal: the masked-convolution
// autoregressive network (training: forward, backward, Adam; the wavefront
// sampler; log q of given configurations, a whole lattice at a time) and
// the Metropolis-Hastings acceptance of whole-lattice proposals.
//
// The network's parameters are bfloat16; the kernels read the float32
// expansion of those bfloat16 values (`wexp`, exactly the same numbers) and
// accumulate in float32.
#include "nn.hpp"

namespace ising {

namespace {

constexpr int C = kNNChannels;
constexpr int NTB = 5;  // taps of mask B; mask A is its first four
// (dy, dx) of the taps: above-left, above, above-right, left, centre
__device__ __forceinline__ int tap_dy(int t) { return t < 3 ? -1 : 0; }
__device__ __forceinline__ int tap_dx(int t) { return t < 3 ? t - 1 : (t == 3 ? -1 : 0); }

struct NNOff {
    static constexpr int W1 = 0, B1 = W1 + C * 4;
    static constexpr int W2 = B1 + C, B2 = W2 + C * C * NTB;
    static constexpr int W3 = B2 + C, B3 = W3 + C * C * NTB;
    static constexpr int W4 = B3 + C, B4 = W4 + C * NTB;
    static constexpr int P = B4 + 1;
};
static_assert(NNOff::P == 2753, "parameter layout");

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round to nearest even (finite inputs; NaN is kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu))
        return (uint16_t)((u >> 16) | 0x40u);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

__device__ __forceinline__ float log_sigmoid(float v) {
    // log(1 / (1 + e^-v)) = -(max(-v, 0) + log1p(e^-|v|))
    return -(fmaxf(-v, 0.f) + log1pf(expf(-fabsf(v))));
}

__global__ void k_nn_round(const float* master, uint16_t* w, float* wexp, int P) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) {
        const uint16_t h = f32_to_bf16(master[i]);
        w[i] = h;
        wexp[i] = bf16_to_f32(h);
    }
}

__global__ void k_nn_adam(float* master, float* m, float* v, const float* g, uint16_t* w,
                          float* wexp, int P, float lr, float b1, float b2, float eps, float c1,
                          float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float x = master[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    master[i] = x;
    const uint16_t h = f32_to_bf16(x);
    w[i] = h;
    wexp[i] = bf16_to_f32(h);
}

// Wavefront evaluation of the network, for sampling and for log q (which
// k_nn_lattice computes instead, with the same bits, up to L = 32).
//
// The factorisation is over sites in raster order, and the logits of site
// (y, x) depend on the sites whose activations its taps read: (y-1, x-1),
// (y-1, x), (y-1, x+1), (y, x-1) and, above layer 1, (y, x) itself.  All
// of these lie on earlier anti-diagonals t = x + 2y, so the sites of one
// anti-diagonal (at most ceil(L/2), one per row) are evaluated together,
// 3L - 2 steps instead of L^2, and the draws and results are those of the
// site-by-site order.
//
// One wave per configuration and sign.  Lane l = m + 16 kk serves site
// slot m of each 16-slot tile and, of that site, channels 4 kk .. 4 kk + 3.
// Each layer is a set of products D[out channel][site] = sum_k A[out
// channel][k] B[k][site] on the matrix cores, with the sites of a tile as
// the 16 columns.  Layer 1 (four mask-A taps of +-1 spins) is one float32
// product v_mfma_f32_16x16x4_f32, exact.  Layers 2, 3 and 4 take one
// bfloat16 product v_mfma_f32_16x16x32_bf16 per mask-B tap, with float32
// accumulation: the weights are bfloat16 already; each float32 activation
// a enters as two bfloat16 terms, hi = bf16(a) and lo = bf16(a - hi), both
// against the same weight, so that the products see a to within 2^-17 of
// it (the network's float32 arithmetic to well within the log q tolerance,
// where bfloat16 activations alone would not be).  The K = 32 of a tap are
// its 16 channels x the two terms, ordered so that lane (m, kk) supplies
// the hi and lo terms of channels 4 kk .. 4 kk + 3: exactly what the lane
// holds of its own site after the previous layer.  The centre tap thus
// passes from layer to layer in registers, and only the four taps on
// earlier anti-diagonals read LDS, all at the start of a step.  Layer 4 (one
// output) has its weights in every row, so that every lane of a site
// receives its z.
// Activations live in LDS for only four columns (x mod 4): a row reads the
// row above at x-1..x+1 while that row writes x+2.  A site keeps 64 bytes,
// [hi of channels 4c..4c+3, lo of the same] for c = 0..3, which its four
// lanes write with one 16-byte store each at the end of the step.  Rows
// share R = floor((L+1)/2) + 1 ring entries: row y + R starts after row
// y + 1 has read the last columns of row y.  The ring is stored as four
// planes, one per lane group kk, each [layer][column][ring row] of 16
// bytes: the 16 lanes of a group serve consecutive rows, whose entries are
// then 16 bytes apart in one column, and the columns of neighbouring rows
// (x and x - 2) are 2 (R + 2) entries apart, an even number, so that the
// lanes' 16-byte pieces fall on distinct banks.  Each column has two rows
// past the ring: row R is zero (read for taps outside the lattice) and row
// R + 1 takes the writes of idle slots, so that every layer's access is
// one offset from the layer-0 one.  The spins use row stride L + 3
// for the same reason (rows one apart, columns two apart: 33 words at
// L = 32).  The draws do not depend on the network, so in sampling mode up
// to L = 32 all of them are taken before the first step, into a table of
// one 32-bit uniform per site after the rings (predraw).
//
// With `symmetric`, a second wave evaluates the negated configuration in
// step with the first, and the result is log q_sym = log((q(s) + q(-s)) / 2).
// Each wave adds its log-likelihood terms after the per-step barrier, in
// the same order in every mode, so that sampling and teacher-forced
// evaluation of the same configuration give the same bits.

struct WaveSlot {
    int y, x;
    bool on;
};

// Row slot s (0 <= s < S, S a power of two >= ceil(L/2)) at step t: the
// active row congruent to s mod S, if any.
__device__ __forceinline__ WaveSlot wave_slot(int s, int t, int L, int S) {
    int ylo = (t - L + 2) >> 1;  // ceil((t - L + 1) / 2)
    ylo = ylo < 0 ? 0 : ylo;
    const int yhi = (t >> 1) < L - 1 ? (t >> 1) : L - 1;
    WaveSlot r;
    r.y = ylo + ((s - ylo) & (S - 1));
    r.x = t - 2 * r.y;
    r.on = r.y <= yhi;
    return r;
}

constexpr int kSiteBytes = 64;  // 16 channels x (bf16 hi + bf16 lo)

// Byte offset of ring row ry, column c of layer 0 in a plane of 3 layers x
// 4 columns x Rp = R + 2 rows (24-bit products: full-rate multiplies).
__device__ __forceinline__ int ring_at(int Rp, int ry, int c) { return (__mul24(c, Rp) + ry) * 16; }

// log sigmoid(v) = -(max(-v, 0) + log1p(e^-|v|)), with log1p(e) taken as
// log(u) - ((u - 1) - e) / u for u = 1 + e (the rounding of u corrected
// to first order) on the hardware exp and log.
__device__ __forceinline__ float log_sigmoid_hw(float v) {
    const float e = __expf(-fabsf(v));
    const float u = 1.f + e;
    return -(fmaxf(-v, 0.f) + (__logf(u) - __fdividef((u - 1.f) - e, u)));
}

// Two float32 values rounded to bfloat16 (nearest even), packed: the first
// in the low half.
__device__ __forceinline__ uint32_t bf16_pair(float x, float y) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2{x, y}, bf16x2));
}

// The four float32 activations of this lane's channels as the operand of
// the next layer's centre tap: their hi terms hi = bf16(a), then their lo
// terms bf16(a - hi) (a - hi is exact in float32).
__device__ __forceinline__ bf16x8 act_terms(const f4& a) {
    bf16x8 r;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        r[v] = (__bf16)a[v];
        r[4 + v] = (__bf16)(a[v] - (float)r[v]);
    }
    return r;
}

// The same terms, two values per conversion, hi read back from the packed
// bits: fewer instructions where many sites are converted at once.
__device__ __forceinline__ bf16x8 act_terms_pk(const f4& a) {
    const uint32_t h01 = bf16_pair(a[0], a[1]), h23 = bf16_pair(a[2], a[3]);
    const uint32_t l01 = bf16_pair(a[0] - __uint_as_float(h01 << 16),
                                   a[1] - __uint_as_float(h01 & 0xFFFF0000u));
    const uint32_t l23 = bf16_pair(a[2] - __uint_as_float(h23 << 16),
                                   a[3] - __uint_as_float(h23 & 0xFFFF0000u));
    return __builtin_bit_cast(bf16x8, uint4{h01, h23, l01, l23});
}

// Operand A of tap t of a mask-B layer (weights at wo) for lane (m, kk):
// row co = m (every row the single output with kOut1), elements e = 0..7
// the weight of channel 4 kk + (e & 3), once for the hi and once for the
// lo term.
template <bool kOut1>
__device__ __forceinline__ bf16x8 weights_tap(const float* wexp, int wo, int m, int kk, int t) {
    bf16x8 a;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int ci = 4 * kk + (e & 3);
        a[e] = (__bf16)(kOut1 ? wexp[wo + ci * NTB + t] : wexp[wo + (m * C + ci) * NTB + t]);
    }
    return a;
}

template <int T>
__global__ void __launch_bounds__(128) k_nn_wave(const float* __restrict__ wexp, int L, int sample,
                                                 int predraw, int symmetric, const int8_t* s_in,
                                                 int64_t in_stride, Key key, uint32_t chain0,
                                                 uint32_t draw, int8_t* s_out, int64_t out_stride,
                                                 float* logq_out) {
    extern __shared__ __align__(16) float sh[];  // 16-byte accesses of eight bfloat16 terms
    __shared__ float red[2];
    constexpr int S = 16 * T;
    const int W2 = L + 3, R = (L + 1) / 2 + 1, Rp = R + 2;
    const int sb_floats = (L * W2 + 3) & ~3;
    const int layer_step = Rp * 4 * 16;  // one layer within a plane
    const int plane = 3 * layer_step;    // one lane group's plane
    float* sb = sh;  // [L][L + 3] spins as +-1.0 (unsigned), zero columns 0, L + 1, L + 2
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int m = lane & 15, kk = lane >> 4;
    // per wave: the four planes of its ring; this lane's plane, and its
    // zero and junk entries (column 0 of layer 0)
    char* act = reinterpret_cast<char*>(sh + sb_floats) + w * (4 * plane) + kk * plane;
    const int zero_off = R * 16, junk_off = (R + 1) * 16;
    // with predraw, every site's uniform draw, taken before the first step
    uint32_t* ru = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(sh + sb_floats) +
                                               (blockDim.x >> 6) * (4 * plane));
    const float sigma = w == 0 ? 1.f : -1.f;
    const int b = blockIdx.x;
    for (int i = threadIdx.x; i < sb_floats; i += blockDim.x) {
        float v = 0.f;
        const int y = i / W2, xc = i - y * W2;
        if (!sample && y < L && xc >= 1 && xc <= L)
            v = (float)s_in[(int64_t)b * in_stride + y * L + xc - 1];
        sb[i] = v;
    }
    // the zero row of each layer, in each lane group's plane
    if (m == 0)
        for (int l = 0; l < 3; ++l)
            *reinterpret_cast<f4*>(act + zero_off + l * layer_step) = f4{0.f, 0.f, 0.f, 0.f};
    // matrix-core operands A: row co = m of every product
    const float wa1 = wexp[NNOff::W1 + m * 4 + kk];
    bf16x8 wa2[NTB], wa3[NTB], wa4[NTB];
#pragma unroll
    for (int t = 0; t < NTB; ++t) {
        wa2[t] = weights_tap<false>(wexp, NNOff::W2, m, kk, t);
        wa3[t] = weights_tap<false>(wexp, NNOff::W3, m, kk, t);
        wa4[t] = weights_tap<true>(wexp, NNOff::W4, m, kk, t);
    }
    f4 bias1, bias2, bias3;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        bias1[v] = wexp[NNOff::B1 + 4 * kk + v];
        bias2[v] = wexp[NNOff::B2 + 4 * kk + v];
        bias3[v] = wexp[NNOff::B3 + 4 * kk + v];
    }
    const float bias4 = wexp[NNOff::B4];
    const RoundKeys rk = round_keys(key);
    const uint32_t chain = chain0 + (uint32_t)b;
    // symmetric sampling writes the configuration negated with probability 1/2
    float out_sign = 1.f;
    if (sample && symmetric) {
        const U4 o = philox4x32_10({0xFFFFFFFFu, chain, draw, kTagNNSample}, rk);
        out_sign = (o.x >> 31) ? -1.f : 1.f;
    }
    // the draws do not depend on the network: with predraw they are all
    // taken here, off the steps' critical path (block j serves sites 4j..4j+3)
    if (predraw)
        for (int j = threadIdx.x; 4 * j < L * L; j += blockDim.x) {
            const U4 o = philox4x32_10({(uint32_t)j, chain, draw, kTagNNSample}, rk);
            ru[4 * j] = o.x;
            ru[4 * j + 1] = o.y;
            ru[4 * j + 2] = o.z;
            ru[4 * j + 3] = o.w;
        }
    __syncthreads();
    float lq[T];
#pragma unroll
    for (int u = 0; u < T; ++u)
        lq[u] = 0.f;
    const f4 zero4 = {0.f, 0.f, 0.f, 0.f};
    const int steps = 3 * L - 2;
    for (int t = 0; t < steps; ++t) {
        // Geometry of the step, per tile: this lane's site, the LDS byte
        // offsets of its part of the four earlier taps (zero site outside
        // the lattice or for an idle slot) and of its own part, its layer-1
        // input (tap kk of mask A) and its spin.
        WaveSlot g[T];
        int nb[T][4], own[T], spin_in[T], spin_at[T];
#pragma unroll
        for (int u = 0; u < T; ++u) {
            g[u] = wave_slot(16 * u + m, t, L, S);
            const int y = g[u].y, x = g[u].x;
            // ring rows of y and y - 1 (y < L < 2R); columns of x - 1, x, x + 1
            const int ry = y < R ? y : y - R, ryu = y - 1 < R ? y - 1 : y - 1 - R;
            const int cl = (x - 1) & 3, cm = x & 3, cr = (x + 1) & 3;
            const bool up = g[u].on && y > 0, lf = x > 0, rt = x + 1 < L;
            // the four earlier taps: (-1, -1), (-1, 0), (-1, +1), (0, -1)
            nb[u][0] = up && lf ? ring_at(Rp, ryu, cl) : zero_off;
            nb[u][1] = up ? ring_at(Rp, ryu, cm) : zero_off;
            nb[u][2] = up && rt ? ring_at(Rp, ryu, cr) : zero_off;
            nb[u][3] = g[u].on && lf ? ring_at(Rp, ry, cl) : zero_off;
            own[u] = g[u].on ? ring_at(Rp, ry, cm) : junk_off;
            // index 0 is the zero column of row 0
            const int dy = kk < 3 ? -1 : 0, dx = kk < 3 ? kk - 1 : -1;
            const bool ok = g[u].on && y + dy >= 0;
            spin_in[u] = ok ? __mul24(y + dy, W2) + x + dx + 1 : 0;
            spin_at[u] = g[u].on ? __mul24(y, W2) + x + 1 : 0;
        }
        // the sampling draws of the step do not depend on z: taken first,
        // they overlap the products' latency
        uint32_t r[T];
        if (sample && w == 0) {
#pragma unroll
            for (int u = 0; u < T; ++u) {
                const int i = __mul24(g[u].y, L) + g[u].x;
                if (predraw) {
                    r[u] = ru[g[u].on ? i : 0];
                } else {
                    const U4 o = philox4x32_10({(uint32_t)(i >> 2), chain, draw, kTagNNSample}, rk);
                    r[u] = u4_get(o, i & 3);
                }
            }
        }
        // every LDS read of the step, before any of its writes: layer-1
        // inputs and the earlier taps of layers 2, 3 and 4
        float sp_in[T];
        bf16x8 ta[T][3][4];
#pragma unroll
        for (int u = 0; u < T; ++u) {
            sp_in[u] = sb[spin_in[u]];
#pragma unroll
            for (int l = 0; l < 3; ++l)
#pragma unroll
                for (int tp = 0; tp < 4; ++tp)
                    ta[u][l][tp] = *reinterpret_cast<const bf16x8*>(act + nb[u][tp] + l * layer_step);
        }
        bf16x8 outs[T][3];
        float z[T];
#pragma unroll
        for (int u = 0; u < T; ++u) {
            // layer 1 (mask A): B[k = kk][site m] is tap kk of site m
            f4 acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wa1, sigma * sp_in[u], zero4, 0, 0, 0);
            f4 a;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                a[v] = fmaxf(acc[v] + bias1[v], 0.f);
            outs[u][0] = act_terms(a);
            // layers 2 and 3: the earlier taps first, the centre tap (this
            // lane's own output of the layer below) last
#pragma unroll
            for (int l = 1; l < 3; ++l) {
                const bf16x8* wl = l == 1 ? wa2 : wa3;
                acc = zero4;
#pragma unroll
                for (int tp = 0; tp < 4; ++tp)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl[tp], ta[u][l - 1][tp], acc, 0,
                                                                  0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl[4], outs[u][l - 1], acc, 0, 0, 0);
                const f4 bl = l == 1 ? bias2 : bias3;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    a[v] = fmaxf(acc[v] + bl[v], 0.f);
                outs[u][l] = act_terms(a);
            }
            // layer 4: every row holds z of the column's site
            acc = zero4;
#pragma unroll
            for (int tp = 0; tp < 4; ++tp)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa4[tp], ta[u][2][tp], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa4[4], outs[u][2], acc, 0, 0, 0);
            z[u] = acc[0] + bias4;
        }
        if (sample && w == 0) {
#pragma unroll
            for (int u = 0; u < T; ++u) {
                if (g[u].on) {
                    const float pplus = 1.f / (1.f + expf(-z[u]));
                    const float sp = ((double)r[u] < (double)pplus * 4294967296.0) ? 1.f : -1.f;
                    if (kk == 0) {
                        sb[spin_at[u]] = sp;
                        s_out[(int64_t)b * out_stride + g[u].y * L + g[u].x] =
                            (int8_t)(out_sign * sp);
                    }
                }
            }
        }
        // this step's activations, for the taps of later steps
#pragma unroll
        for (int u = 0; u < T; ++u)
#pragma unroll
            for (int l = 0; l < 3; ++l)
                *reinterpret_cast<bf16x8*>(act + own[u] + l * layer_step) = outs[u][l];
        if (sample) {
            // the second wave reads the spins the first one drew
            __syncthreads();
        } else {
            // the spins are inputs and each wave has its own ring: the
            // waves need not wait for each other
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const float term = log_sigmoid_hw(sigma * sb[spin_at[u]] * z[u]);
            lq[u] += g[u].on ? term : 0.f;
        }
    }
    float tot = lq[0];
#pragma unroll
    for (int u = 1; u < T; ++u)
        tot += lq[u];
#pragma unroll
    for (int off = 1; off < 16; off <<= 1)
        tot += __shfl_xor(tot, off, 64);
    if (lane == 0)
        red[w] = tot;
    __syncthreads();
    if (threadIdx.x == 0 && logq_out) {
        float r = red[0];
        if (symmetric) {
            const float x = red[0], y = red[1];
            r = fmaxf(x, y) + log1pf(expf(-fabsf(x - y))) - 0.69314718055994531f;
        }
        logq_out[b] = r;
    }
}

// Teacher-forced log q of configurations that fit in LDS whole (L <= 32).
//
// With every spin given, nothing orders the sites: each layer is computed
// for the whole lattice at once and its activations go to LDS for the taps
// of the next layer.  The per-site arithmetic is k_nn_wave's: the same
// operands in the same lanes, the same products in the same order (earlier
// taps, then the centre tap from registers) and the same rounding of the
// activations into hi and lo terms.  The log-likelihood terms are added in
// k_nn_wave's order too: for L <= 32 the wavefront gives row slot s the
// rows s and s + 16, summed in raster order from zero, and combines the 16
// slots by a butterfly.  Here lane s (one sign) or s + 16 (the other) of
// the first wave adds its slot's terms in that order, and the butterfly is
// the same.  The result is therefore bitwise the wavefront's, and the
// sampler's log q of a proposal is the one this kernel gives it.
//
// Wave w computes rows w and w + 16 as tiles of 16 columns (x0 = 0, 16):
// kT = 4 tiles for L > 16, one for L <= 16.  A tile past the lattice (rows
// w + 16 >= L) runs like the others on a harmless site and writes nothing,
// so that a wave's tiles are straight-line code whose products and LDS
// accesses interleave.  Grids in LDS carry a zero border, so that every
// tap is one fixed offset from its site: row stride L + 1, a zero row above
// row 0 and a zero column 0 that also serves as column L of the row above.
// The spins are floats on such a grid; an activation buffer is four planes
// (one per lane group kk: the hi and lo terms of channels 4 kk .. 4 kk + 3,
// 16 bytes per site) of such grids, so that the 16 lanes of a group access
// consecutive bytes, each plane padded to a multiple of kLatticePlaneAlign
// bytes.  The first sign runs layer 1 -> A, 2 -> B, 3 -> A, 4 from A, the
// second the other way round, so that its layer 1 may start while slower
// waves still read A.  The weights of layers 2-4 are kept as bfloat16
// [layer][tap][out][in] (layer 4: [tap][in]).  About 160 KB at L = 32: one
// workgroup per CU, persistent over the batch, each configuration's spins
// fetched into registers while the one before is evaluated.
constexpr int kLatticePrefetch = 2;  // spins per thread: (L + 1)^2 <= 2 x 64 min(L, 16)
constexpr int kLatticePlaneAlign = 256;

// Row stride of the terms: a multiple of 4 floats past L (16-byte rows whose
// padding reads as zeros), plus 4 to spread the rows over the banks.
__host__ __device__ inline int lattice_term_stride(int L) { return ((L + 3) & ~3) + 4; }

struct LatticeLds {
    int grid;   // (L + 1)^2 entries per grid
    int plane;  // bytes of one plane of an activation buffer
    int wts;    // byte offsets: bfloat16 weights of layers 2-4
    int par;    // float [64] layer-1 weights in lane order, [3][16] biases, bias of layer 4
    int buf[2];
    int junk;
    int terms;  // float [2 signs][L][lattice_term_stride(L)]
    int bytes;
};
__host__ __device__ inline LatticeLds lattice_lds(int L) {
    LatticeLds d;
    d.grid = (L + 1) * (L + 1);
    d.plane = (16 * d.grid + kLatticePlaneAlign - 1) / kLatticePlaneAlign * kLatticePlaneAlign;
    d.wts = (d.grid * 4 + 15) & ~15;  // the spins first
    d.par = d.wts + (2 * NTB * C * C + NTB * C) * 2;
    d.buf[0] = (d.par + (64 + 3 * C + 4) * 4 + kLatticePlaneAlign - 1) / kLatticePlaneAlign *
               kLatticePlaneAlign;
    d.buf[1] = d.buf[0] + 4 * d.plane;
    d.junk = d.buf[1] + 4 * d.plane;
    d.terms = d.junk + kSiteBytes;
    d.bytes = d.terms + 2 * L * lattice_term_stride(L) * 4;
    return d;
}

template <int kT>
__global__ void __launch_bounds__(1024) k_nn_lattice(const float* __restrict__ wexp, int L, int B,
                                                     int symmetric, const int8_t* __restrict__ s_in,
                                                     int64_t in_stride, float* __restrict__ logq_out) {
    extern __shared__ __align__(16) float sh[];
    const LatticeLds d = lattice_lds(L);
    const int L1 = L + 1, RS = lattice_term_stride(L);
    char* base = reinterpret_cast<char*>(sh);
    float* sb = sh;  // spins as +-1.0 (unsigned) on the bordered grid
    uint16_t* wts = reinterpret_cast<uint16_t*>(base + d.wts);
    float* par = reinterpret_cast<float*>(base + d.par);
    float* terms = reinterpret_cast<float*>(base + d.terms);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int m = lane & 15, kk = lane >> 4;
    // bfloat16 weights (exact: wexp holds bfloat16 values)
    for (int i = threadIdx.x; i < 2 * NTB * C * C + NTB * C; i += blockDim.x) {
        float v;
        if (i < 2 * NTB * C * C) {
            const int l = i / (NTB * C * C), t = (i / (C * C)) % NTB, co = (i / C) % C, ci = i % C;
            v = wexp[(l == 0 ? NNOff::W2 : NNOff::W3) + (co * C + ci) * NTB + t];
        } else {
            const int j = i - 2 * NTB * C * C, t = j / C, ci = j % C;
            v = wexp[NNOff::W4 + ci * NTB + t];
        }
        wts[i] = (uint16_t)(__float_as_uint(v) >> 16);
    }
    // operand A of layer 1 for lane (m, kk), then the biases of layers 1-4
    for (int i = threadIdx.x; i < 64 + 3 * C + 1; i += blockDim.x)
        par[i] = i < 64 ? wexp[NNOff::W1 + (i & 15) * 4 + (i >> 4)]
                 : i < 64 + 3 * C
                     ? wexp[(i < 64 + C ? NNOff::B1 : i < 64 + 2 * C ? NNOff::B2 : NNOff::B3) +
                            (i - 64) % C]
                     : wexp[NNOff::B4];
    // the borders of every plane of both buffers, and the term padding
    for (int i = threadIdx.x; i < 8 * (2 * L + 1); i += blockDim.x) {
        const int p = i / (2 * L + 1), j = i % (2 * L + 1);
        const int q = j <= L ? j : (j - L) * L1;
        *reinterpret_cast<f4*>(base + ((p >> 2) ? d.buf[1] : d.buf[0]) + (p & 3) * d.plane +
                               16 * q) = f4{0.f, 0.f, 0.f, 0.f};
    }
    for (int i = threadIdx.x; i < 2 * L * RS; i += blockDim.x)
        terms[i] = 0.f;
    // Tile i of wave w: row sy(i) = w + 16 (i >> 1), columns 16 (i & 1) + m.
    // Grid index of this lane's site, or of the last site where there is
    // none (its reads then stay inside the grid and its writes go to junk).
    bool on[kT];
    int q[kT];
#pragma unroll
    for (int i = 0; i < kT; ++i) {
        const int y = w + 16 * (i >> 1), x = 16 * (i & 1) + m;
        on[i] = y < L && x < L;
        q[i] = on[i] ? (y + 1) * L1 + x + 1 : d.grid - 1;
    }
    // tap kk of mask A, and the four earlier taps of mask B, as offsets
    const int qa = kk < 3 ? -L1 + kk - 1 : -1;
    // spins of the next configuration, fetched a configuration ahead
    float pre[kLatticePrefetch];
    auto fetch = [&](int b) {
#pragma unroll
        for (int k = 0; k < kLatticePrefetch; ++k) {
            const int i = threadIdx.x + k * blockDim.x;
            const int y = i / L1 - 1, x = i % L1 - 1;
            pre[k] = b < B && i < d.grid && y >= 0 && x >= 0
                         ? (float)s_in[(int64_t)b * in_stride + y * L + x]
                         : 0.f;
        }
    };
    fetch(blockIdx.x);
    const f4 zero4 = {0.f, 0.f, 0.f, 0.f};
    const int signs = symmetric ? 2 : 1;
    const int pk = kk * d.plane;
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
#pragma unroll
        for (int k = 0; k < kLatticePrefetch; ++k) {
            const int i = threadIdx.x + k * blockDim.x;
            if (i < d.grid)
                sb[i] = pre[k];
        }
        fetch(b + gridDim.x);
        __syncthreads();
        for (int sg = 0; sg < signs; ++sg) {
            const float sigma = sg == 0 ? 1.f : -1.f;
            const int bA = sg == 0 ? d.buf[0] : d.buf[1], bB = sg == 0 ? d.buf[1] : d.buf[0];
            bf16x8 prev[kT];
            // layer 1 (mask A)
            const float wa1 = par[lane];
            const f4 bias1 = *reinterpret_cast<const f4*>(par + 64 + 4 * kk);
#pragma unroll
            for (int i = 0; i < kT; ++i) {
                const float sp = sb[on[i] ? q[i] + qa : 0];
                const f4 acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wa1, sigma * sp, zero4, 0, 0, 0);
                f4 a;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    a[v] = fmaxf(acc[v] + bias1[v], 0.f);
                prev[i] = act_terms_pk(a);
                *reinterpret_cast<bf16x8*>(base + (on[i] ? bA + pk + 16 * q[i] : d.junk)) = prev[i];
            }
            __syncthreads();
            // layers 2, 3 and 4 (mask B): the four earlier taps from the
            // buffer the layer below wrote, the centre tap from registers
#pragma unroll
            for (int l = 1; l < 4; ++l) {
                const int in_off = ((l & 1) ? bA : bB) + pk, out_off = ((l & 1) ? bB : bA) + pk;
                // operand A of tap t: weights of channels 4 kk .. 4 kk + 3
                // for output m (layer 4: its one output), once for the hi
                // and once for the lo terms
                bf16x8 wl[NTB];
#pragma unroll
                for (int t = 0; t < NTB; ++t) {
                    const int o = l < 3 ? (((l - 1) * NTB + t) * C + m) * C + 4 * kk
                                        : 2 * NTB * C * C + t * C + 4 * kk;
                    const uint2 u = *reinterpret_cast<const uint2*>(wts + o);
                    wl[t] = __builtin_bit_cast(bf16x8, uint4{u.x, u.y, u.x, u.y});
                }
                const f4 bl = *reinterpret_cast<const f4*>(par + 64 + (l < 3 ? l : 0) * C + 4 * kk);
                const float bias4 = par[64 + 3 * C];
#pragma unroll
                for (int i = 0; i < kT; ++i) {
                    bf16x8 ta[4];
#pragma unroll
                    for (int tp = 0; tp < 4; ++tp)
                        ta[tp] = *reinterpret_cast<const bf16x8*>(
                            base + in_off + 16 * (q[i] + tap_dy(tp) * L1 + tap_dx(tp)));
                    f4 acc = zero4;
#pragma unroll
                    for (int tp = 0; tp < 4; ++tp)
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl[tp], ta[tp], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl[4], prev[i], acc, 0, 0, 0);
                    if (l < 3) {
                        f4 a;
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            a[v] = fmaxf(acc[v] + bl[v], 0.f);
                        prev[i] = act_terms_pk(a);
                        *reinterpret_cast<bf16x8*>(base + (on[i] ? out_off + 16 * q[i] : d.junk)) =
                            prev[i];
                    } else {
                        const float z = acc[0] + bias4;
                        const float t = log_sigmoid_hw(sigma * sb[q[i]] * z);
                        if (on[i] && kk == 0)
                            terms[(sg * L + w + 16 * (i >> 1)) * RS + 16 * (i & 1) + m] = t;
                    }
                }
                if (l < 3)
                    __syncthreads();
            }
        }
        __syncthreads();
        // lane s + 16 sg of the first wave: slot s of sign sg, its rows in
        // raster order (the padding adds zeros), then the butterfly
        if (w == 0) {
            float tot = 0.f;
            if (lane < 32)
                for (int y = lane & 15; y < L; y += 16) {
                    const f4* row = reinterpret_cast<const f4*>(terms + ((lane >> 4) * L + y) * RS);
                    for (int x4 = 0; x4 < (L + 3) / 4; ++x4) {
                        const f4 v = row[x4];
                        tot += v[0];
                        tot += v[1];
                        tot += v[2];
                        tot += v[3];
                    }
                }
#pragma unroll
            for (int off = 1; off < 16; off <<= 1)
                tot += __shfl_xor(tot, off, 64);
            const float r1 = __shfl(tot, 16, 64);
            if (lane == 0 && logq_out) {
                float r = tot;
                if (symmetric) {
                    const float x = tot, y = r1;
                    r = fmaxf(x, y) + log1pf(expf(-fabsf(x - y))) - 0.69314718055994531f;
                }
                logq_out[b] = r;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Training: forward and backward passes over a batch of B configurations.
//
// Activations and their gradients live in the workspace as float32
// [B][N][C]: the 16 channels of a site are 64 contiguous bytes, and the
// flattened site index e = b N + p runs over the whole batch.  The
// convolutions of layers 2 and 3 and their transposes run on the matrix
// cores as in the sampler, with 16 consecutive sites as the columns of a
// tile: D[out channel][site] = sum_k A[out channel][k] B[k][site] over
// k = (tap, in channel), A the bfloat16 weights and B the three bfloat16
// terms that sum exactly to each float32 activation or gradient.  The weight gradients
// contract over sites, where neither operand is bfloat16: they use the
// float32 product v_mfma_f32_16x16x4_f32 (four sites per product, exact
// products, float32 accumulation).
// ---------------------------------------------------------------------------

constexpr int kTile = 16;  // sites per matrix-core tile

// Operand A of the products of a mask-B layer (weights at wo) for lane
// (m, kk): row = output channel m; product j, elements e = 0..7 are
// k = 32 j + 8 kk + e, i.e. channel 8 (kk & 1) + e of tap 2 j + (kk >> 1)
// (zero past the fifth tap).
__device__ __forceinline__ bf16x8 weights_b(const float* wexp, int wo, int m, int kk, int j) {
    bf16x8 b;
    const int tap = 2 * j + (kk >> 1);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int ci = 8 * (kk & 1) + e;
        // exact: the values are bfloat16 already
        b[e] = (__bf16)(tap < NTB ? wexp[wo + (m * C + ci) * NTB + tap] : 0.f);
    }
    return b;
}

struct TSite {
    int y, x;
};
// Row and column of flattened site e.
__device__ __forceinline__ TSite tsite(int e, int N, int L) {
    const int p = e % N;
    const int y = p / L;
    return {y, p - y * L};
}
__device__ __forceinline__ bool tinside(const TSite& q, int L, int dy, int dx) {
    return (unsigned)(q.y + dy) < (unsigned)L && (unsigned)(q.x + dx) < (unsigned)L;
}

// A lane's site in a contiguous run of sites: flattened index e = b N + p,
// row y and column x of p.  Divides once, at the start of the run.
struct RunSite {
    int e, b, p, y, x;
    __device__ __forceinline__ void start(int e0, int N, int L) {
        e = e0;
        b = e0 / N;
        p = e0 - b * N;
        y = p / L;
        x = p - y * L;
    }
    __device__ __forceinline__ void advance(int k, int N, int L) {
        e += k;
        p += k;
        x += k;
        while (x >= L) {
            x -= L;
            if (++y == L) {
                y = 0;
                p -= N;
                ++b;
            }
        }
    }
    // Whether the neighbour (y + dy, x + dx) of tap t of mask B exists,
    // from the three edge flags; tap 5 (padding) never does.
    __device__ __forceinline__ bool tap_ok(int t, int L) const {
        const bool up = y > 0, left = x > 0, right = x < L - 1;
        return t == 0 ? up && left : t == 1 ? up : t == 2 ? up && right : t == 3 ? left : t == 4;
    }
    // The same for the neighbour (y - dy, x - dx) that tap t reads from.
    __device__ __forceinline__ bool tap_ok_rev(int t, int L) const {
        const bool down = y < L - 1, left = x > 0, right = x < L - 1;
        return t == 0 ? down && right : t == 1 ? down : t == 2 ? down && left : t == 3 ? right : t == 4;
    }
};

// Contiguous run of tiles [t0, t1) of wave `wave` of `waves`.
__device__ __forceinline__ void tile_run(int tiles, int wave, int waves, int& t0, int& t1) {
    const int per = (tiles + waves - 1) / waves;
    t0 = wave * per;
    t1 = t0 + per < tiles ? t0 + per : tiles;
}

// Eight float32 values v as three bfloat16 vectors with hi + mid + lo = v
// exactly: hi keeps the leading 8 significant bits of v (truncated), mid
// the leading 8 of the remainder v - hi (exact in float32), and lo the
// rest, at most 8 significant bits and so a bfloat16 itself.  The products
// on the matrix cores then see the float32 operand unchanged.
__device__ __forceinline__ void split3_bf16(const f4& a, const f4& b, bf16x8& hi, bf16x8& mid,
                                            bf16x8& lo) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float v = e < 4 ? a[e] : b[e - 4];
        const uint32_t uh = __float_as_uint(v) & 0xFFFF0000u;
        const float r = v - __uint_as_float(uh);
        const uint32_t um = __float_as_uint(r) & 0xFFFF0000u;
        const uint32_t ul = __float_as_uint(r - __uint_as_float(um));
        hi[e] = __builtin_bit_cast(__bf16, (uint16_t)(uh >> 16));
        mid[e] = __builtin_bit_cast(__bf16, (uint16_t)(um >> 16));
        lo[e] = __builtin_bit_cast(__bf16, (uint16_t)(ul >> 16));
    }
}

// Operand A of the transposed convolution by the layer weights at wo, for
// this lane: row ci = m; elements e = 0..7 are k = 32 j + 8 kk + e, i.e.
// output channel 8 (kk & 1) + e of tap 2 j + (kk >> 1) (zero past the fifth).
__device__ __forceinline__ bf16x8 weights_t(const float* wexp, int wo, int m, int kk, int j) {
    bf16x8 a;
    const int tap = 2 * j + (kk >> 1);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int co = 8 * (kk & 1) + e;
        a[e] = (__bf16)(tap < NTB ? wexp[wo + (co * C + m) * NTB + tap] : 0.f);
    }
    return a;
}

// Layer 1 (mask A, 1 -> C, ReLU) from the int8 spins times sign: thread i
// computes channels 4 (i & 3) .. + 3 of site i >> 2.  Also clears the 64
// zero bytes that the later passes read for taps outside the lattice.
__global__ void k_nn_fwd1(const int8_t* s, int64_t stride, int total, int N, int L, float sign,
                          const float* __restrict__ w, float* __restrict__ h1,
                          float* __restrict__ zero) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < C)
        zero[i] = 0.f;
    if (i >= (int64_t)total * 4)
        return;
    const int e = (int)(i >> 2), c0 = 4 * (int)(i & 3);
    const int b = e / N, p = e - b * N;
    const TSite q{p / L, p % L};
    const int8_t* sb = s + (int64_t)b * stride;
    float in[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        in[t] = tinside(q, L, tap_dy(t), tap_dx(t))
                    ? sign * (float)sb[p + tap_dy(t) * L + tap_dx(t)]
                    : 0.f;
    f4 out;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float a = w[NNOff::B1 + c0 + c];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            a = fmaf(w[NNOff::W1 + (c0 + c) * 4 + t], in[t], a);
        out[c] = fmaxf(a, 0.f);
    }
    *reinterpret_cast<f4*>(h1 + (size_t)e * C + c0) = out;
}

// Layers 2 and 3 (mask B, C -> C, ReLU): each wave takes a contiguous run
// of 16-site tiles.  Lane (m, kk) gathers the eight input channels
// 8 (kk & 1) .. of tap 2 j + (kk >> 1) of site m for product j, and
// receives output channels 4 kk .. 4 kk + 3 of site m.  Loads are
// unconditional (a tap outside the lattice reads `zero`, 64 zero bytes),
// so that the loads of a tile are in flight together.
__global__ void __launch_bounds__(256) k_nn_fwd_mid(const float* __restrict__ hin,
                                                    const float* __restrict__ zero, int total,
                                                    int N, int L, const float* __restrict__ wexp,
                                                    int wo, int bo, float* __restrict__ hout) {
    const int lane = threadIdx.x & 63, m = lane & 15, kk = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    bf16x8 wa[3];
    int off[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        wa[j] = weights_b(wexp, wo, m, kk, j);
        const int tap = 2 * j + (kk >> 1);
        off[j] = tap < NTB ? tap_dy(tap) * L + tap_dx(tap) : 0;
    }
    f4 bias;
#pragma unroll
    for (int v = 0; v < 4; ++v)
        bias[v] = wexp[bo + 4 * kk + v];
    int t0, t1;
    tile_run((total + kTile - 1) / kTile, blockIdx.x * (blockDim.x >> 6) + w,
             gridDim.x * (blockDim.x >> 6), t0, t1);
    if (t0 >= t1)
        return;
    RunSite q;
    q.start(t0 * kTile + m, N, L);
    // the loads of kU tiles are issued before their products (a tile past
    // the run reads the zero site and stores nothing)
    constexpr int kU = 2;
    for (int tile = t0; tile < t1; tile += kU) {
        f4 src_v[kU][3][2];
        int e[kU];
        bool on[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            on[u] = tile + u < t1 && q.e < total;
            e[u] = q.e;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const bool ok = on[u] && q.tap_ok(2 * j + (kk >> 1), L);
                const f4* src = reinterpret_cast<const f4*>(
                    (ok ? hin + (size_t)(q.e + off[j]) * C : zero) + 8 * (kk & 1));
                src_v[u][j][0] = src[0];
                src_v[u][j][1] = src[1];
            }
            q.advance(kTile, N, L);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            f4 hi = {0.f, 0.f, 0.f, 0.f}, mid = hi, lo = hi;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                bf16x8 bh, bm, bl;
                split3_bf16(src_v[u][j][0], src_v[u][j][1], bh, bm, bl);
                hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], bh, hi, 0, 0, 0);
                mid = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], bm, mid, 0, 0, 0);
                lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], bl, lo, 0, 0, 0);
            }
            f4 d = hi + (mid + lo) + bias;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                d[v] = fmaxf(d[v], 0.f);
            if (on[u])
                *reinterpret_cast<f4*>(hout + (size_t)e[u] * C + 4 * kk) = d;
        }
    }
}

// Layer 4 (mask B, C -> 1) and the likelihood: one workgroup per batch
// element.  logq[b] = sum_p log sigmoid(s_p z_p); with dz, also
// dz[b][p] = d(-mean_b log q)/dz_p = -s_p sigmoid(-s_p z_p) / B.  The
// configuration is sign * s (sign = -1 evaluates the negated lattice).
__global__ void k_nn_out(const float* __restrict__ h3, const int8_t* s, int64_t stride, int B, int L,
                         float sign, const float* __restrict__ w, float* logq, float* dz) {
    __shared__ float red[16];
    // the layer's 80 weights and its bias, read from LDS by every lane (kept
    // in scalar registers they overflowed them)
    __shared__ float w4[C * NTB + 1];
    for (int i = threadIdx.x; i < C * NTB + 1; i += blockDim.x)
        w4[i] = w[NNOff::W4 + i];
    __syncthreads();
    const int N = L * L, b = blockIdx.x;
    const float* xb = h3 + (size_t)b * N * C;
    const int8_t* sb = s + (int64_t)b * stride;
    float lq = 0.f;
    for (int p = threadIdx.x; p < N; p += blockDim.x) {
        const TSite q{p / L, p % L};
        float z = w4[C * NTB];  // B4 follows W4
#pragma unroll
        for (int t = 0; t < NTB; ++t) {
            if (!tinside(q, L, tap_dy(t), tap_dx(t)))
                continue;
            const f4* src =
                reinterpret_cast<const f4*>(xb + (size_t)(p + tap_dy(t) * L + tap_dx(t)) * C);
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4) {
                const f4 a = src[c4];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    z = fmaf(w4[(4 * c4 + c) * NTB + t], a[c], z);
            }
        }
        const float sp = sign * (float)sb[p];
        lq += log_sigmoid(sp * z);
        if (dz)
            dz[(size_t)b * N + p] = -sp / (1.f + expf(sp * z)) / (float)B;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        lq += __shfl_xor(lq, off, 64);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = lq;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i)
            t += red[i];
        logq[b] = t;
    }
}

// Mean negative log-likelihood from logq[0..B-1] in a fixed order.
__global__ void k_nn_loss(const float* logq, int B, float* loss) {
    __shared__ float red[4];
    float t = 0.f;
    for (int b = threadIdx.x; b < B; b += blockDim.x)
        t += logq[b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        t += __shfl_xor(t, off, 64);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0)
        *loss = -(red[0] + red[1] + red[2] + red[3]) / (float)B;
}

// Gradient into the input of layer 4: g3[e][ci] = [h3 > 0] sum_t W4[ci][t]
// dz[e - d_t]; thread i computes channels 4 (i & 3) .. + 3 of site i >> 2.
__global__ void k_nn_bwd_out(const float* __restrict__ dz, const float* __restrict__ h3, int total,
                             int N, int L, const float* __restrict__ w, float* __restrict__ g3) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)total * 4)
        return;
    const int e = (int)(i >> 2), c0 = 4 * (int)(i & 3);
    const TSite q = tsite(e, N, L);
    float g[NTB];
#pragma unroll
    for (int t = 0; t < NTB; ++t)
        g[t] = tinside(q, L, -tap_dy(t), -tap_dx(t)) ? dz[e - tap_dy(t) * L - tap_dx(t)] : 0.f;
    const f4 h = *reinterpret_cast<const f4*>(h3 + (size_t)e * C + c0);
    f4 o;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float a = 0.f;
#pragma unroll
        for (int t = 0; t < NTB; ++t)
            a = fmaf(w[NNOff::W4 + (c0 + c) * NTB + t], g[t], a);
        o[c] = h[c] > 0.f ? a : 0.f;
    }
    *reinterpret_cast<f4*>(g3 + (size_t)e * C + c0) = o;
}

// Gradient into the input of layer 3 or 2 (the transposed convolution):
// gprev[e][ci] = [hprev > 0] sum_{t, co} W[co][ci][t] gout[e - d_t][co],
// organised as k_nn_fwd_mid.
__global__ void __launch_bounds__(256) k_nn_bwd_mid(const float* __restrict__ gout,
                                                    const float* __restrict__ zero,
                                                    const float* __restrict__ hprev, int total,
                                                    int N, int L, const float* __restrict__ wexp,
                                                    int wo, float* __restrict__ gprev) {
    const int lane = threadIdx.x & 63, m = lane & 15, kk = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    bf16x8 wa[3];
    int off[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        wa[j] = weights_t(wexp, wo, m, kk, j);
        const int tap = 2 * j + (kk >> 1);
        off[j] = tap < NTB ? -(tap_dy(tap) * L + tap_dx(tap)) : 0;
    }
    int t0, t1;
    tile_run((total + kTile - 1) / kTile, blockIdx.x * (blockDim.x >> 6) + w,
             gridDim.x * (blockDim.x >> 6), t0, t1);
    if (t0 >= t1)
        return;
    RunSite q;
    q.start(t0 * kTile + m, N, L);
    // the loads of kU tiles are issued before their products (a tile past
    // the run reads the zero site and stores nothing)
    constexpr int kU = 2;
    for (int tile = t0; tile < t1; tile += kU) {
        f4 src_v[kU][3][2], h[kU];
        int e[kU];
        bool on[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            on[u] = tile + u < t1 && q.e < total;
            e[u] = q.e;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const bool ok = on[u] && q.tap_ok_rev(2 * j + (kk >> 1), L);
                const f4* src = reinterpret_cast<const f4*>(
                    (ok ? gout + (size_t)(q.e + off[j]) * C : zero) + 8 * (kk & 1));
                src_v[u][j][0] = src[0];
                src_v[u][j][1] = src[1];
            }
            h[u] = *reinterpret_cast<const f4*>(on[u] ? hprev + (size_t)q.e * C + 4 * kk : zero);
            q.advance(kTile, N, L);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            f4 hi = {0.f, 0.f, 0.f, 0.f}, mid = hi, lo = hi;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                bf16x8 bh, bm, bl;
                split3_bf16(src_v[u][j][0], src_v[u][j][1], bh, bm, bl);
                hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], bh, hi, 0, 0, 0);
                mid = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], bm, mid, 0, 0, 0);
                lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], bl, lo, 0, 0, 0);
            }
            if (on[u]) {
                f4 d = hi + (mid + lo);
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    d[v] = h[u][v] > 0.f ? d[v] : 0.f;
                *reinterpret_cast<f4*>(gprev + (size_t)e[u] * C + 4 * kk) = d;
            }
        }
    }
}

// Weight gradient of one layer, partial sums per workgroup: dW[co][ci][t] =
// sum_e g[e][co] x[e + d_t][ci] and db[co] = sum_e g[e][co] over the
// workgroup's sites, written into row blockIdx.x of partial[rows][P] at
// the layer's parameter offsets wo and bo.  Each product takes four sites
// k: A[co][k] = g of site k, B[k][ci] = x at tap t of site k; lane (m, kk)
// loads channel m of site kk of both and receives D[4 kk + v][m].  Each
// wave takes a contiguous run of 16-site tiles; loads are unconditional as
// in k_nn_fwd_mid (lanes without a value read `zero`).
// kCout = C: g is [B][N][C]; kCout = 1 (layer 4): g is dz, [B][N].
// kIn = C: x is [B][N][C], one product per tap; kIn = 1 (layer 1): x is the
// int8 spins, the four taps of mask A in the columns of one product.
template <int kCout, int kIn>
__global__ void __launch_bounds__(256) k_nn_wgrad(const float* __restrict__ g,
                                                  const float* __restrict__ zero,
                                                  const float* __restrict__ x,
                                                  const int8_t* __restrict__ s, int64_t stride,
                                                  int total, int N, int L, int wo, int bo, int P,
                                                  float* __restrict__ partial) {
    constexpr int kT = kIn == 1 ? 1 : NTB;
    __shared__ float red[4][4 * kT + 1][64];
    const int lane = threadIdx.x & 63, m = lane & 15, kk = lane >> 4;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    f4 acc[kT];
#pragma unroll
    for (int t = 0; t < kT; ++t)
        acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    float accb = 0.f;
    int off[NTB];
#pragma unroll
    for (int t = 0; t < NTB; ++t)
        off[t] = tap_dy(t) * L + tap_dx(t);
    // layer 1: column m holds tap m of mask A
    const int off1 = m < 4 ? tap_dy(m) * L + tap_dx(m) : 0;
    int t0, t1;
    tile_run((total + kTile - 1) / kTile, blockIdx.x * 4 + w, gridDim.x * 4, t0, t1);
    if (t0 < t1) {
        RunSite q;
        q.start(t0 * kTile + kk, N, L);
        // kU steps of four sites at a time: every load of the kU steps is
        // issued before their products, so that a wave keeps 6 kU loads in
        // flight.  A step past the run loads the zero site: it adds exact
        // zeros, and the sums are those of the step-by-step loop.
        constexpr int kU = 4;
        for (int k4 = 4 * t0; k4 < 4 * t1; k4 += kU) {
            float a[kU], bv[kU][kT];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const bool on = k4 + u < 4 * t1 && q.e < total;
                a[u] = kCout == 1 ? *(on && m == 0 ? g + q.e : zero)
                                  : *(on ? g + (size_t)q.e * C + m : zero);
                if constexpr (kIn == 1) {
                    const bool ok = on && m < 4 && q.tap_ok(m, L);
                    bv[u][0] = (float)*(ok ? s + (int64_t)q.b * stride + q.p + off1
                                           : reinterpret_cast<const int8_t*>(zero));
                } else {
#pragma unroll
                    for (int t = 0; t < NTB; ++t) {
                        const bool ok = on && q.tap_ok(t, L);
                        bv[u][t] = *(ok ? x + (size_t)(q.e + off[t]) * C + m : zero);
                    }
                }
                q.advance(4, N, L);
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                accb += a[u];
#pragma unroll
                for (int t = 0; t < kT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], bv[u][t], acc[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            red[w][4 * t + v][lane] = acc[t][v];
    red[w][4 * kT][lane] = accb;
    __syncthreads();
    if (w != 0)
        return;
    float* out = partial + (size_t)blockIdx.x * P;
#pragma unroll
    for (int t = 0; t < kT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 4 * t + v, co = 4 * kk + v;
            const float d = ((red[0][r][lane] + red[1][r][lane]) + red[2][r][lane]) + red[3][r][lane];
            if (kIn == 1) {
                if (m < 4)
                    out[wo + co * 4 + m] = d;
            } else if (kCout == 1) {
                if (co == 0)
                    out[wo + m * NTB + t] = d;
            } else {
                out[wo + (co * C + m) * NTB + t] = d;
            }
        }
    float bs = ((red[0][4 * kT][lane] + red[1][4 * kT][lane]) + red[2][4 * kT][lane]) +
               red[3][4 * kT][lane];
    bs += __shfl_xor(bs, 16, 64);
    bs += __shfl_xor(bs, 32, 64);
    if (kk == 0 && (kCout != 1 || m == 0))
        out[bo + m] = bs;
}

// grad[i] = sum over rows r of partial[r][i] in a fixed order: thread
// (o, seg) sums rows seg, seg + 8, .. of output 32 blockIdx.x + o, and the
// eight segments are added in order.
__global__ void k_nn_reduce(const float* __restrict__ partial, int rows, int P,
                            float* __restrict__ grad) {
    __shared__ float red[8][32];
    const int o = threadIdx.x & 31, seg = threadIdx.x >> 5;
    const int i = blockIdx.x * 32 + o;
    float t = 0.f;
    if (i < P) {
#pragma unroll 8
        for (int r = seg; r < rows; r += 8)
            t += partial[(size_t)r * P + i];
    }
    red[seg][o] = t;
    __syncthreads();
    if (seg == 0 && i < P) {
        float u = red[0][o];
#pragma unroll
        for (int k = 1; k < 8; ++k)
            u += red[k][o];
        grad[i] = u;
    }
}

// E of an L x L int8 lattice (periodic right and down bonds), summed by
// the workgroup into thread 0.
__device__ __forceinline__ long long energy_to0(const int8_t* s, int L, long long* red) {
    long long e = 0;
    const int N = L * L;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int y = i / L, x = i - y * L;
        e -= s[i] * (s[y * L + (x + 1 == L ? 0 : x + 1)] + s[(y + 1 == L ? 0 : y + 1) * L + x]);
    }
    e = wave_sum_i64(e);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = e;
    __syncthreads();
    long long t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
            t += red[w];
    return t;
}

// Independent-proposal Metropolis-Hastings, one workgroup per lattice.
__global__ void k_batch_mh(unsigned char* ws, int count, uint64_t spins_bytes, int max_L,
                           int8_t* spins, int L_prop, const int8_t* prop, int64_t pstride,
                           const float* lq_cur, const float* lq_prop, const double* beta, Key key,
                           uint32_t draw, int32_t* accepted) {
    __shared__ long long red[16];
    __shared__ int acc_s;
    const BatchHeaderView hv(ws);
    const int j = blockIdx.x;
    const BatchDesc d = reinterpret_cast<const BatchDesc*>(ws + BatchWs::desc_offset(count))[j];
    // the checks a sweep's prepare step makes, for this lattice: the batch
    // is set up, its descriptor fits the spins buffer and max_L, and its
    // side is the proposals'
    const uint32_t* mc = reinterpret_cast<const uint32_t*>(ws + BatchWs::kMagic);
    const bool set_up = mc[0] == kBatchMagic && mc[1] == (uint32_t)count;
    const bool fits = d.L >= 8 && d.L <= max_L && (d.L & 7) == 0 && (d.off & 255u) == 0 &&
                      d.off + (uint64_t)d.L * (uint64_t)d.L <= spins_bytes;
    if (!set_up || !fits || d.L != L_prop) {
        if (threadIdx.x == 0) {
            atomicOr(hv.err, !set_up ? kBatchErrNotSetUp : !fits ? kBatchErrDescriptor : kBatchErrShape);
            if (accepted)
                accepted[j] = 0;
        }
        return;
    }
    int8_t* s = spins + d.off;
    const int8_t* sp = prop + (int64_t)j * pstride;
    const long long E0 = energy_to0(s, L_prop, red);
    const long long E1 = energy_to0(sp, L_prop, red);
    if (threadIdx.x == 0) {
#pragma clang fp contract(off)
        // ((-beta dE) + log q(s)) - log q(s'), each operation rounded (no FMA)
        const double lr = -beta[j] * (double)(E1 - E0) + (double)lq_cur[j] - (double)lq_prop[j];
        const U4 o = philox4x32_10({d.lid, draw, 0u, kTagMH}, key);
        const double thr = exp(lr < 0.0 ? lr : 0.0) * 4294967296.0;
        acc_s = (double)o.x < thr ? 1 : 0;
        if (accepted)
            accepted[j] = acc_s;
    }
    __syncthreads();
    if (acc_s) {
        const int N = L_prop * L_prop;
        for (int i = threadIdx.x; i < N; i += blockDim.x)
            s[i] = sp[i];
    }
}

}  // namespace

NNWs nn_ws_layout(int L, int max_batch) {
    NNWs w;
    const size_t N = (size_t)L * L;
    const size_t act = (size_t)max_batch * C * N * 4;
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t o = 0;
    w.wexp = o;
    o += up((size_t)NNOff::P * 4);
    w.h[0] = o;
    o += up(act);
    w.h[1] = o;
    o += up(act);
    w.h[2] = o;
    o += up(act);
    w.g[0] = o;
    o += up(act);
    w.g[1] = o;
    o += up(act);
    w.dz = o;
    o += up((size_t)max_batch * N * 4);
    w.logq = o;
    o += up((size_t)max_batch * 4);
    w.zero = o;
    o += up((size_t)C * 4);
    w.rows = nn_grad_rows(L, max_batch);
    w.partial = o;
    o += up((size_t)w.rows * NNOff::P * 4);
    w.bytes = o;
    return w;
}

int nn_param_count() { return NNOff::P; }

int nn_grad_rows(int L, int B) {
    const int64_t tiles = ((int64_t)B * L * L + kTile - 1) / kTile;
    const int64_t wgs = (tiles + 3) / 4;
    return (int)(wgs < kNNGradBlocks ? wgs : kNNGradBlocks);
}

namespace {
// Workgroups of 256 threads for a pass of one wave per 16-site tile.
dim3 tile_grid(int total) {
    const int tiles = (total + kTile - 1) / kTile;
    const int wgs = (tiles + 3) / 4;
    return dim3((unsigned)(wgs < 2048 ? wgs : 2048));
}
// One thread per 4 channels of a site.
dim3 quad_grid(int total) { return dim3((unsigned)(((int64_t)total * 4 + 255) / 256)); }
}  // namespace

hipError_t launch_nn_round(const float* master, uint16_t* w, float* wexp, hipStream_t st) {
    hipLaunchKernelGGL(k_nn_round, dim3((NNOff::P + 255) / 256), dim3(256), 0, st, master, w, wexp,
                       NNOff::P);
    return hipGetLastError();
}

hipError_t launch_nn_forward(const int8_t* s, int64_t stride, int B, int L, const NNWs& lay,
                             unsigned char* ws, float* logq, bool with_dz, float sign,
                             hipStream_t st) {
    const float* wexp = reinterpret_cast<const float*>(ws + lay.wexp);
    float* h[3] = {reinterpret_cast<float*>(ws + lay.h[0]), reinterpret_cast<float*>(ws + lay.h[1]),
                   reinterpret_cast<float*>(ws + lay.h[2])};
    float* zero = reinterpret_cast<float*>(ws + lay.zero);
    const int N = L * L, total = B * N;
    hipLaunchKernelGGL(k_nn_fwd1, quad_grid(total), dim3(256), 0, st, s, stride, total, N, L, sign,
                       wexp, h[0], zero);
    hipLaunchKernelGGL(k_nn_fwd_mid, tile_grid(total), dim3(256), 0, st, h[0], zero, total, N, L,
                       wexp, NNOff::W2, NNOff::B2, h[1]);
    hipLaunchKernelGGL(k_nn_fwd_mid, tile_grid(total), dim3(256), 0, st, h[1], zero, total, N, L,
                       wexp, NNOff::W3, NNOff::B3, h[2]);
    hipLaunchKernelGGL(k_nn_out, dim3(B), dim3(256), 0, st, h[2], s, stride, B, L, sign, wexp, logq,
                       with_dz ? reinterpret_cast<float*>(ws + lay.dz) : nullptr);
    return hipGetLastError();
}

hipError_t launch_nn_backward(const int8_t* s, int64_t stride, int B, int L, const NNWs& lay,
                              unsigned char* ws, float* grad, float* loss, hipStream_t st) {
    const float* wexp = reinterpret_cast<const float*>(ws + lay.wexp);
    const float* h[3] = {reinterpret_cast<const float*>(ws + lay.h[0]),
                         reinterpret_cast<const float*>(ws + lay.h[1]),
                         reinterpret_cast<const float*>(ws + lay.h[2])};
    float* g[2] = {reinterpret_cast<float*>(ws + lay.g[0]), reinterpret_cast<float*>(ws + lay.g[1])};
    const float* dz = reinterpret_cast<const float*>(ws + lay.dz);
    float* partial = reinterpret_cast<float*>(ws + lay.partial);
    const float* zero = reinterpret_cast<const float*>(ws + lay.zero);
    const int N = L * L, total = B * N, P = NNOff::P;
    // every layer's weight-gradient pass fills its parameters' columns of
    // the same rows of partial, so one reduction gives the whole gradient
    const dim3 rows(nn_grad_rows(L, B));
    if (loss)
        hipLaunchKernelGGL(k_nn_loss, dim3(1), dim3(256), 0, st,
                           reinterpret_cast<const float*>(ws + lay.logq), B, loss);
    // layer 4: weights from dz and h3, then the gradient into h3
    hipLaunchKernelGGL((k_nn_wgrad<1, C>), rows, dim3(256), 0, st, dz, zero, h[2], s, stride, total,
                       N, L, NNOff::W4, NNOff::B4, P, partial);
    hipLaunchKernelGGL(k_nn_bwd_out, quad_grid(total), dim3(256), 0, st, dz, h[2], total, N, L, wexp,
                       g[0]);
    // layer 3: g[0] is the gradient at its pre-activation output
    hipLaunchKernelGGL((k_nn_wgrad<C, C>), rows, dim3(256), 0, st, g[0], zero, h[1], s, stride,
                       total, N, L, NNOff::W3, NNOff::B3, P, partial);
    hipLaunchKernelGGL(k_nn_bwd_mid, tile_grid(total), dim3(256), 0, st, g[0], zero, h[1], total, N,
                       L, wexp, NNOff::W3, g[1]);
    // layer 2
    hipLaunchKernelGGL((k_nn_wgrad<C, C>), rows, dim3(256), 0, st, g[1], zero, h[0], s, stride,
                       total, N, L, NNOff::W2, NNOff::B2, P, partial);
    hipLaunchKernelGGL(k_nn_bwd_mid, tile_grid(total), dim3(256), 0, st, g[1], zero, h[0], total, N,
                       L, wexp, NNOff::W2, g[0]);
    // layer 1 (input: the spins)
    hipLaunchKernelGGL((k_nn_wgrad<C, 1>), rows, dim3(256), 0, st, g[0], zero, nullptr, s, stride,
                       total, N, L, NNOff::W1, NNOff::B1, P, partial);
    hipLaunchKernelGGL(k_nn_reduce, dim3((P + 31) / 32), dim3(256), 0, st, partial, (int)rows.x, P,
                       grad);
    return hipGetLastError();
}

hipError_t launch_nn_adam(float* master, float* m, float* v, const float* g, uint16_t* w,
                          float* wexp, float lr, float b1, float b2, float eps, float c1, float c2,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_nn_adam, dim3((NNOff::P + 255) / 256), dim3(256), 0, st, master, m, v, g, w,
                       wexp, NNOff::P, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

size_t nn_wave_lds_bytes(int L, int symmetric, int predraw) {
    const size_t sb = ((size_t)L * (L + 3) + 3) & ~(size_t)3;
    const size_t Rp = (size_t)(L + 1) / 2 + 3;  // ring rows + a zero and a junk row
    return sb * sizeof(float) + (size_t)(symmetric ? 2 : 1) * 4 * (3 * 4 * Rp * 16) +
           (predraw ? (((size_t)L * L + 3) & ~(size_t)3) * sizeof(uint32_t) : 0);
}

hipError_t launch_nn_wave(const float* wexp, int L, int B, int sample, int symmetric,
                          const int8_t* s_in, int64_t in_stride, Key key, uint32_t chain0,
                          uint32_t draw, int8_t* s_out, int64_t out_stride, float* logq,
                          hipStream_t st) {
    const int rows = (L + 1) / 2;  // sites of one anti-diagonal, at most
    const dim3 block(symmetric ? 128 : 64);
    // draws taken up front where their table is small (4 KB at L = 32)
    const int predraw = sample && L <= 32;
    const size_t lds = nn_wave_lds_bytes(L, symmetric, predraw);
    if (rows <= 16)
        hipLaunchKernelGGL(k_nn_wave<1>, dim3(B), block, lds, st, wexp, L, sample, predraw,
                           symmetric, s_in, in_stride, key, chain0, draw, s_out, out_stride, logq);
    else if (rows <= 32)
        hipLaunchKernelGGL(k_nn_wave<2>, dim3(B), block, lds, st, wexp, L, sample, predraw,
                           symmetric, s_in, in_stride, key, chain0, draw, s_out, out_stride, logq);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

size_t nn_lattice_lds_bytes(int L) {
    if (L < 2 || L > kNNLatticeMaxL)
        return 0;
    return (size_t)lattice_lds(L).bytes;
}

hipError_t launch_nn_lattice(const float* wexp, int L, int B, int symmetric, const int8_t* s_in,
                             int64_t in_stride, float* logq, int grid, hipStream_t st) {
    const size_t lds = nn_lattice_lds_bytes(L);
    if (!lds || grid < 1)
        return hipErrorInvalidValue;
    // wave w evaluates rows w and w + 16: L waves up to 16
    const int waves = L < 16 ? L : 16;
    const int threads = 64 * waves;
    if ((L + 1) * (L + 1) > kLatticePrefetch * threads)
        return hipErrorInvalidValue;
    const dim3 g(grid < B ? grid : B);
    if (L > 16)
        hipLaunchKernelGGL(k_nn_lattice<4>, g, dim3(threads), lds, st, wexp, L, B, symmetric, s_in,
                           in_stride, logq);
    else
        hipLaunchKernelGGL(k_nn_lattice<1>, g, dim3(threads), lds, st, wexp, L, B, symmetric, s_in,
                           in_stride, logq);
    return hipGetLastError();
}

hipError_t launch_batch_mh(unsigned char* ws, int count, uint64_t spins_bytes, int max_L,
                           int8_t* spins, int L_prop, const int8_t* prop, int64_t pstride,
                           const float* lq_cur, const float* lq_prop, const double* beta, Key key,
                           uint32_t draw, int32_t* accepted, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_mh, dim3(count), dim3(256), 0, st, ws, count, spins_bytes, max_L,
                       spins, L_prop, prop, pstride, lq_cur, lq_prop, beta, key, draw, accepted);
    return hipGetLastError();
}

}  // namespace ising
