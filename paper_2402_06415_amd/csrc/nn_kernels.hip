// Kernels of the learned whole-lattice proposal: the masked-convolution
// autoregressive network (forward, backward, Adam, incremental sampling)
// and the Metropolis-Hastings acceptance of whole-lattice proposals.
//
// Tensors of a batch live in the workspace as float32 [B][C][N] with
// N = L*L sites in raster order.  The network's parameters are bfloat16;
// the kernels read the float32 expansion of those bfloat16 values (`wexp`,
// exactly the same numbers), because uniform float loads become scalar
// operands of the FMAs, and accumulate in float32.
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

// Site p of a batch element: (y, x), and whether (y + dy, x + dx) is inside.
struct Site {
    int y, x;
};
__device__ __forceinline__ bool inside(const Site& q, int L, int dy, int dx) {
    return (unsigned)(q.y + dy) < (unsigned)L && (unsigned)(q.x + dx) < (unsigned)L;
}

// Layer 1 (mask A, 1 -> C, ReLU) from the int8 spins.
__global__ void k_nn_fwd1(const int8_t* s, int64_t stride, int B, int L, float sign,
                          const float* __restrict__ w, float* h1) {
    const int N = L * L;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * N)
        return;
    const int b = (int)(e / N), p = (int)(e - (int64_t)b * N);
    const Site q{p / L, p % L};
    const int8_t* sb = s + (int64_t)b * stride;
    float in[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        in[t] = inside(q, L, tap_dy(t), tap_dx(t)) ? sign * (float)sb[p + tap_dy(t) * L + tap_dx(t)]
                                                   : 0.f;
    float* out = h1 + (int64_t)b * C * N + p;
#pragma unroll
    for (int co = 0; co < C; ++co) {
        float a = w[NNOff::B1 + co];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            a = fmaf(w[NNOff::W1 + co * 4 + t], in[t], a);
        out[(int64_t)co * N] = fmaxf(a, 0.f);
    }
}

// Layers 2 and 3 (mask B, C -> C, ReLU).
__global__ void k_nn_fwd_mid(const float* hin, int B, int L, const float* __restrict__ w, int wo,
                             int bo, float* hout) {
    const int N = L * L;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * N)
        return;
    const int b = (int)(e / N), p = (int)(e - (int64_t)b * N);
    const Site q{p / L, p % L};
    const float* xb = hin + (int64_t)b * C * N;
    float in[C][NTB];
#pragma unroll
    for (int ci = 0; ci < C; ++ci)
#pragma unroll
        for (int t = 0; t < NTB; ++t)
            in[ci][t] = inside(q, L, tap_dy(t), tap_dx(t))
                            ? xb[(int64_t)ci * N + p + tap_dy(t) * L + tap_dx(t)]
                            : 0.f;
    float* out = hout + (int64_t)b * C * N + p;
#pragma unroll
    for (int co = 0; co < C; ++co) {
        float a = w[bo + co];
#pragma unroll
        for (int ci = 0; ci < C; ++ci)
#pragma unroll
            for (int t = 0; t < NTB; ++t)
                a = fmaf(w[wo + (co * C + ci) * NTB + t], in[ci][t], a);
        out[(int64_t)co * N] = fmaxf(a, 0.f);
    }
}

// Layer 4 (mask B, C -> 1) and the likelihood: one workgroup per batch
// element.  logq[b] = sum_p log sigmoid(s_p z_p); with dz, also
// dz[b][p] = d(-mean_b log q)/dz_p = -s_p sigmoid(-s_p z_p) / B.  The
// configuration is sign * s (sign = -1 evaluates the negated lattice).
__global__ void k_nn_out(const float* h3, const int8_t* s, int64_t stride, int B, int L, float sign,
                         const float* __restrict__ w, float* logq, float* dz) {
    __shared__ float red[16];
    const int N = L * L, b = blockIdx.x;
    const float* xb = h3 + (int64_t)b * C * N;
    const int8_t* sb = s + (int64_t)b * stride;
    float lq = 0.f;
    for (int p = threadIdx.x; p < N; p += blockDim.x) {
        const Site q{p / L, p % L};
        float z = w[NNOff::B4];
#pragma unroll
        for (int ci = 0; ci < C; ++ci)
#pragma unroll
            for (int t = 0; t < NTB; ++t)
                if (inside(q, L, tap_dy(t), tap_dx(t)))
                    z = fmaf(w[NNOff::W4 + ci * NTB + t],
                             xb[(int64_t)ci * N + p + tap_dy(t) * L + tap_dx(t)], z);
        const float sp = sign * (float)sb[p];
        lq += log_sigmoid(sp * z);
        if (dz)
            dz[(int64_t)b * N + p] = -sp / (1.f + expf(sp * z)) / (float)B;
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

// Gradient into the input of layer 4: g3[ci][p] = [h3 > 0] sum_t W4[ci][t] dz[p - d_t].
__global__ void k_nn_bwd_out(const float* dz, const float* h3, int B, int L,
                             const float* __restrict__ w, float* g3) {
    const int N = L * L;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * N)
        return;
    const int b = (int)(e / N), p = (int)(e - (int64_t)b * N);
    const Site q{p / L, p % L};
    float g[NTB];
#pragma unroll
    for (int t = 0; t < NTB; ++t)
        g[t] = inside(q, L, -tap_dy(t), -tap_dx(t))
                   ? dz[(int64_t)b * N + p - tap_dy(t) * L - tap_dx(t)]
                   : 0.f;
    const float* hb = h3 + (int64_t)b * C * N + p;
    float* ob = g3 + (int64_t)b * C * N + p;
#pragma unroll
    for (int ci = 0; ci < C; ++ci) {
        float a = 0.f;
#pragma unroll
        for (int t = 0; t < NTB; ++t)
            a = fmaf(w[NNOff::W4 + ci * NTB + t], g[t], a);
        ob[(int64_t)ci * N] = hb[(int64_t)ci * N] > 0.f ? a : 0.f;
    }
}

// Gradient into the input of layer 3 or 2:
// gprev[ci][p] = [hprev > 0] sum_co sum_t W[co][ci][t] gout[co][p - d_t].
__global__ void k_nn_bwd_mid(const float* gout, const float* hprev, int B, int L,
                             const float* __restrict__ w, int wo, float* gprev) {
    const int N = L * L;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * N)
        return;
    const int b = (int)(e / N), p = (int)(e - (int64_t)b * N);
    const Site q{p / L, p % L};
    const float* gb = gout + (int64_t)b * C * N;
    float g[C][NTB];
#pragma unroll
    for (int co = 0; co < C; ++co)
#pragma unroll
        for (int t = 0; t < NTB; ++t)
            g[co][t] = inside(q, L, -tap_dy(t), -tap_dx(t))
                           ? gb[(int64_t)co * N + p - tap_dy(t) * L - tap_dx(t)]
                           : 0.f;
    const float* hb = hprev + (int64_t)b * C * N + p;
    float* ob = gprev + (int64_t)b * C * N + p;
#pragma unroll
    for (int ci = 0; ci < C; ++ci) {
        float a = 0.f;
#pragma unroll
        for (int co = 0; co < C; ++co)
#pragma unroll
            for (int t = 0; t < NTB; ++t)
                a = fmaf(w[wo + (co * C + ci) * NTB + t], g[co][t], a);
        ob[(int64_t)ci * N] = hb[(int64_t)ci * N] > 0.f ? a : 0.f;
    }
}

// Weight gradient of one layer, partial sums: block (chunk, co) sums
// gout[co][p] x[ci][p + d_t] (and gout for the bias) over its chunk of
// (b, p) and writes partial[chunk][co][ci * NT + t], bias last.
// kIn: 1 (int8 spins, layer 1) or C; kNT: 4 or 5.
template <int kIn, int kNT>
__global__ void k_nn_wgrad(const float* gout, int cout, const float* xin, const int8_t* s,
                           int64_t stride, int B, int L, int per_thread, float* partial) {
    constexpr int K = kIn * kNT + 1;
    __shared__ float red[16][K];
    const int N = L * L, co = blockIdx.y;
    float acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        acc[k] = 0.f;
    const int64_t total = (int64_t)B * N;
    const int64_t base = (int64_t)blockIdx.x * blockDim.x * per_thread;
    for (int r = 0; r < per_thread; ++r) {
        const int64_t e = base + (int64_t)r * blockDim.x + threadIdx.x;
        if (e >= total)
            break;
        const int b = (int)(e / N), p = (int)(e - (int64_t)b * N);
        const Site q{p / L, p % L};
        const float g = gout[((int64_t)b * cout + co) * N + p];
#pragma unroll
        for (int ci = 0; ci < kIn; ++ci)
#pragma unroll
            for (int t = 0; t < kNT; ++t) {
                float x = 0.f;
                if (inside(q, L, tap_dy(t), tap_dx(t))) {
                    const int pp = p + tap_dy(t) * L + tap_dx(t);
                    x = kIn == 1 ? (float)s[(int64_t)b * stride + pp]
                                 : xin[((int64_t)b * kIn + ci) * N + pp];
                }
                acc[ci * kNT + t] = fmaf(g, x, acc[ci * kNT + t]);
            }
        acc[K - 1] += g;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float v = acc[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            v += __shfl_xor(v, off, 64);
        if (lane == 0)
            red[wave][k] = v;
    }
    __syncthreads();
    const int nw = blockDim.x >> 6;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        float t = 0.f;
        for (int i = 0; i < nw; ++i)
            t += red[i][k];
        partial[((int64_t)blockIdx.x * cout + co) * K + k] = t;
    }
}

// grad[W(co, k)] and grad[b(co)] = sum over chunks of partial[chunk][co][k].
__global__ void k_nn_reduce(const float* partial, int chunks, int cout, int K, float* grad,
                            int wo, int bo) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cout * K)
        return;
    const int co = i / K, k = i - co * K;
    float t = 0.f;
    for (int c = 0; c < chunks; ++c)
        t += partial[((int64_t)c * cout + co) * K + k];
    if (k == K - 1)
        grad[bo + co] = t;
    else
        grad[wo + co * (K - 1) + k] = t;
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

// Wavefront evaluation of the network, for sampling and for log q.
//
// The factorisation is over sites in raster order, and the logits of site
// (y, x) depend on the sites whose activations its taps read: (y-1, x-1),
// (y-1, x), (y-1, x+1), (y, x-1) and, above layer 1, (y, x) itself.  All
// of these lie on earlier anti-diagonals t = x + 2y, so the sites of one
// anti-diagonal (at most ceil(L/2), one per row) are evaluated together,
// 3L - 2 steps instead of L^2, and the draws and results are those of the
// site-by-site order.
//
// One wave per configuration and sign.  Lane l = m + 16 kk serves row slot
// m of each 16-slot tile; each step runs, per tile, the 16 sites as the 16
// rows of matrix products on the matrix cores.  Layer 1 (four mask-A taps
// of +-1 spins) is one float32 product v_mfma_f32_16x16x4_f32, exact.
// Layers 2, 3 and 4 are bfloat16 products v_mfma_f32_16x16x32_bf16 over
// K = 5 taps x 16 channels (padded to 96: three products of K = 32, the
// k-th input being channel k mod 16 of tap k / 16), with float32
// accumulation: the weights are bfloat16 already; each float32 activation
// a enters as two bfloat16 terms, hi = bf16(a) and lo = bf16(a - hi), each
// with its own accumulation chain, so that the products see a to within
// 2^-17 of it (the network's float32 arithmetic to well within the log q
// tolerance, where bfloat16 activations alone would not be).  Layer 4 (one
// output) uses the same products with its weights in every column.
// Activations live in LDS for only four columns (x mod 4): a row reads the
// row above at x-1..x+1 while that row writes x+2; each site keeps its 16
// channels as 16 bfloat16 hi terms and 16 lo terms (64 bytes), so that one
// 16-byte read gives a lane the eight channels of its part of K.  Rows
// share R = floor((L+1)/2) + 1 ring entries: row y + R starts after row
// y + 1 has read the last columns of row y.
//
// With `symmetric`, a second wave evaluates the negated configuration in
// step with the first, and the result is log q_sym = log((q(s) + q(-s)) / 2).
// Each wave adds its log-likelihood terms after the per-step barrier, in
// the same order in every mode, so that sampling and teacher-forced
// evaluation of the same configuration give the same bits.
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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

// Byte offset of the activations of site (y, x) of layer `layer` in the ring.
__device__ __forceinline__ int act_at(int layer, int R, int y, int x) {
    const int ry = y < R ? y : y - R;  // y mod R, as y < L < 2R
    return ((layer * R + ry) * 4 + (x & 3)) * kSiteBytes;
}

// log sigmoid(v) = -(max(-v, 0) + log1p(e^-|v|)), with log1p(e) taken as
// log(u) - ((u - 1) - e) / u for u = 1 + e (the rounding of u corrected
// to first order) on the hardware exp and log.
__device__ __forceinline__ float log_sigmoid_hw(float v) {
    const float e = __expf(-fabsf(v));
    const float u = 1.f + e;
    return -(fmaxf(-v, 0.f) + (__logf(u) - __fdividef((u - 1.f) - e, u)));
}

__device__ __forceinline__ __bf16 bf16_bits(uint16_t h) {
    return __builtin_bit_cast(__bf16, h);
}

// Store the float32 activation a of channel ch at site byte offset o as its
// two bfloat16 terms.
__device__ __forceinline__ void store_act(char* act, int o, int ch, float a) {
    const __bf16 hi = (__bf16)a;
    const __bf16 lo = (__bf16)(a - (float)hi);  // a - hi is exact in float32
    *reinterpret_cast<__bf16*>(act + o + 2 * ch) = hi;
    *reinterpret_cast<__bf16*>(act + o + 32 + 2 * ch) = lo;
}

// The bfloat16 operand B of layer weights for this lane: product j,
// elements e = 0..7 are k = 32 j + 8 kk + e, i.e. channel 8 (kk & 1) + e of
// tap 2 j + (kk >> 1) (zero past the fifth tap), column `col`.
template <bool kOut1>
__device__ __forceinline__ bf16x8 weights_b(const float* wexp, int wo, int col, int kk, int j) {
    bf16x8 b;
    const int tap = 2 * j + (kk >> 1);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int ci = 8 * (kk & 1) + e;
        float w = 0.f;
        if (tap < NTB)
            w = kOut1 ? wexp[wo + ci * NTB + tap] : wexp[wo + (col * C + ci) * NTB + tap];
        b[e] = (__bf16)w;  // exact: the values are bfloat16 already
    }
    return b;
}

// One layer's products for the 16 sites of a tile: sum over the three
// K = 32 chunks of A (the gathered activations, hi and lo terms) times B.
__device__ __forceinline__ f4 layer_products(const char* act, const int (&src)[3],
                                             const bf16x8 (&b)[3]) {
    f4 hi = {0.f, 0.f, 0.f, 0.f}, lo = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(act + src[j]);
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(act + src[j] + 32);
        hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b[j], hi, 0, 0, 0);
        lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b[j], lo, 0, 0, 0);
    }
    return hi + lo;
}

template <int T>
__global__ void __launch_bounds__(128) k_nn_wave(const float* __restrict__ wexp, int L, int sample,
                                                 int symmetric, const int8_t* s_in,
                                                 int64_t in_stride, Key key, uint32_t chain0,
                                                 uint32_t draw, int8_t* s_out, int64_t out_stride,
                                                 float* logq_out) {
    extern __shared__ __align__(16) float sh[];  // 16-byte reads of eight bfloat16 terms
    __shared__ float red[2];
    constexpr int S = 16 * T;
    const int W2 = L + 2, R = (L + 1) / 2 + 1;
    const int sb_floats = (L * W2 + 3) & ~3;
    const int layer_bytes = R * 4 * kSiteBytes;
    float* sb = sh;  // [L][L + 2] spins as +-1.0 (unsigned), zero columns 0 and L + 1
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 15, kk = lane >> 4;
    // per wave: activations [3][R][4] sites of 64 bytes, then one zero site
    // (read for taps outside the lattice) and one junk site that absorbs
    // the writes of idle rows
    char* act = reinterpret_cast<char*>(sh + sb_floats) + w * (3 * layer_bytes + 2 * kSiteBytes);
    const int zero_off = 3 * layer_bytes, junk_off = zero_off + kSiteBytes;
    const float sigma = w == 0 ? 1.f : -1.f;
    const int b = blockIdx.x;
    for (int i = threadIdx.x; i < sb_floats; i += blockDim.x) {
        float v = 0.f;
        const int y = i / W2, xc = i - y * W2;
        if (!sample && y < L && xc >= 1 && xc <= L)
            v = (float)s_in[(int64_t)b * in_stride + y * L + xc - 1];
        sb[i] = v;
    }
    if (lane < kSiteBytes / 4)
        reinterpret_cast<float*>(act + zero_off)[lane] = 0.f;
    // matrix-core operands: B[k][j = m] of every product
    const float wb1 = wexp[NNOff::W1 + m * 4 + kk];
    bf16x8 wb2[3], wb3[3], wb4[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        wb2[j] = weights_b<false>(wexp, NNOff::W2, m, kk, j);
        wb3[j] = weights_b<false>(wexp, NNOff::W3, m, kk, j);
        wb4[j] = weights_b<true>(wexp, NNOff::W4, m, kk, j);
    }
    const float bias1 = wexp[NNOff::B1 + m], bias2 = wexp[NNOff::B2 + m];
    const float bias3 = wexp[NNOff::B3 + m], bias4 = wexp[NNOff::B4];
    const RoundKeys rk = round_keys(key);
    const uint32_t chain = chain0 + (uint32_t)b;
    // symmetric sampling writes the configuration negated with probability 1/2
    float out_sign = 1.f;
    if (sample && symmetric) {
        const U4 o = philox4x32_10({0xFFFFFFFFu, chain, draw, kTagNNSample}, rk);
        out_sign = (o.x >> 31) ? -1.f : 1.f;
    }
    __syncthreads();
    float lq[T];
#pragma unroll
    for (int u = 0; u < T; ++u)
        lq[u] = 0.f;
    // the lane holding z of site slot m after the layer-4 products: column
    // m, rows 4 (m >> 2) .. 4 (m >> 2) + 3 (all columns hold z)
    const int zsrc = m + 16 * (m >> 2);
    const int steps = 3 * L - 2;
    for (int t = 0; t < steps; ++t) {
        // Geometry of the step: for this lane's site of each tile, the LDS
        // byte offsets of the taps its part of K reads (tap 2 j + (kk >> 1)
        // in product j, channels 8 (kk & 1) ..; -1 for the zero site: tap
        // outside the lattice, slot idle or past the fifth tap), of its
        // layer-1 input and of its spin; for the four product rows this
        // lane receives, where their results go.
        WaveSlot g[T];
        int src[T][3], doff[T][4], spin_in[T], spin_at[T];
#pragma unroll
        for (int u = 0; u < T; ++u) {
            g[u] = wave_slot(16 * u + m, t, L, S);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int tap = 2 * j + (kk >> 1);
                const int yy = g[u].y + tap_dy(tap), xx = g[u].x + tap_dx(tap);
                const bool ok = tap < NTB && g[u].on && yy >= 0 && (unsigned)xx < (unsigned)L;
                src[u][j] = ok ? act_at(0, R, yy, xx) + 16 * (kk & 1) : -1;
            }
            {
                // layer-1 input of this lane: tap kk (mask A) of its site;
                // index 0 is the zero column of row 0
                const int dy = kk < 3 ? -1 : 0, dx = kk < 3 ? kk - 1 : -1;
                const bool ok = g[u].on && g[u].y + dy >= 0;
                spin_in[u] = ok ? (g[u].y + dy) * W2 + g[u].x + dx + 1 : 0;
                spin_at[u] = g[u].on ? g[u].y * W2 + g[u].x + 1 : 0;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const WaveSlot d = wave_slot(16 * u + 4 * kk + v, t, L, S);
                doff[u][v] = d.on ? act_at(0, R, d.y, d.x) : -1;
            }
        }
        // layer 1 (mask A): A[i = m][k = kk] is tap kk of site m
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const float a = sigma * sb[spin_in[u]];
            f4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, wb1, acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v)
                store_act(act, doff[u][v] < 0 ? junk_off : doff[u][v], m,
                          fmaxf(acc[v] + bias1, 0.f));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // layers 2 and 3 (mask B)
#pragma unroll
        for (int layer = 1; layer < 3; ++layer) {
#pragma unroll
            for (int u = 0; u < T; ++u) {
                int o[3];
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    o[j] = src[u][j] < 0 ? zero_off : src[u][j] + (layer - 1) * layer_bytes;
                const f4 acc = layer_products(act, o, layer == 1 ? wb2 : wb3);
                const float bias = layer == 1 ? bias2 : bias3;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    store_act(act, doff[u][v] < 0 ? junk_off : doff[u][v] + layer * layer_bytes, m,
                              fmaxf(acc[v] + bias, 0.f));
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // layer 4: the same products with W4 in every column, then each lane
        // takes z of its site slot from the lane that holds it
        float z[T];
#pragma unroll
        for (int u = 0; u < T; ++u) {
            int o[3];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                o[j] = src[u][j] < 0 ? zero_off : src[u][j] + 2 * layer_bytes;
            const f4 acc = layer_products(act, o, wb4);
            const int v = lane & 3;
            const float mine = v == 0 ? acc[0] : v == 1 ? acc[1] : v == 2 ? acc[2] : acc[3];
            z[u] = __shfl(mine, zsrc, 64) + bias4;
        }
        if (sample && w == 0) {
#pragma unroll
            for (int u = 0; u < T; ++u) {
                if (g[u].on) {
                    const int i = g[u].y * L + g[u].x;
                    const U4 o = philox4x32_10({(uint32_t)(i >> 2), chain, draw, kTagNNSample}, rk);
                    const uint32_t r = u4_get(o, i & 3);
                    const float pplus = 1.f / (1.f + expf(-z[u]));
                    const float sp = ((double)r < (double)pplus * 4294967296.0) ? 1.f : -1.f;
                    if (kk == 0) {
                        sb[spin_at[u]] = sp;
                        s_out[(int64_t)b * out_stride + i] = (int8_t)(out_sign * sp);
                    }
                }
            }
        }
        __syncthreads();
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
__global__ void k_batch_mh(unsigned char* ws, int count, int8_t* spins, int L_prop,
                           const int8_t* prop, int64_t pstride, const float* lq_cur,
                           const float* lq_prop, const double* beta, Key key, uint32_t draw,
                           int32_t* accepted) {
    __shared__ long long red[16];
    __shared__ int acc_s;
    const BatchHeaderView hv(ws);
    if (*hv.ok == 0)
        return;
    const int j = blockIdx.x;
    const BatchDesc d = reinterpret_cast<const BatchDesc*>(ws + BatchWs::desc_offset(count))[j];
    if (d.L != L_prop) {
        if (threadIdx.x == 0) {
            atomicOr(hv.err, kBatchErrShape);
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
    w.chunks = nn_wgrad_chunks(L, max_batch);
    w.partial = o;
    o += up((size_t)w.chunks * C * (C * NTB + 1) * 4);
    w.bytes = o;
    return w;
}

int nn_param_count() { return NNOff::P; }

int nn_wgrad_chunks(int L, int B) {
    const int64_t total = (int64_t)B * L * L;
    return (int)((total + kNNWgradPerBlock - 1) / kNNWgradPerBlock);
}

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
    const int64_t total = (int64_t)B * L * L;
    const dim3 grid((unsigned)((total + 255) / 256));
    hipLaunchKernelGGL(k_nn_fwd1, grid, dim3(256), 0, st, s, stride, B, L, sign, wexp, h[0]);
    hipLaunchKernelGGL(k_nn_fwd_mid, grid, dim3(256), 0, st, h[0], B, L, wexp, NNOff::W2,
                       NNOff::B2, h[1]);
    hipLaunchKernelGGL(k_nn_fwd_mid, grid, dim3(256), 0, st, h[1], B, L, wexp, NNOff::W3,
                       NNOff::B3, h[2]);
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
    const int64_t total = (int64_t)B * L * L;
    const dim3 grid((unsigned)((total + 255) / 256));
    const int chunks = nn_wgrad_chunks(L, B);
    const int per = kNNWgradPerBlock / 256;
    constexpr int KB = C * NTB + 1, KA = 4 + 1, K4 = C * NTB + 1;
    if (loss)
        hipLaunchKernelGGL(k_nn_loss, dim3(1), dim3(256), 0, st,
                           reinterpret_cast<const float*>(ws + lay.logq), B, loss);
    // layer 4: weights from dz and h3, then the gradient into h3
    hipLaunchKernelGGL((k_nn_wgrad<C, NTB>), dim3(chunks, 1), dim3(256), 0, st, dz, 1, h[2], s,
                       stride, B, L, per, partial);
    hipLaunchKernelGGL(k_nn_reduce, dim3((K4 + 255) / 256), dim3(256), 0, st, partial, chunks, 1, K4,
                       grad, NNOff::W4, NNOff::B4);
    hipLaunchKernelGGL(k_nn_bwd_out, grid, dim3(256), 0, st, dz, h[2], B, L, wexp, g[0]);
    // layer 3: g[0] is the gradient at its pre-activation output
    hipLaunchKernelGGL((k_nn_wgrad<C, NTB>), dim3(chunks, C), dim3(256), 0, st, g[0], C, h[1], s,
                       stride, B, L, per, partial);
    hipLaunchKernelGGL(k_nn_reduce, dim3((C * KB + 255) / 256), dim3(256), 0, st, partial, chunks, C,
                       KB, grad, NNOff::W3, NNOff::B3);
    hipLaunchKernelGGL(k_nn_bwd_mid, grid, dim3(256), 0, st, g[0], h[1], B, L, wexp, NNOff::W3,
                       g[1]);
    // layer 2
    hipLaunchKernelGGL((k_nn_wgrad<C, NTB>), dim3(chunks, C), dim3(256), 0, st, g[1], C, h[0], s,
                       stride, B, L, per, partial);
    hipLaunchKernelGGL(k_nn_reduce, dim3((C * KB + 255) / 256), dim3(256), 0, st, partial, chunks, C,
                       KB, grad, NNOff::W2, NNOff::B2);
    hipLaunchKernelGGL(k_nn_bwd_mid, grid, dim3(256), 0, st, g[1], h[0], B, L, wexp, NNOff::W2,
                       g[0]);
    // layer 1 (input: the spins)
    hipLaunchKernelGGL((k_nn_wgrad<1, 4>), dim3(chunks, C), dim3(256), 0, st, g[0], C, nullptr, s,
                       stride, B, L, per, partial);
    hipLaunchKernelGGL(k_nn_reduce, dim3((C * KA + 255) / 256), dim3(256), 0, st, partial, chunks, C,
                       KA, grad, NNOff::W1, NNOff::B1);
    return hipGetLastError();
}

hipError_t launch_nn_adam(float* master, float* m, float* v, const float* g, uint16_t* w,
                          float* wexp, float lr, float b1, float b2, float eps, float c1, float c2,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_nn_adam, dim3((NNOff::P + 255) / 256), dim3(256), 0, st, master, m, v, g, w,
                       wexp, NNOff::P, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

size_t nn_wave_lds_bytes(int L, int symmetric) {
    const size_t sb = ((size_t)L * (L + 2) + 3) & ~(size_t)3;
    const size_t R = (size_t)(L + 1) / 2 + 1;
    return sb * sizeof(float) +
           (size_t)(symmetric ? 2 : 1) * (3 * R * 4 + 2) * (size_t)kSiteBytes;
}

hipError_t launch_nn_wave(const float* wexp, int L, int B, int sample, int symmetric,
                          const int8_t* s_in, int64_t in_stride, Key key, uint32_t chain0,
                          uint32_t draw, int8_t* s_out, int64_t out_stride, float* logq,
                          hipStream_t st) {
    const int rows = (L + 1) / 2;  // sites of one anti-diagonal, at most
    const dim3 block(symmetric ? 128 : 64);
    const size_t lds = nn_wave_lds_bytes(L, symmetric);
    if (rows <= 16)
        hipLaunchKernelGGL(k_nn_wave<1>, dim3(B), block, lds, st, wexp, L, sample, symmetric, s_in,
                           in_stride, key, chain0, draw, s_out, out_stride, logq);
    else if (rows <= 32)
        hipLaunchKernelGGL(k_nn_wave<2>, dim3(B), block, lds, st, wexp, L, sample, symmetric, s_in,
                           in_stride, key, chain0, draw, s_out, out_stride, logq);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_batch_mh(unsigned char* ws, int count, int8_t* spins, int L_prop,
                           const int8_t* prop, int64_t pstride, const float* lq_cur,
                           const float* lq_prop, const double* beta, Key key, uint32_t draw,
                           int32_t* accepted, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_mh, dim3(count), dim3(256), 0, st, ws, count, spins, L_prop, prop,
                       pstride, lq_cur, lq_prop, beta, key, draw, accepted);
    return hipGetLastError();
}

}  // namespace ising
