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

// log q_sym = log((q(s) + q(-s)) / 2) from a = log q(s), b = log q(-s).
__global__ void k_nn_logsym(const float* a, const float* b, float* out, int B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) {
        const float x = a[i], y = b[i];
        out[i] = fmaxf(x, y) + log1pf(expf(-fabsf(x - y))) - 0.69314718055994531f;
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

// Incremental autoregressive sampling: one wave per configuration.  Each
// step computes the four layers at the new site only; the earlier sites'
// activations come from two-row ring buffers in LDS (the masks reach one
// row up at most), with a zero column on each side for the padding.
// Lane l holds, for the whole run, the weights it multiplies: layers 2 and
// 3 split as (co = l / 4, ci in 4 (l % 4) .. +3), layers 1 and 4 use lanes
// 0..15 (one output channel or one input channel each).
__global__ void __launch_bounds__(64) k_nn_sample(const float* __restrict__ wexp, int L, Key key,
                                                  uint32_t chain0, uint32_t draw, int symmetric,
                                                  int8_t* s_out, int64_t stride, float* logq_out) {
    extern __shared__ float sh[];
    const int W2 = L + 2;               // padded row
    float* sb = sh;                     // [2][W2] spins as +-1.0
    float* hb[3] = {sb + 2 * W2, sb + 2 * W2 + C * 2 * W2, sb + 2 * W2 + 2 * C * 2 * W2};
    const int lane = threadIdx.x;
    const int total = 2 * W2 + 3 * C * 2 * W2;
    for (int i = lane; i < total; i += 64)
        sh[i] = 0.f;
    // per-lane weights
    const int co = lane >> 2, part = lane & 3;
    float w1[4] = {0.f, 0.f, 0.f, 0.f}, b1 = 0.f, w4[NTB] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (lane < C) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
            w1[t] = wexp[NNOff::W1 + lane * 4 + t];
        b1 = wexp[NNOff::B1 + lane];
#pragma unroll
        for (int t = 0; t < NTB; ++t)
            w4[t] = wexp[NNOff::W4 + lane * NTB + t];
    }
    float wm[2][4][NTB], bm[2];
#pragma unroll
    for (int l = 0; l < 2; ++l) {
        const int wo = l == 0 ? NNOff::W2 : NNOff::W3;
        bm[l] = wexp[(l == 0 ? NNOff::B2 : NNOff::B3) + co];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int t = 0; t < NTB; ++t)
                wm[l][j][t] = wexp[wo + (co * C + part * 4 + j) * NTB + t];
    }
    const float b4 = wexp[NNOff::B4];
    const RoundKeys rk = round_keys(key);
    const uint32_t chain = chain0 + blockIdx.x;
    int8_t* out = s_out + (int64_t)blockIdx.x * stride;
    // symmetric: the configuration is written negated with probability 1/2
    // (the network still conditions on the drawn, unnegated spins)
    float out_sign = 1.f;
    if (symmetric) {
        const U4 o = philox4x32_10({0xFFFFFFFFu, chain, draw, kTagNNSample}, rk);
        out_sign = (o.x >> 31) ? -1.f : 1.f;
    }
    __syncthreads();
    float lq = 0.f;
    U4 rr = {0u, 0u, 0u, 0u};
    int y = 0, x = 0;
    const int N = L * L;
    for (int i = 0; i < N; ++i) {
        const int cur = y & 1, prv = cur ^ 1, col = x + 1;
        // offsets of the five taps inside one channel's [2][W2] buffer
        const int o0 = prv * W2 + col - 1, o1 = prv * W2 + col, o2 = prv * W2 + col + 1;
        const int o3 = cur * W2 + col - 1, o4 = cur * W2 + col;
        if (lane < C) {
            float a = b1;
            a = fmaf(w1[0], sb[o0], a);
            a = fmaf(w1[1], sb[o1], a);
            a = fmaf(w1[2], sb[o2], a);
            a = fmaf(w1[3], sb[o3], a);
            hb[0][lane * 2 * W2 + o4] = fmaxf(a, 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            const float* hin = hb[l];
            float a = 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float* c0 = hin + (part * 4 + j) * 2 * W2;
                a = fmaf(wm[l][j][0], c0[o0], a);
                a = fmaf(wm[l][j][1], c0[o1], a);
                a = fmaf(wm[l][j][2], c0[o2], a);
                a = fmaf(wm[l][j][3], c0[o3], a);
                a = fmaf(wm[l][j][4], c0[o4], a);
            }
            a += __shfl_xor(a, 1, 64);
            a += __shfl_xor(a, 2, 64);
            if (part == 0)
                hb[l + 1][co * 2 * W2 + o4] = fmaxf(a + bm[l], 0.f);
            __syncthreads();
        }
        float zp = 0.f;
        if (lane < C) {
            const float* c0 = hb[2] + lane * 2 * W2;
            zp = fmaf(w4[0], c0[o0], zp);
            zp = fmaf(w4[1], c0[o1], zp);
            zp = fmaf(w4[2], c0[o2], zp);
            zp = fmaf(w4[3], c0[o3], zp);
            zp = fmaf(w4[4], c0[o4], zp);
        }
#pragma unroll
        for (int off = 1; off < 16; off <<= 1)
            zp += __shfl_xor(zp, off, 64);
        const float z = __shfl(zp, 0, 64) + b4;
        if ((i & 3) == 0)
            rr = philox4x32_10({(uint32_t)(i >> 2), chain, draw, kTagNNSample}, rk);
        const uint32_t r = u4_get(rr, i & 3);
        const float pplus = 1.f / (1.f + expf(-z));
        const float sp = ((double)r < (double)pplus * 4294967296.0) ? 1.f : -1.f;
        lq += log_sigmoid(sp * z);
        if (lane == 0) {
            sb[o4] = sp;
            out[i] = (int8_t)(out_sign * sp);
        }
        __syncthreads();
        if (++x == L) {
            x = 0;
            ++y;
        }
    }
    if (lane == 0 && logq_out)
        logq_out[blockIdx.x] = lq;
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
    w.logq2 = o;
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

hipError_t launch_nn_logq_sym(const int8_t* s, int64_t stride, int B, int L, const NNWs& lay,
                              unsigned char* ws, float* logq, hipStream_t st) {
    float* a = reinterpret_cast<float*>(ws + lay.logq);
    float* b = reinterpret_cast<float*>(ws + lay.logq2);
    hipError_t e = launch_nn_forward(s, stride, B, L, lay, ws, a, false, 1.f, st);
    if (e == hipSuccess)
        e = launch_nn_forward(s, stride, B, L, lay, ws, b, false, -1.f, st);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_nn_logsym, dim3((B + 255) / 256), dim3(256), 0, st, a, b, logq, B);
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

size_t nn_sample_lds_bytes(int L) { return (size_t)(2 * (L + 2) + 3 * C * 2 * (L + 2)) * 4; }

hipError_t launch_nn_sample(const float* wexp, int L, int B, Key key, uint32_t chain0,
                            uint32_t draw, int symmetric, int8_t* s_out, int64_t stride,
                            float* logq, hipStream_t st) {
    hipLaunchKernelGGL(k_nn_sample, dim3(B), dim3(64), nn_sample_lds_bytes(L), st, wexp, L, key,
                       chain0, draw, symmetric, s_out, stride, logq);
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
