/*
 * ising_nn.h - learned whole-lattice proposals for the Metropolis chains of
 * libising.so (C ABI; same conventions, status codes and error reporting as
 * ising.h).
 *
 * The proposal q(s) is an autoregressive network over the spins of an L x L
 * lattice in raster order (site i = y*L + x): q(s) = prod_i q(s_i | s_<i),
 * q(s_i = +1 | s_<i) = sigmoid(z_i).  The logits z come from four masked 3x3
 * convolutions with zero padding outside the lattice:
 *   layer 1: taps (dy,dx) = (-1,-1) (-1,0) (-1,1) (0,-1)   1 -> C, ReLU
 *   layers 2, 3: the same taps plus (0,0)                  C -> C, ReLU
 *   layer 4: the same five taps                            C -> 1
 * Parameters are one flat vector: per layer W[out][in][tap], then b[out]
 * (ising_nn_param_count values).  Every kernel computes with the weights
 * rounded to bfloat16 (round to nearest even) and accumulates in float32;
 * training keeps float32 master weights and Adam moments.
 *
 * A whole-lattice move draws s' ~ q independently of the current state s
 * and accepts it with the Metropolis-Hastings probability
 *   min(1, exp(-beta (E' - E) + log q(s) - log q(s'))),
 * E and E' the integer energies (ising.h), which leaves the Boltzmann
 * distribution exp(-beta E) invariant for any q.  The plain checkerboard
 * sweeps of ising.h run between such moves.  This extends the paper's
 * single-spin-flip Metropolis step (Fig. 2c; accept iff p < P) to one
 * proposal for all N spins with the Hastings correction for q.
 *
 * Draws: Philox4x32-10 keyed by (seed lo, seed hi) as in ising.h;
 *   sampling site i of chain c in draw k: r = out[i & 3] of counter
 *     (i >> 2, c, k, 6), and s_i = +1 iff r < q(s_i = +1 | s_<i) * 2^32
 *     (q as float32, the comparison exact);
 *   the acceptance of chain c in draw k: r = out[0] of counter (c, k, 0, 7),
 *     accepted iff r < exp(min(0, log ratio)) * 2^32 (double).
 */
#ifndef ISING_NN_H
#define ISING_NN_H

#include "ising.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ISING_NN_CHANNELS 16 /* C: the kernels are built for 16 channels */
#define ISING_NN_MAX_L 64

typedef struct ising_nn {
    int32_t abi_version; /* must equal ISING_ABI_VERSION                       */
    int32_t L;           /* lattice side, 2..ISING_NN_MAX_L                    */
    int32_t channels;    /* must equal ISING_NN_CHANNELS                       */
    int32_t max_batch;   /* configurations per call, 1..65536                  */
    float *master;       /* device float32[P]: master parameters               */
    uint16_t *weights;   /* device bfloat16[P]: the parameters the kernels use */
    float *grad;         /* device float32[P]: gradient of the last grad call  */
    float *adam_m;       /* device float32[P]: Adam first moment               */
    float *adam_v;       /* device float32[P]: Adam second moment              */
    void *workspace;     /* device, 256-B aligned,
                            >= ising_nn_workspace_bytes(L, channels, max_batch) */
} ising_nn;

/* P, the number of parameters for `channels` (0 unless 16). */
ISING_API int32_t ising_nn_param_count(int32_t channels);

/* Device workspace: activations and gradients of max_batch configurations,
 * the float32 expansion of the bfloat16 weights, partial sums.  0 if
 * invalid. */
ISING_API size_t ising_nn_workspace_bytes(int32_t L, int32_t channels, int32_t max_batch);

/* weights = bfloat16(master) (round to nearest even).  Call after writing
 * master directly; ising_nn_adam does it by itself. */
ISING_API int ising_nn_round_weights(const ising_nn *net, void *hip_stream);

/* log q(s) of `batch` configurations: configuration b is the int8 L x L
 * row-major +1/-1 array at s_dev + b * stride (bytes, >= L*L).  With the
 * spins given (teacher forcing) the sites need no order: up to L = 32 each
 * configuration is held in LDS whole and evaluated a layer at a time over
 * all sites, above that by the sampler's own wavefront code.  Either way
 * every site's products, roundings and the order of the sum over sites are
 * the sampler's, so that for a configuration written by ising_nn_sample
 * with the same `symmetric` the result is bitwise the logq_out the sampler
 * returned.  With symmetric = 1 the result is
 * log q_sym(s) = log((q(s) + q(-s)) / 2), the Z2-symmetrised proposal
 * (sample from q, negate the whole lattice with probability 1/2).
 * logq_dev: device float32[batch].  Errors: batch outside 1..max_batch,
 * stride < L*L, symmetric not 0 or 1, NULL pointers, invalid net ->
 * ISING_E_INVALID. */
ISING_API int ising_nn_logq(const ising_nn *net, const int8_t *s_dev, int64_t stride,
                            int32_t batch, int32_t symmetric, float *logq_dev, void *hip_stream);

/* Mean negative log-likelihood of the batch (loss_dev: device float32[1],
 * may be NULL) and its gradient with respect to the parameters into
 * net->grad (overwritten), by backpropagation through the four layers.
 * The sums over the batch run in a fixed order: the result does not
 * depend on timing. */
ISING_API int ising_nn_grad(const ising_nn *net, const int8_t *s_dev, int64_t stride,
                            int32_t batch, float *loss_dev, void *hip_stream);

/* One Adam step (Kingma and Ba) on the master parameters from net->grad,
 * step >= 1 (bias correction 1 - b^step), then weights = bfloat16(master).
 * Errors: step < 1, lr <= 0 or not finite, b1 or b2 outside [0, 1),
 * eps <= 0 -> ISING_E_INVALID. */
ISING_API int ising_nn_adam(const ising_nn *net, float lr, float b1, float b2, float eps,
                            int32_t step, void *hip_stream);

/* Draw `batch` configurations from q, site by site: the sites of one
 * anti-diagonal x + 2y = t are drawn together for t = 0, 1, ..., 3L - 3,
 * which respects every dependency of the raster-order factorisation (the
 * masks reach the row above up to x + 1 and the left neighbour), so the
 * configuration is the one raster-order sampling gives for the same draws.
 * Configuration b goes to s_out + b * stride and uses chain id chain0 + b
 * in the Philox counter, draw index `draw`.  With symmetric = 1 each
 * configuration is written negated when the top bit of out[0] of counter
 * (2^32 - 1, chain, draw, 6) is set.  logq_out (float32[batch], may be
 * NULL) receives log q of the configuration written (log q_sym with
 * symmetric = 1), bitwise equal to ising_nn_logq of it. */
ISING_API int ising_nn_sample(const ising_nn *net, int32_t batch, uint64_t seed, uint32_t chain0,
                              uint32_t draw, int32_t symmetric, int8_t *s_out, int64_t stride,
                              float *logq_out, void *hip_stream);

/* Metropolis-Hastings with independent proposals on the lattices of a
 * batch (ising.h): lattice j (side L_prop, else a device error) is
 * replaced by the proposal at prop_dev + j * prop_stride when accepted,
 * with E recounted for both.  logq_cur_dev / logq_prop_dev: device
 * float32[count] (ising_nn_logq of the current lattices and of the
 * proposals); beta_dev: device double[count]; accepted_dev: device
 * int32[count] receiving 1 or 0, may be NULL.  The acceptance draw of
 * lattice j uses chain id lattice_id0 + j and draw index `draw`.  Only
 * kernel launches: may be captured in a HIP graph. */
ISING_API int ising_batch_mh(const ising_batch *b, int32_t L_prop, const int8_t *prop_dev,
                             int64_t prop_stride, const float *logq_cur_dev,
                             const float *logq_prop_dev, const double *beta_dev, uint32_t draw,
                             int32_t *accepted_dev, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ISING_NN_H */
