// Host-side launchers of the learned proposal network and of whole-lattice
// Metropolis-Hastings moves (internal to libising.so).
#pragma once

#include "batch.hpp"

namespace ising {

constexpr int kNNChannels = 16;
constexpr int kNNGradBlocks = 1024;  // most workgroups of a weight-gradient pass
// Byte offsets of the network workspace of max_batch configurations.
struct NNWs {
    size_t wexp = 0;          // float[P]: the bfloat16 weights as float
    size_t h[3] = {0, 0, 0};  // float[B][N][C]: post-ReLU outputs of layers 1-3
    size_t g[2] = {0, 0};     // float[B][N][C]: gradients, ping-pong
    size_t dz = 0;            // float[B][N]: gradient of the loss at the logits
    size_t logq = 0;          // float[B]
    size_t zero = 0;          // float[C]: zeros, read for taps outside the lattice
    size_t partial = 0;       // float[rows][P]: weight-gradient partial sums per workgroup
    int rows = 0;
    size_t bytes = 0;
};
NNWs nn_ws_layout(int L, int max_batch);
int nn_param_count();
// Workgroups (rows of partial) of the weight-gradient passes over B
// configurations: one per four 16-site tiles, at most kNNGradBlocks.
int nn_grad_rows(int L, int B);
hipError_t launch_nn_round(const float* master, uint16_t* w, float* wexp, hipStream_t st);
// Forward pass of B configurations; logq[b] = log q(s_b); with_dz also
// writes the loss gradient at the logits (for launch_nn_backward).
hipError_t launch_nn_forward(const int8_t* s, int64_t stride, int B, int L, const NNWs& lay,
                             unsigned char* ws, float* logq, bool with_dz, float sign,
                             hipStream_t st);
// Backward pass after launch_nn_forward(with_dz, logq = ws + lay.logq):
// writes the gradient into grad and the mean NLL into loss (may be NULL).
hipError_t launch_nn_backward(const int8_t* s, int64_t stride, int B, int L, const NNWs& lay,
                              unsigned char* ws, float* grad, float* loss, hipStream_t st);
hipError_t launch_nn_adam(float* master, float* m, float* v, const float* g, uint16_t* w,
                          float* wexp, float lr, float b1, float b2, float eps, float c1, float c2,
                          hipStream_t st);
// Wavefront evaluation (sites of one anti-diagonal x + 2y at a time, on the
// matrix cores): with sample = 1 draws B configurations into s_out, else
// evaluates the B configurations at s_in (teacher forcing); logq (may be
// NULL in sampling) receives log q, or log q_sym with symmetric = 1.  The
// two modes give the same bits for the same configuration.  L <= 64.
size_t nn_wave_lds_bytes(int L, int symmetric, int predraw);
hipError_t launch_nn_wave(const float* wexp, int L, int B, int sample, int symmetric,
                          const int8_t* s_in, int64_t in_stride, Key key, uint32_t chain0,
                          uint32_t draw, int8_t* s_out, int64_t out_stride, float* logq,
                          hipStream_t st);
// Teacher-forced log q (log q_sym with symmetric = 1) of B configurations
// held whole in LDS, a layer at a time over all sites: bitwise the result
// of launch_nn_wave for the same configuration.  2 <= L <= kNNLatticeMaxL;
// nn_lattice_lds_bytes gives its LDS per workgroup (0 outside that range).
// grid: workgroups (one per CU), each taking configurations blockIdx,
// blockIdx + grid, ...
constexpr int kNNLatticeMaxL = 32;
size_t nn_lattice_lds_bytes(int L);
hipError_t launch_nn_lattice(const float* wexp, int L, int B, int symmetric, const int8_t* s_in,
                             int64_t in_stride, float* logq, int grid, hipStream_t st);
// Metropolis-Hastings on the lattices of a batch; each workgroup checks its
// own lattice's setup and descriptor (no prepare launch).
hipError_t launch_batch_mh(unsigned char* ws, int count, uint64_t spins_bytes, int max_L,
                           int8_t* spins, int L_prop, const int8_t* prop, int64_t pstride,
                           const float* lq_cur, const float* lq_prop, const double* beta, Key key,
                           uint32_t draw, int32_t* accepted, hipStream_t st);

}  // namespace ising
