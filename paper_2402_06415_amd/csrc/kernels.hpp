// Host-side launchers of the sweep kernels (internal to libising.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace ising {

// Workspace layout (device bytes, caller-owned, 256-B aligned base).
struct WsLayout {
    static constexpr size_t kAcc = 0;          // int64[4]: raw E, raw M, E0, M0
    static constexpr size_t kErr = 64;         // uint32 device error word
    static constexpr size_t kRngBlocks = 256;  // uint64[64]: Philox blocks drawn since init
    static constexpr int kRngSlots = 64;       // workgroup b adds into slot b % 64
    static constexpr size_t kClearBytes = 768; // cleared by init: acc, error word, counters
    static constexpr size_t kHalo = 1024;      // uint64 halo slots of the tile sweep
    static constexpr int kMaxTiles = 1024;
    // [tiles][2 colours][first, last row][L/64 words] of (tag << 32 | word)
    static size_t halo_bytes(int L) { return (size_t)kMaxTiles * 2 * 2 * (size_t)(L / 64) * 8; }
};

// INT8 layout ---------------------------------------------------------------
hipError_t launch_init_int8(int8_t* s, int L, int start, Key key, uint32_t lid,
                            hipStream_t st);
hipError_t launch_sweep_int8_resident(int8_t* s, int L, int64_t n, uint32_t t0, Key key,
                                      uint32_t lid, Accept acc, int64_t* Etr, int64_t* Mtr,
                                      unsigned long long* nblk, hipStream_t st);
bool int8_resident_fits(int L);
hipError_t launch_halfsweep_int8(int8_t* s, int L, int c, uint32_t h, Key key, uint32_t lid,
                                 Accept acc, long long* dE, long long* dM,
                                 unsigned long long* nblk, hipStream_t st);
hipError_t launch_measure_int8(const int8_t* s, int L, long long* acc, hipStream_t st);
hipError_t launch_convert_int8(const int8_t* in, int8_t* out, int64_t N, hipStream_t st);

// BIT1 layout ---------------------------------------------------------------
hipError_t launch_init_bit1(uint32_t* planes, int L, int start, Key key, uint32_t lid,
                            hipStream_t st);
hipError_t launch_halfsweep_bit1(uint32_t* planes, int L, int c, uint32_t h, Key key,
                                 uint32_t lid, Accept acc, long long* dE, long long* dM,
                                 unsigned long long* nblk, hipStream_t st);
hipError_t launch_measure_bit1(const uint32_t* planes, int L, long long* acc, hipStream_t st);
hipError_t launch_to_int8_bit1(const uint32_t* planes, int L, int8_t* out, hipStream_t st);
hipError_t launch_from_int8_bit1(uint32_t* planes, int L, const int8_t* in, hipStream_t st);

// Persistent tile-resident sweep (BIT1); returns hipErrorNotSupported when
// the lattice does not fit the resident scheme on this device.
struct Bit1TilePlan {
    int ntiles = 0;     // workgroups, one tile of rows each
    int rows = 0;       // rows per tile
    int threads = 0;    // workgroup size: one wave per row, at most 16 waves
    size_t lds = 0;     // dynamic LDS bytes
};
// tiles_per_cu: how many tiles (workgroups) may share one CU.
bool plan_bit1_tiles(int L, int device_cus, int tiles_per_cu, Bit1TilePlan* plan);
hipError_t launch_sweep_bit1_tiles(uint32_t* planes, int L, const Bit1TilePlan& plan,
                                   int64_t n, uint32_t t0, Key key, uint32_t lid, Accept acc,
                                   long long* dE, long long* dM, unsigned char* ws,
                                   uint32_t spin_limit, hipStream_t st);

// Batches of small INT8 lattices -----------------------------------------------
// Workspace of a batch (device bytes, caller-owned, 256-B aligned base).
struct BatchWs {
    static constexpr size_t kMagic = 0;       // uint32 magic, uint32 count (written by setup)
    static constexpr size_t kT = 8;           // uint64 sweep index of the batch
    static constexpr size_t kTScratch = 16;   // uint64 sweep index used by the autotuner
    static constexpr size_t kOk = 24;         // uint32: the last prepare found everything valid
    static constexpr size_t kQueue = 32;      // uint32 work-queue head (cleared per launch)
    static constexpr size_t kErr = 40;        // uint32 device error word
    static constexpr size_t kRngBlocks = 256; // uint64[64] Philox blocks since init
    static constexpr size_t kRngScratch = 768;// uint64[64] Philox blocks of autotuner runs
    static constexpr size_t kOrder = 1280;    // int32[count]: queue position -> lattice
    __host__ __device__ static size_t desc_offset(int count) { return kOrder + (((size_t)count * 4 + 255) & ~(size_t)255); }
    __host__ __device__ static size_t bytes(int count) {
        return (desc_offset(count) + (size_t)count * 32 + 255) & ~(size_t)255;
    }
};
constexpr uint32_t kBatchMagic = 0x31425349u;  // "ISB1"
// Error bits of the batch error word.
constexpr uint32_t kBatchErrNotSetUp = 1u;     // magic or count does not match
constexpr uint32_t kBatchErrDescriptor = 2u;   // a descriptor does not fit spins / max_L
constexpr uint32_t kBatchErrSweepIndex = 4u;   // t + n > 2^31
constexpr uint32_t kBatchErrShape = 8u;        // a lattice's side differs from the proposals'

// Device view of the ok and error words of a batch workspace.
struct BatchHeaderView {
    const uint32_t* ok;
    uint32_t* err;
    __device__ explicit BatchHeaderView(unsigned char* ws)
        : ok(reinterpret_cast<const uint32_t*>(ws + BatchWs::kOk)),
          err(reinterpret_cast<uint32_t*>(ws + BatchWs::kErr)) {}
};

// One lattice of a batch (32 bytes, written by the host at setup).
struct BatchDesc {
    uint64_t off;     // byte offset of the lattice in the spins buffer
    int32_t L;        // side (multiple of 8)
    uint32_t lid;     // Philox lattice id
    uint32_t T2, T4;  // acceptance thresholds for u = 2 and u = 4
    uint32_t always;  // bit 0: u = 2 always flips; bit 1: u = 4 always flips
    uint32_t pad;
};
static_assert(sizeof(BatchDesc) == 32, "descriptor layout");

enum BatchPrepareMode { kPrepareSweep = 0, kPrepareInit = 1, kPrepareMeasure = 2 };
// Validate the workspace against (count, spins_bytes, max_L) and, for a
// sweep, t + n; write the ok word; init mode also zeroes t and the draw
// counters, sweep mode clears the queue head.  One small workgroup.
hipError_t launch_batch_prepare(unsigned char* ws, bool scratch_t, int count, uint64_t spins_bytes,
                                int max_L, int64_t n, int mode, hipStream_t st);
hipError_t launch_batch_init(unsigned char* ws, int count, int8_t* spins, int start, Key key,
                             hipStream_t st);
// Threads per workgroup and workgroups of the persistent sweep.
hipError_t launch_batch_sweep(unsigned char* ws, bool scratch_t, int count, int8_t* spins,
                              int max_L, int64_t n, Key key, int64_t* moments, int64_t* trace,
                              int threads, int blocks, hipStream_t st);
hipError_t launch_batch_advance(unsigned char* ws, int64_t n, hipStream_t st);
hipError_t launch_batch_measure(unsigned char* ws, int count, const int8_t* spins, int64_t* E,
                                int64_t* M, hipStream_t st);
size_t batch_lds_bytes(int max_L);

// Learned proposal network (16 channels) ------------------------------------
constexpr int kNNChannels = 16;
constexpr int kNNWgradPerBlock = 4096;  // (b, p) pairs per weight-gradient block
// Byte offsets of the network workspace of max_batch configurations.
struct NNWs {
    size_t wexp = 0;          // float[P]: the bfloat16 weights as float
    size_t h[3] = {0, 0, 0};  // float[B][C][N]: post-ReLU outputs of layers 1-3
    size_t g[2] = {0, 0};     // float[B][C][N]: gradients, ping-pong
    size_t dz = 0;            // float[B][N]: gradient of the loss at the logits
    size_t logq = 0;          // float[B]
    size_t logq2 = 0;         // float[B]: log q of the negated configurations
    size_t partial = 0;       // float[chunks][C][C*5+1]: weight-gradient partial sums
    int chunks = 0;
    size_t bytes = 0;
};
NNWs nn_ws_layout(int L, int max_batch);
int nn_param_count();
int nn_wgrad_chunks(int L, int B);
hipError_t launch_nn_round(const float* master, uint16_t* w, float* wexp, hipStream_t st);
// Forward pass of B configurations; logq[b] = log q(s_b); with_dz also
// writes the loss gradient at the logits (for launch_nn_backward).
hipError_t launch_nn_forward(const int8_t* s, int64_t stride, int B, int L, const NNWs& lay,
                             unsigned char* ws, float* logq, bool with_dz, float sign,
                             hipStream_t st);
// log q_sym(s) = log((q(s) + q(-s)) / 2): two forward passes and a combine.
hipError_t launch_nn_logq_sym(const int8_t* s, int64_t stride, int B, int L, const NNWs& lay,
                              unsigned char* ws, float* logq, hipStream_t st);
// Backward pass after launch_nn_forward(with_dz, logq = ws + lay.logq):
// writes the gradient into grad and the mean NLL into loss (may be NULL).
hipError_t launch_nn_backward(const int8_t* s, int64_t stride, int B, int L, const NNWs& lay,
                              unsigned char* ws, float* grad, float* loss, hipStream_t st);
hipError_t launch_nn_adam(float* master, float* m, float* v, const float* g, uint16_t* w,
                          float* wexp, float lr, float b1, float b2, float eps, float c1, float c2,
                          hipStream_t st);
size_t nn_sample_lds_bytes(int L);
hipError_t launch_nn_sample(const float* wexp, int L, int B, Key key, uint32_t chain0,
                            uint32_t draw, int symmetric, int8_t* s_out, int64_t stride,
                            float* logq, hipStream_t st);
hipError_t launch_batch_mh(unsigned char* ws, int count, int8_t* spins, int L_prop,
                           const int8_t* prop, int64_t pstride, const float* lq_cur,
                           const float* lq_prop, const double* beta, Key key, uint32_t draw,
                           int32_t* accepted, hipStream_t st);

// 3D Edwards-Anderson spin glass with replica exchange --------------------
constexpr uint32_t kEaMagic = 0x31414549u;  // "IEA1"
constexpr int kEaSwapTable = 4096;          // swap thresholds tabulated per pair
constexpr uint32_t kEaErrNotSetUp = 1u;
constexpr uint32_t kEaErrSweepIndex = 4u;
constexpr uint32_t kEaErrEnergy = 16u;      // an energy difference not a multiple of 4
enum EaPrepareMode { kEaPrepareSweep = 0, kEaPrepareInit = 1, kEaPrepareMeasure = 2 };
// Swap thresholds of one pair: T(q) for D = 4q, q < len, from the table;
// 1 for len <= q < zero_from; 0 beyond (exp underflows).
struct EaSwapMeta {
    uint64_t len;
    uint64_t zero_from;
};
// Workspace of a spin-glass run (byte offsets); the header (magic, R,
// sweep index, ok and error words) is at 0.
struct EaLayout {
    size_t perm = 0, tidx = 0, E = 0, accepts = 0, thr = 0, swap_meta = 0, swap_tab = 0;
    size_t partial = 0, partial_blk = 0, rng_blocks = 0, bytes = 0;
    int bpr = 0;           // blocks per replica of a half-sweep
    int plane_blocks = 0;  // blocks per z-plane of a replica
};
EaLayout ea_ws_layout(int L, int R);
hipError_t launch_ea_prepare(unsigned char* ws, const EaLayout& lay, int R, int64_t n, int mode,
                             hipStream_t st);
hipError_t launch_ea_init(unsigned char* ws, int8_t* spins, int L, int R, int start, Key key,
                          hipStream_t st);
hipError_t launch_ea_energy(unsigned char* ws, const int8_t* spins, const int8_t* bonds, int L,
                            int R, long long* out, hipStream_t st);
// One sweep of all replicas, the energy update and the exchange step.
hipError_t launch_ea_sweep(unsigned char* ws, const EaLayout& lay, int8_t* spins,
                           const int8_t* bonds, int L, int R, int every, Key key, int64_t* trace,
                           hipStream_t st);

// 2D XY model (double precision) --------------------------------------------
constexpr uint32_t kXyMagic = 0x31595849u;   // "IXY1"
constexpr uint32_t kXyErrNotInit = 1u;
constexpr uint32_t kXyErrSweepIndex = 4u;
constexpr size_t kXyAccepted = 256;          // uint64[count]: accepted rotations
size_t xy_workspace_bytes(int count);
hipError_t launch_xy_init(unsigned char* ws, double* theta, int L, int count, int start, Key key,
                          uint32_t lid0, hipStream_t st);
// prepare (validate, note t), the persistent sweep kernel, advance t
hipError_t launch_xy_sweep(unsigned char* ws, double* theta, int L, int count, int64_t n,
                           double beta, Key key, uint32_t lid0, double* E_trace, hipStream_t st);
hipError_t launch_xy_energy(const double* theta, int L, int count, double* E_out, hipStream_t st);

// Shared small kernels ------------------------------------------------------
hipError_t launch_fill_i64(long long* p, int64_t n, long long v, hipStream_t st);
// out[j] = base + sum_{i<=j} d[i] in place (d == out allowed); base read
// from device memory.
hipError_t launch_prefix_i64(long long* d, int64_t n, const long long* base, hipStream_t st);
// E_out = a*acc[0] + b ; M_out = c*acc[1] + d   (either output may be NULL)
hipError_t launch_finish_measure(const long long* acc, long long aE, long long bE, long long aM,
                                 long long bM, long long* E_out, long long* M_out,
                                 long long* E_copy, long long* M_copy, hipStream_t st);

}  // namespace ising
