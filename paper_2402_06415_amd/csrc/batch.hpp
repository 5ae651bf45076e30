// Host-side launchers of batches of small INT8 lattices (internal to libising.so).
#pragma once

#include "kernels.hpp"

namespace ising {

// Workspace of a batch (device bytes, caller-owned, 256-B aligned base).
struct BatchWs {
    static constexpr size_t kMagic = 0;       // uint32 magic, uint32 count (written by setup)
    static constexpr size_t kT = 8;           // uint64 sweep index of the batch
    static constexpr size_t kTScratch = 16;   // uint64 sweep index used by the autotuner
    static constexpr size_t kOk = 24;         // uint32: the last prepare found everything valid
    static constexpr size_t kQueue = 32;      // uint32 work-queue head (cleared per launch)
    static constexpr size_t kErr = 40;        // uint32 device error word
    static constexpr size_t kDraws = 52;      // uint32: the draw mode given at setup
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
constexpr uint32_t kBatchErrDraws = 16u;       // draw mode differs from setup's, or an L unfit for it

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
// draws: the sweep's draw mode (0 site, 1 plane), checked against setup's in
// sweep mode.
hipError_t launch_batch_prepare(unsigned char* ws, bool scratch_t, int count, uint64_t spins_bytes,
                                int max_L, int64_t n, int mode, int draws, hipStream_t st);
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
// Bit-plane draws: lattices of side 32 or a multiple of 64, kept in LDS as
// colour bit planes and updated 32 sites per lane (bitslice.hpp); each
// workgroup runs its share of the lattices together, as many at once as fit
// lds_bytes of dynamic LDS (at least batch_bit_lds_bytes).
hipError_t launch_batch_sweep_bit(unsigned char* ws, bool scratch_t, int count, int8_t* spins,
                                  int64_t n, Key key, int64_t* moments, int64_t* trace,
                                  int threads, int blocks, size_t lds_bytes, hipStream_t st);
size_t batch_bit_lds_bytes(int threads, int max_L);

}  // namespace ising
