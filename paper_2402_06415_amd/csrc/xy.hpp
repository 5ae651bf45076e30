// Host-side launchers of the 2D XY model (internal to libising.so).
#pragma once

#include "kernels.hpp"

namespace ising {

constexpr uint32_t kXyMagic = 0x31595849u;   // "IXY1"
constexpr uint32_t kXyErrNotInit = 1u;
constexpr uint32_t kXyErrSweepIndex = 4u;
constexpr uint32_t kXyErrHandoff = 8u;  // a band waited too long for a neighbour
constexpr size_t kXyAccepted = 256;          // uint64[count]: accepted rotations
// double[2][count]: per-lattice energy sums of the global-memory sweep
inline size_t xy_energy_sums_offset(int count) {
    return kXyAccepted + (((size_t)count * 8 + 255) & ~(size_t)255);
}
size_t xy_workspace_bytes(int L, int count);
hipError_t launch_xy_init(unsigned char* ws, double* theta, int L, int count, int start, Key key,
                          uint32_t lid0, hipStream_t st);
// prepare (validate, note t), the persistent sweep kernel, advance t
hipError_t launch_xy_sweep(unsigned char* ws, double* theta, int L, int count, int64_t n,
                           double beta, Key key, uint32_t lid0, double* E_trace, hipStream_t st);
hipError_t launch_xy_energy(const double* theta, int L, int count, double* E_out, hipStream_t st);

}  // namespace ising
