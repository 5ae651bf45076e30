// Host-side launchers of the 3D Edwards-Anderson spin glass with replica
// exchange (internal to libising.so).
#pragma once

#include "kernels.hpp"

namespace ising {

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
    size_t partial = 0, partial_blk = 0, rng_blocks = 0;
    size_t sbits = 0;  // plane draws: uint32 [R][2][L^3/64], spins by colour, bit 1 = s = -1
    size_t jbits = 0;  // plane draws: uint32 [3][2][L^3/64], couplings J_d(n) by colour of n
    size_t bytes = 0;
    int bpr = 0;           // blocks per replica of a half-sweep (site draws)
    int plane_blocks = 0;  // blocks per z-plane of a replica (site draws)
    int bpr_bit = 0;       // blocks per replica of a half-sweep (plane draws)
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
// Plane draws (L >= 64): the INT8 spins and couplings are packed into colour
// bit planes in the workspace, swept there 32 sites per lane, and the spins
// unpacked again; pack_bonds / pack_spins before the sweeps of a call,
// unpack_spins after them.
hipError_t launch_ea_pack_bonds(unsigned char* ws, const EaLayout& lay, const int8_t* bonds, int L,
                                hipStream_t st);
hipError_t launch_ea_pack_spins(unsigned char* ws, const EaLayout& lay, const int8_t* spins, int L,
                                int R, hipStream_t st);
hipError_t launch_ea_unpack_spins(unsigned char* ws, const EaLayout& lay, int8_t* spins, int L,
                                  int R, hipStream_t st);
hipError_t launch_ea_sweep_bit(unsigned char* ws, const EaLayout& lay, int L, int R, int every,
                               Key key, int64_t* trace, hipStream_t st);

}  // namespace ising
