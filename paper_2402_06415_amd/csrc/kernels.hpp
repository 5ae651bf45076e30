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
// Persistent tile-resident INT8 sweep (L % 8 == 0, L <= kInt8TilesMaxL).
constexpr int kInt8TilesMaxL = 4096;
struct Int8TilePlan {
    int ntiles = 0;   // workgroups, one tile of full rows each
    int rows = 0;     // rows per tile
    int threads = 0;  // workgroup size
    size_t lds = 0;   // dynamic LDS bytes: (rows + 2) * L
};
// max_lds: LDS bytes one workgroup may use on the device.
bool plan_int8_tiles(int L, int device_cus, int max_lds, Int8TilePlan* plan);
// Bytes of tagged halo slots the plan's tiles use (after WsLayout::kHalo).
size_t int8_halo_bytes(int L, int ntiles);
int int8_tiles_resident(const Int8TilePlan& plan, bool obs);
hipError_t launch_sweep_int8_tiles(int8_t* s, int L, const Int8TilePlan& plan, int64_t n,
                                   uint32_t t0, Key key, uint32_t lid, Accept acc, long long* dE,
                                   long long* dM, unsigned char* ws, uint32_t spin_limit,
                                   hipStream_t st);
hipError_t launch_convert_int8(const int8_t* in, int8_t* out, int64_t N, hipStream_t st);

// BIT1 layout ---------------------------------------------------------------
hipError_t launch_init_bit1(uint32_t* planes, int L, int start, Key key, uint32_t lid,
                            hipStream_t st);
hipError_t launch_halfsweep_bit1(uint32_t* planes, int L, int c, uint32_t h, Key key,
                                 uint32_t lid, Accept acc, long long* dE, long long* dM,
                                 unsigned long long* nblk, bool count, hipStream_t st);
hipError_t launch_measure_bit1(const uint32_t* planes, int L, long long* acc, hipStream_t st);
hipError_t launch_to_int8_bit1(const uint32_t* planes, int L, int8_t* out, hipStream_t st);
hipError_t launch_from_int8_bit1(uint32_t* planes, int L, const int8_t* in, hipStream_t st);

// Persistent tile-resident sweep (BIT1); returns hipErrorNotSupported when
// the lattice does not fit the resident scheme on this device.
struct Bit1TilePlan {
    int ntiles = 0;     // workgroups, one tile of rows each
    int rows = 0;       // rows per tile
    int threads = 0;    // workgroup size: one wave per row, at most 16 waves per CU
    size_t lds = 0;     // dynamic LDS bytes
};
bool plan_bit1_tiles(int L, int device_cus, Bit1TilePlan* plan);
// LDS bytes of a tile of `rows` rows (both colours, one halo row each side).
size_t tile_lds_bytes(int L, int rows);
// How many tiles of this plan the device holds at once (0 if the query
// fails) in the kernel variant of (traces, always-flip classes, counting);
// every tile must be resident for the inter-tile hand-off.
int bit1_tiles_resident(int L, const Bit1TilePlan& plan, bool obs, bool general, bool count);
// count: add the Philox blocks drawn to the workspace's counters.
hipError_t launch_sweep_bit1_tiles(uint32_t* planes, int L, const Bit1TilePlan& plan,
                                   int64_t n, uint32_t t0, Key key, uint32_t lid, Accept acc,
                                   long long* dE, long long* dM, unsigned char* ws,
                                   uint32_t spin_limit, bool count, hipStream_t st);

// Shared small kernels ------------------------------------------------------
hipError_t launch_fill_i64(long long* p, int64_t n, long long v, hipStream_t st);
// *dst = *src (one word, device to device) as a kernel.
hipError_t launch_copy_u32(const uint32_t* src, uint32_t* dst, hipStream_t st);
// out[j] = base + sum_{i<=j} d[i] in place (d == out allowed); base read
// from device memory.
hipError_t launch_prefix_i64(long long* d, int64_t n, const long long* base, hipStream_t st);
// E_out = a*acc[0] + b ; M_out = c*acc[1] + d   (either output may be NULL)
hipError_t launch_finish_measure(const long long* acc, long long aE, long long bE, long long aM,
                                 long long bM, long long* E_out, long long* M_out,
                                 long long* E_copy, long long* M_copy, hipStream_t st);

}  // namespace ising
