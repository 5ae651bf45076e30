// extern "C" entry points of libising.so (declared in include/ising.h):
// argument validation, the host-side acceptance table, and dispatch of the
// kernels on the caller's stream.  No call allocates device memory; the
// only library-held device memory is the static scratch array of
// ising_sweep_noalloc.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "abi_common.hpp"
#include "ising.h"
#include "kernels.hpp"

namespace ising {
namespace abi {

namespace {
thread_local std::string g_last_error;
}

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return set_error(ISING_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int device_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 0;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return cus;
}

int device_max_lds() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 0;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    return lds;
}

const char* last_error() { return g_last_error.c_str(); }

}  // namespace abi
}  // namespace ising

namespace {

using ising::abi::aligned256;
using ising::abi::device_cus;
using ising::abi::device_max_lds;
using ising::abi::set_error;

constexpr int kMaxL = 65536;

bool valid_shape(int32_t dim, int32_t L, int32_t layout) {
    if (dim != 2)
        return false;
    if (L < 4 || L > kMaxL || (L & 1))
        return false;
    if (layout == ISING_LAYOUT_INT8)
        return true;
    if (layout == ISING_LAYOUT_BIT1)
        return (L % 64) == 0;
    return false;
}

int validate(const ising_lattice* lat, bool need_workspace = true) {
    if (!lat)
        return set_error(ISING_E_INVALID, "lattice pointer is NULL");
    if (lat->abi_version != ISING_ABI_VERSION)
        return set_error(ISING_E_INVALID, "abi_version %d, library has %d", lat->abi_version,
                         ISING_ABI_VERSION);
    if (lat->dim != 2)
        return set_error(ISING_E_UNSUPPORTED, "dim %d: only dim = 2 is built", lat->dim);
    if (lat->layout != ISING_LAYOUT_INT8 && lat->layout != ISING_LAYOUT_BIT1)
        return set_error(ISING_E_INVALID, "unknown layout %d", lat->layout);
    if (!valid_shape(lat->dim, lat->L, lat->layout))
        return set_error(ISING_E_INVALID,
                         "L = %d invalid for layout %d (even, 4..65536; BIT1 needs L %% 64 == 0)",
                         lat->L, lat->layout);
    if (lat->flags & ~(uint32_t)(ISING_FLAG_GLOBAL_HALFSWEEP | ISING_FLAG_COUNT_DRAWS))
        return set_error(ISING_E_INVALID, "unknown flag bits 0x%x", lat->flags);
    if (!lat->spins || !aligned256(lat->spins))
        return set_error(ISING_E_INVALID, "spins must be a non-NULL 256-byte aligned device pointer");
    size_t ws = ising_workspace_bytes(lat->dim, lat->L, lat->layout);
    if (need_workspace && ws && (!lat->workspace || !aligned256(lat->workspace)))
        return set_error(ISING_E_INVALID,
                         "workspace must be a non-NULL 256-byte aligned device pointer");
    if (lat->sweep_index > (1ull << 31))
        return set_error(ISING_E_INVALID, "sweep_index %llu exceeds 2^31",
                         (unsigned long long)lat->sweep_index);
    return ISING_OK;
}

ising::Key key_of(const ising_lattice* lat) {
    return ising::Key{(uint32_t)(lat->seed & 0xFFFFFFFFu), (uint32_t)(lat->seed >> 32)};
}

unsigned char* ws_of(const ising_lattice* lat) {
    return reinterpret_cast<unsigned char*>(lat->workspace);
}
long long* ws_acc(unsigned char* ws) {
    return reinterpret_cast<long long*>(ws + ising::WsLayout::kAcc);
}
unsigned long long* ws_blocks(unsigned char* ws) {
    return reinterpret_cast<unsigned long long*>(ws + ising::WsLayout::kRngBlocks);
}

// Scratch of ising_sweep_noalloc: the workspace of one sweep call (the
// header of accumulators, device error word and draw counters, then the
// tagged halo slots of the tile kernel) as a static device array, so that
// the call allocates nothing.  Each GPU the library runs on holds its own
// copy until the process ends.  Its size bounds BIT1 lattices to
// L <= kNoAllocMaxL (1024 tiles x 2 colours x 2 edge rows x L/64 words x
// 8 bytes of halo slots); the other paths need only the header.
constexpr int kNoAllocMaxL = 8192;
constexpr size_t kScratchBytes =
    ising::WsLayout::kHalo + (size_t)ising::WsLayout::kMaxTiles * 2 * 2 * (kNoAllocMaxL / 64) * 8;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (the array's name is only a host-side stand-in).
int scratch_of_current_device(unsigned char** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(ISING_E_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p)
            return set_error(ISING_E_HIP, "hipGetSymbolAddress(scratch) gave NULL");
        g_scratch_dev[dev] = reinterpret_cast<unsigned char*>(p);
    }
    *out = g_scratch_dev[dev];
    return ISING_OK;
}

// Spin limit of the inter-tile waits (each spin sleeps ~64 clocks); a
// healthy wait lasts microseconds, so this only ends a broken run.
constexpr uint32_t kSpinLimit = 1u << 24;

// Zero acc[0..1] and recount E, M of the current spins into acc (raw
// counts) then finish into E_out/M_out and copies.
int measure_into(const ising_lattice* lat, unsigned char* ws, long long* E_out, long long* M_out,
                 long long* E_copy, long long* M_copy, hipStream_t st) {
    long long* acc = ws_acc(ws);
    HIP_TRY(ising::launch_fill_i64(acc, 2, 0, st), "fill");
    const long long N = (long long)lat->L * lat->L;
    if (lat->layout == ISING_LAYOUT_INT8) {
        HIP_TRY(ising::launch_measure_int8(reinterpret_cast<const int8_t*>(lat->spins), lat->L, acc,
                                           st),
                "measure_int8");
        HIP_TRY(ising::launch_finish_measure(acc, 1, 0, 1, 0, E_out, M_out, E_copy, M_copy, st),
                "finish_measure");
    } else {
        HIP_TRY(ising::launch_measure_bit1(reinterpret_cast<const uint32_t*>(lat->spins), lat->L,
                                           acc, st),
                "measure_bit1");
        // E = 2 * (anti-aligned bonds) - 2N ; M = N - 2 * (set bits)
        HIP_TRY(ising::launch_finish_measure(acc, 2, -2 * N, -2, N, E_out, M_out, E_copy, M_copy,
                                             st),
                "finish_measure");
    }
    return ISING_OK;
}

}  // namespace

extern "C" {

int32_t ising_abi_version(void) { return ISING_ABI_VERSION; }

const char* ising_last_error(void) { return ising::abi::last_error(); }

size_t ising_spins_bytes(int32_t dim, int32_t L, int32_t layout) {
    if (!valid_shape(dim, L, layout))
        return 0;
    const size_t N = (size_t)L * (size_t)L;
    return layout == ISING_LAYOUT_INT8 ? N : N / 8;
}

size_t ising_workspace_bytes(int32_t dim, int32_t L, int32_t layout) {
    if (!valid_shape(dim, L, layout))
        return 0;
    size_t bytes = ising::WsLayout::kHalo;
    if (layout == ISING_LAYOUT_BIT1)
        bytes += ising::WsLayout::halo_bytes(L);
    else if ((L & 7) == 0 && L <= ising::kInt8TilesMaxL)
        bytes += ising::int8_halo_bytes(L, ising::WsLayout::kMaxTiles);
    return (bytes + 255) & ~(size_t)255;
}

int ising_thresholds(double beta, uint32_t T[5], uint8_t always_flip[5]) {
    if (!T || !always_flip)
        return set_error(ISING_E_INVALID, "NULL output");
    if (!(beta >= 0.0) || isinf(beta))
        return set_error(ISING_E_INVALID, "beta must be finite and >= 0 (got %g)", beta);
    for (int k = 0; k < 5; ++k) {
        const int u = 2 * k - 4;  // u = s_i h_i, dE = 2u
        T[k] = 0;
        always_flip[k] = 0;
        if (u <= 0) {
            always_flip[k] = 1;  // P(dE) >= 1
            continue;
        }
        const double P = exp(-beta * (double)(2 * u));
        const double t = ceil(ldexp(P, 32));  // p = r/2^32 < P  <=>  r < t
        if (t >= 4294967296.0)
            always_flip[k] = 1;
        else
            T[k] = (uint32_t)t;
    }
    return ISING_OK;
}

int ising_init(ising_lattice* lat, int32_t start, void* hip_stream) {
    int rc = validate(lat);
    if (rc)
        return rc;
    if (start != ISING_START_COLD_UP && start != ISING_START_RANDOM)
        return set_error(ISING_E_INVALID, "unknown start %d", start);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    // clear the accumulators, the device error word and the draw counters
    HIP_TRY(ising::launch_fill_i64(ws_acc(ws_of(lat)), ising::WsLayout::kClearBytes / 8, 0, st),
            "fill");
    if (lat->layout == ISING_LAYOUT_INT8)
        HIP_TRY(ising::launch_init_int8(reinterpret_cast<int8_t*>(lat->spins), lat->L, start,
                                        key_of(lat), lat->lattice_id, st),
                "init_int8");
    else
        HIP_TRY(ising::launch_init_bit1(reinterpret_cast<uint32_t*>(lat->spins), lat->L, start,
                                        key_of(lat), lat->lattice_id, st),
                "init_bit1");
    lat->sweep_index = 0;
    return ISING_OK;
}

// The sweep of ising_sweep and ising_sweep_tiles: `forced` (BIT1 only)
// replaces the library's tile plan.
// The kernels use the lattice's workspace, or `scratch` when it is given
// (the library's static scratch of ising_sweep_noalloc; lat->workspace is
// then not used and may be NULL).
static int sweep_impl(ising_lattice* lat, unsigned char* scratch, double beta, int64_t n,
                      int64_t* E_dev, int64_t* M_dev, void* hip_stream,
                      const ising::Bit1TilePlan* forced,
                      const ising::Int8TilePlan* forced8 = nullptr) {
    int rc = validate(lat, scratch == nullptr);
    if (rc)
        return rc;
    unsigned char* ws = scratch ? scratch : ws_of(lat);
    if (n < 0)
        return set_error(ISING_E_INVALID, "n = %lld < 0", (long long)n);
    if (lat->sweep_index + (uint64_t)n > (1ull << 31))
        return set_error(ISING_E_INVALID, "sweep_index + n exceeds 2^31");
    uint32_t T[5];
    uint8_t alw[5];
    rc = ising_thresholds(beta, T, alw);
    if (rc)
        return rc;
    if (n == 0)
        return ISING_OK;
    ising::Accept acc{T[3], T[4], alw[3], alw[4]};
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const ising::Key key = key_of(lat);
    const uint32_t t0 = (uint32_t)lat->sweep_index;
    const int L = lat->L;
    long long* Etr = reinterpret_cast<long long*>(E_dev);
    long long* Mtr = reinterpret_cast<long long*>(M_dev);
    const bool trace = Etr || Mtr;
    long long* acc_ws = ws_acc(ws);

    const bool global_only = (lat->flags & ISING_FLAG_GLOBAL_HALFSWEEP) != 0;
    // the no-alloc scratch's counters are cleared per call: nothing counts there
    const bool count = (lat->flags & ISING_FLAG_COUNT_DRAWS) != 0 && !scratch;
    // INT8 lattices above L = 64 (L % 8 == 0) run the tile kernel when it
    // fits the device and the workspace holds its halo slots: up to L = 128
    // one workgroup could hold the lattice, but its threads then take
    // several spans each per half-sweep (L = 128: 5.3 us a sweep, against
    // about 2.5 for one-row tiles on as many CUs)
    ising::Int8TilePlan plan8;
    bool tiles8 = false;
    if (lat->layout == ISING_LAYOUT_INT8) {
        if (forced8) {
            plan8 = *forced8;
            tiles8 = true;
        } else if (!global_only && (L > 64 || !ising::int8_resident_fits(L)) &&
                   ising::plan_int8_tiles(L, device_cus(), device_max_lds(), &plan8)) {
            const size_t room = scratch ? kScratchBytes - ising::WsLayout::kHalo
                                        : ising::int8_halo_bytes(L, ising::WsLayout::kMaxTiles);
            tiles8 = ising::int8_halo_bytes(L, plan8.ntiles) <= room &&
                     ising::int8_tiles_resident(plan8, E_dev || M_dev) >= plan8.ntiles;
        }
    }
    if (lat->layout == ISING_LAYOUT_INT8 && !tiles8 && !global_only &&
        ising::int8_resident_fits(L)) {
        HIP_TRY(ising::launch_sweep_int8_resident(reinterpret_cast<int8_t*>(lat->spins), L, n, t0,
                                                  key, lat->lattice_id, acc, E_dev, M_dev,
                                                  ws_blocks(ws), st),
                "sweep_int8_resident");
        lat->sweep_index += (uint64_t)n;
        return ISING_OK;
    }
    // Multi-workgroup paths: per-sweep changes are accumulated into the
    // traces, then turned into running values from a recount at the start.
    if (trace) {
        rc = measure_into(lat, ws, nullptr, nullptr, acc_ws + 2, acc_ws + 3, st);
        if (rc)
            return rc;
        if (Etr)
            HIP_TRY(ising::launch_fill_i64(Etr, n, 0, st), "fill");
        if (Mtr)
            HIP_TRY(ising::launch_fill_i64(Mtr, n, 0, st), "fill");
    }
    if (tiles8) {
        HIP_TRY(ising::launch_sweep_int8_tiles(reinterpret_cast<int8_t*>(lat->spins), L, plan8, n,
                                               t0, key, lat->lattice_id, acc, Etr, Mtr, ws,
                                               kSpinLimit, st),
                "sweep_int8_tiles");
    } else if (lat->layout == ISING_LAYOUT_INT8) {
        int8_t* s = reinterpret_cast<int8_t*>(lat->spins);
        for (int64_t j = 0; j < n; ++j)
            for (int c = 0; c < 2; ++c)
                HIP_TRY(ising::launch_halfsweep_int8(s, L, c, 2u * (t0 + (uint32_t)j) + (uint32_t)c,
                                                     key, lat->lattice_id, acc,
                                                     Etr ? Etr + j : nullptr,
                                                     Mtr ? Mtr + j : nullptr, ws_blocks(ws), st),
                        "halfsweep_int8");
    } else {
        uint32_t* planes = reinterpret_cast<uint32_t*>(lat->spins);
        ising::Bit1TilePlan plan;
        bool tiles = false;
        if (forced) {
            plan = *forced;
            tiles = true;
        } else if (!global_only) {
            tiles = ising::plan_bit1_tiles(L, device_cus(), &plan);
        }
        if (tiles) {
            HIP_TRY(ising::launch_sweep_bit1_tiles(planes, L, plan, n, t0, key, lat->lattice_id,
                                                   acc, Etr, Mtr, ws, kSpinLimit, count, st),
                    "sweep_bit1_tiles");
        } else {
            for (int64_t j = 0; j < n; ++j)
                for (int c = 0; c < 2; ++c)
                    HIP_TRY(ising::launch_halfsweep_bit1(
                                planes, L, c, 2u * (t0 + (uint32_t)j) + (uint32_t)c, key,
                                lat->lattice_id, acc, Etr ? Etr + j : nullptr,
                                Mtr ? Mtr + j : nullptr, ws_blocks(ws), count, st),
                            "halfsweep_bit1");
        }
    }
    if (Etr)
        HIP_TRY(ising::launch_prefix_i64(Etr, n, acc_ws + 2, st), "prefix");
    if (Mtr)
        HIP_TRY(ising::launch_prefix_i64(Mtr, n, acc_ws + 3, st), "prefix");
    lat->sweep_index += (uint64_t)n;
    return ISING_OK;
}

int ising_sweep(ising_lattice* lat, double beta, int64_t n, int64_t* E_dev, int64_t* M_dev,
                void* hip_stream) {
    return sweep_impl(lat, nullptr, beta, n, E_dev, M_dev, hip_stream, nullptr);
}

int ising_sweep_noalloc(ising_lattice* lat, double beta, int64_t n, int64_t* E_dev,
                        int64_t* M_dev, uint32_t* status_dev, void* hip_stream) {
    int rc = validate(lat, false);
    if (rc)
        return rc;
    if (lat->layout == ISING_LAYOUT_BIT1 && lat->L > kNoAllocMaxL)
        return set_error(ISING_E_UNSUPPORTED,
                         "ising_sweep_noalloc: BIT1 L = %d exceeds the scratch limit L <= %d "
                         "(%zu bytes); use ising_sweep with a workspace",
                         lat->L, kNoAllocMaxL, kScratchBytes);
    if (status_dev && (reinterpret_cast<uintptr_t>(status_dev) & 3u))
        return set_error(ISING_E_INVALID, "status_dev must be 4-byte aligned");
    if (n < 0)
        return set_error(ISING_E_INVALID, "n = %lld < 0", (long long)n);
    if (lat->sweep_index + (uint64_t)n > (1ull << 31))
        return set_error(ISING_E_INVALID, "sweep_index + n exceeds 2^31");
    uint32_t T[5];
    uint8_t alw[5];
    rc = ising_thresholds(beta, T, alw);
    if (rc)
        return rc;
    unsigned char* ws = nullptr;
    rc = scratch_of_current_device(&ws);
    if (rc)
        return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    // the array keeps the last call's contents: clear the accumulators, the
    // error word and the draw counters (the tile kernel clears its halo)
    HIP_TRY(ising::launch_fill_i64(ws_acc(ws), ising::WsLayout::kClearBytes / 8, 0, st), "fill");
    rc = sweep_impl(lat, ws, beta, n, E_dev, M_dev, hip_stream, nullptr);
    if (rc)
        return rc;
    if (status_dev)
        HIP_TRY(ising::launch_copy_u32(reinterpret_cast<const uint32_t*>(ws + ising::WsLayout::kErr),
                                       status_dev, st),
                "copy status");
    return ISING_OK;
}

int ising_sweep_tiles(ising_lattice* lat, double beta, int64_t n, int32_t rows, int32_t waves,
                      int64_t* E_dev, int64_t* M_dev, void* hip_stream) {
    int rc = validate(lat);
    if (rc)
        return rc;
    const int L = lat->L;
    if (lat->layout == ISING_LAYOUT_INT8) {
        if ((L & 7) != 0 || L > ising::kInt8TilesMaxL)
            return set_error(ISING_E_INVALID,
                             "ising_sweep_tiles: INT8 needs L %% 8 == 0 and L <= %d (L = %d)",
                             ising::kInt8TilesMaxL, L);
        if (rows < 1 || L % rows != 0 || L / rows < 2 || L / rows > ising::WsLayout::kMaxTiles)
            return set_error(ISING_E_INVALID, "rows = %d: must divide L = %d into 2..%d tiles",
                             rows, L, ising::WsLayout::kMaxTiles);
        if (waves < 1 || waves > 16)
            return set_error(ISING_E_INVALID, "waves = %d: must be in 1..16", waves);
        ising::Int8TilePlan p8;
        p8.ntiles = L / rows;
        p8.rows = rows;
        p8.threads = 64 * waves;
        p8.lds = (size_t)(rows + 2) * (size_t)L;
        if (p8.lds > (size_t)device_max_lds())
            return set_error(ISING_E_UNSUPPORTED, "a tile of %d rows needs %zu bytes of LDS",
                             rows, p8.lds);
        const int resident = ising::int8_tiles_resident(p8, E_dev || M_dev);
        if (resident < p8.ntiles)
            return set_error(ISING_E_UNSUPPORTED,
                             "%d tiles of %d rows x %d waves: only %d fit the device at once",
                             p8.ntiles, rows, waves, resident);
        return sweep_impl(lat, nullptr, beta, n, E_dev, M_dev, hip_stream, nullptr, &p8);
    }
    if (lat->layout != ISING_LAYOUT_BIT1)
        return set_error(ISING_E_INVALID, "unknown layout");
    if (rows < 1 || L % rows != 0 || L / rows < 2 || L / rows > ising::WsLayout::kMaxTiles)
        return set_error(ISING_E_INVALID,
                         "rows = %d: must divide L = %d into 2..%d tiles", rows, L,
                         ising::WsLayout::kMaxTiles);
    if (waves < 1 || waves > 16 || waves > rows)
        return set_error(ISING_E_INVALID, "waves = %d: must be in 1..min(16, rows = %d)", waves,
                         rows);
    ising::Bit1TilePlan plan;
    plan.ntiles = L / rows;
    plan.rows = rows;
    plan.threads = 64 * waves;
    plan.lds = ising::tile_lds_bytes(L, rows);
    if (plan.lds > (size_t)64 * 1024)
        return set_error(ISING_E_UNSUPPORTED, "a tile of %d rows needs %zu bytes of LDS (> 64 KiB)",
                         rows, plan.lds);
    uint32_t T[5];
    uint8_t alw[5];
    rc = ising_thresholds(beta, T, alw);
    if (rc)
        return rc;
    const int resident = ising::bit1_tiles_resident(
        L, plan, E_dev || M_dev, alw[3] || alw[4], (lat->flags & ISING_FLAG_COUNT_DRAWS) != 0);
    if (resident < plan.ntiles)
        return set_error(ISING_E_UNSUPPORTED,
                         "%d tiles of %d rows x %d waves: only %d fit the device at once",
                         plan.ntiles, rows, waves, resident);
    return sweep_impl(lat, nullptr, beta, n, E_dev, M_dev, hip_stream, &plan);
}

int ising_measure(const ising_lattice* lat, int64_t* E_dev, int64_t* M_dev, void* hip_stream) {
    int rc = validate(lat);
    if (rc)
        return rc;
    return measure_into(lat, ws_of(lat), reinterpret_cast<long long*>(E_dev),
                        reinterpret_cast<long long*>(M_dev), nullptr, nullptr,
                        reinterpret_cast<hipStream_t>(hip_stream));
}

int ising_to_int8(const ising_lattice* lat, int8_t* out_dev, void* hip_stream) {
    int rc = validate(lat);
    if (rc)
        return rc;
    if (!out_dev || (reinterpret_cast<uintptr_t>(out_dev) & 3u))
        return set_error(ISING_E_INVALID, "out_dev must be a non-NULL 4-byte aligned pointer");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    if (lat->layout == ISING_LAYOUT_INT8)
        HIP_TRY(ising::launch_convert_int8(reinterpret_cast<const int8_t*>(lat->spins), out_dev,
                                           (int64_t)lat->L * lat->L, st),
                "to_int8");
    else
        HIP_TRY(ising::launch_to_int8_bit1(reinterpret_cast<const uint32_t*>(lat->spins), lat->L,
                                           out_dev, st),
                "to_int8_bit1");
    return ISING_OK;
}

int ising_from_int8(ising_lattice* lat, const int8_t* in_dev, void* hip_stream) {
    int rc = validate(lat);
    if (rc)
        return rc;
    if (!in_dev || (reinterpret_cast<uintptr_t>(in_dev) & 3u))
        return set_error(ISING_E_INVALID, "in_dev must be a non-NULL 4-byte aligned pointer");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    if (lat->layout == ISING_LAYOUT_INT8)
        HIP_TRY(ising::launch_convert_int8(in_dev, reinterpret_cast<int8_t*>(lat->spins),
                                           (int64_t)lat->L * lat->L, st),
                "from_int8");
    else
        HIP_TRY(ising::launch_from_int8_bit1(reinterpret_cast<uint32_t*>(lat->spins), lat->L,
                                             in_dev, st),
                "from_int8_bit1");
    return ISING_OK;
}

int ising_rng_blocks(const ising_lattice* lat, uint64_t* blocks_host, void* hip_stream) {
    int rc = validate(lat);
    if (rc)
        return rc;
    if (!blocks_host)
        return set_error(ISING_E_INVALID, "blocks_host is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    uint64_t v[ising::WsLayout::kRngSlots] = {};
    HIP_TRY(hipMemcpyAsync(v, ws_blocks(ws_of(lat)), sizeof v, hipMemcpyDeviceToHost, st),
            "read block counters");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    uint64_t total = 0;
    for (uint64_t x : v)
        total += x;
    *blocks_host = total;
    return ISING_OK;
}

int ising_check_device_error(const ising_lattice* lat, void* hip_stream) {
    int rc = validate(lat);
    if (rc)
        return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    uint32_t* errp = reinterpret_cast<uint32_t*>(ws_of(lat) + ising::WsLayout::kErr);
    uint32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, errp, sizeof err, hipMemcpyDeviceToHost, st), "read error word");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    if (err) {
        const uint32_t zero = 0;
        HIP_TRY(hipMemcpyAsync(errp, &zero, sizeof zero, hipMemcpyHostToDevice, st),
                "clear error word");
        HIP_TRY(hipStreamSynchronize(st), "synchronise");
        return set_error(ISING_E_STATE,
                         "device error word 0x%x: an inter-tile wait timed out; spins undefined",
                         err);
    }
    return ISING_OK;
}

}  // extern "C"
