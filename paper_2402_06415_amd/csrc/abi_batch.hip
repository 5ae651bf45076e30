// extern "C" entry points of the batch API (include/ising.h, "Batches of
// small lattices"): validation, descriptor tables, launch shapes and the
// autotuner.  No device memory is allocated here.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "abi_common.hpp"
#include "ising.h"
#include "batch.hpp"

namespace {

using ising::BatchDesc;
using ising::BatchWs;
using ising::abi::aligned256;
using ising::abi::device_cus;
using ising::abi::set_error;

constexpr size_t kLdsPerCU = 160 * 1024;  // gfx950
constexpr int kThreadsPerCU = 2048;       // 32 waves of 64

bool valid_batch_L(int32_t L, int32_t max_L) {
    return L >= 8 && L <= max_L && (L % 8) == 0;
}

int validate(const ising_batch* b) {
    if (!b)
        return set_error(ISING_E_INVALID, "batch pointer is NULL");
    if (b->abi_version != ISING_ABI_VERSION)
        return set_error(ISING_E_INVALID, "abi_version %d, library has %d", b->abi_version,
                         ISING_ABI_VERSION);
    if (b->count < 1 || b->count > ISING_BATCH_MAX_COUNT)
        return set_error(ISING_E_INVALID, "count %d outside 1..%d", b->count,
                         ISING_BATCH_MAX_COUNT);
    if ((uint64_t)b->lattice_id0 + (uint64_t)b->count - 1 > 0xFFFFFFFFull)
        return set_error(ISING_E_INVALID, "lattice_id0 + count - 1 exceeds 2^32 - 1");
    if (!valid_batch_L(b->max_L, ISING_BATCH_MAX_L))
        return set_error(ISING_E_INVALID, "max_L = %d: must be a multiple of 8 in 8..%d",
                         b->max_L, ISING_BATCH_MAX_L);
    if (b->threads != 0 && (b->threads < 64 || b->threads > 1024 || b->threads % 64))
        return set_error(ISING_E_INVALID, "threads = %d: 0 or a multiple of 64 in 64..1024",
                         b->threads);
    if (b->groups_per_cu < 0 || b->groups_per_cu > 16)
        return set_error(ISING_E_INVALID, "groups_per_cu = %d outside 0..16", b->groups_per_cu);
    if (b->draws != ISING_DRAWS_SITE && b->draws != ISING_DRAWS_PLANE)
        return set_error(ISING_E_INVALID, "draws = %d: ISING_DRAWS_SITE or ISING_DRAWS_PLANE",
                         b->draws);
    if (b->reserved != 0)
        return set_error(ISING_E_INVALID, "reserved must be 0");
    if (!b->spins || !aligned256(b->spins))
        return set_error(ISING_E_INVALID, "spins must be a non-NULL 256-byte aligned device pointer");
    if (!b->workspace || !aligned256(b->workspace))
        return set_error(ISING_E_INVALID,
                         "workspace must be a non-NULL 256-byte aligned device pointer");
    return ISING_OK;
}

ising::Key key_of(const ising_batch* b) {
    return ising::Key{(uint32_t)(b->seed & 0xFFFFFFFFu), (uint32_t)(b->seed >> 32)};
}

unsigned char* ws_of(const ising_batch* b) { return reinterpret_cast<unsigned char*>(b->workspace); }

struct Shape {
    int threads, groups_per_cu;
};

// Workgroups per CU that fit LDS and the thread limit for this shape.
int fit_groups(int threads, int want, int max_L, int draws) {
    const size_t lds = (draws == ISING_DRAWS_PLANE ? ising::batch_bit_lds_bytes(threads, max_L)
                                                   : ising::batch_lds_bytes(max_L)) +
                       2048;  // + static LDS of the kernel
    int g = want;
    g = std::min<int>(g, (int)(kLdsPerCU / lds));
    g = std::min<int>(g, kThreadsPerCU / threads);
    return std::max(g, 1);
}

// The launch shape of a batch: its own fields, else 512 threads and as
// many workgroups per CU as fit.
Shape shape_of(const ising_batch* b) {
    Shape s;
    s.threads = b->threads ? b->threads : 512;
    s.groups_per_cu =
        fit_groups(s.threads, b->groups_per_cu ? b->groups_per_cu : 16, b->max_L, b->draws);
    return s;
}

int grid_of(const ising_batch* b, const Shape& s) {
    const int cus = std::max(device_cus(), 1);
    return std::max(1, std::min(b->count, cus * s.groups_per_cu));
}

// Dynamic LDS of a plane-draw workgroup: its share of the CU's LDS (at most
// 128 KiB), and at least both planes of one lattice of side max_L.
size_t plane_lds_bytes(const ising_batch* b, const Shape& s) {
    const size_t need = ising::batch_bit_lds_bytes(s.threads, b->max_L);
    size_t share = kLdsPerCU / (size_t)s.groups_per_cu;
    share = share > 2048 ? share - 2048 : 0;  // static LDS of the kernel
    share = std::min<size_t>(share, 128 * 1024) & ~(size_t)255;
    return std::max(need, share);
}

// The sweep kernel of the batch's draw mode.
hipError_t launch_sweep_of(const ising_batch* b, unsigned char* ws, bool scratch_t, int8_t* spins,
                           int64_t n, int64_t* moments, int64_t* trace, const Shape& s, int grid,
                           hipStream_t st) {
    if (b->draws == ISING_DRAWS_PLANE)
        return ising::launch_batch_sweep_bit(ws, scratch_t, b->count, spins, n, key_of(b),
                                             moments, trace, s.threads, grid,
                                             plane_lds_bytes(b, s), st);
    return ising::launch_batch_sweep(ws, scratch_t, b->count, spins, b->max_L, n, key_of(b),
                                     moments, trace, s.threads, grid, st);
}

}  // namespace

extern "C" {

size_t ising_batch_spins_bytes(int32_t count, const int32_t* L_host, uint64_t* offsets_host) {
    if (count < 1 || count > ISING_BATCH_MAX_COUNT || !L_host)
        return 0;
    uint64_t off = 0;
    for (int32_t j = 0; j < count; ++j) {
        if (!valid_batch_L(L_host[j], ISING_BATCH_MAX_L))
            return 0;
        if (offsets_host)
            offsets_host[j] = off;
        off += ((uint64_t)L_host[j] * (uint64_t)L_host[j] + 255u) & ~(uint64_t)255u;
    }
    return (size_t)off;
}

size_t ising_batch_workspace_bytes(int32_t count) {
    if (count < 1 || count > ISING_BATCH_MAX_COUNT)
        return 0;
    return BatchWs::bytes(count);
}

int ising_batch_setup(const ising_batch* b, const int32_t* L_host, const double* beta_host,
                      void* hip_stream) {
    int rc = validate(b);
    if (rc)
        return rc;
    if (!L_host || !beta_host)
        return set_error(ISING_E_INVALID, "L_host and beta_host must be non-NULL");
    const int count = b->count;
    if (b->draws == ISING_DRAWS_PLANE)
        for (int j = 0; j < count; ++j)
            if (L_host[j] != 32 && L_host[j] % 64 != 0)
                return set_error(ISING_E_INVALID,
                                 "L[%d] = %d: plane draws need L = 32 or a multiple of 64", j,
                                 L_host[j]);
    std::vector<uint64_t> off(count);
    for (int j = 0; j < count; ++j)
        if (L_host[j] > b->max_L && valid_batch_L(L_host[j], ISING_BATCH_MAX_L))
            return set_error(ISING_E_INVALID, "L[%d] = %d exceeds max_L = %d", j, L_host[j],
                             b->max_L);
    const size_t need = ising_batch_spins_bytes(count, L_host, off.data());
    if (need == 0)
        return set_error(ISING_E_INVALID, "every L must be a multiple of 8 in 8..%d",
                         ISING_BATCH_MAX_L);
    if (need > b->spins_bytes)
        return set_error(ISING_E_INVALID, "spins_bytes %llu < %zu needed",
                         (unsigned long long)b->spins_bytes, need);
    std::vector<BatchDesc> desc(count);
    for (int j = 0; j < count; ++j) {
        uint32_t T[5];
        uint8_t alw[5];
        rc = ising_thresholds(beta_host[j], T, alw);
        if (rc)
            return set_error(ISING_E_INVALID, "beta[%d] = %g: must be finite and >= 0", j,
                             beta_host[j]);
        BatchDesc& d = desc[j];
        d.off = off[j];
        d.L = L_host[j];
        d.lid = b->lattice_id0 + (uint32_t)j;
        d.T2 = T[3];
        d.T4 = T[4];
        d.always = (alw[3] ? 1u : 0u) | (alw[4] ? 2u : 0u);
        d.pad = 0;
    }
    // queue order: largest lattice first (longest-processing-time), ties by index
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t c) { return L_host[a] > L_host[c]; });
    const uint32_t draws = (uint32_t)b->draws;
    const uint32_t head[2] = {ising::kBatchMagic, (uint32_t)count};
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = ws_of(b);
    HIP_TRY(hipMemcpyAsync(ws + BatchWs::kDraws, &draws, sizeof draws, hipMemcpyHostToDevice, st),
            "copy draw mode");
    HIP_TRY(hipMemcpyAsync(ws + BatchWs::kOrder, order.data(), order.size() * 4,
                           hipMemcpyHostToDevice, st),
            "copy queue order");
    HIP_TRY(hipMemcpyAsync(ws + BatchWs::desc_offset(count), desc.data(),
                           desc.size() * sizeof(BatchDesc), hipMemcpyHostToDevice, st),
            "copy descriptors");
    HIP_TRY(hipMemcpyAsync(ws + BatchWs::kMagic, head, sizeof head, hipMemcpyHostToDevice, st),
            "copy header");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    return ISING_OK;
}

int ising_batch_init(const ising_batch* b, int32_t start, void* hip_stream) {
    int rc = validate(b);
    if (rc)
        return rc;
    if (start != ISING_START_COLD_UP && start != ISING_START_RANDOM)
        return set_error(ISING_E_INVALID, "unknown start %d", start);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    HIP_TRY(ising::launch_batch_prepare(ws_of(b), false, b->count, b->spins_bytes, b->max_L, 0,
                                        ising::kPrepareInit, b->draws, st),
            "batch prepare");
    HIP_TRY(ising::launch_batch_init(ws_of(b), b->count, b->spins, start, key_of(b), st),
            "batch init");
    return ISING_OK;
}

int ising_batch_sweep(const ising_batch* b, int64_t n, int64_t* moments_dev, int64_t* trace_dev,
                      void* hip_stream) {
    int rc = validate(b);
    if (rc)
        return rc;
    if (n < 0 || n > (1ll << 31))
        return set_error(ISING_E_INVALID, "n = %lld outside 0..2^31", (long long)n);
    if (n == 0)
        return ISING_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const Shape s = shape_of(b);
    HIP_TRY(ising::launch_batch_prepare(ws_of(b), false, b->count, b->spins_bytes, b->max_L, n,
                                        ising::kPrepareSweep, b->draws, st),
            "batch prepare");
    HIP_TRY(launch_sweep_of(b, ws_of(b), false, b->spins, n, moments_dev, trace_dev, s,
                            grid_of(b, s), st),
            "batch sweep");
    HIP_TRY(ising::launch_batch_advance(ws_of(b), n, st), "batch advance");
    return ISING_OK;
}

int ising_batch_measure(const ising_batch* b, int64_t* E_dev, int64_t* M_dev, void* hip_stream) {
    int rc = validate(b);
    if (rc)
        return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    HIP_TRY(ising::launch_batch_prepare(ws_of(b), false, b->count, b->spins_bytes, b->max_L, 0,
                                        ising::kPrepareMeasure, b->draws, st),
            "batch prepare");
    HIP_TRY(ising::launch_batch_measure(ws_of(b), b->count, b->spins, E_dev, M_dev, st),
            "batch measure");
    return ISING_OK;
}

int ising_batch_sweep_index(const ising_batch* b, uint64_t* t_host, void* hip_stream) {
    int rc = validate(b);
    if (rc)
        return rc;
    if (!t_host)
        return set_error(ISING_E_INVALID, "t_host is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipMemcpyAsync(t_host, ws_of(b) + BatchWs::kT, 8, hipMemcpyDeviceToHost, st),
            "read sweep index");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    return ISING_OK;
}

int ising_batch_rng_blocks(const ising_batch* b, uint64_t* blocks_host, void* hip_stream) {
    int rc = validate(b);
    if (rc)
        return rc;
    if (!blocks_host)
        return set_error(ISING_E_INVALID, "blocks_host is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    uint64_t v[64] = {};
    HIP_TRY(hipMemcpyAsync(v, ws_of(b) + BatchWs::kRngBlocks, sizeof v, hipMemcpyDeviceToHost, st),
            "read block counters");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    uint64_t total = 0;
    for (uint64_t x : v)
        total += x;
    *blocks_host = total;
    return ISING_OK;
}

int ising_batch_check_device_error(const ising_batch* b, void* hip_stream) {
    int rc = validate(b);
    if (rc)
        return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    uint32_t* errp = reinterpret_cast<uint32_t*>(ws_of(b) + BatchWs::kErr);
    uint32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, errp, sizeof err, hipMemcpyDeviceToHost, st), "read error word");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    if (err) {
        const uint32_t zero = 0;
        HIP_TRY(hipMemcpyAsync(errp, &zero, sizeof zero, hipMemcpyHostToDevice, st),
                "clear error word");
        HIP_TRY(hipStreamSynchronize(st), "synchronise");
        return set_error(ISING_E_STATE, "batch device error word 0x%x:%s%s%s%s%s", err,
                         (err & ising::kBatchErrNotSetUp) ? " workspace not set up for this batch;" : "",
                         (err & ising::kBatchErrDescriptor) ? " descriptor outside spins or max_L;" : "",
                         (err & ising::kBatchErrSweepIndex) ? " sweep index + n exceeds 2^31;" : "",
                         (err & ising::kBatchErrShape) ? " a lattice's side differs from the proposals';" : "",
                         (err & ising::kBatchErrDraws) ? " draw mode differs from setup's;" : "");
    }
    return ISING_OK;
}

int ising_batch_autotune(ising_batch* b, int8_t* scratch_spins, int64_t probe_sweeps,
                         double* times_ms_host, int32_t max_times, int32_t* n_times,
                         void* hip_stream) {
    int rc = validate(b);
    if (rc)
        return rc;
    if (probe_sweeps < 1 || probe_sweeps > 1000000)
        return set_error(ISING_E_INVALID, "probe_sweeps = %lld outside 1..10^6",
                         (long long)probe_sweeps);
    if (!scratch_spins || !aligned256(scratch_spins) || scratch_spins == b->spins)
        return set_error(ISING_E_INVALID,
                         "scratch_spins must be a 256-byte aligned device buffer other than spins");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = ws_of(b);
    std::vector<Shape> cand;
    for (int threads : {128, 256, 512, 1024})
        for (int g : {1, 2, 4, 8, 16}) {
            const int fit = fit_groups(threads, g, b->max_L, b->draws);
            if (fit != g)
                continue;
            cand.push_back({threads, g});
        }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0), "event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(ISING_E_HIP, "event");
    }
    ising_batch probe = *b;
    probe.spins = scratch_spins;
    Shape best{0, 0};
    float best_ms = 0.f;
    int timed = 0;
    hipError_t err = hipSuccess;
    for (const Shape& s : cand) {
        // the probe starts from the batch's spins and sweep index each time
        err = hipMemcpyAsync(scratch_spins, b->spins, b->spins_bytes, hipMemcpyDeviceToDevice, st);
        if (err == hipSuccess)
            err = hipMemcpyAsync(ws + BatchWs::kTScratch, ws + BatchWs::kT, 8,
                                 hipMemcpyDeviceToDevice, st);
        if (err == hipSuccess)
            err = ising::launch_batch_prepare(ws, true, b->count, b->spins_bytes, b->max_L,
                                              probe_sweeps, ising::kPrepareSweep, b->draws, st);
        if (err == hipSuccess)
            err = hipEventRecord(e0, st);
        probe.threads = s.threads;
        probe.groups_per_cu = s.groups_per_cu;
        if (err == hipSuccess)
            err = launch_sweep_of(b, ws, true, scratch_spins, probe_sweeps, nullptr, nullptr, s,
                                  grid_of(&probe, s), st);
        if (err == hipSuccess)
            err = hipEventRecord(e1, st);
        if (err == hipSuccess)
            err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess)
            err = hipEventElapsedTime(&ms, e0, e1);
        if (err != hipSuccess)
            break;
        if (times_ms_host && timed < max_times) {
            times_ms_host[3 * timed + 0] = s.threads;
            times_ms_host[3 * timed + 1] = s.groups_per_cu;
            times_ms_host[3 * timed + 2] = ms;
        }
        ++timed;
        if (best.threads == 0 || ms < best_ms) {
            best = s;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess)
        return ising::abi::hip_fail(err, "autotune");
    if (n_times)
        *n_times = timed;
    b->threads = best.threads;
    b->groups_per_cu = best.groups_per_cu;
    return ISING_OK;
}

}  // extern "C"
