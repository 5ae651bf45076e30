// extern "C" entry points of the 2D XY model (include/ising_xy.h):
// validation and dispatch.  No device memory is allocated here.
#include <math.h>

#include "abi_common.hpp"
#include "ising_xy.h"
#include "xy.hpp"

namespace {

using ising::abi::aligned256;
using ising::abi::set_error;

int validate(const ising_xy* xy) {
    if (!xy)
        return set_error(ISING_E_INVALID, "XY pointer is NULL");
    if (xy->abi_version != ISING_ABI_VERSION)
        return set_error(ISING_E_INVALID, "abi_version %d, library has %d", xy->abi_version,
                         ISING_ABI_VERSION);
    if (xy->L < 2 || xy->L > ISING_XY_MAX_L || (xy->L & 1))
        return set_error(ISING_E_INVALID, "L = %d: even, 2..%d", xy->L, ISING_XY_MAX_L);
    if (xy->count < 1 || xy->count > ISING_XY_MAX_COUNT)
        return set_error(ISING_E_INVALID, "count = %d outside 1..%d", xy->count,
                         ISING_XY_MAX_COUNT);
    if ((uint64_t)xy->lattice_id0 + (uint64_t)xy->count - 1 > 0xFFFFFFFFull)
        return set_error(ISING_E_INVALID, "lattice_id0 + count - 1 exceeds 2^32 - 1");
    if (!xy->theta || !aligned256(xy->theta) || !xy->workspace || !aligned256(xy->workspace))
        return set_error(ISING_E_INVALID,
                         "theta and workspace must be non-NULL 256-byte aligned device pointers");
    return ISING_OK;
}

ising::Key key_of(const ising_xy* xy) {
    return ising::Key{(uint32_t)(xy->seed & 0xFFFFFFFFu), (uint32_t)(xy->seed >> 32)};
}

unsigned char* ws_of(const ising_xy* xy) { return reinterpret_cast<unsigned char*>(xy->workspace); }

}  // namespace

extern "C" {

size_t ising_xy_workspace_bytes(int32_t L, int32_t count) {
    if (L < 2 || L > ISING_XY_MAX_L || (L & 1) || count < 1 || count > ISING_XY_MAX_COUNT)
        return 0;
    return ising::xy_workspace_bytes(L, count);
}

int ising_xy_init(const ising_xy* xy, int32_t start, void* hip_stream) {
    int rc = validate(xy);
    if (rc)
        return rc;
    if (start != ISING_START_COLD_UP && start != ISING_START_RANDOM)
        return set_error(ISING_E_INVALID, "unknown start %d", start);
    HIP_TRY(ising::launch_xy_init(ws_of(xy), xy->theta, xy->L, xy->count, start, key_of(xy),
                                  xy->lattice_id0, reinterpret_cast<hipStream_t>(hip_stream)),
            "xy init");
    return ISING_OK;
}

int ising_xy_sweep(const ising_xy* xy, double beta, int64_t n, double* E_trace_dev,
                   void* hip_stream) {
    int rc = validate(xy);
    if (rc)
        return rc;
    if (!(beta >= 0.0) || isinf(beta))
        return set_error(ISING_E_INVALID, "beta must be finite and >= 0 (got %g)", beta);
    if (n < 0 || n > (1ll << 31))
        return set_error(ISING_E_INVALID, "n = %lld outside 0..2^31", (long long)n);
    if (n == 0)
        return ISING_OK;
    HIP_TRY(ising::launch_xy_sweep(ws_of(xy), xy->theta, xy->L, xy->count, n, beta, key_of(xy),
                                   xy->lattice_id0, E_trace_dev,
                                   reinterpret_cast<hipStream_t>(hip_stream)),
            "xy sweep");
    return ISING_OK;
}

int ising_xy_energy(const ising_xy* xy, double* E_dev, void* hip_stream) {
    int rc = validate(xy);
    if (rc)
        return rc;
    if (!E_dev)
        return set_error(ISING_E_INVALID, "E_dev is NULL");
    HIP_TRY(ising::launch_xy_energy(xy->theta, xy->L, xy->count, E_dev,
                                    reinterpret_cast<hipStream_t>(hip_stream)),
            "xy energy");
    return ISING_OK;
}

int ising_xy_state(const ising_xy* xy, uint64_t* t_host, uint64_t* accepted_host,
                   void* hip_stream) {
    int rc = validate(xy);
    if (rc)
        return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    if (t_host)
        HIP_TRY(hipMemcpyAsync(t_host, ws_of(xy) + 8, 8, hipMemcpyDeviceToHost, st), "read t");
    if (accepted_host)
        HIP_TRY(hipMemcpyAsync(accepted_host, ws_of(xy) + ising::kXyAccepted,
                               (size_t)xy->count * 8, hipMemcpyDeviceToHost, st),
                "read counters");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    return ISING_OK;
}

int ising_xy_check_device_error(const ising_xy* xy, void* hip_stream) {
    int rc = validate(xy);
    if (rc)
        return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    uint32_t* errp = reinterpret_cast<uint32_t*>(ws_of(xy) + 28);
    uint32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, errp, 4, hipMemcpyDeviceToHost, st), "read error word");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    if (err) {
        const uint32_t zero = 0;
        HIP_TRY(hipMemcpyAsync(errp, &zero, 4, hipMemcpyHostToDevice, st), "clear error word");
        HIP_TRY(hipStreamSynchronize(st), "synchronise");
        return set_error(ISING_E_STATE, "XY device error word 0x%x:%s%s%s", err,
                         (err & ising::kXyErrNotInit) ? " workspace not initialised;" : "",
                         (err & ising::kXyErrSweepIndex) ? " sweep index + n exceeds 2^31;" : "",
                         (err & ising::kXyErrHandoff) ? " hand-off between bands timed out;" : "");
    }
    return ISING_OK;
}

}  // extern "C"
