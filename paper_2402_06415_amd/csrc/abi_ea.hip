// extern "C" entry points of the spin glass with replica exchange
// (include/ising_ea.h): validation, threshold and swap tables, dispatch.
// No device memory is allocated here.
#include <math.h>

#include <vector>

#include "abi_common.hpp"
#include "ising_ea.h"
#include "ea.hpp"

namespace {

using ising::EaLayout;
using ising::EaSwapMeta;
using ising::abi::aligned256;
using ising::abi::set_error;

int validate(const ising_ea* ea) {
    if (!ea)
        return set_error(ISING_E_INVALID, "spin-glass pointer is NULL");
    if (ea->abi_version != ISING_ABI_VERSION)
        return set_error(ISING_E_INVALID, "abi_version %d, library has %d", ea->abi_version,
                         ISING_ABI_VERSION);
    if (ea->L < 8 || ea->L > ISING_EA_MAX_L || (ea->L & (ea->L - 1)))
        return set_error(ISING_E_INVALID, "L = %d: a power of two in 8..%d", ea->L,
                         ISING_EA_MAX_L);
    if (ea->replicas < 1 || ea->replicas > ISING_EA_MAX_REPLICAS)
        return set_error(ISING_E_INVALID, "replicas = %d outside 1..%d", ea->replicas,
                         ISING_EA_MAX_REPLICAS);
    if (ea->draws != ISING_DRAWS_SITE && ea->draws != ISING_DRAWS_PLANE)
        return set_error(ISING_E_INVALID, "draws = %d: ISING_DRAWS_SITE or ISING_DRAWS_PLANE",
                         ea->draws);
    if (ea->draws == ISING_DRAWS_PLANE && ea->L < 64)
        return set_error(ISING_E_INVALID, "L = %d: plane draws need L >= 64", ea->L);
    if (!ea->spins || !aligned256(ea->spins) || !ea->bonds || !aligned256(ea->bonds) ||
        !ea->workspace || !aligned256(ea->workspace))
        return set_error(ISING_E_INVALID,
                         "spins, bonds and workspace must be non-NULL 256-byte aligned pointers");
    return ISING_OK;
}

ising::Key key_of(const ising_ea* ea) {
    return ising::Key{(uint32_t)(ea->seed & 0xFFFFFFFFu), (uint32_t)(ea->seed >> 32)};
}

unsigned char* ws_of(const ising_ea* ea) { return reinterpret_cast<unsigned char*>(ea->workspace); }

// ceil(2^32 exp(-x)) as the acceptance threshold of a draw; false if it
// rounds up to 2^32 (the move would always be accepted).
bool threshold(double x, uint32_t* T) {
    const double t = ceil(ldexp(exp(-x), 32));
    if (t >= 4294967296.0)
        return false;
    *T = (uint32_t)t;
    return true;
}

}  // namespace

extern "C" {

size_t ising_ea_spins_bytes(int32_t L, int32_t replicas) {
    if (L < 8 || L > ISING_EA_MAX_L || (L & (L - 1)) || replicas < 1 ||
        replicas > ISING_EA_MAX_REPLICAS)
        return 0;
    return (size_t)replicas * (size_t)L * L * L;
}

size_t ising_ea_workspace_bytes(int32_t L, int32_t replicas) {
    if (ising_ea_spins_bytes(L, replicas) == 0)
        return 0;
    return ising::ea_ws_layout(L, replicas).bytes;
}

int ising_ea_setup(const ising_ea* ea, const double* beta_host, void* hip_stream) {
    int rc = validate(ea);
    if (rc)
        return rc;
    if (!beta_host)
        return set_error(ISING_E_INVALID, "beta_host is NULL");
    const int R = ea->replicas;
    for (int k = 0; k < R; ++k) {
        if (!(beta_host[k] >= 0.0) || isinf(beta_host[k]))
            return set_error(ISING_E_INVALID, "beta[%d] = %g: must be finite and >= 0", k,
                             beta_host[k]);
        if (k > 0 && !(beta_host[k] > beta_host[k - 1]))
            return set_error(ISING_E_INVALID, "the betas must increase strictly (index %d)", k);
    }
    const EaLayout lay = ising::ea_ws_layout(ea->L, R);
    // Metropolis thresholds per temperature: T2, T4, T6 as compared, and the
    // need of each class (0 where the class always flips)
    std::vector<uint32_t> thr((size_t)R * 6);
    for (int k = 0; k < R; ++k) {
        const uint32_t need[3] = {0x01010101u, 0x02020202u, 0x03030303u};
        for (int i = 0; i < 3; ++i) {
            const int u = 2 * (i + 1);
            uint32_t T = 0;
            const bool drawn = threshold(beta_host[k] * (double)(2 * u), &T);
            thr[(size_t)k * 6 + i] = drawn ? T : 0xFFFFFFFFu;
            thr[(size_t)k * 6 + 3 + i] = drawn ? need[i] : 0u;
        }
    }
    // swap thresholds per pair for D = 4q: the exact host values
    std::vector<EaSwapMeta> meta((size_t)R);
    std::vector<uint32_t> tab((size_t)R * ising::kEaSwapTable, 0u);
    for (int k = 0; k + 1 < R; ++k) {
        const double lo = beta_host[k], hi = beta_host[k + 1];
        auto T_of = [&](uint64_t q, uint32_t* T) {
            return threshold((hi - lo) * (double)(4 * q), T);
        };
        uint64_t q = 1;
        for (;; ++q) {
            uint32_t T = 0;
            if (!T_of(q, &T))
                return set_error(ISING_E_UNSUPPORTED, "betas %g and %g too close for the swap table",
                                 lo, hi);
            if (T == 1)
                break;
            if (q >= (uint64_t)ising::kEaSwapTable)
                return set_error(ISING_E_UNSUPPORTED,
                                 "betas %g and %g: swap table longer than %d entries", lo, hi,
                                 ising::kEaSwapTable);
            tab[(size_t)k * ising::kEaSwapTable + q] = T;
        }
        meta[k].len = q;
        // first q with T = 0 (exp underflows); T is non-increasing in q
        uint64_t a = q, b = q;
        uint32_t T = 1;
        while (T_of(b, &T) && T != 0 && b < (1ull << 61))
            b *= 2;
        if (T != 0) {
            meta[k].zero_from = ~0ull;
        } else {
            while (b - a > 1) {
                const uint64_t mid = a + (b - a) / 2;
                uint32_t Tm = 1;
                T_of(mid, &Tm);
                if (Tm == 0)
                    b = mid;
                else
                    a = mid;
            }
            meta[k].zero_from = b;
        }
    }
    const uint32_t head[2] = {ising::kEaMagic, (uint32_t)R};
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = ws_of(ea);
    HIP_TRY(hipMemcpyAsync(ws + lay.thr, thr.data(), thr.size() * 4, hipMemcpyHostToDevice, st),
            "copy thresholds");
    HIP_TRY(hipMemcpyAsync(ws + lay.swap_meta, meta.data(), meta.size() * sizeof(EaSwapMeta),
                           hipMemcpyHostToDevice, st),
            "copy swap metadata");
    HIP_TRY(hipMemcpyAsync(ws + lay.swap_tab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, st),
            "copy swap table");
    HIP_TRY(hipMemcpyAsync(ws, head, sizeof head, hipMemcpyHostToDevice, st), "copy header");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    return ISING_OK;
}

int ising_ea_init(const ising_ea* ea, int32_t start, void* hip_stream) {
    int rc = validate(ea);
    if (rc)
        return rc;
    if (start != ISING_START_COLD_UP && start != ISING_START_RANDOM)
        return set_error(ISING_E_INVALID, "unknown start %d", start);
    const EaLayout lay = ising::ea_ws_layout(ea->L, ea->replicas);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = ws_of(ea);
    HIP_TRY(ising::launch_ea_prepare(ws, lay, ea->replicas, 0, ising::kEaPrepareInit, st),
            "ea prepare");
    HIP_TRY(ising::launch_ea_init(ws, ea->spins, ea->L, ea->replicas, start, key_of(ea), st),
            "ea init");
    HIP_TRY(ising::launch_ea_energy(ws, ea->spins, ea->bonds, ea->L, ea->replicas,
                                    reinterpret_cast<long long*>(ws + lay.E), st),
            "ea energy");
    return ISING_OK;
}

int ising_ea_sweep(const ising_ea* ea, int64_t n, int32_t every, int64_t* trace_dev,
                   void* hip_stream) {
    int rc = validate(ea);
    if (rc)
        return rc;
    if (n < 0 || n > (1ll << 31))
        return set_error(ISING_E_INVALID, "n = %lld outside 0..2^31", (long long)n);
    if (every < 0)
        return set_error(ISING_E_INVALID, "every = %d < 0", every);
    if (n == 0)
        return ISING_OK;
    const EaLayout lay = ising::ea_ws_layout(ea->L, ea->replicas);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = ws_of(ea);
    HIP_TRY(ising::launch_ea_prepare(ws, lay, ea->replicas, n, ising::kEaPrepareSweep, st),
            "ea prepare");
    if (ea->draws == ISING_DRAWS_PLANE) {
        HIP_TRY(ising::launch_ea_pack_bonds(ws, lay, ea->bonds, ea->L, st), "ea pack couplings");
        HIP_TRY(ising::launch_ea_pack_spins(ws, lay, ea->spins, ea->L, ea->replicas, st),
                "ea pack spins");
        for (int64_t j = 0; j < n; ++j)
            HIP_TRY(ising::launch_ea_sweep_bit(ws, lay, ea->L, ea->replicas, every, key_of(ea),
                                               trace_dev, st),
                    "ea sweep");
        HIP_TRY(ising::launch_ea_unpack_spins(ws, lay, ea->spins, ea->L, ea->replicas, st),
                "ea unpack spins");
        return ISING_OK;
    }
    for (int64_t j = 0; j < n; ++j)
        HIP_TRY(ising::launch_ea_sweep(ws, lay, ea->spins, ea->bonds, ea->L, ea->replicas, every,
                                       key_of(ea), trace_dev, st),
                "ea sweep");
    return ISING_OK;
}

int ising_ea_measure(const ising_ea* ea, int64_t* E_dev, void* hip_stream) {
    int rc = validate(ea);
    if (rc)
        return rc;
    if (!E_dev)
        return set_error(ISING_E_INVALID, "E_dev is NULL");
    const EaLayout lay = ising::ea_ws_layout(ea->L, ea->replicas);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    HIP_TRY(ising::launch_ea_prepare(ws_of(ea), lay, ea->replicas, 0, ising::kEaPrepareMeasure, st),
            "ea prepare");
    HIP_TRY(ising::launch_ea_energy(ws_of(ea), ea->spins, ea->bonds, ea->L, ea->replicas,
                                    reinterpret_cast<long long*>(E_dev), st),
            "ea energy");
    return ISING_OK;
}

int ising_ea_state(const ising_ea* ea, uint64_t* t_host, int32_t* perm_host, int64_t* E_host,
                   uint64_t* accepts_host, void* hip_stream) {
    int rc = validate(ea);
    if (rc)
        return rc;
    const int R = ea->replicas;
    const EaLayout lay = ising::ea_ws_layout(ea->L, R);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = ws_of(ea);
    if (t_host)
        HIP_TRY(hipMemcpyAsync(t_host, ws + 8, 8, hipMemcpyDeviceToHost, st), "read t");
    if (perm_host)
        HIP_TRY(hipMemcpyAsync(perm_host, ws + lay.perm, (size_t)R * 4, hipMemcpyDeviceToHost, st),
                "read order");
    if (E_host)
        HIP_TRY(hipMemcpyAsync(E_host, ws + lay.E, (size_t)R * 8, hipMemcpyDeviceToHost, st),
                "read energies");
    if (accepts_host && R > 1)
        HIP_TRY(hipMemcpyAsync(accepts_host, ws + lay.accepts, (size_t)(R - 1) * 8,
                               hipMemcpyDeviceToHost, st),
                "read swap counts");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    return ISING_OK;
}

int ising_ea_rng_blocks(const ising_ea* ea, uint64_t* blocks_host, void* hip_stream) {
    int rc = validate(ea);
    if (rc)
        return rc;
    if (!blocks_host)
        return set_error(ISING_E_INVALID, "blocks_host is NULL");
    const EaLayout lay = ising::ea_ws_layout(ea->L, ea->replicas);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipMemcpyAsync(blocks_host, ws_of(ea) + lay.rng_blocks, 8, hipMemcpyDeviceToHost, st),
            "read block counter");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    return ISING_OK;
}

int ising_ea_check_device_error(const ising_ea* ea, void* hip_stream) {
    int rc = validate(ea);
    if (rc)
        return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    uint32_t* errp = reinterpret_cast<uint32_t*>(ws_of(ea) + 28);
    uint32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, errp, 4, hipMemcpyDeviceToHost, st), "read error word");
    HIP_TRY(hipStreamSynchronize(st), "synchronise");
    if (err) {
        const uint32_t zero = 0;
        HIP_TRY(hipMemcpyAsync(errp, &zero, 4, hipMemcpyHostToDevice, st), "clear error word");
        HIP_TRY(hipStreamSynchronize(st), "synchronise");
        return set_error(ISING_E_STATE, "spin-glass device error word 0x%x:%s%s%s", err,
                         (err & ising::kEaErrNotSetUp) ? " workspace not set up;" : "",
                         (err & ising::kEaErrSweepIndex) ? " sweep index + n exceeds 2^31;" : "",
                         (err & ising::kEaErrEnergy) ? " energy difference not a multiple of 4;" : "");
    }
    return ISING_OK;
}

}  // extern "C"
