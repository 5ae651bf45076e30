// Hand-off of rows between the workgroups of a persistent sweep (internal to
// libising.so).
//
// A row is handed over through slots of 64-bit words, each carrying a
// 32-bit data word and, in the high half, a tag: the number of the
// half-sweep that produced it plus one.  A reader polls its own word until
// the tag is the one it expects, so each hand-off involves a single memory
// location (relaxed agent-scope atomics: no cache write-back or
// invalidation, no grid-wide barrier).  Waits are bounded: on time-out
// `code` is or-ed into the device error word and the word read last is
// used, so the kernel still runs to completion.
#pragma once

#include "common.hpp"

namespace ising {

__device__ __forceinline__ uint32_t wait_slot(const unsigned long long* slot, uint32_t tag,
                                              uint32_t limit, uint32_t* err, uint32_t code = 1u) {
    uint32_t spins = 0;
    unsigned long long v;
    for (;;) {
        v = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == tag)
            break;
        if (++spins > limit) {
            atomicOr(err, code);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return (uint32_t)v;
}

__device__ __forceinline__ void publish_slot(unsigned long long* slot, uint32_t tag,
                                             uint32_t word) {
    __hip_atomic_store(slot, ((unsigned long long)tag << 32) | word, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// The rest of a wait whose first load was issued early: poll the slot until
// its tag is the one expected (bounded; on time-out the device error word is
// set and the word read last is used).
__device__ __forceinline__ uint32_t finish_wait(unsigned long long v,
                                                const unsigned long long* slot, uint32_t tag,
                                                uint32_t limit, uint32_t* err) {
    uint32_t spins = 0;
    while ((uint32_t)(v >> 32) != tag) {
        if (++spins > limit) {
            atomicOr(err, 1u);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return (uint32_t)v;
}

}  // namespace ising
