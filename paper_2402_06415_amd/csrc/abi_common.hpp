// Helpers shared by the extern "C" entry points of libising.so: the
// thread-local error message, HIP error mapping and device queries.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising.h"

namespace ising {
namespace abi {

// Record a message for ising_last_error() and return `code`.
int set_error(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// ISING_E_HIP with the HIP error string.
int hip_fail(hipError_t e, const char* what);
// Compute units of the current device (0 if the query fails).
int device_cus();
// LDS bytes one workgroup may use on the current device (0 if the query fails).
int device_max_lds();
// Thread-local message of the last failure ("" if none).
const char* last_error();

inline bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

}  // namespace abi
}  // namespace ising

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess)                        \
            return ::ising::abi::hip_fail(e_, what); \
    } while (0)
