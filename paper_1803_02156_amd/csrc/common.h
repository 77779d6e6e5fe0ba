// Internal helpers shared by the libchebfd translation units: status/error
// reporting, HIP call checking, device properties and launch geometry.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/chebfd.h"

namespace chebfd {

void set_error(const char *fmt, ...);
void clear_error();

// Return `code` after recording a formatted message.
#define CHEBFD_FAIL(code, ...)          \
    do {                                \
        ::chebfd::set_error(__VA_ARGS__); \
        return (code);                  \
    } while (0)

#define CHEBFD_REQUIRE(cond, ...)                           \
    do {                                                    \
        if (!(cond)) CHEBFD_FAIL(CHEBFD_EINVAL, __VA_ARGS__); \
    } while (0)

#define CHEBFD_HIP(call)                                                          \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            CHEBFD_FAIL(CHEBFD_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Properties of the current device (cached per device id).
struct DeviceProps {
    int id;
    int num_cus;
    int max_threads_per_cu;
    char name[256];
};
int device_props(DeviceProps *out);

inline bool aligned(const void *p, size_t a) {
    return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

inline bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + nb && pb < pa + na;
}

inline size_t vec_elem_bytes(int prec) { return prec == CHEBFD_PREC_FP64 ? 16 : 8; }

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace chebfd
