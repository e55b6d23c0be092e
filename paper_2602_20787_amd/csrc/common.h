// Shared host-side helpers of the steps_cyl library: status handling, the
// per-thread error message and the device check done before launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cmath>
#include <cstdio>
#include <string>

#include "../../include/steps_cyl.h"

#define STEPS_API extern "C" __attribute__((visibility("default")))

namespace steps {

// Records `msg` as the calling thread's last error and returns `code`.
int fail(int code, const char *fmt, ...);
void clear_error();

// STEPS_OK when the current device is a gfx950; otherwise records why not.
int require_device();

// Converts a HIP status into STEPS_OK / STEPS_EHIP with a message.
int hip_status(hipError_t e, const char *what);

inline bool finite_positive(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace steps

#define STEPS_CHECK_HIP(expr)                                          \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return ::steps::hip_status(e_, #expr);   \
    } while (0)
