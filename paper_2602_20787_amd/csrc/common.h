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

// The positions 0..n_tgt-1 of a target list (targets, or 0..N-1 when NULL)
// in spatial order of the targets (see target_order.hip): *perm points into
// stream-ordered scratch that the caller releases with hipFreeAsync after
// the launches that read it.  STEPS_OK or an error status.
int order_targets(const double *pos, int64_t N, double L, const int64_t *targets, int64_t n_tgt, hipStream_t stream,
                  void **scratch, const int **perm);

// target lists at least this long are walked in spatial order
constexpr int64_t kOrderTargetsMin = 4096;

// The pairwise path (forces_pairwise.hip) for all N particles: every
// unordered pair once, exact images |n| <= n_img, or with a table (non-null)
// images |n| <= 1 plus its far images (order 1 CIC, 2 TSC).  Arguments are
// validated by the caller.
int launch_forces_pairwise(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                           int n_img, const steps_cyl_table *table, int order, float *out_acc, float *out_pot,
                           hipStream_t stream);

// The learned correction's pairwise path for all N particles
// (forces_learned.hip); arguments validated by the caller.
int launch_forces_learned_pairwise(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                                   const steps_cyl_mlp *net, float *out_acc, float *out_pot, hipStream_t stream);

}  // namespace steps

#define STEPS_CHECK_HIP(expr)                                          \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return ::steps::hip_status(e_, #expr);   \
    } while (0)
