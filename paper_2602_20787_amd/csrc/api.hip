// C entry points of the force sums: host-side argument validation, the
// device check, and dispatch to the kernels.
#include "common.h"

namespace steps {
int launch_forces_exact(const double *pos, const double *mass, const double *eps, int64_t N,
                        double L, int n_img, const int64_t *targets, int64_t n_tgt, int mode,
                        float *out_acc, float *out_pot, hipStream_t stream);
int launch_forces_f64(const double *pos, const double *mass, const double *eps, int64_t N,
                      double L, int n_img, const int64_t *targets, int64_t n_tgt, double *out_acc,
                      double *out_pot, hipStream_t stream);

int launch_forces_learned(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                          const steps_cyl_mlp *net, const int64_t *targets, int64_t n_tgt, int mode,
                          float *out_acc, float *out_pot, hipStream_t stream);

namespace {

int check_common(const void *pos, const void *mass, const void *eps, int64_t N, double L,
                 int n_img, const void *targets, int64_t n_targets, const void *out_acc) {
    if (!pos || !mass || !eps) return fail(STEPS_EINVAL, "pos, mass and eps must be non-null");
    if (!out_acc) return fail(STEPS_EINVAL, "out_acc must be non-null");
    if (N < 1 || N > STEPS_MAX_N) return fail(STEPS_EINVAL, "N=%lld outside [1, 2^29]", (long long)N);
    if (!finite_positive(L)) return fail(STEPS_EINVAL, "L must be finite and > 0");
    if (n_img < 0 || n_img > STEPS_MAX_NIMG)
        return fail(STEPS_EINVAL, "n_img=%d outside [0, %d]", n_img, STEPS_MAX_NIMG);
    if (n_targets < 1 || n_targets > STEPS_MAX_N)
        return fail(STEPS_EINVAL, "n_targets=%lld outside [1, 2^29]", (long long)n_targets);
    if (!targets && n_targets != N)
        return fail(STEPS_EINVAL, "targets is NULL, so n_targets must equal N");
    return STEPS_OK;
}

}  // namespace
}  // namespace steps

using namespace steps;

STEPS_API int steps_cyl_forces(const double *pos, const double *mass, const double *eps, int64_t N,
                               double L, int n_img, float *out_acc, float *out_pot,
                               hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, n_img, nullptr, N, out_acc);
    if (rc) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    return launch_forces_pairwise(pos, mass, eps, N, L, n_img, nullptr, 0, out_acc, out_pot, stream);
}

STEPS_API int steps_cyl_forces_ex(const double *pos, const double *mass, const double *eps,
                                  int64_t N, double L, int n_img, const int64_t *targets,
                                  int64_t n_targets, int mode, float *out_acc, float *out_pot,
                                  hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, n_img, targets, n_targets, out_acc);
    if (rc) return rc;
    if (mode != STEPS_SUM_COMPENSATED && mode != STEPS_SUM_PLAIN && mode != STEPS_SUM_PAIRWISE)
        return fail(STEPS_EINVAL, "mode=%d is not a summation mode", mode);
    if (mode == STEPS_SUM_PAIRWISE && targets)
        return fail(STEPS_EINVAL, "STEPS_SUM_PAIRWISE needs every particle as a target (targets NULL)");
    if ((rc = require_device())) return rc;
    clear_error();
    if (mode == STEPS_SUM_PAIRWISE)
        return launch_forces_pairwise(pos, mass, eps, N, L, n_img, nullptr, 0, out_acc, out_pot, stream);
    return launch_forces_exact(pos, mass, eps, N, L, n_img, targets, n_targets, mode, out_acc,
                               out_pot, stream);
}

STEPS_API int steps_cyl_forces_f64(const double *pos, const double *mass, const double *eps,
                                   int64_t N, double L, int n_img, const int64_t *targets,
                                   int64_t n_targets, double *out_acc, double *out_pot,
                                   hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, n_img, targets, n_targets, out_acc);
    if (rc) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    return launch_forces_f64(pos, mass, eps, N, L, n_img, targets, n_targets, out_acc, out_pot,
                             stream);
}

STEPS_API int steps_cyl_forces_learned(const double *pos, const double *mass, const double *eps, int64_t N,
                                       double L, const steps_cyl_mlp *net, float *out_acc, float *out_pot,
                                       hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, 1, nullptr, N, out_acc);
    if (rc) return rc;
    if (!net) return fail(STEPS_EINVAL, "net must be non-null");
    if ((rc = require_device())) return rc;
    clear_error();
    return launch_forces_learned_pairwise(pos, mass, eps, N, L, net, out_acc, out_pot, stream);
}

STEPS_API int steps_cyl_forces_learned_ex(const double *pos, const double *mass, const double *eps,
                                          int64_t N, double L, const steps_cyl_mlp *net,
                                          const int64_t *targets, int64_t n_targets, int mode,
                                          float *out_acc, float *out_pot, hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, 1, targets, n_targets, out_acc);
    if (rc) return rc;
    if (!net) return fail(STEPS_EINVAL, "net must be non-null");
    if (mode != STEPS_SUM_COMPENSATED && mode != STEPS_SUM_PLAIN && mode != STEPS_SUM_PAIRWISE)
        return fail(STEPS_EINVAL, "mode=%d is not a summation mode", mode);
    if (mode == STEPS_SUM_PAIRWISE && targets)
        return fail(STEPS_EINVAL, "STEPS_SUM_PAIRWISE needs every particle as a target (targets NULL)");
    if ((rc = require_device())) return rc;
    clear_error();
    if (mode == STEPS_SUM_PAIRWISE)
        return launch_forces_learned_pairwise(pos, mass, eps, N, L, net, out_acc, out_pot, stream);
    return launch_forces_learned(pos, mass, eps, N, L, net, targets, n_targets, mode, out_acc, out_pot,
                                 stream);
}
