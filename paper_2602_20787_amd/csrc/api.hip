// C entry points of the force sums: host-side argument validation, the
// device check, the workspace (the caller's, or stream-ordered memory for
// the allocating forms) and dispatch to the kernels.
#include "common.h"

namespace steps {
int launch_forces_exact(const double *pos, const double *mass, const double *eps, int64_t N,
                        double L, int n_img, const int64_t *targets, int64_t n_tgt, int mode,
                        float *out_acc, float *out_pot, Workspace &ws, hipStream_t stream);
size_t f64_bytes(int64_t N, int64_t n_tgt);
int launch_forces_f64(const double *pos, const double *mass, const double *eps, int64_t N,
                      double L, int n_img, const int64_t *targets, int64_t n_tgt, double *out_acc,
                      double *out_pot, Workspace &ws, hipStream_t stream);
int launch_forces_learned(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                          const steps_cyl_mlp *net, const int64_t *targets, int64_t n_tgt, int mode,
                          float *out_acc, float *out_pot, Workspace &ws, hipStream_t stream);
size_t table_forces_bytes(int64_t N, const steps_cyl_table *t, int order, bool all_targets, int64_t n_targets,
                          bool pot);
size_t exact_per_target_bytes(int64_t N, int64_t n_tgt);
size_t learned_per_target_bytes(int64_t N, int64_t n_tgt);

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

int check_mode(int mode, const void *targets) {
    if (mode != STEPS_SUM_COMPENSATED && mode != STEPS_SUM_PLAIN && mode != STEPS_SUM_PAIRWISE)
        return fail(STEPS_EINVAL, "mode=%d is not a summation mode", mode);
    if (mode == STEPS_SUM_PAIRWISE && targets)
        return fail(STEPS_EINVAL, "STEPS_SUM_PAIRWISE needs every particle as a target (targets NULL)");
    return STEPS_OK;
}

Workspace caller_workspace(void *p, size_t bytes) {
    Workspace ws;
    ws.base = (char *)p;
    ws.size = p ? bytes : 0;
    return ws;
}

// the exact path of steps_cyl_forces_ex (validated arguments)
size_t exact_bytes(int64_t N, int n_img, bool all_targets, int64_t n_targets, int mode, bool pot) {
    if (mode == STEPS_SUM_PAIRWISE) return pairwise_bytes(N, n_img, nullptr, 0, pot);
    return exact_per_target_bytes(N, all_targets ? N : n_targets);
}

int run_exact(const double *pos, const double *mass, const double *eps, int64_t N, double L, int n_img,
              const int64_t *targets, int64_t n_targets, int mode, float *out_acc, float *out_pot, Workspace &ws,
              hipStream_t stream) {
    if (mode == STEPS_SUM_PAIRWISE)
        return launch_forces_pairwise(pos, mass, eps, N, L, n_img, nullptr, 0, out_acc, out_pot, ws, stream);
    return launch_forces_exact(pos, mass, eps, N, L, n_img, targets, n_targets, mode, out_acc, out_pot, ws,
                               stream);
}

size_t learned_bytes(int64_t N, bool all_targets, int64_t n_targets, int mode) {
    if (mode == STEPS_SUM_PAIRWISE) return learned_pairwise_bytes(N);
    return learned_per_target_bytes(N, all_targets ? N : n_targets);
}

int run_learned(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                const steps_cyl_mlp *net, const int64_t *targets, int64_t n_targets, int mode, float *out_acc,
                float *out_pot, Workspace &ws, hipStream_t stream) {
    if (mode == STEPS_SUM_PAIRWISE)
        return launch_forces_learned_pairwise(pos, mass, eps, N, L, net, out_acc, out_pot, ws, stream);
    return launch_forces_learned(pos, mass, eps, N, L, net, targets, n_targets, mode, out_acc, out_pot, ws,
                                 stream);
}

}  // namespace
}  // namespace steps

using namespace steps;

STEPS_API int steps_cyl_forces_workspace(int path, int64_t N, int n_img, int64_t n_targets, int mode,
                                         const steps_cyl_table *table, int order, int potential, size_t *bytes) {
    if (!bytes) return fail(STEPS_EINVAL, "bytes must be non-null");
    *bytes = 0;
    if (N < 1 || N > STEPS_MAX_N) return fail(STEPS_EINVAL, "N=%lld outside [1, 2^29]", (long long)N);
    if (n_targets < 0 || n_targets > STEPS_MAX_N)
        return fail(STEPS_EINVAL, "n_targets=%lld outside [0, 2^29]", (long long)n_targets);
    if (n_img < 0 || n_img > STEPS_MAX_NIMG)
        return fail(STEPS_EINVAL, "n_img=%d outside [0, %d]", n_img, STEPS_MAX_NIMG);
    const bool all = (n_targets == 0);
    int rc;
    switch (path) {
        case STEPS_PATH_EXACT:
        case STEPS_PATH_LEARNED:
            if ((rc = check_mode(mode, all ? nullptr : (const void *)1))) return rc;
            break;
        case STEPS_PATH_TABLE:
            if (!table) return fail(STEPS_EINVAL, "a table path needs the table");
            if (order != 1 && order != 2) return fail(STEPS_EINVAL, "order=%d: 1 (CIC) or 2 (TSC)", order);
            break;
        case STEPS_PATH_F64:
            break;
        default:
            return fail(STEPS_EINVAL, "path=%d is not a force path", path);
    }
    if ((rc = require_device())) return rc;
    clear_error();
    const bool pot = potential != 0;
    size_t b = 0;
    switch (path) {
        case STEPS_PATH_EXACT: b = exact_bytes(N, n_img, all, n_targets, mode, pot); break;
        case STEPS_PATH_LEARNED: b = learned_bytes(N, all, n_targets, mode); break;
        case STEPS_PATH_TABLE: b = table_forces_bytes(N, table, order, all, n_targets, pot); break;
        default: b = f64_bytes(N, all ? N : n_targets); break;
    }
    *bytes = b;
    return STEPS_OK;
}

STEPS_API int steps_cyl_forces_ws(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                                  int n_img, float *out_acc, float *out_pot, void *workspace,
                                  size_t workspace_bytes, hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, n_img, nullptr, N, out_acc);
    if (rc) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    Workspace ws = caller_workspace(workspace, workspace_bytes);
    return launch_forces_pairwise(pos, mass, eps, N, L, n_img, nullptr, 0, out_acc, out_pot, ws, stream);
}

STEPS_API int steps_cyl_forces(const double *pos, const double *mass, const double *eps, int64_t N,
                               double L, int n_img, float *out_acc, float *out_pot,
                               hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, n_img, nullptr, N, out_acc);
    if (rc) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    return with_stream_workspace(pairwise_bytes(N, n_img, nullptr, 0, out_pot != nullptr), stream,
                                 [&](Workspace &ws) {
                                     return launch_forces_pairwise(pos, mass, eps, N, L, n_img, nullptr, 0,
                                                                   out_acc, out_pot, ws, stream);
                                 });
}

STEPS_API int steps_cyl_forces_ex_ws(const double *pos, const double *mass, const double *eps, int64_t N,
                                     double L, int n_img, const int64_t *targets, int64_t n_targets, int mode,
                                     float *out_acc, float *out_pot, void *workspace, size_t workspace_bytes,
                                     hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, n_img, targets, n_targets, out_acc);
    if (rc) return rc;
    if ((rc = check_mode(mode, targets))) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    Workspace ws = caller_workspace(workspace, workspace_bytes);
    return run_exact(pos, mass, eps, N, L, n_img, targets, n_targets, mode, out_acc, out_pot, ws, stream);
}

STEPS_API int steps_cyl_forces_ex(const double *pos, const double *mass, const double *eps,
                                  int64_t N, double L, int n_img, const int64_t *targets,
                                  int64_t n_targets, int mode, float *out_acc, float *out_pot,
                                  hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, n_img, targets, n_targets, out_acc);
    if (rc) return rc;
    if ((rc = check_mode(mode, targets))) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    const size_t bytes = exact_bytes(N, n_img, targets == nullptr, n_targets, mode, out_pot != nullptr);
    return with_stream_workspace(bytes, stream, [&](Workspace &ws) {
        return run_exact(pos, mass, eps, N, L, n_img, targets, n_targets, mode, out_acc, out_pot, ws, stream);
    });
}

STEPS_API int steps_cyl_forces_f64_ws(const double *pos, const double *mass, const double *eps, int64_t N,
                                      double L, int n_img, const int64_t *targets, int64_t n_targets,
                                      double *out_acc, double *out_pot, void *workspace, size_t workspace_bytes,
                                      hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, n_img, targets, n_targets, out_acc);
    if (rc) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    Workspace ws = caller_workspace(workspace, workspace_bytes);
    return launch_forces_f64(pos, mass, eps, N, L, n_img, targets, n_targets, out_acc, out_pot, ws, stream);
}

STEPS_API int steps_cyl_forces_f64(const double *pos, const double *mass, const double *eps,
                                   int64_t N, double L, int n_img, const int64_t *targets,
                                   int64_t n_targets, double *out_acc, double *out_pot,
                                   hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, n_img, targets, n_targets, out_acc);
    if (rc) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    return with_stream_workspace(f64_bytes(N, n_targets), stream, [&](Workspace &ws) {
        return launch_forces_f64(pos, mass, eps, N, L, n_img, targets, n_targets, out_acc, out_pot, ws, stream);
    });
}

STEPS_API int steps_cyl_forces_learned_ws(const double *pos, const double *mass, const double *eps, int64_t N,
                                          double L, const steps_cyl_mlp *net, float *out_acc, float *out_pot,
                                          void *workspace, size_t workspace_bytes, hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, 1, nullptr, N, out_acc);
    if (rc) return rc;
    if (!net) return fail(STEPS_EINVAL, "net must be non-null");
    if ((rc = require_device())) return rc;
    clear_error();
    Workspace ws = caller_workspace(workspace, workspace_bytes);
    return launch_forces_learned_pairwise(pos, mass, eps, N, L, net, out_acc, out_pot, ws, stream);
}

STEPS_API int steps_cyl_forces_learned(const double *pos, const double *mass, const double *eps, int64_t N,
                                       double L, const steps_cyl_mlp *net, float *out_acc, float *out_pot,
                                       hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, 1, nullptr, N, out_acc);
    if (rc) return rc;
    if (!net) return fail(STEPS_EINVAL, "net must be non-null");
    if ((rc = require_device())) return rc;
    clear_error();
    return with_stream_workspace(learned_pairwise_bytes(N), stream, [&](Workspace &ws) {
        return launch_forces_learned_pairwise(pos, mass, eps, N, L, net, out_acc, out_pot, ws, stream);
    });
}

STEPS_API int steps_cyl_forces_learned_ex_ws(const double *pos, const double *mass, const double *eps,
                                             int64_t N, double L, const steps_cyl_mlp *net,
                                             const int64_t *targets, int64_t n_targets, int mode, float *out_acc,
                                             float *out_pot, void *workspace, size_t workspace_bytes,
                                             hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, 1, targets, n_targets, out_acc);
    if (rc) return rc;
    if (!net) return fail(STEPS_EINVAL, "net must be non-null");
    if ((rc = check_mode(mode, targets))) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    Workspace ws = caller_workspace(workspace, workspace_bytes);
    return run_learned(pos, mass, eps, N, L, net, targets, n_targets, mode, out_acc, out_pot, ws, stream);
}

STEPS_API int steps_cyl_forces_learned_ex(const double *pos, const double *mass, const double *eps,
                                          int64_t N, double L, const steps_cyl_mlp *net,
                                          const int64_t *targets, int64_t n_targets, int mode,
                                          float *out_acc, float *out_pot, hipStream_t stream) {
    int rc = check_common(pos, mass, eps, N, L, 1, targets, n_targets, out_acc);
    if (rc) return rc;
    if (!net) return fail(STEPS_EINVAL, "net must be non-null");
    if ((rc = check_mode(mode, targets))) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    return with_stream_workspace(learned_bytes(N, targets == nullptr, n_targets, mode), stream,
                                 [&](Workspace &ws) {
                                     return run_learned(pos, mass, eps, N, L, net, targets, n_targets, mode,
                                                        out_acc, out_pot, ws, stream);
                                 });
}
