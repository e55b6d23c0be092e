// Shared host-side helpers of the steps_cyl library: status handling, the
// per-thread error message and the device check done before launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cmath>
#include <cstdio>
#include <string>
#include <initializer_list>

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

// Device workspace of one force call, handed out in 256-byte aligned
// pieces.  The kernels of a call use nothing else: the caller's buffer (the
// *_ws entry points), stream-ordered memory of the allocating entry points,
// or the library's static scratch (steps_cyl_forces_noalloc).
constexpr size_t kWsAlign = 256;
inline size_t ws_round(size_t n) { return (n + kWsAlign - 1) & ~(kWsAlign - 1); }

struct Workspace {
    char *base = nullptr;
    size_t size = 0, used = 0;
    // n bytes at the next aligned address, or nullptr when they do not fit
    void *take(size_t n) {
        const uintptr_t b = (uintptr_t)base;
        const size_t off = (size_t)(((b + used + kWsAlign - 1) & ~(uintptr_t)(kWsAlign - 1)) - b);
        if (off > size || n > size - off) return nullptr;
        used = off + n;
        return base + off;
    }
};

// Bytes a call needs when its pieces are n1, n2, ...: each rounded up to the
// alignment, plus one alignment step for an unaligned base.
inline size_t ws_total(std::initializer_list<size_t> pieces) {
    size_t t = kWsAlign;
    for (size_t n : pieces) t += ws_round(n);
    return t;
}

// Workspace of order_targets for a list of n_tgt targets.
size_t order_targets_bytes(int64_t n_tgt);

// The positions 0..n_tgt-1 of a target list (targets, or 0..N-1 when NULL)
// in spatial order of the targets (see target_order.hip): *perm points into
// the workspace (order_targets_bytes(n_tgt) bytes of it).  STEPS_OK or an
// error status.
int order_targets(const double *pos, int64_t N, double L, const int64_t *targets, int64_t n_tgt, hipStream_t stream,
                  Workspace &ws, const int **perm);

// target lists at least this long are walked in spatial order
constexpr int64_t kOrderTargetsMin = 4096;

// Workspace of the per-target force kernels for n_tgt targets (the spatial
// order of long lists).
inline size_t per_target_bytes(int64_t n_tgt) {
    return n_tgt >= kOrderTargetsMin ? order_targets_bytes(n_tgt) : 0;
}

// STEPS_EINVAL unless `ws` holds `need` bytes.
int check_workspace(const Workspace &ws, size_t need);

// The pairwise path (forces_pairwise.hip) for all N particles: every
// unordered pair once, exact images |n| <= n_img, or with a table (non-null)
// images |n| <= 1 plus its far images (order 1 CIC, 2 TSC).  Arguments are
// validated by the caller; pairwise_bytes() is the workspace it takes.
// s_cap > 0 caps the parts per group (S, a power of two up to 16), which
// sets the sum slots (2S per particle); pairwise_bytes_S() is the workspace
// with S parts per group.
size_t pairwise_bytes(int64_t N, int n_img, const steps_cyl_table *table, int order, bool pot);
size_t pairwise_bytes_S(int64_t N, int S);
int launch_forces_pairwise(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                           int n_img, const steps_cyl_table *table, int order, float *out_acc, float *out_pot,
                           Workspace &ws, hipStream_t stream, int s_cap = 0);

// The learned correction's pairwise path for all N particles
// (forces_learned.hip); arguments validated by the caller.
size_t learned_pairwise_bytes(int64_t N);
int launch_forces_learned_pairwise(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                                   const steps_cyl_mlp *net, float *out_acc, float *out_pot, Workspace &ws,
                                   hipStream_t stream);

// Runs f(ws) with `bytes` of stream-ordered device memory (none when 0),
// released on the stream after the launches f makes: the allocating entry
// points.
template <class F>
int with_stream_workspace(size_t bytes, hipStream_t stream, F &&f) {
    Workspace ws;
    if (bytes > 0) {
        void *p = nullptr;
        if (hipMallocAsync(&p, bytes, stream) != hipSuccess)
            return fail(STEPS_ENOMEM, "workspace of %zu bytes", bytes);
        ws.base = (char *)p;
        ws.size = bytes;
    }
    const int rc = f(ws);
    if (ws.base) {
        const hipError_t e = hipFreeAsync(ws.base, stream);
        if (rc == STEPS_OK && e != hipSuccess) return hip_status(e, "workspace release");
    }
    return rc;
}

}  // namespace steps

#define STEPS_CHECK_HIP(expr)                                          \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return ::steps::hip_status(e_, #expr);   \
    } while (0)
