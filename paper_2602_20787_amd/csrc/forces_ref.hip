// FP64 reference of the exact image sum on the GPU: every operation of the
// pair sum in FP64 with the spline law on every image (same definitions as
// the FP32 kernel).  A slow precision yardstick, one thread per target,
// sources staged through LDS in tiles of 256.
#include "common.h"
#include "pair_f64.h"

namespace steps {

namespace {

constexpr int kBlock = 256;

struct RefArgs {
    const double *x, *y, *z, *m, *h;
    const int64_t *targets;
    double *ax, *ay, *az, *pot;
    double L, invL;
    int N, n_tgt, n_img;
};

__global__ __launch_bounds__(kBlock) void forces_f64_kernel(RefArgs a) {
    __shared__ double tx[kBlock], ty[kBlock], tz[kBlock], tm[kBlock], th[kBlock];
    const int tid = threadIdx.x;
    const int k = blockIdx.x * kBlock + tid;
    const bool active = k < a.n_tgt;
    const int64_t i = active ? (a.targets ? a.targets[k] : (int64_t)k) : 0;
    const double xi = a.x[i], yi = a.y[i], zi = wrap_z(a.z[i], a.L), hi = a.h[i];
    double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
    for (int base = 0; base < a.N; base += kBlock) {
        const int j = base + tid;
        if (j < a.N) {
            tx[tid] = a.x[j];
            ty[tid] = a.y[j];
            tz[tid] = wrap_z(a.z[j], a.L);
            tm[tid] = a.m[j];
            th[tid] = a.h[j];
        }
        __syncthreads();
        const int cnt = min(kBlock, a.N - base);
        for (int s = 0; s < cnt; ++s) {
            if ((int64_t)(base + s) == i) continue;
            const double dx = xi - tx[s], dy = yi - ty[s];
            const double d = min_image(zi - tz[s], a.L, a.invL);
            double S, Fz, P;
            pair_spline_f64(dx, dy, d, hi + th[s], a.L, a.n_img, S, Fz, P);
            sx += tm[s] * S * dx;
            sy += tm[s] * S * dy;
            sz += tm[s] * Fz;
            sp += tm[s] * P;
        }
        __syncthreads();
    }
    if (active) {
        a.ax[k] = -sx;
        a.ay[k] = -sy;
        a.az[k] = -sz;
        if (a.pot) a.pot[k] = -sp;
    }
}

}  // namespace

int launch_forces_f64(const double *pos, const double *mass, const double *eps, int64_t N,
                      double L, int n_img, const int64_t *targets, int64_t n_tgt, double *out_acc,
                      double *out_pot, hipStream_t stream) {
    RefArgs a;
    a.x = pos;
    a.y = pos + N;
    a.z = pos + 2 * N;
    a.m = mass;
    a.h = eps;
    a.targets = targets;
    a.ax = out_acc;
    a.ay = out_acc + n_tgt;
    a.az = out_acc + 2 * n_tgt;
    a.pot = out_pot;
    a.L = L;
    a.invL = 1.0 / L;
    a.N = (int)N;
    a.n_tgt = (int)n_tgt;
    a.n_img = n_img;
    const int grid = (int)((n_tgt + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(forces_f64_kernel, dim3(grid), dim3(kBlock), 0, stream, a);
    return hip_status(hipGetLastError(), "forces_f64 launch");
}

}  // namespace steps
