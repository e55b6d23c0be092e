// FP64 reference of the exact image sum on the GPU: every operation of the
// pair sum in FP64 with the spline law on every image (same definitions as
// the FP32 kernel).  A precision yardstick for sampled targets: the sources
// are split into chunks over the grid's second dimension so that a few
// thousand targets still fill the GPU, each (target block, chunk) writes
// FP64 partial sums, and a second pass adds the chunks in order.
#include "common.h"
#include "pair_f64.h"

namespace steps {

namespace {

constexpr int kBlock = 256;

struct RefArgs {
    const double *x, *y, *z, *m, *h;
    const int64_t *targets;
    double *part;  // [chunks][4][n_tgt]
    double L, invL;
    int N, n_tgt, n_img, chunk;
};

// 1/sqrt(x) to FP64 precision: FP32 hardware estimate and two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    y = y * (1.5 - 0.5 * x * y * y);
    return y * (1.5 - 0.5 * x * y * y);
}

// All images of one pair; images farther than the softening length use
// the Newtonian terms, the others the spline law.
__device__ __forceinline__ void pair_f64(double dx, double dy, double d, double h, double L, int n_img,
                                         double &s, double &fz, double &p) {
    const double rho2 = dx * dx + dy * dy;
    const double h2 = h * h;
    if (rho2 >= h2) {
        s = fz = p = 0.0;
        for (int n = -n_img; n <= n_img; ++n) {
            const double dz = d - (double)n * L;
            const double ri = rsqrt_nr(rho2 + dz * dz);
            const double ri3 = ri * ri * ri;
            s += ri3;
            fz += ri3 * dz;
            p += ri;
        }
        return;
    }
    pair_spline_f64(dx, dy, d, h, L, n_img, s, fz, p);
}

__global__ __launch_bounds__(kBlock) void forces_f64_kernel(RefArgs a) {
    __shared__ double tx[kBlock], ty[kBlock], tz[kBlock], tm[kBlock], th[kBlock];
    const int tid = threadIdx.x;
    const int k = blockIdx.x * kBlock + tid;
    const bool active = k < a.n_tgt;
    const int64_t i = active ? (a.targets ? a.targets[k] : (int64_t)k) : 0;
    const double xi = a.x[i], yi = a.y[i], zi = wrap_z(a.z[i], a.L), hi = a.h[i];
    const int c0 = blockIdx.y * a.chunk, c1 = min(a.N, c0 + a.chunk);
    double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
    for (int base = c0; base < c1; base += kBlock) {
        const int j = base + tid;
        if (j < c1) {
            tx[tid] = a.x[j];
            ty[tid] = a.y[j];
            tz[tid] = wrap_z(a.z[j], a.L);
            tm[tid] = a.m[j];
            th[tid] = a.h[j];
        }
        __syncthreads();
        const int cnt = min(kBlock, c1 - base);
        for (int s = 0; s < cnt; ++s) {
            if ((int64_t)(base + s) == i) continue;
            const double dx = xi - tx[s], dy = yi - ty[s];
            const double d = min_image(zi - tz[s], a.L, a.invL);
            double S, Fz, P;
            pair_f64(dx, dy, d, hi + th[s], a.L, a.n_img, S, Fz, P);
            sx += tm[s] * S * dx;
            sy += tm[s] * S * dy;
            sz += tm[s] * Fz;
            sp += tm[s] * P;
        }
        __syncthreads();
    }
    if (active) {
        double *q = a.part + (int64_t)blockIdx.y * 4 * a.n_tgt;
        q[k] = sx;
        q[a.n_tgt + k] = sy;
        q[2 * a.n_tgt + k] = sz;
        q[3 * a.n_tgt + k] = sp;
    }
}

__global__ void reduce_chunks_kernel(const double *part, int chunks, int n_tgt, double *acc, double *pot) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_tgt) return;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < chunks; ++c)
        for (int q = 0; q < 4; ++q) v[q] += part[((int64_t)c * 4 + q) * n_tgt + k];
    acc[k] = -v[0];
    acc[n_tgt + k] = -v[1];
    acc[2 * (int64_t)n_tgt + k] = -v[2];
    if (pot) pot[k] = -v[3];
}

}  // namespace

// Source chunks of the FP64 reference for n_tgt targets: enough (target
// block, chunk) pairs to fill the GPU, chunks of at least 256 sources.
void f64_chunks(int64_t N, int64_t n_tgt, int *chunks, int *chunk) {
    const int tblocks = (int)((n_tgt + kBlock - 1) / kBlock);
    int c = (4096 + tblocks - 1) / tblocks;
    const int max_chunks = (int)((N + kBlock - 1) / kBlock);
    if (c > max_chunks) c = max_chunks;
    if (c < 1) c = 1;
    *chunk = (int)(((N + c - 1) / c + kBlock - 1) / kBlock * kBlock);
    *chunks = (int)((N + *chunk - 1) / *chunk);
}

size_t f64_bytes(int64_t N, int64_t n_tgt) {
    int chunks = 1, chunk = 1;
    f64_chunks(N, n_tgt, &chunks, &chunk);
    return ws_total({sizeof(double) * 4 * (size_t)chunks * n_tgt});
}

int launch_forces_f64(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                      int n_img, const int64_t *targets, int64_t n_tgt, double *out_acc, double *out_pot,
                      Workspace &ws, hipStream_t stream) {
    int rc = check_workspace(ws, f64_bytes(N, n_tgt));
    if (rc) return rc;
    RefArgs a;
    a.x = pos;
    a.y = pos + N;
    a.z = pos + 2 * N;
    a.m = mass;
    a.h = eps;
    a.targets = targets;
    a.L = L;
    a.invL = 1.0 / L;
    a.N = (int)N;
    a.n_tgt = (int)n_tgt;
    a.n_img = n_img;
    const int tblocks = (int)((n_tgt + kBlock - 1) / kBlock);
    int chunks = 1;
    f64_chunks(N, n_tgt, &chunks, &a.chunk);
    a.part = (double *)ws.take(sizeof(double) * 4 * (size_t)chunks * n_tgt);
    if (!a.part) return fail(STEPS_EINVAL, "workspace too small for the FP64 reference");
    hipLaunchKernelGGL(forces_f64_kernel, dim3(tblocks, chunks), dim3(kBlock), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(reduce_chunks_kernel, dim3(tblocks), dim3(kBlock), 0, stream, a.part, chunks,
                           (int)n_tgt, out_acc, out_pot);
        e = hipGetLastError();
    }
    return hip_status(e, "forces_f64 launch");
}

}  // namespace steps
