// Tabulated far-image correction (Sect. 2.2, eq. S1R2EwaldCorrectionTable):
// the image band of one unit mass on an equally spaced grid in
// delta = |d|/L in [0, 1/2] and r = rho/L in [0, r_max], with one ghost node
// beyond every edge, interpolated with cloud-in-cell (bilinear) or
// triangular-shaped-cloud (quadratic B-spline, 3 x 3 nodes) weights and
// added to the exact images |n| <= 1.
//
// Two kinds of table:
//  * band: the images 2 <= |n| <= n_far, summed directly in FP64;
//  * complete: every image |n| >= 2 (N_cut -> infinity), from the Ewald split
//    of Sect. 2.2 (eqs. cylindricalEwaldSplit, EwaldRealSum, EwaldRecSum):
//    a real-space sum over n = -n_max..n_max weighted by
//    Q(3/2, alpha^2 r^2) = erfc(alpha r) + 2 alpha r exp(-alpha^2 r^2)/sqrt(pi),
//    Fourier modes m = 1..m_max, and the m = 0 mode
//    -2 (1 - exp(-alpha^2 rho^2)) / rho.  The Fourier kernel is either the
//    incomplete Bessel function
//        B(k, rho) = int_{1/(4 alpha^2)}^inf exp(-k^2 t - rho^2/(4 t)) dt/(2 t)
//    that Poisson summation of the smooth part gives for one periodic
//    direction (force (4/L) grad[cos(k d) B]), or, for comparison, the kernel
//    as printed in eq. Bkernel with its printed prefactor (-(2/L)), which
//    only matches the complete sum where its modes are negligible.  The
//    three nearest images enter the real-space sum as (Ewald - Newton),
//    -P(3/2, alpha^2 r^2), so the node values carry no cancellation.
//    Pairs beyond r_max use the line-mass limit of the complete sum,
//    F = (0, -2/rho) per G m / L, minus the three nearest images: the
//    modes decay as exp(-2 pi rho/L), below 1e-10 for rho_max >= 4 L.
//
// The nodes are built on the GPU in FP64, one wave per node (the image or
// mode range split over the lanes, then a fixed-order reduction), kept in
// FP64 for inspection and stored as FP32 pairs (T_z, T_rho) for the force
// kernel; at 146 x 131 nodes (the paper's 144 x 128 grid plus ghosts) the
// FP32 table is 153 KB and stays in L2.  The force kernel maps one target
// per thread like the exact kernel; sources come through LDS tiles, the
// table through the vector caches.  Pairs of a band table beyond r_max take
// the exact band, shared by the 64 lanes of the wave.
#include "table_pair.h"

namespace steps {

namespace {

constexpr int kBlock = 256;
constexpr int kSub = 32;

__device__ __forceinline__ double rsqrt_f64(double x) {
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    y = y * (1.5 - 0.5 * x * y * y);
    return y * (1.5 - 0.5 * x * y * y);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ void store_node(float2 *nodes, double2 *nodes64, int k, double tz, double tr) {
    if ((threadIdx.x & 63) == 0) {
        nodes64[k] = make_double2(tz, tr);
        nodes[k] = make_float2((float)tz, (float)tr);
    }
}

// band 2 <= |n| <= n_far, one wave per node; each lane sums its images from
// the far end inwards (smallest terms first)
__global__ __launch_bounds__(64) void build_band_kernel(float2 *nodes, double2 *nodes64, int n_d, double h_d,
                                                        double h_r, int n_far) {
    const int w = n_d + 3;
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    const int i = k % w - 1, j = k / w - 1;
    const double delta = i * h_d, r = j * h_r, r2 = r * r;
    double tz = 0.0, tr = 0.0;
    for (int q = n_far - lane; q >= 2; q -= 64) {
        const double up = delta - (double)q, um = delta + (double)q;
        const double ip = rsqrt_f64(up * up + r2), im = rsqrt_f64(um * um + r2);
        const double ip3 = ip * ip * ip, im3 = im * im * im;
        tz += -up * ip3 - um * im3;
        tr += -r * (ip3 + im3);
    }
    store_node(nodes, nodes64, k, wave_sum(tz), wave_sum(tr));
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoOverSqrtPi = 1.12837916709551257390;

// P(3/2, x^2) = erf(x) - 2 x exp(-x^2)/sqrt(pi): by its power series
// x^3 exp(-x^2)/Gamma(5/2) * sum_j x^2j / ((5/2)(7/2)...(3/2+j)) for x < 1
// (all terms positive), directly beyond
__device__ double gamma_p32(double x) {
    const double y = x * x;
    if (x < 1.0) {
        double term = 1.0, sum = 1.0;
        for (int j = 1; j < 40; ++j) {
            term *= y / (1.5 + j);
            sum += term;
            if (term < 1e-17 * sum) break;
        }
        return x * y * exp(-y) * sum / (0.75 * 1.77245385090551602730);
    }
    return erf(x) - kTwoOverSqrtPi * x * exp(-y);
}

// (B, dB/drho) of the incomplete-Bessel kernel.  With s = ln(4 alpha^2 t),
// c = k^2/(4 alpha^2) and b = alpha^2 rho^2:
//   B = 1/2 int_0^inf exp(-c e^s - b e^-s) ds,
//   dB/drho = -alpha^2 rho int_0^inf exp(-c e^s - b e^-s - s) ds.
// The exponent has its minimum E0 at s0 = max(0, ln(b/c)/2); the integral is
// taken where it stays below E0 + 45, by 8-point Gauss-Legendre on panels of
// width at most 1/16 (the integrand is analytic and varies on the scale
// 1/(c e^s + b e^-s) there).
__device__ void kernel_bessel(double k, double rho, double alpha, double &B, double &dB) {
    const double c = k * k / (4.0 * alpha * alpha), b = alpha * alpha * rho * rho;
    const double s0 = (b > c) ? 0.5 * log(b / c) : 0.0;
    const double E0 = c * exp(s0) + b * exp(-s0);
    B = 0.0;
    dB = 0.0;
    if (E0 > 700.0) return;
    const double s_hi = log((E0 + 45.0) / c);
    const double s_lo = (b > E0 + 45.0) ? log(b / (E0 + 45.0)) : 0.0;
    const int panels = max(1, (int)ceil((s_hi - s_lo) * 16.0));
    const double hw = 0.5 * (s_hi - s_lo) / panels;
    // Gauss-Legendre, 8 points on [-1, 1] (symmetric pairs)
    const double gx[4] = {0.18343464249564980494, 0.52553240991632898582, 0.79666647741362673959,
                          0.96028985649753623168};
    const double gw[4] = {0.36268378337836198297, 0.31370664587788728734, 0.22238103445337447054,
                          0.10122853629037625915};
    double sb = 0.0, sd = 0.0;
    for (int p = 0; p < panels; ++p) {
        const double mid = s_lo + (2 * p + 1) * hw;
        for (int q = 0; q < 4; ++q) {
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                const double s = mid + sgn * hw * gx[q];
                const double es = exp(s);
                const double f = gw[q] * exp(-c * es - b / es);
                sb += f;
                sd += f / es;
            }
        }
    }
    B = 0.5 * hw * sb;
    dB = -alpha * alpha * rho * hw * sd;
}

// (B_p, dB_p/drho) of the printed kernel; exp(k rho) erfc(a+) written as
// exp(-k^2/(4 alpha^2) - alpha^2 rho^2) erfcx(a+) so that nothing overflows,
// and the Gaussian terms of the two derivatives cancel
__device__ void kernel_printed(double k, double rho, double alpha, double &B, double &dB) {
    const double ap = k / (2.0 * alpha) + alpha * rho, am = k / (2.0 * alpha) - alpha * rho;
    const double t1 = exp(-k * k / (4.0 * alpha * alpha) - alpha * alpha * rho * rho) * erfcx(ap);
    const double t2 = exp(-k * rho) * erfc(am);
    B = t1 + t2;
    dB = k * (t1 - t2);
}

// complete band (every |n| >= 2) at (delta, |r|) by the Ewald split, one wave
// per node: lane l takes the real-space images n = -n_max + l + 64 t and the
// modes m = 1 + l + 64 t
__global__ __launch_bounds__(64) void build_ewald_kernel(float2 *nodes, double2 *nodes64, int n_d, double h_d,
                                                         double h_r, double alpha, int n_max, int m_max,
                                                         int printed) {
    const int w = n_d + 3;
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    const int i = k % w - 1, j = k / w - 1;
    const double delta = i * h_d, rs = j * h_r, r = fabs(rs), r2 = r * r;
    double tz = 0.0, tr = 0.0;
    for (int n = -n_max + lane; n <= n_max; n += 64) {
        const double u = delta - (double)n;
        const double q2 = u * u + r2;
        if (q2 == 0.0) continue;  // the subtracted n = 0 term tends to zero with s_n
        const double q = sqrt(q2), x = alpha * q;
        const double p = gamma_p32(x);
        // |n| >= 2: Q = 1 - P; |n| <= 1: Q - 1 = -P (Newton's term removed)
        const double wgt = (n >= -1 && n <= 1) ? -p : erfc(x) + kTwoOverSqrtPi * x * exp(-x * x);
        const double inv3 = 1.0 / (q2 * q);
        tz -= u * inv3 * wgt;
        tr -= r * inv3 * wgt;
    }
    for (int m = 1 + lane; m <= m_max; m += 64) {
        const double km = 2.0 * kPi * m;
        double B, dB, pre;
        if (printed) {
            kernel_printed(km, r, alpha, B, dB);
            pre = -2.0;
        } else {
            kernel_bessel(km, r, alpha, B, dB);
            pre = 4.0;
        }
        double sn, cs;
        sincos(km * delta, &sn, &cs);
        tz += pre * (-km * sn) * B;
        tr += pre * cs * dB;
    }
    tz = wave_sum(tz);
    tr = wave_sum(tr);
    if (r > 0.0) tr += 2.0 * expm1(-alpha * alpha * r2) / r;  // m = 0
    store_node(nodes, nodes64, k, tz, rs < 0.0 ? -tr : tr);
}

struct TableArgs {
    const double *x, *y, *z, *m, *h;
    const int64_t *targets;
    const int *perm;  // list positions in spatial order of their targets, or null
    float *ax, *ay, *az, *pot;
    TableView tv;
    PeriodConsts pc;
    int N, n_tgt;
};

template <int ORDER, bool POT, bool COMPLETE>
__global__ __launch_bounds__(kBlock) void forces_table_kernel(TableArgs a) {
    __shared__ SrcRec tile[kBlock];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int k = blockIdx.x * kBlock + tid;
    const bool active = k < a.n_tgt;
    const int64_t kk = active ? (a.perm ? (int64_t)a.perm[k] : (int64_t)k) : 0;  // position in the list
    const int64_t i = a.targets ? a.targets[kk] : kk;
    const double xi = a.x[i], yi = a.y[i], zi = wrap_z(a.z[i], a.pc.L);
    const float hi = (float)a.h[i];
    float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f;
    float cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;
    for (int base = 0; base < a.N; base += kBlock) {
        __syncthreads();
        const int j = base + tid;
        if (j < a.N) {
            SrcRec r;
            r.x = a.x[j];
            r.y = a.y[j];
            r.z = wrap_z(a.z[j], a.pc.L);
            r.m = (float)a.m[j];
            r.h = (float)a.h[j];
            tile[tid] = r;
        }
        __syncthreads();
        const int cnt = min(kBlock, a.N - base);
        for (int s0 = 0; s0 < cnt; s0 += kSub) {
            const int e = min(kSub, cnt - s0);
            float px = 0.f, py = 0.f, pz = 0.f, pp = 0.f;
            for (int s = 0; s < e; ++s) {
                const SrcRec src = tile[s0 + s];
                const bool self = (int64_t)(base + s0 + s) == i;
                table_pair<ORDER, POT, COMPLETE>(a.tv, a.pc, xi, yi, zi, hi, src, self, active, px, py, pz, pp);
            }
            kahan_add(sx, cx, px);
            kahan_add(sy, cy, py);
            kahan_add(sz, cz, pz);
            if (POT) kahan_add(sp, cp, pp);
        }
    }
    if (active) {
        const int64_t o = kk;
        a.ax[o] = -(sx - cx);
        a.ay[o] = -(sy - cy);
        a.az[o] = -(sz - cz);
        if (POT) a.pot[o] = -(sp - cp);
    }
}


template <int ORDER, bool POT>
hipError_t launch_t(const TableArgs &a, hipStream_t stream) {
    const int grid = (a.n_tgt + kBlock - 1) / kBlock;
    if (a.tv.complete)
        hipLaunchKernelGGL((forces_table_kernel<ORDER, POT, true>), dim3(grid), dim3(kBlock), 0, stream, a);
    else
        hipLaunchKernelGGL((forces_table_kernel<ORDER, POT, false>), dim3(grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace
}  // namespace steps

using namespace steps;

namespace {

steps_cyl_table *new_table(int n_delta, int n_rho, double rho_max, int n_far, int complete) {
    steps_cyl_table *t = new (std::nothrow) steps_cyl_table();
    if (!t) return nullptr;
    t->n_d = n_delta;
    t->n_r = n_rho;
    t->r_max = rho_max;
    t->n_far = n_far;
    t->complete = complete;
    const size_t nodes = (size_t)(n_delta + 3) * (n_rho + 3);
    if (hipMalloc(&t->nodes, nodes * sizeof(float2)) != hipSuccess) {
        delete t;
        return nullptr;
    }
    if (hipMalloc(&t->nodes64, nodes * sizeof(double2)) != hipSuccess) {
        (void)hipFree(t->nodes);
        delete t;
        return nullptr;
    }
    return t;
}

int finish_build(steps_cyl_table *t, hipStream_t stream, steps_cyl_table **out) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        steps_cyl_table_destroy(t);
        return hip_status(e, "table build");
    }
    *out = t;
    return STEPS_OK;
}

int check_grid(int n_delta, int n_rho, double rho_max) {
    if (n_delta < 2 || n_delta > 4096 || n_rho < 2 || n_rho > 4096)
        return fail(STEPS_EINVAL, "grid sizes must lie in [2, 4096]");
    if (!finite_positive(rho_max) || rho_max > 1e4) return fail(STEPS_EINVAL, "rho_max must be finite and > 0");
    return STEPS_OK;
}

}  // namespace

STEPS_API int steps_cyl_table_create(int n_delta, int n_rho, double rho_max, int n_far, hipStream_t stream,
                                     steps_cyl_table **out) {
    if (!out) return fail(STEPS_EINVAL, "out must be non-null");
    int rc = check_grid(n_delta, n_rho, rho_max);
    if (rc) return rc;
    if (n_far < 2 || n_far > STEPS_TABLE_MAX_FAR)
        return fail(STEPS_EINVAL, "n_far=%d outside [2, %d]", n_far, STEPS_TABLE_MAX_FAR);
    if ((rc = require_device())) return rc;
    clear_error();
    steps_cyl_table *t = new_table(n_delta, n_rho, rho_max, n_far, 0);
    if (!t) return fail(STEPS_ENOMEM, "table allocation failed");
    const int nodes = (n_delta + 3) * (n_rho + 3);
    hipLaunchKernelGGL(build_band_kernel, dim3(nodes), dim3(64), 0, stream, t->nodes, t->nodes64, n_delta,
                       0.5 / n_delta, rho_max / n_rho, n_far);
    return finish_build(t, stream, out);
}

STEPS_API int steps_cyl_table_create_ewald(int n_delta, int n_rho, double rho_max, double alpha, int n_max,
                                           int m_max, int kernel, hipStream_t stream, steps_cyl_table **out) {
    if (!out) return fail(STEPS_EINVAL, "out must be non-null");
    int rc = check_grid(n_delta, n_rho, rho_max);
    if (rc) return rc;
    if (rho_max < 4.0) return fail(STEPS_EINVAL, "a complete table needs rho_max >= 4 (got %g)", rho_max);
    if (!finite_positive(alpha) || alpha > 64.0) return fail(STEPS_EINVAL, "alpha must lie in (0, 64]");
    if (n_max < 1 || n_max > 1024) return fail(STEPS_EINVAL, "n_max=%d outside [1, 1024]", n_max);
    if (m_max < 0 || m_max > 1024) return fail(STEPS_EINVAL, "m_max=%d outside [0, 1024]", m_max);
    if (kernel != STEPS_EWALD_BESSEL && kernel != STEPS_EWALD_PRINTED)
        return fail(STEPS_EINVAL, "kernel=%d: STEPS_EWALD_BESSEL or STEPS_EWALD_PRINTED", kernel);
    if ((rc = require_device())) return rc;
    clear_error();
    steps_cyl_table *t = new_table(n_delta, n_rho, rho_max, 0, 1);
    if (!t) return fail(STEPS_ENOMEM, "table allocation failed");
    const int nodes = (n_delta + 3) * (n_rho + 3);
    hipLaunchKernelGGL(build_ewald_kernel, dim3(nodes), dim3(64), 0, stream, t->nodes, t->nodes64, n_delta,
                       0.5 / n_delta, rho_max / n_rho, alpha, n_max, m_max, kernel == STEPS_EWALD_PRINTED);
    return finish_build(t, stream, out);
}

STEPS_API void steps_cyl_table_destroy(steps_cyl_table *t) {
    if (!t) return;
    (void)hipFree(t->nodes);
    (void)hipFree(t->nodes64);
    delete t;
}

STEPS_API int steps_cyl_table_values(const steps_cyl_table *t, float *host_out) {
    if (!t || !host_out) return fail(STEPS_EINVAL, "table and host_out must be non-null");
    clear_error();
    const size_t nodes = (size_t)(t->n_d + 3) * (t->n_r + 3);
    STEPS_CHECK_HIP(hipMemcpy(host_out, t->nodes, nodes * sizeof(float2), hipMemcpyDeviceToHost));
    return STEPS_OK;
}

STEPS_API int steps_cyl_table_values_f64(const steps_cyl_table *t, double *host_out) {
    if (!t || !host_out) return fail(STEPS_EINVAL, "table and host_out must be non-null");
    clear_error();
    const size_t nodes = (size_t)(t->n_d + 3) * (t->n_r + 3);
    STEPS_CHECK_HIP(hipMemcpy(host_out, t->nodes64, nodes * sizeof(double2), hipMemcpyDeviceToHost));
    return STEPS_OK;
}

STEPS_API int steps_cyl_table_info(const steps_cyl_table *t, int *n_delta, int *n_rho, double *rho_max,
                                   int *n_far) {
    if (!t) return fail(STEPS_EINVAL, "table must be non-null");
    clear_error();
    if (n_delta) *n_delta = t->n_d;
    if (n_rho) *n_rho = t->n_r;
    if (rho_max) *rho_max = t->r_max;
    if (n_far) *n_far = t->complete ? -1 : t->n_far;
    return STEPS_OK;
}

namespace steps {

int check_table_call(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                     const steps_cyl_table *t, int order, const int64_t *targets, int64_t n_targets,
                     const float *out_acc) {
    if (!pos || !mass || !eps || !out_acc || !t)
        return fail(STEPS_EINVAL, "pos, mass, eps, out_acc and table must be non-null");
    if (N < 1 || N > STEPS_MAX_N) return fail(STEPS_EINVAL, "N=%lld outside [1, 2^29]", (long long)N);
    if (!finite_positive(L)) return fail(STEPS_EINVAL, "L must be finite and > 0");
    if (order != 1 && order != 2) return fail(STEPS_EINVAL, "order=%d: 1 (CIC) or 2 (TSC)", order);
    if (n_targets < 1 || n_targets > STEPS_MAX_N) return fail(STEPS_EINVAL, "n_targets out of range");
    if (!targets && n_targets != N) return fail(STEPS_EINVAL, "targets is NULL, so n_targets must equal N");
    return STEPS_OK;
}

size_t table_forces_bytes(int64_t N, const steps_cyl_table *t, int order, bool all_targets, int64_t n_targets,
                          bool pot) {
    return all_targets ? pairwise_bytes(N, 1, t, order, pot) : per_target_bytes(n_targets);
}

// The tabulated forces (arguments validated): the pairwise path for every
// particle, the per-target kernel for a list.
int launch_forces_table(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                        const steps_cyl_table *t, int order, const int64_t *targets, int64_t n_targets,
                        float *out_acc, float *out_pot, Workspace &ws, hipStream_t stream) {
    // every particle a target: each unordered pair once
    if (!targets) return launch_forces_pairwise(pos, mass, eps, N, L, 1, t, order, out_acc, out_pot, ws, stream);
    int rc = check_workspace(ws, per_target_bytes(n_targets));
    if (rc) return rc;
    TableArgs a;
    a.x = pos;
    a.y = pos + N;
    a.z = pos + 2 * N;
    a.m = mass;
    a.h = eps;
    a.targets = targets;
    a.ax = out_acc;
    a.ay = out_acc + n_targets;
    a.az = out_acc + 2 * n_targets;
    a.pot = out_pot;
    a.tv = table_view(t);
    a.pc = period_consts(L);
    a.N = (int)N;
    a.n_tgt = (int)n_targets;
    a.perm = nullptr;
    // walk the targets in spatial order (keys and order in the workspace)
    if (n_targets >= kOrderTargetsMin && (rc = order_targets(pos, N, L, targets, n_targets, stream, ws, &a.perm)))
        return rc;
    hipError_t e;
    if (order == 1)
        e = out_pot ? launch_t<1, true>(a, stream) : launch_t<1, false>(a, stream);
    else
        e = out_pot ? launch_t<2, true>(a, stream) : launch_t<2, false>(a, stream);
    return hip_status(e, "forces_table launch");
}

}  // namespace steps

STEPS_API int steps_cyl_forces_table_ws(const double *pos, const double *mass, const double *eps, int64_t N,
                                        double L, const steps_cyl_table *t, int order, const int64_t *targets,
                                        int64_t n_targets, float *out_acc, float *out_pot, void *workspace,
                                        size_t workspace_bytes, hipStream_t stream) {
    int rc = check_table_call(pos, mass, eps, N, L, t, order, targets, n_targets, out_acc);
    if (rc) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    Workspace ws;
    ws.base = (char *)workspace;
    ws.size = workspace ? workspace_bytes : 0;
    return launch_forces_table(pos, mass, eps, N, L, t, order, targets, n_targets, out_acc, out_pot, ws, stream);
}

STEPS_API int steps_cyl_forces_table(const double *pos, const double *mass, const double *eps, int64_t N,
                                     double L, const steps_cyl_table *t, int order, const int64_t *targets,
                                     int64_t n_targets, float *out_acc, float *out_pot, hipStream_t stream) {
    int rc = check_table_call(pos, mass, eps, N, L, t, order, targets, n_targets, out_acc);
    if (rc) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    const size_t bytes = table_forces_bytes(N, t, order, targets == nullptr, n_targets, out_pot != nullptr);
    return with_stream_workspace(bytes, stream, [&](Workspace &ws) {
        return launch_forces_table(pos, mass, eps, N, L, t, order, targets, n_targets, out_acc, out_pot, ws,
                                   stream);
    });
}
