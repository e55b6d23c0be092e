// Kick-drift-kick leapfrog in cosmic time for the comoving S1 x R2 equations
// of motion (Sect. 2.1, eq. ComovingEquationsOfMotionCylindrical and the
// integrator named after it; background from Sect. 2.3, eqs. Friedmann,
// DEdensity, CPLw0wa):
//
//     dp/dt = (g(x) - F_h(x)) / a,    dx/dt = p / a^2,    p = a^2 dx/dt,
//
// where g is the pair-sum acceleration at unit scale factor (the force
// kernels) and F_h the field of the homogeneous cylinder that the truncated
// image sum pulls every particle with.  Writing the momentum as p = a^2 dx/dt
// absorbs the Hubble drag -2H dx/dt exactly; F_h carries the same a^-3 as
// the pair term so that a homogeneous load feels no net force at any epoch.
//
// Host: the step length dt = t(a_end) - t(a_begin) by Gauss-Legendre
// quadrature in ln a, then the Friedmann equation da/dt = a H(a) advanced by
// fourth-order Runge-Kutta together with int dt/a and int dt/a^2 over the
// two half steps.  Device (FP64): kick, drift with the z wrap, and F_h.
//
// F_h in the mid-plane of a cylinder of radius R, half-height Z, density
// rho0 (per particle at radius rho):
//   F_h = 2 G rho0 (2 A - B),  B = pi rho (rho <= R) or pi R^2 / rho,
//   A = int_0^{pi/2} log1p(delta(theta)) R cos(theta) dtheta,
//   delta = 4 rho R cos(theta) / ((s+ + s-)(s- + Z)),  s+- = sqrt(Z^2 + w+-),
//   w+- = R^2 + rho^2 +- 2 rho R cos(theta),
// the line-element integral over disk chords with Y = R sin(theta), written
// without cancellation; A is evaluated with 64-point Gauss-Legendre.
#include <cmath>
#include <vector>

#include "common.h"

namespace steps {


namespace {

constexpr int kGL = 64;
constexpr double kPi = 3.14159265358979323846;

struct Quad {
    double x[kGL];  // nodes in [0, pi/2]
    double w[kGL];
};

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

const Quad &theta_rule() {
    static Quad q = [] {
        Quad r;
        double x[kGL], w[kGL];
        gauss_legendre(kGL, x, w);
        for (int i = 0; i < kGL; ++i) {  // map [-1, 1] -> [0, pi/2]
            r.x[i] = 0.25 * kPi * (x[i] + 1.0);
            r.w[i] = 0.25 * kPi * w[i];
        }
        return r;
    }();
    return q;
}

struct Rule16 {
    double x[16], w[16];  // on [-1, 1]
};

// initialised once, thread-safe (function-local static)
const Rule16 &rule16() {
    static const Rule16 r = [] {
        Rule16 q;
        gauss_legendre(16, q.x, q.w);
        return q;
    }();
    return r;
}

struct CompArgs {
    Quad q;
    double R, Z, rho0;  // G = 1
};

// F_h(rho) per unit G (radial component, negative = inward)
__device__ double cylinder_field(double rho, const CompArgs &c) {
    if (rho <= 0.0) return 0.0;
    const double R = c.R, Z = c.Z, Z2 = Z * Z;
    double A = 0.0;
    for (int i = 0; i < kGL && Z < INFINITY; ++i) {  // A -> 0 for an infinite cylinder
        const double ct = cos(c.q.x[i]);
        const double t = 2.0 * rho * R * ct;
        const double base = R * R + rho * rho;
        const double sp = sqrt(Z2 + base + t), sm = sqrt(Z2 + base - t);
        const double delta = 2.0 * t / ((sp + sm) * (sm + Z));
        A += c.q.w[i] * log1p(delta) * R * ct;
    }
    const double B = (rho <= R) ? kPi * rho : kPi * R * R / rho;
    return 2.0 * c.rho0 * (2.0 * A - B);
}

__global__ void compensation_kernel(const double *pos, int64_t N, CompArgs c, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double x = pos[i], y = pos[N + i];
    const double rho = sqrt(x * x + y * y);
    const double f = cylinder_field(rho, c);
    const double s = rho > 0.0 ? f / rho : 0.0;
    out[i] = s * x;
    out[N + i] = s * y;
    out[2 * N + i] = 0.0;
}

// p += K (g - F_h(x))
__global__ void kick_kernel(const double *pos, double *mom, const float *acc, int64_t N, double K,
                            CompArgs c, int compensate) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double cx = 0.0, cy = 0.0;
    if (compensate) {
        const double x = pos[i], y = pos[N + i];
        const double rho = sqrt(x * x + y * y);
        const double s = rho > 0.0 ? cylinder_field(rho, c) / rho : 0.0;
        cx = s * x;
        cy = s * y;
    }
    mom[i] += K * ((double)acc[i] - cx);
    mom[N + i] += K * ((double)acc[N + i] - cy);
    mom[2 * N + i] += K * (double)acc[2 * N + i];
}

// x += D p, z wrapped into [0, L)
__global__ void drift_kernel(double *pos, const double *mom, int64_t N, double D, double L) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    pos[i] += D * mom[i];
    pos[N + i] += D * mom[N + i];
    double z = pos[2 * N + i] + D * mom[2 * N + i];
    z = z - L * floor(z / L);
    pos[2 * N + i] = (z >= L) ? 0.0 : z;
}

// ---------------------------------------------------------------- background
struct Background {
    double H0, Om, OL, Or, Ok, w0, wa;
    double hubble(double a) const {
        // CPL: Omega_DE(a) = Omega_DE,0 a^{-3(1+w0+wa)} exp(3 wa (a - 1))
        const double de = OL * std::pow(a, -3.0 * (1.0 + w0 + wa)) * std::exp(3.0 * wa * (a - 1.0));
        return H0 * std::sqrt(Or / (a * a * a * a) + Om / (a * a * a) + Ok / (a * a) + de);
    }
};

// t(a1) - t(a0) = int_{ln a0}^{ln a1} dln a / H(a), composite Gauss-Legendre
double step_length(const Background &bg, double a0, double a1) {
    const Rule16 &g = rule16();
    const double *x = g.x, *w = g.w;
    const double l0 = std::log(a0), l1 = std::log(a1);
    const int panels = 64;
    const double hw = (l1 - l0) / panels;
    double sum = 0.0;
    for (int p = 0; p < panels; ++p) {
        const double mid = l0 + (p + 0.5) * hw;
        for (int i = 0; i < 16; ++i) sum += 0.5 * hw * w[i] / bg.hubble(std::exp(mid + 0.5 * hw * x[i]));
    }
    return sum;
}

// RK4 on (a, int dt/a, int dt/a^2) over `span` of cosmic time from a0
void advance(const Background &bg, double a0, double span, int n_sub, double out[3]) {
    double y[3] = {a0, 0.0, 0.0};
    const double h = span / n_sub;
    auto f = [&](const double *s, double *d) {
        d[0] = s[0] * bg.hubble(s[0]);
        d[1] = 1.0 / s[0];
        d[2] = 1.0 / (s[0] * s[0]);
    };
    for (int k = 0; k < n_sub; ++k) {
        double k1[3], k2[3], k3[3], k4[3], t[3];
        f(y, k1);
        for (int q = 0; q < 3; ++q) t[q] = y[q] + 0.5 * h * k1[q];
        f(t, k2);
        for (int q = 0; q < 3; ++q) t[q] = y[q] + 0.5 * h * k2[q];
        f(t, k3);
        for (int q = 0; q < 3; ++q) t[q] = y[q] + h * k3[q];
        f(t, k4);
        for (int q = 0; q < 3; ++q) y[q] += h / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
    }
    for (int q = 0; q < 3; ++q) out[q] = y[q];
}

// the force and compensation settings, common to both ways of giving the factors
int check_force_params(const steps_cyl_kdk_params *p) {
    if (p->compensate && (!finite_positive(p->R_cyl) || !std::isfinite(p->rho0) || p->rho0 < 0.0))
        return fail(STEPS_EINVAL, "compensation needs R_cyl > 0 and rho0 >= 0");
    if (p->net && p->table) return fail(STEPS_EINVAL, "give a network or a table, not both");
    if (p->tree && !p->table) return fail(STEPS_EINVAL, "a tree needs a table");
    if (p->tree && (!std::isfinite(p->theta) || p->theta < 0.0 || !std::isfinite(p->tree_shift) ||
                    !std::isfinite(p->tree_angle)))
        return fail(STEPS_EINVAL, "tree: theta >= 0, shift and angle finite");
    if (p->table && p->table_order != 1 && p->table_order != 2)
        return fail(STEPS_EINVAL, "table_order=%d: 1 (CIC) or 2 (TSC)", p->table_order);
    if (!p->net && !p->table && (p->n_img < 0 || p->n_img > STEPS_MAX_NIMG))
        return fail(STEPS_EINVAL, "n_img=%d outside [0, %d]", p->n_img, STEPS_MAX_NIMG);
    return STEPS_OK;
}

int check_params(const steps_cyl_kdk_params *p) {
    if (!p) return fail(STEPS_EINVAL, "params must be non-null");
    if (p->factors) {
        for (int q = 0; q < 3; ++q)
            if (!std::isfinite(p->factors[q])) return fail(STEPS_EINVAL, "non-finite step factor");
        return check_force_params(p);
    }
    const double v[] = {p->a_begin, p->a_end, p->H0, p->Omega_m, p->Omega_L, p->Omega_r, p->Omega_k, p->w0, p->wa};
    for (double x : v)
        if (!std::isfinite(x)) return fail(STEPS_EINVAL, "non-finite background parameter");
    if (!(p->a_begin > 0.0) || !(p->a_end > 0.0)) return fail(STEPS_EINVAL, "scale factors must be > 0");
    if (!(p->H0 > 0.0)) return fail(STEPS_EINVAL, "H0 must be > 0");
    // H^2 must stay positive over the step
    Background bg{p->H0, p->Omega_m, p->Omega_L, p->Omega_r, p->Omega_k, p->w0, p->wa};
    const double lo = std::fmin(p->a_begin, p->a_end), hi = std::fmax(p->a_begin, p->a_end);
    for (int i = 0; i <= 32; ++i) {
        const double a = lo * std::pow(hi / lo, i / 32.0);
        const double H = bg.hubble(a);
        if (!std::isfinite(H) || !(H > 0.0)) return fail(STEPS_EDOMAIN, "H(a) is not positive at a=%g", a);
    }
    return check_force_params(p);
}

void factors(const steps_cyl_kdk_params *p, double out[3]) {
    if (p->factors) {
        out[0] = p->factors[0];
        out[1] = p->factors[1];
        out[2] = p->factors[2];
        return;
    }
    Background bg{p->H0, p->Omega_m, p->Omega_L, p->Omega_r, p->Omega_k, p->w0, p->wa};
    const double dt = step_length(bg, p->a_begin, p->a_end);
    double h1[3], h2[3];
    advance(bg, p->a_begin, 0.5 * dt, 64, h1);
    advance(bg, h1[0], 0.5 * dt, 64, h2);
    out[0] = h1[1];
    out[1] = h1[2] + h2[2];
    out[2] = h2[1];
}

// ---------------------------------------------------------------- tabulated history
// a(t) on [t_k, t_k+1]: Lagrange polynomial through nodes k..k+1 (order 1),
// k..k+2 (order 2) or k-1..k+2 (order 3), shifted inwards at the table ends.
struct History {
    const double *t, *a;
    int64_t n;
    int order;
    double eval(double x) const {
        int64_t lo = 0, hi = n - 1;  // k: last node with t_k <= x, clamped to [0, n-2]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            if (t[mid] <= x) lo = mid; else hi = mid;
        }
        int64_t k = lo;
        if (k > n - 2) k = n - 2;
        int64_t first = (order == 3) ? k - 1 : k;
        if (first > n - 1 - order) first = n - 1 - order;
        if (first < 0) first = 0;
        double v = 0.0;
        for (int64_t p = first; p <= first + order; ++p) {
            double w = 1.0;
            for (int64_t q = first; q <= first + order; ++q)
                if (q != p) w *= (x - t[q]) / (t[p] - t[q]);
            v += w * a[p];
        }
        return v;
    }
    // t with a(t) = target by bisection on the (monotonic) interpolant
    double invert(double target) const {
        double lo = t[0], hi = t[n - 1];
        for (int it = 0; it < 200 && hi - lo > 1e-15 * std::fabs(hi); ++it) {
            const double mid = 0.5 * (lo + hi);
            if (eval(mid) < target) lo = mid; else hi = mid;
        }
        return 0.5 * (lo + hi);
    }
    // int_{x0}^{x1} a(t)^-p dt: 16-point Gauss-Legendre on every piece between nodes
    double integral(double x0, double x1, int p) const {
        const Rule16 &g = rule16();
        const double *gx = g.x, *gw = g.w;
        const double sgn = x1 >= x0 ? 1.0 : -1.0;
        const double lo = std::fmin(x0, x1), hi = std::fmax(x0, x1);
        double sum = 0.0, a0 = lo;
        int64_t k = 0;
        while (k < n && t[k] <= lo) ++k;
        while (a0 < hi) {
            const double b0 = (k < n && t[k] < hi) ? t[k] : hi;
            const double hw = 0.5 * (b0 - a0), mid = 0.5 * (a0 + b0);
            for (int i = 0; i < 16; ++i) sum += hw * gw[i] * std::pow(eval(mid + hw * gx[i]), -p);
            a0 = b0;
            ++k;
        }
        return sgn * sum;
    }
};

CompArgs comp_args(double R, double Z, double rho0) {
    CompArgs c;
    c.q = theta_rule();
    c.R = R;
    c.Z = Z;
    c.rho0 = rho0;
    return c;
}

}  // namespace
}  // namespace steps

using namespace steps;

STEPS_API int steps_cyl_kdk_factors(const steps_cyl_kdk_params *params, double *out) {
    int rc = check_params(params);
    if (rc) return rc;
    if (!out) return fail(STEPS_EINVAL, "out must be non-null");
    clear_error();
    factors(params, out);
    return STEPS_OK;
}

STEPS_API int steps_cyl_history_factors(const double *t, const double *a, int64_t n, int order,
                                        double a_begin, double a_end, double *out) {
    if (!t || !a || !out) return fail(STEPS_EINVAL, "t, a and out must be non-null");
    if (order < 1 || order > 3) return fail(STEPS_EINVAL, "order=%d: 1, 2 or 3", order);
    if (n < order + 1) return fail(STEPS_EINVAL, "n=%lld: at least order+1 nodes", (long long)n);
    for (int64_t k = 0; k < n; ++k) {
        if (!std::isfinite(t[k]) || !std::isfinite(a[k]) || !(a[k] > 0.0))
            return fail(STEPS_EINVAL, "node %lld is not finite or has a <= 0", (long long)k);
        if (k > 0 && !(t[k] > t[k - 1] && a[k] > a[k - 1]))
            return fail(STEPS_EINVAL, "t and a must increase strictly (node %lld)", (long long)k);
    }
    const double lo = std::fmin(a_begin, a_end), hi = std::fmax(a_begin, a_end);
    if (!(lo >= a[0] && hi <= a[n - 1]))
        return fail(STEPS_EDOMAIN, "the step [%g, %g] leaves the table [%g, %g]", a_begin, a_end, a[0], a[n - 1]);
    clear_error();
    const History H{t, a, n, order};
    const double t0 = H.invert(a_begin), t1 = H.invert(a_end), tm = 0.5 * (t0 + t1);
    out[0] = H.integral(t0, tm, 1);
    out[1] = H.integral(t0, t1, 2);
    out[2] = H.integral(tm, t1, 1);
    return STEPS_OK;
}

STEPS_API int steps_cyl_compensation(const double *pos, int64_t N, double R_cyl, double Z, double rho0,
                                     double *out, hipStream_t stream) {
    if (!pos || !out) return fail(STEPS_EINVAL, "pos and out must be non-null");
    if (N < 1 || N > STEPS_MAX_N) return fail(STEPS_EINVAL, "N=%lld outside [1, 2^29]", (long long)N);
    if (!finite_positive(R_cyl) || !(Z > 0.0) || !std::isfinite(rho0) || rho0 < 0.0)
        return fail(STEPS_EINVAL, "need R_cyl > 0 finite, Z > 0 (infinity allowed) and rho0 >= 0");
    int rc = require_device();
    if (rc) return rc;
    clear_error();
    hipLaunchKernelGGL(compensation_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream, pos, N,
                       comp_args(R_cyl, Z, rho0), out);
    return hip_status(hipGetLastError(), "compensation kernel");
}

STEPS_API int steps_cyl_kdk_step(double *pos, double *mom, const double *mass, const double *eps, int64_t N,
                                 double L, const steps_cyl_kdk_params *params, float *acc_inout,
                                 hipStream_t stream) {
    if (!pos || !mom || !mass || !eps || !acc_inout)
        return fail(STEPS_EINVAL, "pos, mom, mass, eps and acc_inout must be non-null");
    if (N < 1 || N > STEPS_MAX_N) return fail(STEPS_EINVAL, "N=%lld outside [1, 2^29]", (long long)N);
    if (!finite_positive(L)) return fail(STEPS_EINVAL, "L must be finite and > 0");
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = require_device())) return rc;
    clear_error();
    double f[3];
    factors(params, f);
    double Z = (params->n_img + 0.5) * L;
    if (params->net) {
        Z = 1024.5 * L;
    } else if (params->table) {
        int n_far = 0;
        if ((rc = steps_cyl_table_info(params->table, nullptr, nullptr, nullptr, &n_far))) return rc;
        Z = n_far < 0 ? INFINITY : (n_far + 0.5) * L;
    }
    const CompArgs c = comp_args(params->R_cyl, Z, params->rho0);
    const dim3 grid((unsigned)((N + 255) / 256)), block(256);
    hipLaunchKernelGGL(kick_kernel, grid, block, 0, stream, pos, mom, acc_inout, N, f[0], c, params->compensate);
    STEPS_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(drift_kernel, grid, block, 0, stream, pos, mom, N, f[1], L);
    STEPS_CHECK_HIP(hipGetLastError());
    if (params->net)
        rc = with_stream_workspace(learned_pairwise_bytes(N), stream, [&](Workspace &ws) {
            return launch_forces_learned_pairwise(pos, mass, eps, N, L, params->net, acc_inout, nullptr, ws,
                                                  stream);
        });
    else if (params->tree)
        rc = steps_cyl_tree_forces(params->tree, pos, mass, eps, N, L, params->R_cyl, params->table,
                                   params->table_order, params->theta, params->tree_shift, params->tree_angle,
                                   params->tree_correct, acc_inout, stream);
    else if (params->table)
        rc = steps_cyl_forces_table(pos, mass, eps, N, L, params->table, params->table_order, nullptr, N,
                                    acc_inout, nullptr, stream);
    else
        rc = with_stream_workspace(pairwise_bytes(N, params->n_img, nullptr, 0, false), stream, [&](Workspace &ws) {
            return launch_forces_pairwise(pos, mass, eps, N, L, params->n_img, nullptr, 0, acc_inout, nullptr, ws,
                                          stream);
        });
    if (rc) return rc;
    hipLaunchKernelGGL(kick_kernel, grid, block, 0, stream, pos, mom, acc_inout, N, f[2], c, params->compensate);
    return hip_status(hipGetLastError(), "kick kernel");
}
