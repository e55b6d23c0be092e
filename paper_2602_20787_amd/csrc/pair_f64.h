// FP64 evaluation of one pair over all its images with the cubic-spline law
// (Sect. 2.1, eq. Force_spline_kernel for F; P is its potential, dP/dr = F,
// P(inf) = 0).  Used by the rare softened branch of the FP32 kernels and by
// the FP64 reference kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace steps {

// Returns s = sum_n F(r_n)/r_n, fz = sum_n F(r_n)/r_n (d - nL) and
// p = -sum_n P(r_n) for n = -n_img..n_img, r_n^2 = dx^2 + dy^2 + (d - nL)^2.
// A zero separation contributes no force and -P(0) = 2.8/h.
__device__ __forceinline__ void pair_spline_f64(double dx, double dy, double d, double h,
                                                double L, int n_img, double &s, double &fz,
                                                double &p) {
    const double rho2 = dx * dx + dy * dy;
    const double ih = 1.0 / h;
    s = 0.0;
    fz = 0.0;
    p = 0.0;
    for (int n = -n_img; n <= n_img; ++n) {
        const double dz = d - (double)n * L;
        const double r2 = rho2 + dz * dz;
        double f_over_r, pe;
        if (r2 < h * h) {
            const double r = sqrt(r2);
            const double u = r * ih;
            if (u < 0.5) {
                // F/r = (32/3 - 38.4 u^2 + 32 u^3) / h^3
                f_over_r = (32.0 / 3.0 + u * u * (-38.4 + 32.0 * u)) * ih * ih * ih;
                pe = -(-2.8 + u * u * (16.0 / 3.0 + u * u * (-9.6 + 6.4 * u))) * ih;
            } else {
                // F = M(<r)/r^2 with the enclosed spline mass
                // M = 1 - w^4 (16 - w (25.6 - 32/3 w)), w = 1 - u (no cancellation)
                const double w = 1.0 - u;
                const double M = 1.0 - w * w * w * w * (16.0 - w * (25.6 - 32.0 / 3.0 * w));
                f_over_r = M / (r2 * r);
                pe = -(-3.2 + 1.0 / (15.0 * u) +
                       u * u * (32.0 / 3.0 + u * (-16.0 + u * (9.6 - 32.0 / 15.0 * u)))) * ih;
            }
        } else {
            const double ri = 1.0 / sqrt(r2);
            f_over_r = ri * ri * ri;
            pe = ri;
        }
        s += f_over_r;
        fz += f_over_r * dz;
        p += pe;
    }
}

// z wrapped into [0, L): z - L floor(z / L), with an exact L mapped to 0.
__device__ __forceinline__ double wrap_z(double z, double L) {
    double w = z - L * floor(z / L);
    return (w >= L) ? 0.0 : w;
}

// Minimum-image separation t - L floor(t/L + 1/2), with 1/L precomputed.
__device__ __forceinline__ double min_image(double t, double L, double invL) {
    return __builtin_fma(-L, floor(__builtin_fma(t, invL, 0.5)), t);
}

}  // namespace steps
