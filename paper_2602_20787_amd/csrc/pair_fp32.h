// FP32 pair kernel of the image sum shared by the exact and learned force
// kernels: source records staged in LDS, the Newtonian fast path over the
// images |n| <= n_img, the rare FP64 spline branch, and Kahan accumulation.
#pragma once

#include <hip/hip_runtime.h>

#include "pair_f64.h"

namespace steps {

struct alignas(16) SrcRec {
    double x, y, z;
    float m, h;
};
static_assert(sizeof(SrcRec) == 32, "source record must be 32 bytes");

struct ImageConsts {
    float Lf, L2f, m2Lf;  // L, L^2, -2L in FP32
    int n_img;            // used when the image count is not a template constant
};

struct PairSums {
    float S, Fz, P;
};

// The whole pair in FP64 with the spline law on every image; returns
// S = sum F(r)/r, Fz = sum F(r)/r (d - nL) and P = -sum P(r).
__device__ __noinline__ PairSums pair_general_f64(double dx, double dy, double d, double h, double L,
                                                  int n_img) {
    double s, fz, p;
    pair_spline_f64(dx, dy, d, h, L, n_img, s, fz, p);
    return PairSums{(float)s, (float)fz, (float)p};
}

__device__ __forceinline__ void kahan_add(float &sum, float &c, float x) {
    const float y = x - c;
    const float t = sum + y;
    c = (t - sum) - y;
    sum = t;
}

// Newtonian terms of one pair over n = -n_img..n_img (NIMG >= 0: image count
// fixed at compile time; NIMG < 0: c.n_img at run time).  S = sum r^-3,
// Fz = sum r^-3 (d - nL), P = sum r^-1.
template <int NIMG, bool POT>
__device__ __forceinline__ void pair_fast(float dx, float dy, float d, const ImageConsts &c, float &S,
                                          float &Fz, float &P) {
    const int n_img = (NIMG >= 0) ? NIMG : c.n_img;
    const float rho2 = __builtin_fmaf(dx, dx, dy * dy);
    const float r2_0 = __builtin_fmaf(d, d, rho2);
    const float ri0 = __builtin_amdgcn_rsqf(r2_0);
    // the sums start at -0: x + (-0) = x for every x, so the first additions
    // fold away (a +0 start would cost an add per sum: +0 + -0 is +0, not -0)
    float Tp = -0.f, Tm = -0.f, Up = -0.f, Um = -0.f, Pp = -0.f, Pm = -0.f;
    if (n_img >= 2) {
        const float B = d * c.m2Lf;  // -2 L d
#pragma unroll
        for (int n = n_img; n >= 2; --n) {
            const float nf = (float)n;
            const float Cn = __builtin_fmaf(nf * nf, c.L2f, r2_0);
            const float r2p = __builtin_fmaf(B, nf, Cn);   // image +n: dz = d - nL
            const float r2m = __builtin_fmaf(B, -nf, Cn);  // image -n: dz = d + nL
            const float rip = __builtin_amdgcn_rsqf(r2p);
            const float rim = __builtin_amdgcn_rsqf(r2m);
            Tp = __builtin_fmaf(rip * rip, rip, Tp);
            Tm = __builtin_fmaf(rim * rim, rim, Tm);
            Up += Tp;
            Um += Tm;
            if (POT) {
                Pp += rip;
                Pm += rim;
            }
        }
    }
    if (n_img >= 1) {
        // n = +-1 directly: the shared-C form would lose ~3 bits here
        const float dzp = d - c.Lf, dzm = d + c.Lf;
        const float rip = __builtin_amdgcn_rsqf(__builtin_fmaf(dzp, dzp, rho2));
        const float rim = __builtin_amdgcn_rsqf(__builtin_fmaf(dzm, dzm, rho2));
        Tp = __builtin_fmaf(rip * rip, rip, Tp);
        Tm = __builtin_fmaf(rim * rim, rim, Tm);
        Up += Tp;
        Um += Tm;
        if (POT) {
            Pp += rip;
            Pm += rim;
        }
    }
    S = __builtin_fmaf(ri0 * ri0, ri0, Tp + Tm);
    Fz = __builtin_fmaf(d, S, -c.Lf * (Up - Um));
    if (POT) P = ri0 + (Pp + Pm);
}

}  // namespace steps
