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

// Newtonian terms of the images n != 0 of one pair (NIMG >= 0: image count
// fixed at compile time; NIMG < 0: c.n_img at run time), from rho^2, the
// minimum-image offset d and r2_0 = rho^2 + d^2: T = sum_{n != 0} r^-3,
// U = sum_{n > 0} n (r_n^-3 - r_-n^-3) and Q = sum_{n != 0} r^-1, so that
// with an n = 0 term s0 (r^-3, or the softened F/r) and p0 (r^-1, or -P)
// the pair sums are S = s0 + T, Fz = d S - L U and P = p0 + Q.
template <int NIMG, bool POT>
__device__ __forceinline__ void pair_images(float rho2, float d, float r2_0, const ImageConsts &c, float &T,
                                            float &U, float &Q) {
    const int n_img = (NIMG >= 0) ? NIMG : c.n_img;
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
    T = Tp + Tm;
    U = Up - Um;
    Q = POT ? (Pp + Pm) : 0.f;
}

// Newtonian terms of one pair over n = -n_img..n_img.  S = sum r^-3,
// Fz = sum r^-3 (d - nL), P = sum r^-1.
template <int NIMG, bool POT>
__device__ __forceinline__ void pair_fast(float dx, float dy, float d, const ImageConsts &c, float &S,
                                          float &Fz, float &P) {
    const float rho2 = __builtin_fmaf(dx, dx, dy * dy);
    const float r2_0 = __builtin_fmaf(d, d, rho2);
    const float ri0 = __builtin_amdgcn_rsqf(r2_0);
    float T, U, Q;
    pair_images<NIMG, POT>(rho2, d, r2_0, c, T, U, Q);
    S = __builtin_fmaf(ri0 * ri0, ri0, T);
    Fz = __builtin_fmaf(d, S, -c.Lf * U);
    if (POT) P = ri0 + Q;
}

// The n = 0 term of the cubic-spline law in FP32 (Sect. 2.1, eq.
// Force_spline_kernel): F(r)/r and -P(r) at r^2 = r2 for softening length
// h (r < h; a zero separation gives F/r = 32/(3 h^3) and -P = 2.8/h, so a
// coincident pair feels no force).
__device__ __forceinline__ void spline_n0(float r2, float h, float &f_over_r, float &pe) {
    const float ih = __builtin_amdgcn_rcpf(h);
    const float r = __builtin_sqrtf(r2);
    const float u = r * ih;
    const float ih3 = ih * ih * ih;
    if (u < 0.5f) {
        const float u2 = u * u;
        f_over_r = __builtin_fmaf(u2, __builtin_fmaf(32.0f, u, -38.4f), 32.0f / 3.0f) * ih3;
        pe = -__builtin_fmaf(u2, __builtin_fmaf(u2, __builtin_fmaf(6.4f, u, -9.6f), 16.0f / 3.0f), -2.8f) * ih;
    } else {
        // F = M(<r)/r^2, M = 1 - w^4 (16 - w (25.6 - 32/3 w)), w = 1 - u
        const float w = 1.0f - u;
        const float w2 = w * w;
        const float M = __builtin_fmaf(-w2 * w2, __builtin_fmaf(-w, __builtin_fmaf(-32.0f / 3.0f, w, 25.6f), 16.0f),
                                       1.0f);
        const float ir = __builtin_amdgcn_rcpf(r);
        f_over_r = M * ir * ir * ir;
        const float poly = __builtin_fmaf(
            u * u, __builtin_fmaf(u, __builtin_fmaf(u, __builtin_fmaf(-32.0f / 15.0f, u, 9.6f), -16.0f), 32.0f / 3.0f),
            -3.2f);
        pe = -(poly + __builtin_amdgcn_rcpf(15.0f * u)) * ih;
    }
}

}  // namespace steps
