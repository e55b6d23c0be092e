// The learned far-image correction as a function of one pair (units of L,
// force per unit G m_j / L^2): network features, output scale and the fixed
// analytic baseline (rods of image mass from 1.5 L to 1024.5 L on both sides
// plus the first midpoint-rule end correction at 1.5 L).  The network adds
// s(r) o to the baseline; the fit target is (exact band - baseline) / s.
#pragma once

#include <hip/hip_runtime.h>

#include "mlp_device.h"

namespace steps {
namespace mlp {

// features: f1 = 4 delta - 1, f2 = 2 ln(r / 0.05) / ln 400 - 1
__device__ __forceinline__ void features_f32(float delta, float r, float &f1, float &f2) {
    f1 = __builtin_fmaf(4.0f, delta, -1.0f);
    // ln(r/0.05) / ln 400 = log2(r / 0.05) / log2(400)
    f2 = __builtin_fmaf(2.0f / 8.643856189774724f, __builtin_amdgcn_logf(r * 20.0f), -1.0f);
}

__device__ __forceinline__ float out_scale_f32(float r) {
    return kOutScale * __builtin_amdgcn_rcpf(__builtin_fmaf(r, r, 1.0f));
}

// Baseline in FP32, written without cancellation: differences of the rod
// end terms are rearranged so that no two nearly equal numbers are
// subtracted (rho -> 0 and delta -> 0 keep full relative precision).
__device__ __forceinline__ void baseline_f32(float delta, float r, float &bz, float &br) {
    const float S1 = (float)kRodInner, S2 = (float)kFarImages + 0.5f;
    const float r2 = r * r;
    // distances of the four rod ends: a = S -+ delta
    const float a1m = S1 - delta, a1p = S1 + delta, a2m = S2 - delta, a2p = S2 + delta;
    const float i1m = __builtin_amdgcn_rsqf(__builtin_fmaf(a1m, a1m, r2));
    const float i1p = __builtin_amdgcn_rsqf(__builtin_fmaf(a1p, a1p, r2));
    const float i2m = __builtin_amdgcn_rsqf(__builtin_fmaf(a2m, a2m, r2));
    const float i2p = __builtin_amdgcn_rsqf(__builtin_fmaf(a2p, a2p, r2));
    // z: [1/A(S1-d) - 1/A(S1+d)] - [1/A(S2-d) - 1/A(S2+d)], 1/A - 1/B = (b^2-a^2) iA^2 iB^2/(iA+iB)
    const float q1 = (4.0f * S1 * delta) * (i1m * i1m) * (i1p * i1p) * __builtin_amdgcn_rcpf(i1m + i1p);
    const float q2 = (4.0f * S2 * delta) * (i2m * i2m) * (i2p * i2p) * __builtin_amdgcn_rcpf(i2m + i2p);
    bz = q1 - q2;
    // rho: -(1/r)[c(a2) - c(a1)] per side, c(a) = a/A(a), rewritten as
    // -r (a2^2 - a1^2) iA1^2 iA2^2 / (c1 + c2)
    const float cm1 = a1m * i1m, cm2 = a2m * i2m, cp1 = a1p * i1p, cp2 = a2p * i2p;
    const float dm = (S2 - S1) * (a2m + a1m);
    const float dp = (S2 - S1) * (a2p + a1p);
    br = -r * (dm * (i1m * i1m) * (i2m * i2m) * __builtin_amdgcn_rcpf(cm1 + cm2) +
               dp * (i1p * i1p) * (i2p * i2p) * __builtin_amdgcn_rcpf(cp1 + cp2));
    // first midpoint-rule correction at the inner ends, u = +-S1 - delta
    const float i1m2 = i1m * i1m, i1p2 = i1p * i1p;
    const float q5m = i1m2 * i1m2 * i1m, q5p = i1p2 * i1p2 * i1p;
    const float um = a1m, up = -a1p;  // + side u = S1 - d, - side u = -S1 - d
    bz += (1.0f / 24.0f) * ((r2 - 2.0f * um * um) * q5m - (r2 - 2.0f * up * up) * q5p);
    br += (1.0f / 24.0f) * (3.0f * r * um * q5m - 3.0f * r * up * q5p);
}

// Same baseline in FP64 (training targets).
__device__ __forceinline__ void baseline_f64(double delta, double r, double &bz, double &br) {
    const double S1 = kRodInner, S2 = (double)kFarImages + 0.5;
    auto inv = [&](double u) { return 1.0 / sqrt(u * u + r * r); };
    bz = inv(S1 - delta) - inv(S2 - delta) - inv(S1 + delta) + inv(S2 + delta);
    br = -(1.0 / r) * ((S2 - delta) * inv(S2 - delta) - (S1 - delta) * inv(S1 - delta) +
                       (S2 + delta) * inv(S2 + delta) - (S1 + delta) * inv(S1 + delta));
    for (int side = 1; side >= -1; side -= 2) {
        const double u = side * S1 - delta;
        const double q = inv(u);
        const double q5 = q * q * q * q * q;
        bz += side * (r * r - 2.0 * u * u) * q5 / 24.0;
        br += side * 3.0 * r * u * q5 / 24.0;
    }
}

}  // namespace mlp
}  // namespace steps
