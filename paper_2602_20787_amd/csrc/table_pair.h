// Device side of the tabulated far-image correction, shared by the table
// force kernel and the octree walk: the table object, a view of it for
// kernels, the CIC/TSC lookup, the exact band shared by a wave, and the pair
// interaction of the tabulated scheme (exact images |n| <= 1, softened, plus
// the interpolated band; Sect. 2.2, eq. S1R2EwaldCorrectionTable).
#pragma once

#include "common.h"
#include "pair_f64.h"
#include "pair_fp32.h"

struct steps_cyl_table {
    float2 *nodes = nullptr;     // [(n_r + 3) * (n_d + 3)], node (i, j) at (j + 1) * (n_d + 3) + i + 1
    double2 *nodes64 = nullptr;  // the same nodes in FP64
    int n_d = 0, n_r = 0, n_far = 0;
    int complete = 0;            // 1: every image |n| >= 2 (Ewald build)
    double r_max = 0.0;
};

namespace steps {

// what a kernel needs of a table (passed by value)
struct TableView {
    const float2 *T;
    float inv_hd, inv_hr, r_max;
    int n_d, n_r, n_far, w, complete;
};

inline TableView table_view(const steps_cyl_table *t) {
    TableView v;
    v.T = t->nodes;
    v.inv_hd = (float)(2.0 * t->n_d);
    v.inv_hr = (float)(t->n_r / t->r_max);
    v.r_max = (float)t->r_max;
    v.n_d = t->n_d;
    v.n_r = t->n_r;
    v.n_far = t->n_far;
    v.w = t->n_d + 3;
    v.complete = t->complete;
    return v;
}

// period-dependent constants of the pair interaction
struct PeriodConsts {
    double L, invL, halfL;
    float invLf, invL2f;
    ImageConsts c;  // n_img = 1
};

inline PeriodConsts period_consts(double L) {
    PeriodConsts p;
    p.L = L;
    p.invL = 1.0 / L;
    p.halfL = 0.5 * L;
    p.invLf = (float)(1.0 / L);
    p.invL2f = (float)(1.0 / (L * L));
    p.c.Lf = (float)L;
    p.c.L2f = (float)(L * L);
    p.c.m2Lf = (float)(-2.0 * L);
    p.c.n_img = 1;
    return p;
}

// exact band of one pair shared by the wave (see the learned kernel)
__device__ __forceinline__ void band_wave(float delta, float r, int n_far, float &fz, float &fr) {
    const int lane = threadIdx.x & 63;
    const float r2 = r * r;
    float sz = 0.f, sr = 0.f;
    for (int q = 2 + lane + 64 * ((n_far - 2 - lane) / 64 + 1); q >= 2; q -= 64) {
        if (q <= n_far) {
            const float qf = (float)q;
            const float up = delta - qf, um = delta + qf;
            const float ip = __builtin_amdgcn_rsqf(__builtin_fmaf(up, up, r2));
            const float im = __builtin_amdgcn_rsqf(__builtin_fmaf(um, um, r2));
            const float ip3 = ip * ip * ip, im3 = im * im * im;
            sz = __builtin_fmaf(-up, ip3, __builtin_fmaf(-um, im3, sz));
            sr = __builtin_fmaf(-r, ip3 + im3, sr);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        sz += __shfl_xor(sz, off);
        sr += __shfl_xor(sr, off);
    }
    fz = sz;
    fr = sr;
}

template <int ORDER>
__device__ __forceinline__ void lookup(const TableView &a, float delta, float r, float &tz, float &tr) {
    const float x = delta * a.inv_hd, y = r * a.inv_hr;
    tz = 0.f;
    tr = 0.f;
    if (ORDER == 1) {
        // indices clamped into the table whatever the input (NaN included)
        const int i0 = max(0, min((int)x, a.n_d - 1)), j0 = max(0, min((int)y, a.n_r - 1));
        const float fx = x - (float)i0, fy = y - (float)j0;
        const float2 *p = a.T + (j0 + 1) * a.w + (i0 + 1);
        const float2 v00 = p[0], v10 = p[1], v01 = p[a.w], v11 = p[a.w + 1];
        const float z0 = __builtin_fmaf(fx, v10.x - v00.x, v00.x), z1 = __builtin_fmaf(fx, v11.x - v01.x, v01.x);
        const float r0 = __builtin_fmaf(fx, v10.y - v00.y, v00.y), r1 = __builtin_fmaf(fx, v11.y - v01.y, v01.y);
        tz = __builtin_fmaf(fy, z1 - z0, z0);
        tr = __builtin_fmaf(fy, r1 - r0, r0);
    } else {
        const int i0 = max(0, min((int)__builtin_rintf(x), a.n_d));
        const int j0 = max(0, min((int)__builtin_rintf(y), a.n_r));
        const float fx = x - (float)i0, fy = y - (float)j0;
        const float ax0 = 0.5f - fx, ax2 = 0.5f + fx, ay0 = 0.5f - fy, ay2 = 0.5f + fy;
        const float wx[3] = {0.5f * ax0 * ax0, 0.75f - fx * fx, 0.5f * ax2 * ax2};
        const float wy[3] = {0.5f * ay0 * ay0, 0.75f - fy * fy, 0.5f * ay2 * ay2};
        const float2 *p = a.T + j0 * a.w + i0;  // node (i0 - 1, j0 - 1)
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) {
            float rz = 0.f, rr = 0.f;
#pragma unroll
            for (int di = 0; di < 3; ++di) {
                const float2 v = p[dj * a.w + di];
                rz = __builtin_fmaf(wx[di], v.x, rz);
                rr = __builtin_fmaf(wx[di], v.y, rr);
            }
            tz = __builtin_fmaf(wy[dj], rz, tz);
            tr = __builtin_fmaf(wy[dj], rr, tr);
        }
    }
}


// One pair of the tabulated scheme, accumulated as (px, py) += m S_eff (dx, dy),
// pz += m Fz_eff, pp += m P (the caller negates at the end).  Every lane of
// the wave must call it together (the exact band beyond a band table's
// rho_max is shared by the wave); ``active`` marks lanes with a real target.
// COMPLETE: the table holds every image |n| >= 2 (pairs beyond rho_max take
// the line-mass limit) rather than a band.
template <int ORDER, bool POT, bool COMPLETE>
__device__ __forceinline__ void table_pair(const TableView &a, const PeriodConsts &pc, double xi, double yi,
                                           double zi, float hi, const SrcRec &src, bool self, bool active,
                                           float &px, float &py, float &pz, float &pp) {
    const int lane = threadIdx.x & 63;
    const double dx64 = xi - src.x, dy64 = yi - src.y;
    const double d64 = min_image(zi - src.z, pc.L, pc.invL);
    const float dx = (float)dx64, dy = (float)dy64, d = (float)d64;
    const float hij = hi + src.h;
    float S, Fz, Pn = 0.f;
    pair_fast<1, POT>(dx, dy, d, pc.c, S, Fz, Pn);
    const float rho2 = __builtin_fmaf(dx, dx, dy * dy);
    const float r2_0 = __builtin_fmaf(d, d, rho2);
    if (r2_0 < hij * hij || hij > (float)pc.halfL) {
        if (self) {
            S = 0.f;
            Fz = 0.f;
            Pn = 0.f;
        } else {
            const PairSums g = pair_general_f64(dx64, dy64, d64, (double)hi + (double)src.h, pc.L, 1);
            S = g.S;
            Fz = g.Fz;
            Pn = g.P;
        }
    }
    const float rho = __builtin_sqrtf(rho2);
    const float r = rho * pc.invLf;
    const float delta = __builtin_fabsf(d) * pc.invLf;
    const bool inside = (r <= a.r_max) && !self;
    float tz, tr;
    lookup<ORDER>(a, delta, inside ? r : 0.f, tz, tr);
    float Rz = (d > 0.f) ? tz : ((d < 0.f) ? -tz : 0.f);
    float Rr = tr;
    if (!inside) {
        Rz = 0.f;
        Rr = 0.f;
    }
    if (COMPLETE) {
        // line-mass limit of the complete sum minus the three nearest images
        if (!inside && !self) {
            const float ds = d * pc.invLf, r2 = r * r;
            float nz = 0.f, nr = 0.f;
#pragma unroll
            for (int n = -1; n <= 1; ++n) {
                const float u = ds - (float)n;
                const float iq = __builtin_amdgcn_rsqf(__builtin_fmaf(u, u, r2));
                const float iq3 = iq * iq * iq;
                nz = __builtin_fmaf(-u, iq3, nz);
                nr = __builtin_fmaf(-r, iq3, nr);
            }
            Rz = -nz;
            Rr = -2.f * __builtin_amdgcn_rcpf(r) - nr;
        }
    }
    uint64_t outside = COMPLETE ? 0 : __ballot(!inside && !self && active);
    while (outside) {
        const int c = __builtin_ctzll(outside);
        outside &= outside - 1;
        const float dc = __shfl(d * pc.invLf, c), rc = __shfl(r, c);
        float bz, br;
        band_wave(dc, rc, a.n_far, bz, br);
        if (lane == c) {
            Rz = bz;
            Rr = br;
        }
    }
    const float rinv = rho > 0.f ? __builtin_amdgcn_rcpf(rho) : 0.f;
    const float Seff = __builtin_fmaf(-Rr * pc.invL2f, rinv, S);
    const float Fzeff = __builtin_fmaf(-Rz, pc.invL2f, Fz);
    const float mS = src.m * Seff;
    px = __builtin_fmaf(mS, dx, px);
    py = __builtin_fmaf(mS, dy, py);
    pz = __builtin_fmaf(src.m, Fzeff, pz);
    if (POT) pp = __builtin_fmaf(src.m, Pn, pp);
}

}  // namespace steps
