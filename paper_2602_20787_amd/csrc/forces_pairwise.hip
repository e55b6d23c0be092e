// Forces of all N particles with every unordered pair evaluated once
// (Sect. 2.1, eqs. ComovingEquationsOfMotion and ForceCylindrical; with a
// table, the far images of Sect. 2.2, eq. S1R2EwaldCorrectionTable).  The
// pair term is odd in the separation: the image set {d - nL, |n| <= n_img}
// of the pair (j, i) is the negated set of (i, j), so S and P are shared and
// F_z, dx, dy change sign; the table's far-image term is odd in d along z
// and even across, so the same holds with it.  The exception is an axial
// separation of L/2 (up to rounding), where both particles may take a
// minimum image of the same sign; F_z then keeps its sign.  Evaluating each
// pair once halves the arithmetic of the per-target kernels
// (forces_exact.hip, table.hip).
//
// Layout.  The particles are put in spatial (Morton) order and staged as
// 32-byte records {x, y, z wrapped, m, h}; groups of 1024 consecutive
// records (512 with a table) are the unit of work.  Group g pairs with itself (one-sided, all
// ordered pairs, no reaction) and with the next K(g) groups modulo G, where
// K = (G-1)/2 for odd G and G/2 - 1, plus one for the first half of the
// groups, for even G; every unordered pair of groups then meets exactly
// once.  The P workgroups of group g split its list of partner groups.
//
// Workgroup.  256 threads own the particles of their group, 4 each (2 with a
// table), in registers.  Partner records come through LDS in tiles of 256.  For each
// source a thread adds the FP32 pair term to its own FP64 sums and the
// reaction over its particles into one FP64 register set; the wave
// reduces those 4 values over its 64 lanes (a reduce-scatter that leaves
// one component per 16 lanes) and writes them to LDS; after the tile the 4
// waves' values are added and the source's
// reaction goes to FP64 device accumulators with atomic adds.  The owned
// particles' sums join the same accumulators at the end, and a last pass
// converts them to FP32 outputs at the particles' own positions.
#include "common.h"
#include "pair_f64.h"
#include "pair_fp32.h"
#include "table_pair.h"

namespace steps {

namespace {

constexpr int kThreads = 256;           // 4 waves
// particles per thread: 4 for the exact pair (fewer reactions to reduce and
// add per pair); 2 with a table, whose gathers want the occupancy that the
// smaller register set gives
constexpr int particles_per_thread(int torder) { return torder > 0 ? 2 : 4; }
constexpr int kTile = 256;              // sources per LDS tile

struct PairwiseArgs {
    const SrcRec *rec;  // [N] records in spatial order
    double *acc;        // [4][N] sums in spatial order (x, y, z, potential)
    double L, invL, halfL, tie;  // tie: |d| within this of L/2 takes the check
    float tie32;                 // FP32 screen for it: 0.5 L (1 - 1e-6), below every such |d|
    ImageConsts c;
    TableView tv;       // far-image table (table paths only)
    float invLf, invL2f;
    int N, G, P;        // particles, groups, workgroups per group
};

// Exact band 2 <= |n| <= n_far of one pair in one lane (delta = d/L signed,
// r = rho/L; per unit G m / L^2): the rare fallback of band tables for
// pairs beyond the table's rho range.
__device__ __noinline__ void band_serial(float delta, float r, int n_far, float &fz, float &fr) {
    const float r2 = r * r;
    float sz = 0.f, sr = 0.f;
    for (int q = n_far; q >= 2; --q) {
        const float qf = (float)q;
        const float up = delta - qf, um = delta + qf;
        const float ip = __builtin_amdgcn_rsqf(__builtin_fmaf(up, up, r2));
        const float im = __builtin_amdgcn_rsqf(__builtin_fmaf(um, um, r2));
        const float ip3 = ip * ip * ip, im3 = im * im * im;
        sz = __builtin_fmaf(-up, ip3, __builtin_fmaf(-um, im3, sz));
        sr = __builtin_fmaf(-r, ip3 + im3, sr);
    }
    fz = sz;
    fr = sr;
}

__global__ void stage_kernel(const double *pos, const double *mass, const double *eps, int N, double L,
                             const int *perm, SrcRec *rec, double *acc) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int p = perm[k];
    SrcRec r;
    r.x = pos[p];
    r.y = pos[N + p];
    r.z = wrap_z(pos[2 * N + p], L);
    r.m = (float)mass[p];
    r.h = (float)eps[p];
    rec[k] = r;
    acc[k] = 0.0;
    acc[N + k] = 0.0;
    acc[2 * (int64_t)N + k] = 0.0;
    acc[3 * (int64_t)N + k] = 0.0;
}

__global__ void finish_kernel(const double *acc, const int *perm, int N, float *ax, float *ay, float *az,
                              float *pot) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int p = perm[k];
    // attraction: a = -sum m_j S (x_i - x_j), potential = -sum m_j / r
    ax[p] = (float)(-acc[k]);
    ay[p] = (float)(-acc[N + k]);
    az[p] = (float)(-acc[2 * (int64_t)N + k]);
    if (pot) pot[p] = (float)(-acc[3 * (int64_t)N + k]);
}

template <int kR>
struct Owned {
    double x[kR], y[kR], z[kR];
    float h[kR], m[kR];
    int t[kR];  // record index, or N for an empty slot
};

// The sources of one LDS tile against the thread's particles.  REACT: the
// tile belongs to a partner group, so the reactions are reduced and left in
// jpart; otherwise (the group against itself) the self pair is skipped.
// Pair terms are FP32; both sides are summed in FP64 (the records are in
// spatial order, so a particle's near neighbours arrive together and an
// FP32 partial would lose their cancellation).
template <int NIMG, bool POT, int TORDER, bool COMPLETE, bool REACT, int kR = particles_per_thread(TORDER)>
__device__ __forceinline__ void tile_pass(const PairwiseArgs &a, const Owned<kR> &o, const SrcRec *tile, int base,
                                          int cnt, float hmax, double (*acc)[4], double (*jpart)[kTile][4]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float thr2[kR];
    bool wide[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const float hb = o.h[r] + hmax;  // >= h_i + h_j for every source of the tile
        thr2[r] = hb * hb;
        wide[r] = hb > (float)a.halfL;
    }
    for (int si = 0; si < cnt; ++si) {
        const SrcRec src = tile[si];
        double dx64[kR], dy64[kR];
        float S[kR], Fz[kR], P[kR], dr[kR];
        bool tie[kR];
        unsigned soft = 0;  // bit r: the pair (r, src) takes the FP64 spline
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            dx64[r] = o.x[r] - src.x;
            dy64[r] = o.y[r] - src.y;
            const double d64 = min_image(o.z[r] - src.z, a.L, a.invL);
            const float dx = (float)dx64[r], dy = (float)dy64[r], d = (float)d64;
            dr[r] = d;
            P[r] = 0.f;
            pair_fast<NIMG, POT>(dx, dy, d, a.c, S[r], Fz[r], P[r]);
            const float r2_0 = __builtin_fmaf(d, d, __builtin_fmaf(dx, dx, dy * dy));
            const float hij = o.h[r] + src.h;
            if ((wide[r] || r2_0 < thr2[r]) && (r2_0 < hij * hij || hij > (float)a.halfL)) soft |= 1u << r;
            tie[r] = REACT && __builtin_fabsf(d) >= a.tie32;
        }
        while (soft) {
            // rare and divergent: one pair per lane and pass, operands picked
            // by selects so that the spline code exists once
            const int rr = __builtin_ctz(soft);
            soft &= soft - 1;
            double xr = o.x[0], yr = o.y[0], zr = o.z[0];
            float hr = o.h[0];
            int tr = o.t[0];
#pragma unroll
            for (int k = 1; k < kR; ++k)
                if (rr == k) {
                    xr = o.x[k];
                    yr = o.y[k];
                    zr = o.z[k];
                    hr = o.h[k];
                    tr = o.t[k];
                }
            float gS = 0.f, gF = 0.f, gP = 0.f;
            if (REACT || base + si != tr) {
                double gs, gf, gp;
                pair_spline_f64(xr - src.x, yr - src.y, min_image(zr - src.z, a.L, a.invL),
                                (double)hr + (double)src.h, a.L, (NIMG >= 0) ? NIMG : a.c.n_img, gs, gf, gp);
                gS = (float)gs;
                gF = (float)gf;
                gP = (float)gp;
            }
#pragma unroll
            for (int k = 0; k < kR; ++k)
                if (rr == k) {
                    S[k] = gS;
                    Fz[k] = gF;
                    P[k] = gP;
                }
        }
        if (TORDER > 0) {
            // far images from the table (Sect. 2.2, eq. S1R2EwaldCorrectionTable):
            // R_z is odd in d and R_rho even, so the corrected pair keeps the
            // symmetry of the exact one
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const float dx = (float)dx64[r], dy = (float)dy64[r];
                const float rho = __builtin_sqrtf(__builtin_fmaf(dx, dx, dy * dy));
                const float rr = rho * a.invLf;
                const float delta = __builtin_fabsf(dr[r]) * a.invLf;
                const bool self = !REACT && base + si == o.t[r];
                const bool inside = (rr <= a.tv.r_max) && !self;
                float tz, tr;
                lookup<(TORDER > 0 ? TORDER : 1)>(a.tv, delta, inside ? rr : 0.f, tz, tr);
                float Rz = (dr[r] > 0.f) ? tz : ((dr[r] < 0.f) ? -tz : 0.f);
                float Rr = tr;
                if (!inside) {
                    Rz = 0.f;
                    Rr = 0.f;
                    if (!self) {
                        const float ds = dr[r] * a.invLf;
                        if (COMPLETE) {
                            // line-mass limit of the complete sum minus the images |n| <= 1
                            const float r2 = rr * rr;
                            float nz = 0.f, nr = 0.f;
#pragma unroll
                            for (int n = -1; n <= 1; ++n) {
                                const float u = ds - (float)n;
                                const float iq = __builtin_amdgcn_rsqf(__builtin_fmaf(u, u, r2));
                                const float iq3 = iq * iq * iq;
                                nz = __builtin_fmaf(-u, iq3, nz);
                                nr = __builtin_fmaf(-rr, iq3, nr);
                            }
                            Rz = -nz;
                            Rr = -2.f * __builtin_amdgcn_rcpf(rr) - nr;
                        } else {
                            band_serial(ds, rr, a.tv.n_far, Rz, Rr);
                        }
                    }
                }
                const float rinv = rho > 0.f ? __builtin_amdgcn_rcpf(rho) : 0.f;
                S[r] = __builtin_fmaf(-Rr * a.invL2f, rinv, S[r]);
                Fz[r] = __builtin_fmaf(-Rz, a.invL2f, Fz[r]);
            }
        }
        const double ms = (double)src.m;
        double jx = 0.0, jy = 0.0, jz = 0.0, jp = 0.0;
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const double S64 = (double)S[r], Fz64 = (double)Fz[r];
            const double mS = ms * S64;
            acc[r][0] = __builtin_fma(mS, dx64[r], acc[r][0]);
            acc[r][1] = __builtin_fma(mS, dy64[r], acc[r][1]);
            acc[r][2] = __builtin_fma(ms, Fz64, acc[r][2]);
            if (POT) acc[r][3] = __builtin_fma(ms, (double)P[r], acc[r][3]);
            if (REACT) {
                // the source sees -dx, -dy and -d, except where |d| = L/2 up to
                // rounding and its own minimum image has the sign of d
                double fz = Fz64;
                if (tie[r]) {
                    const double d64 = min_image(o.z[r] - src.z, a.L, a.invL);
                    if (__builtin_fabs(__builtin_fabs(d64) - a.halfL) <= a.tie) {
                        const double dji = min_image(src.z - o.z[r], a.L, a.invL);
                        if ((dji < 0.0) == (d64 < 0.0)) fz = -Fz64;
                    }
                }
                const double miS = o.m[r] * S64;
                jx = __builtin_fma(miS, dx64[r], jx);
                jy = __builtin_fma(miS, dy64[r], jy);
                jz = __builtin_fma(o.m[r], fz, jz);
                if (POT) jp = __builtin_fma(o.m[r], (double)P[r], jp);
            }
        }
        if (REACT) {
            // reduce-scatter over the wave: lanes 16q..16q+15 end with
            // component q (x, y, z, potential) summed over all 64 lanes
            const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0;
            double k0 = b5 ? jz : jx, k1 = b5 ? jp : jy;
            k0 += __shfl_xor(b5 ? jx : jz, 32);
            k1 += __shfl_xor(b5 ? jy : jp, 32);
            double kp = b4 ? k1 : k0;
            kp += __shfl_xor(b4 ? k0 : k1, 16);
            kp += __shfl_xor(kp, 8);
            kp += __shfl_xor(kp, 4);
            kp += __shfl_xor(kp, 2);
            kp += __shfl_xor(kp, 1);
            if ((lane & 15) == 0) jpart[wave][si][lane >> 4] = kp;
        }
    }
}

template <int NIMG, bool POT, int TORDER, bool COMPLETE>
__global__ __launch_bounds__(kThreads, 2) void forces_pairwise_kernel(PairwiseArgs a) {
    constexpr int kR = particles_per_thread(TORDER);
    constexpr int kGroup = kThreads * kR;  // particles per group
    __shared__ SrcRec tile[kTile];
    __shared__ float wave_hmax[kThreads / 64];
    __shared__ double jpart[kThreads / 64][kTile][4];
    const int tid = threadIdx.x;
    const int g = blockIdx.x / a.P, q = blockIdx.x % a.P;

    Owned<kR> o;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int64_t t64 = (int64_t)g * kGroup + r * kThreads + tid;
        const int t = t64 < a.N ? (int)t64 : a.N;  // a.N marks an empty slot
        o.t[r] = t;
        if (t < a.N) {
            const SrcRec rr = a.rec[t];
            o.x[r] = rr.x;
            o.y[r] = rr.y;
            o.z[r] = rr.z;
            o.h[r] = rr.h;
            o.m[r] = rr.m;
        } else {
            // an empty slot far from every particle, with no mass: its
            // reactions vanish and its own sums are never written
            o.x[r] = 1e18;
            o.y[r] = 0.0;
            o.z[r] = 0.0;
            o.h[r] = 0.f;
            o.m[r] = 0.f;
        }
    }
    double acc[kR][4];
#pragma unroll
    for (int r = 0; r < kR; ++r)
        for (int k = 0; k < 4; ++k) acc[r][k] = 0.0;

    const int half = a.G / 2;
    const int K = (a.G & 1) ? half : half - 1 + (g < half ? 1 : 0);
    const int U = K + 1;  // the group itself and its K partners
    const int u0 = (int)((int64_t)q * U / a.P), u1 = (int)((int64_t)(q + 1) * U / a.P);
    for (int u = u0; u < u1; ++u) {
        const int h = (g + u) % a.G;
        // index arithmetic that stays below N (no int overflow near 2^31)
        const int gbase = h * kGroup, gend = gbase + min(kGroup, a.N - gbase);
        for (int base = gbase, cnt = 0; base < gend; base += cnt) {
            cnt = min(kTile, gend - base);
            float hj = 0.f;
            if (tid < cnt) {
                const SrcRec rr = a.rec[base + tid];
                hj = rr.h;
                tile[tid] = rr;
            }
            for (int off = 32; off >= 1; off >>= 1) hj = fmaxf(hj, __shfl_xor(hj, off));
            if ((tid & 63) == 0) wave_hmax[tid >> 6] = hj;
            __syncthreads();
            float hmax = wave_hmax[0];
            for (int w = 1; w < kThreads / 64; ++w) hmax = fmaxf(hmax, wave_hmax[w]);
            if (u == 0) {
                tile_pass<NIMG, POT, TORDER, COMPLETE, false>(a, o, tile, base, cnt, hmax, acc, jpart);
                __syncthreads();
            } else {
                tile_pass<NIMG, POT, TORDER, COMPLETE, true>(a, o, tile, base, cnt, hmax, acc, jpart);
                __syncthreads();
                if (tid < cnt) {
                    // reaction on source base + tid, in the owned sums' sign convention
                    const int64_t jj = base + tid;
                    double v[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        v[k] = (jpart[0][tid][k] + jpart[1][tid][k]) + (jpart[2][tid][k] + jpart[3][tid][k]);
                    unsafeAtomicAdd(a.acc + jj, -v[0]);
                    unsafeAtomicAdd(a.acc + a.N + jj, -v[1]);
                    unsafeAtomicAdd(a.acc + 2 * (int64_t)a.N + jj, -v[2]);
                    if (POT) unsafeAtomicAdd(a.acc + 3 * (int64_t)a.N + jj, v[3]);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        if (o.t[r] < a.N) {
            unsafeAtomicAdd(a.acc + o.t[r], acc[r][0]);
            unsafeAtomicAdd(a.acc + a.N + o.t[r], acc[r][1]);
            unsafeAtomicAdd(a.acc + 2 * (int64_t)a.N + o.t[r], acc[r][2]);
            if (POT) unsafeAtomicAdd(a.acc + 3 * (int64_t)a.N + o.t[r], acc[r][3]);
        }
    }
}

template <int NIMG, bool POT, int TORDER, bool COMPLETE>
hipError_t launch_t(const PairwiseArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL((forces_pairwise_kernel<NIMG, POT, TORDER, COMPLETE>), dim3(a.G * a.P), dim3(kThreads), 0,
                       stream, a);
    return hipGetLastError();
}

template <bool POT>
hipError_t launch_nimg(const PairwiseArgs &a, hipStream_t stream) {
    switch (a.c.n_img) {
        case 0: return launch_t<0, POT, 0, false>(a, stream);
        case 1: return launch_t<1, POT, 0, false>(a, stream);
        case 2: return launch_t<2, POT, 0, false>(a, stream);
        case 4: return launch_t<4, POT, 0, false>(a, stream);
        case 8: return launch_t<8, POT, 0, false>(a, stream);
        default: return launch_t<-1, POT, 0, false>(a, stream);
    }
}

template <bool POT>
hipError_t launch_table(const PairwiseArgs &a, int order, bool complete, hipStream_t stream) {
    if (order == 1)
        return complete ? launch_t<1, POT, 1, true>(a, stream) : launch_t<1, POT, 1, false>(a, stream);
    return complete ? launch_t<1, POT, 2, true>(a, stream) : launch_t<1, POT, 2, false>(a, stream);
}

}  // namespace

// Launches the pairwise path for all N particles: exact images |n| <= n_img,
// or (table non-null) images |n| <= 1 plus the table's far images with CIC
// (order 1) or TSC (order 2) interpolation.  Arguments already validated.  Scratch (spatial order, records, FP64 sums) is
// stream-ordered.
int launch_forces_pairwise(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                           int n_img, const steps_cyl_table *table, int order, float *out_acc, float *out_pot,
                           hipStream_t stream) {
    void *order_scratch = nullptr;
    const int *perm = nullptr;
    int rc = order_targets(pos, N, L, nullptr, N, stream, &order_scratch, &perm);
    if (rc) return rc;
    void *buf = nullptr;
    const size_t bytes = (size_t)N * (sizeof(SrcRec) + 4 * sizeof(double));
    hipError_t e = hipMallocAsync(&buf, bytes, stream);
    if (e != hipSuccess) {
        (void)hipFreeAsync(order_scratch, stream);
        return fail(STEPS_ENOMEM, "pairwise scratch (%zu bytes)", bytes);
    }
    PairwiseArgs a;
    a.rec = (const SrcRec *)buf;
    a.acc = (double *)((char *)buf + (size_t)N * sizeof(SrcRec));
    a.L = L;
    a.invL = 1.0 / L;
    a.halfL = 0.5 * L;
    a.tie = 1e-12 * L;
    a.tie32 = (float)(0.5 * L * (1.0 - 1e-6));
    a.c.Lf = (float)L;
    a.c.L2f = (float)(L * L);
    a.c.m2Lf = (float)(-2.0 * L);
    a.c.n_img = table ? 1 : n_img;
    a.invLf = (float)(1.0 / L);
    a.invL2f = (float)(1.0 / (L * L));
    if (table) a.tv = table_view(table);
    a.N = (int)N;
    const int group = kThreads * particles_per_thread(table ? 1 : 0);
    a.G = (int)((N + group - 1) / group);
    // enough workgroups to fill the chip: about 2048, never more than the
    // units of a group's list
    const int units = a.G / 2 + 1;
    a.P = std::max(1, std::min(units, (2048 + a.G - 1) / a.G));
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL(stage_kernel, dim3(nb), dim3(256), 0, stream, pos, mass, eps, (int)N, L, perm,
                       (SrcRec *)buf, a.acc);
    e = hipGetLastError();
    if (e == hipSuccess) {
        if (table)
            e = out_pot ? launch_table<true>(a, order, table->complete != 0, stream)
                        : launch_table<false>(a, order, table->complete != 0, stream);
        else
            e = out_pot ? launch_nimg<true>(a, stream) : launch_nimg<false>(a, stream);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(finish_kernel, dim3(nb), dim3(256), 0, stream, a.acc, perm, (int)N, out_acc,
                           out_acc + N, out_acc + 2 * N, out_pot);
        e = hipGetLastError();
    }
    (void)hipFreeAsync(buf, stream);
    (void)hipFreeAsync(order_scratch, stream);
    return hip_status(e, "forces_pairwise launch");
}

}  // namespace steps
