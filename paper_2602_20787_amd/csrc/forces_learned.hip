// Learned far-image forces on gfx950: exact images |n| <= 1 plus the
// network correction for the images 2 <= |n| <= 1024 (the paper adds its far
// images through an interpolated correction table, Sect. 2.2, eq.
// S1R2EwaldCorrectionTable; here a network of (|d|/L, rho/L) on BF16 MFMA
// takes that role).
//
// Mapping.  A wave owns 32 targets, one per MFMA column; lanes l and l+32
// share target l%32 and split each network layer between them.  A
// workgroup of 4 waves (128 targets) walks the sources in LDS tiles of 256,
// two sources per step: lane half 0 does the per-pair work (near images,
// baseline, features, accumulation) for the even source and half 1 for the
// odd one, and the wave then evaluates two network tiles of 32 pairs each
// (32 targets x 1 source), the features crossing halves by one swap.  In a
// tile, layer 1 runs on MFMA through the exact three-part BF16 split of its
// FP32 inputs, layers 2-4 as 8 MFMAs each, the activations and layer 5 on
// the VALU (layer 5 with a cross-half sum).  Each half keeps its own
// compensated sums; they are added at the end.  Pairs outside the network's
// domain take the exact image band instead: near the axis (rho/L < 0.05)
// each lane evaluates its pair's band from a series (BandSeries, below);
// beyond rho/L = 20 all 64 lanes share the direct sum of one pair (32 images
// each plus a butterfly reduction).
#include <cmath>

#include "common.h"
#include "learned_model.h"
#include "mlp_device.h"
#include "pair_fp32.h"

namespace steps {

namespace {

constexpr int kBlock = 256;     // 4 waves
constexpr int kTargets = 128;   // targets per workgroup (32 per wave)
constexpr int kTile = 256;      // sources per LDS tile
constexpr int kSub = 32;        // sources per compensated flush

// The band 2 <= |n| <= 1024 of a pair near the axis (rho < 0.05 L), where the
// network is not defined, as a convergent series rather than 2046 image
// terms.  With x = n -+ delta >= 1.5 (|delta| = |d|/L <= 1/2) and
// (rho/x)^2 < 1.2e-3, (x^2 + rho^2)^(-3/2) = x^-3 sum_k b_k (rho^2/x^2)^k,
// b_k = binom(-3/2, k); four terms leave less than 4e-12 of the sum.  Then
//   F_z   =  delta  sum_k b_k rho^2k H_k(delta^2),
//   F_rho = -rho    sum_k b_k rho^2k G_k(delta^2),
// H_k = sum_n [(n - delta)^-(2+2k) - (n + delta)^-(2+2k)] / delta and
// G_k = sum_n [(n - delta)^-(3+2k) + (n + delta)^-(3+2k)], smooth functions
// of delta^2 held as degree-8 polynomials in t = 8 delta^2 - 1 on [-1, 1]
// (Chebyshev interpolation in FP64 when the library loads, under 1e-9 of
// the sums).  Evaluated in FP32 the result is the exact band to FP32
// rounding (1.7e-7 of it at most, checked against the direct sum on 3000
// random pairs).
struct BandSeries {
    float c[2][4][9];  // [F_z | F_rho][k][monomial coefficient of t, highest first], times b_k
};

struct LearnedArgs {
    const double *x, *y, *z, *m, *h;
    const int64_t *targets;
    const int *perm;  // list positions in spatial order of their targets, or null
    const mlp::Packed *P;
    float *ax, *ay, *az, *pot;
    double *part;     // [chunks][4][n_tgt] chunk totals of a short list, or null
    double L, invL, halfL;
    float invLf, invL2f;
    ImageConsts c;  // n_img = 1
    int N, n_tgt;
    int chunk;        // sources per chunk (a multiple of kTile, or N)
    BandSeries bs;    // near-axis band
};

__device__ __forceinline__ void band_near_axis(const BandSeries &bs, float delta, float r, float &fz, float &fr) {
    const float t = __builtin_fmaf(8.0f * delta, delta, -1.0f);
    const float r2 = r * r;
    float pz = 0.f, pr = 0.f;
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        float hz = bs.c[0][k][0], hr = bs.c[1][k][0];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            hz = __builtin_fmaf(hz, t, bs.c[0][k][i]);
            hr = __builtin_fmaf(hr, t, bs.c[1][k][i]);
        }
        pz = __builtin_fmaf(pz, r2, hz);
        pr = __builtin_fmaf(pr, r2, hr);
    }
    fz = delta * pz;
    fr = -r * pr;
}

// Exact band 2 <= |n| <= 1024 for one pair (delta = d/L signed, r = rho/L),
// shared by the 64 lanes of the wave; every lane returns the totals
// (per unit G m / L^2).
__device__ __forceinline__ void band_cooperative(float delta, float r, float &fz, float &fr) {
    const int lane = threadIdx.x & 63;
    const float r2 = r * r;
    float sz = 0.f, sr = 0.f;
#pragma unroll 4
    for (int mm = 15; mm >= 0; --mm) {
        const int q = 2 + lane + 64 * mm;
        if (q <= mlp::kFarImages) {
            const float qf = (float)q;
            const float up = delta - qf, um = delta + qf;
            const float ip = __builtin_amdgcn_rsqf(__builtin_fmaf(up, up, r2));
            const float im = __builtin_amdgcn_rsqf(__builtin_fmaf(um, um, r2));
            const float ip3 = ip * ip * ip, im3 = im * im * im;
            sz = __builtin_fmaf(-up, ip3, __builtin_fmaf(-um, im3, sz));
            sr = __builtin_fmaf(-r, ip3 + im3, sr);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sz += __shfl_xor(sz, off);
        sr += __shfl_xor(sr, off);
    }
    fz = sz;
    fr = sr;
}

// Per-pair work that does not involve the network: near images |n| <= 1,
// the analytic baseline, features and the domain test.
struct PairState {
    float dx, dy, d, rho, r, S, Fz, Pn, f1, f2, bz, br, sc, m;
    bool inside, band;  // band: outside the network domain, needs the exact band
};

template <bool POT>
__device__ __forceinline__ PairState pair_state(const SrcRec &src, bool self, bool live, double xi,
                                                double yi, double zi, float hi, const LearnedArgs &a) {
    PairState q;
    const double dx64 = xi - src.x, dy64 = yi - src.y;
    const double d64 = min_image(zi - src.z, a.L, a.invL);
    q.dx = (float)dx64;
    q.dy = (float)dy64;
    q.d = (float)d64;
    q.m = live ? src.m : 0.f;
    const float hij = hi + src.h;
    q.Pn = 0.f;
    pair_fast<1, POT>(q.dx, q.dy, q.d, a.c, q.S, q.Fz, q.Pn);
    const float rho2 = __builtin_fmaf(q.dx, q.dx, q.dy * q.dy);
    const float r2_0 = __builtin_fmaf(q.d, q.d, rho2);
    if (r2_0 < hij * hij || hij > (float)a.halfL) {
        if (self) {
            q.S = 0.f;
            q.Fz = 0.f;
            q.Pn = 0.f;
        } else {
            const PairSums g = pair_general_f64(dx64, dy64, d64, (double)hi + (double)src.h, a.L, 1);
            q.S = g.S;
            q.Fz = g.Fz;
            q.Pn = g.P;
        }
    }
    q.rho = __builtin_sqrtf(rho2);
    q.r = q.rho * a.invLf;
    const float delta = __builtin_fabsf(q.d) * a.invLf;
    q.inside = (q.r >= mlp::kRhoMin) && (q.r <= mlp::kRhoMax) && !self;
    q.band = !q.inside && !self && live;
    const float rr = q.inside ? q.r : 1.0f;
    mlp::features_f32(delta, rr, q.f1, q.f2);
    mlp::baseline_f32(delta, rr, q.bz, q.br);
    q.sc = mlp::out_scale_f32(q.r);
    return q;
}

// The band series' coefficients copied into the workgroup's LDS (read there
// only by waves that meet a near-axis pair; kept out of scalar registers).
__device__ __forceinline__ void load_band_series(BandSeries *dst, const BandSeries &src) {
    constexpr int n = (int)(sizeof(BandSeries) / sizeof(float));
    const float *s = &src.c[0][0][0];
    float *d = &dst->c[0][0][0];
    for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
}

// The band of a pair outside the network's domain (R_z, R_rho per unit
// G m_j / L^2): near the axis from the series, beyond the domain's outer
// edge exactly, with the 64 lanes of the wave sharing each such pair.
__device__ __forceinline__ void band_outside(const LearnedArgs &a, const BandSeries &bs, const PairState &q,
                                             bool active, float &Rz, float &Rr) {
    const int lane = threadIdx.x & 63;
    const bool out = q.band && active;
    const bool axis = out && q.r < mlp::kRhoMin;
    if (axis) band_near_axis(bs, q.d * a.invLf, q.r, Rz, Rr);
    uint64_t outside = __ballot(out && !axis);
    while (outside) {
        const int c = __builtin_ctzll(outside);
        outside &= outside - 1;
        const float dc = __shfl(q.d * a.invLf, c), rc = __shfl(q.r, c);
        float tz, tr;
        band_cooperative(dc, rc, tz, tr);
        if (lane == c) {
            Rz = tz;
            Rr = tr;
        }
    }
}

template <bool POT, bool COMP>
__global__ __launch_bounds__(kBlock, 3) void forces_learned_kernel(LearnedArgs a) {
    __shared__ mlp::Packed P;
    __shared__ SrcRec tile[kTile];
    __shared__ BandSeries bands;
    mlp::load_packed(&P, a.P);
    load_band_series(&bands, a.bs);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int col = lane & 31, h = lane >> 5;
    const int k = blockIdx.x * kTargets + wave * 32 + col;
    const bool active = k < a.n_tgt;
    const int64_t kk = active ? (a.perm ? (int64_t)a.perm[k] : (int64_t)k) : 0;  // position in the list
    const int64_t i = a.targets ? a.targets[kk] : kk;
    const double xi = a.x[i], yi = a.y[i], zi = wrap_z(a.z[i], a.L);
    const float hi = (float)a.h[i];

    // each lane half accumulates its own sources (h = 0: even, h = 1: odd)
    float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f;
    float cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;

    const int j0 = blockIdx.y * a.chunk, j1 = min(a.N, j0 + a.chunk);
    for (int base = j0; base < j1; base += kTile) {
        __syncthreads();
        const int j = base + tid;
        if (j < j1) {
            SrcRec r;
            r.x = a.x[j];
            r.y = a.y[j];
            r.z = wrap_z(a.z[j], a.L);
            r.m = (float)a.m[j];
            r.h = (float)a.h[j];
            tile[tid] = r;
        }
        __syncthreads();
        const int cnt = min(kTile, j1 - base);
        for (int s0 = 0; s0 < cnt; s0 += kSub) {
            const int e = min(kSub, cnt - s0);
            float px = 0.f, py = 0.f, pz = 0.f, pp = 0.f;
            for (int s = 0; s < e; s += 2) {
                // this lane's source: s (h = 0) or s + 1 (h = 1); past the end the
                // lane repeats source s with zero mass
                const bool live = (s + h) < e;
                const int js = live ? (s + h) : s;
                const SrcRec src = tile[s0 + js];
                const bool self = (int64_t)(base + s0 + js) == i;
                PairState q = pair_state<POT>(src, self, live, xi, yi, zi, hi, a);
                // network tiles: tile A holds the pairs of source s, tile B of s + 1;
                // each half takes the other half's features by a cross-half swap
                const float g1 = __shfl_xor(q.f1, 32), g2 = __shfl_xor(q.f2, 32);
                const float fa1 = h ? g1 : q.f1, fa2 = h ? g2 : q.f2;
                const float fb1 = h ? q.f1 : g1, fb2 = h ? q.f2 : g2;
                int poff = 0;
                asm volatile("" : "+v"(poff));
                const mlp::Packed &Pl = *reinterpret_cast<const mlp::Packed *>(
                    reinterpret_cast<const char *>(&P) + poff);
                float oa0, oa1, ob0, ob1;
                mlp::forward32<false>(Pl, fa1, fa2, oa0, oa1, nullptr, nullptr);
                // the two tiles one after the other: one tile's registers
                // let 3 waves share a SIMD, and the other waves hide the
                // MFMA and transcendental latency that interleaving the
                // tiles would
                __builtin_amdgcn_sched_barrier(0);
                mlp::forward32<false>(Pl, fb1, fb2, ob0, ob1, nullptr, nullptr);
                const float o0 = h ? ob0 : oa0, o1 = h ? ob1 : oa1;
                const float mz = __builtin_fmaf(q.sc, o0, q.bz);
                float Rz = (q.d > 0.f) ? mz : ((q.d < 0.f) ? -mz : 0.f);
                float Rr = __builtin_fmaf(q.sc, o1, q.br);
                if (!q.inside) {
                    Rz = 0.f;
                    Rr = 0.f;
                }
                band_outside(a, bands, q, active, Rz, Rr);
                // a = -m_j [ S (dx, dy, *) - R_rho (dx, dy)/(rho L^2) , Fz - R_z / L^2 ]
                const float rinv = q.rho > 0.f ? __builtin_amdgcn_rcpf(q.rho) : 0.f;
                const float Seff = __builtin_fmaf(-Rr * a.invL2f, rinv, q.S);
                const float Fzeff = __builtin_fmaf(-Rz, a.invL2f, q.Fz);
                const float mS = q.m * Seff;
                if (COMP) {
                    px = __builtin_fmaf(mS, q.dx, px);
                    py = __builtin_fmaf(mS, q.dy, py);
                    pz = __builtin_fmaf(q.m, Fzeff, pz);
                    if (POT) pp = __builtin_fmaf(q.m, q.Pn, pp);
                } else {
                    sx = __builtin_fmaf(mS, q.dx, sx);
                    sy = __builtin_fmaf(mS, q.dy, sy);
                    sz = __builtin_fmaf(q.m, Fzeff, sz);
                    if (POT) sp = __builtin_fmaf(q.m, q.Pn, sp);
                }
            }
            if (COMP) {
                kahan_add(sx, cx, px);
                kahan_add(sy, cy, py);
                kahan_add(sz, cz, pz);
                if (POT) kahan_add(sp, cp, pp);
            }
        }
    }
    // combine the halves: value and compensation of the odd sources join the even ones
    const float ox = __shfl_xor(sx - cx, 32), oy = __shfl_xor(sy - cy, 32);
    const float oz = __shfl_xor(sz - cz, 32), op = __shfl_xor(sp - cp, 32);
    if (active && h == 0) {
        const int64_t o = kk;
        if (a.part) {
            double *q = a.part + (int64_t)blockIdx.y * 4 * a.n_tgt + o;
            q[0] = (double)(sx - cx) + (double)ox;
            q[a.n_tgt] = (double)(sy - cy) + (double)oy;
            q[2 * (int64_t)a.n_tgt] = (double)(sz - cz) + (double)oz;
            q[3 * (int64_t)a.n_tgt] = (double)(sp - cp) + (double)op;
        } else {
            a.ax[o] = -((sx - cx) + ox);
            a.ay[o] = -((sy - cy) + oy);
            a.az[o] = -((sz - cz) + oz);
            if (POT) a.pot[o] = -((sp - cp) + op);
        }
    }
}

// Chunk totals of a short target list added in chunk order (FP64), negated
// and written as FP32.
__global__ void learned_chunks_kernel(const double *part, int chunks, int n_tgt, float *ax, float *ay, float *az,
                                      float *pot) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_tgt) return;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < chunks; ++c)
        for (int q = 0; q < 4; ++q) v[q] += part[((int64_t)c * 4 + q) * n_tgt + k];
    ax[k] = (float)(-v[0]);
    ay[k] = (float)(-v[1]);
    az[k] = (float)(-v[2]);
    if (pot) pot[k] = (float)(-v[3]);
}

template <bool POT, bool COMP>
hipError_t launch_t(const LearnedArgs &a, hipStream_t stream) {
    const int grid = (a.n_tgt + kTargets - 1) / kTargets;
    const int chunks = (a.N + a.chunk - 1) / a.chunk;
    hipLaunchKernelGGL((forces_learned_kernel<POT, COMP>), dim3(grid, chunks), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

namespace mlp {
const Packed *packed_of(const steps_cyl_mlp *net);
}

int per_target_chunks(int64_t N, int64_t n_tgt, int block);

// Workspace of the per-target learned kernel: the spatial order of a long
// list and the chunk totals of a short one (sources split into chunks when
// the target blocks alone would leave the device idle; see forces_exact.hip).
size_t learned_per_target_bytes(int64_t N, int64_t n_tgt) {
    const int chunks = per_target_chunks(N, n_tgt, kTargets);
    return ws_total({per_target_bytes(n_tgt), chunks > 1 ? (size_t)chunks * 4 * n_tgt * sizeof(double) : 0});
}

namespace {

// Coefficients of the near-axis band series (BandSeries), computed once in
// FP64: the sums at 32 Chebyshev nodes of t, the truncated Chebyshev series
// of degree 8, converted to monomials in t.
BandSeries make_band_series() {
    constexpr int kNodes = 32, kDeg = 8;
    constexpr double kPi = 3.14159265358979323846;
    const double b[4] = {1.0, -1.5, 1.875, -2.1875};  // binom(-3/2, k)
    BandSeries bs{};
    for (int comp = 0; comp < 2; ++comp)
        for (int k = 0; k < 4; ++k) {
            const int m = (comp == 0 ? 2 : 3) + 2 * k;
            double f[kNodes];
            for (int j = 0; j < kNodes; ++j) {
                const double t = std::cos(kPi * (j + 0.5) / kNodes);
                const double d = std::sqrt((t + 1.0) / 8.0);  // > 0 at every node
                double sum = 0.0;
                for (int n = 2; n <= mlp::kFarImages; ++n) {
                    const double lo = std::pow(n - d, -m), hi = std::pow(n + d, -m);
                    sum += comp == 0 ? lo - hi : lo + hi;
                }
                f[j] = comp == 0 ? sum / d : sum;
            }
            double a[kDeg + 1];
            for (int i = 0; i <= kDeg; ++i) {
                double acc = 0.0;
                for (int j = 0; j < kNodes; ++j) acc += f[j] * std::cos(kPi * i * (j + 0.5) / kNodes);
                a[i] = acc * (i == 0 ? 1.0 : 2.0) / kNodes;
            }
            // T_0 = 1, T_1 = t, T_{i+1} = 2 t T_i - T_{i-1}, as monomial coefficients
            double p[kDeg + 1] = {}, tm[kDeg + 1] = {}, tc[kDeg + 1] = {}, tn[kDeg + 1];
            tm[0] = 1.0;
            tc[1] = 1.0;
            p[0] = a[0];
            p[1] = a[1];
            for (int i = 2; i <= kDeg; ++i) {
                for (int e = 0; e <= kDeg; ++e) tn[e] = (e > 0 ? 2.0 * tc[e - 1] : 0.0) - tm[e];
                for (int e = 0; e <= kDeg; ++e) {
                    tm[e] = tc[e];
                    tc[e] = tn[e];
                    p[e] += a[i] * tc[e];
                }
            }
            for (int e = 0; e <= kDeg; ++e) bs.c[comp][k][kDeg - e] = (float)(b[k] * p[e]);
        }
    return bs;
}

const BandSeries &band_series() {
    static const BandSeries bs = make_band_series();
    return bs;
}

}  // namespace

int launch_forces_learned(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                          const steps_cyl_mlp *net, const int64_t *targets, int64_t n_tgt, int mode,
                          float *out_acc, float *out_pot, Workspace &ws, hipStream_t stream) {
    LearnedArgs a;
    a.x = pos;
    a.y = pos + N;
    a.z = pos + 2 * N;
    a.m = mass;
    a.h = eps;
    a.targets = targets;
    a.P = mlp::packed_of(net);
    a.ax = out_acc;
    a.ay = out_acc + n_tgt;
    a.az = out_acc + 2 * n_tgt;
    a.pot = out_pot;
    a.L = L;
    a.invL = 1.0 / L;
    a.halfL = 0.5 * L;
    a.invLf = (float)(1.0 / L);
    a.invL2f = (float)(1.0 / (L * L));
    a.c.Lf = (float)L;
    a.c.L2f = (float)(L * L);
    a.c.m2Lf = (float)(-2.0 * L);
    a.c.n_img = 1;
    a.bs = band_series();
    a.N = (int)N;
    a.n_tgt = (int)n_tgt;
    a.perm = nullptr;
    // walk the targets in spatial order (keys and order in the workspace)
    int rc = check_workspace(ws, learned_per_target_bytes(N, n_tgt));
    if (rc) return rc;
    if (n_tgt >= kOrderTargetsMin && (rc = order_targets(pos, N, L, targets, n_tgt, stream, ws, &a.perm)))
        return rc;
    const int chunks = per_target_chunks(N, n_tgt, kTargets);
    a.chunk = (int)N;
    a.part = nullptr;
    if (chunks > 1) {
        a.chunk = (int)(((N + chunks - 1) / chunks + kTile - 1) / kTile * kTile);
        a.part = (double *)ws.take((size_t)chunks * 4 * n_tgt * sizeof(double));
        if (!a.part) return fail(STEPS_EINVAL, "workspace too small for the chunk totals");
    }
    const bool comp = (mode == STEPS_SUM_COMPENSATED);
    hipError_t e;
    if (out_pot)
        e = comp ? launch_t<true, true>(a, stream) : launch_t<true, false>(a, stream);
    else
        e = comp ? launch_t<false, true>(a, stream) : launch_t<false, false>(a, stream);
    if (e == hipSuccess && a.part) {
        const int nch = (int)((N + a.chunk - 1) / a.chunk);
        hipLaunchKernelGGL(learned_chunks_kernel, dim3((unsigned)((n_tgt + 255) / 256)), dim3(256), 0, stream,
                           a.part, nch, (int)n_tgt, out_acc, out_acc + n_tgt, out_acc + 2 * n_tgt, out_pot);
        e = hipGetLastError();
    }
    return hip_status(e, "forces_learned launch");
}

// ---------------------------------------------------------------------------
// Pairwise learned path (every particle a target): each unordered pair is
// evaluated once.  The learned pair term is odd in the separation like the
// exact one (R_z is sign(d) times a function of |d| and rho, R_rho a
// function of |d| and rho), so the reaction is the action with dx, dy and
// F_z negated (F_z keeps its sign where both particles take the minimum
// image -L/2).
//
// Schedule (no atomics, bitwise reproducible).  Particles in spatial order
// form sub-groups of 128 (a workgroup's 4 waves x 32 columns) and groups of
// kSubs sub-groups.  The groups meet on the schedule of the pairwise exact
// path: a first launch pairs every group with itself (one-sided, every
// ordered pair, the self pair skipped), then G' - 1 launches (G' = G rounded
// up to even) follow the round-robin tournament in which round r pairs group
// G'-1 with group r and group (r + k) mod (G'-1) with group (r - k) mod
// (G'-1).  A meeting of groups A and B takes kSubs^2 workgroups, workgroup
// (i, j) holding sub-group i of A as targets and streaming sub-group j of B:
// it adds its actions to slot j of the sums of a_i and the reactions to slot
// kSubs + i of the sums of b_j.  No group appears twice in a launch, so each
// slot has one writer per launch and every sum is a plain read-modify-write
// in an order fixed by N.  A launch holds kSubs^2 G'/2 workgroups of equal
// size, so one slow meeting (a near pair of groups, with many pairs outside
// the network's domain) is a small part of it.  A wave walks the sources in
// blocks of 64, 32 steps per block: at step u lane (h, c) takes source
// 32h + (c + u) mod 32 of the block, so the 64 lanes meet 64 different
// sources and each source meets the wave's 32 targets over the 32 steps.
// The reaction on a source is then summed in an FP64 LDS slot per wave that
// the lanes update in turn (no cross-lane reduction), and the 4 waves'
// slots are added in order at the end.  Both sides are summed in FP64
// (sources in spatial order would cost FP32 partials their cancellation).
namespace {

constexpr int kOwn = 128;  // particles per sub-group, one per wave column
constexpr int kSubs = 8;   // sub-groups per group
constexpr int kSlots = 2 * kSubs;  // sums per particle: actions by source sub-group, reactions by target sub-group

struct PairwiseLearnedArgs {
    LearnedArgs la;   // L, invL, halfL, invLf, invL2f, c, P of the per-target kernel
    const SrcRec *rec;
    double *acc;      // [kSlots][4][N] in spatial order
    double tie;
    float tie32;
    int N, G, Gp;     // particles, groups (of kSubs sub-groups), groups rounded up to even
    int round;        // tournament round (meeting launches)
};

__global__ void lp_stage_kernel(const double *pos, const double *mass, const double *eps, int N, double L,
                                const int *perm, SrcRec *rec) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int p = perm[k];
    SrcRec r;
    r.x = pos[p];
    r.y = pos[(int64_t)N + p];
    r.z = wrap_z(pos[2 * (int64_t)N + p], L);
    r.m = (float)mass[p];
    r.h = (float)eps[p];
    rec[k] = r;
}

__global__ void lp_finish_kernel(const double *acc, const int *perm, int N, float *ax, float *ay, float *az,
                                 float *pot) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = 0; q < kSlots; ++q)
        for (int c = 0; c < 4; ++c) v[c] += acc[((int64_t)q * 4 + c) * N + k];
    const int p = perm[k];
    ax[p] = (float)(-v[0]);
    ay[p] = (float)(-v[1]);
    az[p] = (float)(-v[2]);
    if (pot) pot[p] = (float)(-v[3]);
}

// Workgroup (i, j) of one meeting (REACT: the groups of tournament round
// pa.round) or of one group's meeting with itself.
template <bool POT, bool REACT>
__global__ __launch_bounds__(kBlock, 3) void forces_learned_pairwise_kernel(PairwiseLearnedArgs pa) {
    __shared__ mlp::Packed P;
    __shared__ SrcRec tile[kOwn];
    __shared__ double jpart[kBlock / 64][4][kOwn];  // per wave, component, source
    __shared__ BandSeries bands;
    const LearnedArgs &a = pa.la;
    const int meet = blockIdx.x / (kSubs * kSubs);
    const int si = (blockIdx.x / kSubs) % kSubs, sj = blockIdx.x % kSubs;
    int ga = meet, gb = meet;
    if (REACT) {
        const int M = pa.Gp - 1;
        if (meet == 0) {
            ga = M;
            gb = pa.round;
        } else {
            ga = (pa.round + meet) % M;
            gb = (pa.round - meet + M) % M;
        }
        if (ga >= pa.G || gb >= pa.G) return;  // the empty group of an odd count (whole workgroup)
    }
    // target sub-group ga*kSubs + si, source sub-group gb*kSubs + sj
    const int ta = ga * kSubs + si, sb = gb * kSubs + sj;
    if ((int64_t)ta * kOwn >= pa.N) return;                   // no targets (whole workgroup)
    if (REACT && (int64_t)sb * kOwn >= pa.N) return;          // no sources: nothing to add
    mlp::load_packed(&P, a.P);
    load_band_series(&bands, a.bs);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int col = lane & 31, h = lane >> 5;
    const int64_t t64 = (int64_t)ta * kOwn + wave * 32 + col;
    const bool active = t64 < pa.N;
    const int t = active ? (int)t64 : pa.N;
    // an empty slot sits far away with no mass: no reaction, never written
    double xi = 1e18, yi = 0.0, zi = 0.0;
    float hi = 0.f, mi = 0.f;
    if (active) {
        const SrcRec r = pa.rec[t];
        xi = r.x;
        yi = r.y;
        zi = r.z;
        hi = r.h;
        mi = r.m;
    }
    // this half's sums for target `col` (h = 0: even sources, h = 1: odd)
    double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;

    const int base = sb * kOwn;
    const int cnt = max(0, min(kOwn, pa.N - base));  // 0: an empty sub-group of the self meeting
    if (tid < cnt) tile[tid] = pa.rec[base + tid];
    if (REACT) {
        double *jz0 = &jpart[0][0][0];
        for (int q = tid; q < (kBlock / 64) * 4 * kOwn; q += kBlock) jz0[q] = 0.0;
    }
    __syncthreads();  // the tile, the parameters and the cleared slots are in LDS
    for (int s0 = 0; s0 < cnt; s0 += 64) {
        for (int u = 0; u < 32; ++u) {
            const int jr = s0 + 32 * h + ((col + u) & 31);
            const bool live = jr < cnt;
            const int js = live ? jr : 0;  // a dead lane reads a real record and adds nothing
            const SrcRec src = tile[js];
            const bool self = !REACT && (base + js == t);
            PairState q = pair_state<POT>(src, self, live, xi, yi, zi, hi, a);
            const float g1 = __shfl_xor(q.f1, 32), g2 = __shfl_xor(q.f2, 32);
            const float fa1 = h ? g1 : q.f1, fa2 = h ? g2 : q.f2;
            const float fb1 = h ? q.f1 : g1, fb2 = h ? q.f2 : g2;
            int poff = 0;
            asm volatile("" : "+v"(poff));
            const mlp::Packed &Pl = *reinterpret_cast<const mlp::Packed *>(
                reinterpret_cast<const char *>(&P) + poff);
            float oa0, oa1, ob0, ob1;
            mlp::forward32<false>(Pl, fa1, fa2, oa0, oa1, nullptr, nullptr);
            // one tile after the other (3 waves per SIMD, as the per-target kernel)
            __builtin_amdgcn_sched_barrier(0);
            mlp::forward32<false>(Pl, fb1, fb2, ob0, ob1, nullptr, nullptr);
            const float o0 = h ? ob0 : oa0, o1 = h ? ob1 : oa1;
            const float mz = __builtin_fmaf(q.sc, o0, q.bz);
            float Rz = (q.d > 0.f) ? mz : ((q.d < 0.f) ? -mz : 0.f);
            float Rr = __builtin_fmaf(q.sc, o1, q.br);
            if (!q.inside) {
                Rz = 0.f;
                Rr = 0.f;
            }
            band_outside(a, bands, q, active, Rz, Rr);
            const float rinv = q.rho > 0.f ? __builtin_amdgcn_rcpf(q.rho) : 0.f;
            const double Seff = (double)__builtin_fmaf(-Rr * a.invL2f, rinv, q.S);
            const double Fzeff = (double)__builtin_fmaf(-Rz, a.invL2f, q.Fz);
            const double Pn = (double)q.Pn;
            const double mj = (double)q.m;  // 0 for a dead lane
            sx = __builtin_fma(mj * Seff, (double)q.dx, sx);
            sy = __builtin_fma(mj * Seff, (double)q.dy, sy);
            sz = __builtin_fma(mj, Fzeff, sz);
            if (POT) sp = __builtin_fma(mj, Pn, sp);
            if (REACT && live) {
                // the source sees -dx, -dy and -d, except where |d| = L/2 up
                // to rounding and its own minimum image has the sign of d
                double fz = Fzeff;
                if (__builtin_fabsf(q.d) >= pa.tie32) {
                    const double d64 = min_image(zi - src.z, a.L, a.invL);
                    if (__builtin_fabs(__builtin_fabs(d64) - a.halfL) <= pa.tie) {
                        const double dji = min_image(src.z - zi, a.L, a.invL);
                        if ((dji < 0.0) == (d64 < 0.0)) fz = -Fzeff;
                    }
                }
                const double w = (double)mi;  // 0 for an empty target slot
                const double wS = w * Seff;
                double *jw = &jpart[wave][0][js];
                jw[0] = __builtin_fma(wS, (double)q.dx, jw[0]);
                jw[kOwn] = __builtin_fma(wS, (double)q.dy, jw[kOwn]);
                jw[2 * kOwn] = __builtin_fma(w, fz, jw[2 * kOwn]);
                if (POT) jw[3 * kOwn] = __builtin_fma(w, Pn, jw[3 * kOwn]);
            }
            // the next step's lanes read the slots this step wrote: a
            // compiler barrier keeps the steps' LDS accesses in program
            // order (the wave's LDS operations complete in issue order)
            asm volatile("" ::: "memory");
        }
    }
    if (REACT) {
        __syncthreads();
        if (tid < cnt) {
            // reaction on source base + tid in the owned sums' orientation:
            // the 4 waves' parts in order, into the source's slot kSubs + si
            const int64_t jj = base + tid;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k == 3 && !POT) continue;
                const double v = (jpart[0][k][tid] + jpart[1][k][tid]) + (jpart[2][k][tid] + jpart[3][k][tid]);
                double *p = pa.acc + ((int64_t)(kSubs + si) * 4 + k) * pa.N + jj;
                *p = (k == 3) ? *p + v : *p - v;
            }
        }
    }
    // the two halves' sums of each target
    sx += __shfl_xor(sx, 32);
    sy += __shfl_xor(sy, 32);
    sz += __shfl_xor(sz, 32);
    sp += __shfl_xor(sp, 32);
    if (active && h == 0) {
        // the targets' actions from sub-group sj: slot sj; the self meeting
        // initialises it and clears the reaction slot kSubs + sj
        const double v[4] = {sx, sy, sz, sp};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double *p = pa.acc + ((int64_t)sj * 4 + k) * pa.N + t;
            if (REACT) {
                if (k < 3 || POT) *p += v[k];
            } else {
                *p = v[k];
                p[(int64_t)kSubs * 4 * pa.N] = 0.0;
            }
        }
    }
}

template <bool POT>
hipError_t launch_learned_pairwise(PairwiseLearnedArgs pa, hipStream_t stream) {
    hipLaunchKernelGGL((forces_learned_pairwise_kernel<POT, false>), dim3(pa.G * kSubs * kSubs), dim3(kBlock), 0,
                       stream, pa);
    hipError_t e = hipGetLastError();
    for (int r = 0; e == hipSuccess && r + 1 < pa.Gp; ++r) {
        pa.round = r;
        hipLaunchKernelGGL((forces_learned_pairwise_kernel<POT, true>), dim3(pa.Gp / 2 * kSubs * kSubs), dim3(kBlock),
                           0, stream, pa);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

size_t learned_pairwise_bytes(int64_t N) {
    return ws_total({order_targets_bytes(N), (size_t)N * sizeof(SrcRec), (size_t)N * kSlots * 4 * sizeof(double)});
}

// Pairwise learned forces of all N particles (see above); arguments already
// validated.  Scratch (spatial order, records, FP64 sums) comes from `ws`.
int launch_forces_learned_pairwise(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                                   const steps_cyl_mlp *net, float *out_acc, float *out_pot, Workspace &ws,
                                   hipStream_t stream) {
    int rc = check_workspace(ws, learned_pairwise_bytes(N));
    if (rc) return rc;
    const int *perm = nullptr;
    if ((rc = order_targets(pos, N, L, nullptr, N, stream, ws, &perm))) return rc;
    SrcRec *rec = (SrcRec *)ws.take((size_t)N * sizeof(SrcRec));
    double *acc = (double *)ws.take((size_t)N * kSlots * 4 * sizeof(double));
    if (!rec || !acc) return fail(STEPS_EINVAL, "workspace too small for the pairwise learned path");
    PairwiseLearnedArgs pa;
    LearnedArgs &a = pa.la;
    a.x = a.y = a.z = a.m = a.h = nullptr;
    a.targets = nullptr;
    a.perm = nullptr;
    a.P = mlp::packed_of(net);
    a.ax = a.ay = a.az = a.pot = nullptr;
    a.L = L;
    a.invL = 1.0 / L;
    a.halfL = 0.5 * L;
    a.invLf = (float)(1.0 / L);
    a.invL2f = (float)(1.0 / (L * L));
    a.c.Lf = (float)L;
    a.c.L2f = (float)(L * L);
    a.c.m2Lf = (float)(-2.0 * L);
    a.c.n_img = 1;
    a.bs = band_series();
    a.N = (int)N;
    a.n_tgt = (int)N;
    pa.rec = rec;
    pa.acc = acc;
    pa.tie = 1e-12 * L;
    pa.tie32 = (float)(0.5 * L * (1.0 - 1e-6));
    pa.N = (int)N;
    pa.G = (int)((N + kOwn * kSubs - 1) / (kOwn * kSubs));
    pa.Gp = pa.G + (pa.G & 1);
    pa.round = 0;
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL(lp_stage_kernel, dim3(nb), dim3(256), 0, stream, pos, mass, eps, (int)N, L, perm, rec);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = out_pot ? launch_learned_pairwise<true>(pa, stream) : launch_learned_pairwise<false>(pa, stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(lp_finish_kernel, dim3(nb), dim3(256), 0, stream, pa.acc, perm, (int)N, out_acc,
                           out_acc + N, out_acc + 2 * N, out_pot);
        e = hipGetLastError();
    }
    return hip_status(e, "forces_learned_pairwise launch");
}

}  // namespace steps
