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
// tile, layer 1 and the activations run on the VALU, layers 2-4 as 8 MFMAs
// each, layer 5 on the VALU with a cross-half sum.  Each half keeps its own
// compensated sums; they are added at the end.  Pairs outside
// the network's domain (rho/L < 0.05 or > 20) take the exact image band
// instead; all 64 lanes share that sum (32 images each plus a butterfly
// reduction), so a rare outside pair costs about 250 instructions instead
// of a 2046-image serial loop in one lane.
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

struct LearnedArgs {
    const double *x, *y, *z, *m, *h;
    const int64_t *targets;
    const int *perm;  // list positions in spatial order of their targets, or null
    const mlp::Packed *P;
    float *ax, *ay, *az, *pot;
    double L, invL, halfL;
    float invLf, invL2f;
    ImageConsts c;  // n_img = 1
    int N, n_tgt;
};

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

template <bool POT, bool COMP>
__global__ __launch_bounds__(kBlock) void forces_learned_kernel(LearnedArgs a) {
    __shared__ mlp::Packed P;
    __shared__ SrcRec tile[kTile];
    mlp::load_packed(&P, a.P);
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

    for (int base = 0; base < a.N; base += kTile) {
        __syncthreads();
        const int j = base + tid;
        if (j < a.N) {
            SrcRec r;
            r.x = a.x[j];
            r.y = a.y[j];
            r.z = wrap_z(a.z[j], a.L);
            r.m = (float)a.m[j];
            r.h = (float)a.h[j];
            tile[tid] = r;
        }
        __syncthreads();
        const int cnt = min(kTile, a.N - base);
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
                mlp::forward32<false>(Pl, fb1, fb2, ob0, ob1, nullptr, nullptr);
                const float o0 = h ? ob0 : oa0, o1 = h ? ob1 : oa1;
                const float mz = __builtin_fmaf(q.sc, o0, q.bz);
                float Rz = (q.d > 0.f) ? mz : ((q.d < 0.f) ? -mz : 0.f);
                float Rr = __builtin_fmaf(q.sc, o1, q.br);
                if (!q.inside) {
                    Rz = 0.f;
                    Rr = 0.f;
                }
                uint64_t outside = __ballot(q.band && active);
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
        a.ax[o] = -((sx - cx) + ox);
        a.ay[o] = -((sy - cy) + oy);
        a.az[o] = -((sz - cz) + oz);
        if (POT) a.pot[o] = -((sp - cp) + op);
    }
}

template <bool POT, bool COMP>
hipError_t launch_t(const LearnedArgs &a, hipStream_t stream) {
    const int grid = (a.n_tgt + kTargets - 1) / kTargets;
    hipLaunchKernelGGL((forces_learned_kernel<POT, COMP>), dim3(grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

namespace mlp {
const Packed *packed_of(const steps_cyl_mlp *net);
}

int launch_forces_learned(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                          const steps_cyl_mlp *net, const int64_t *targets, int64_t n_tgt, int mode,
                          float *out_acc, float *out_pot, hipStream_t stream) {
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
    a.N = (int)N;
    a.n_tgt = (int)n_tgt;
    a.perm = nullptr;
    // walk the targets in spatial order (scratch is stream-ordered)
    void *scratch = nullptr;
    if (n_tgt >= kOrderTargetsMin) {
        const int rc = order_targets(pos, N, L, targets, n_tgt, stream, &scratch, &a.perm);
        if (rc) return rc;
    }
    const bool comp = (mode == STEPS_SUM_COMPENSATED);
    hipError_t e;
    if (out_pot)
        e = comp ? launch_t<true, true>(a, stream) : launch_t<true, false>(a, stream);
    else
        e = comp ? launch_t<false, true>(a, stream) : launch_t<false, false>(a, stream);
    if (scratch) (void)hipFreeAsync(scratch, stream);
    return hip_status(e, "forces_learned launch");
}

}  // namespace steps
