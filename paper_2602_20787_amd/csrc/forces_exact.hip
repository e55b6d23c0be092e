// Exact image-sum forces on gfx950 (Sect. 2.1, eqs. ComovingEquationsOfMotion,
// Force_spline_kernel, NewtonianForce, ForceCylindrical).
//
// Mapping.  One thread owns one target: its FP64 position, wrapped z and
// softening stay in registers for the whole launch.  A workgroup of 256
// threads walks the N sources in tiles of 256; each thread stages one source
// per tile from the caller's SoA arrays (coalesced FP64 loads), wraps its z
// into [0, L) in FP64 and writes a 32-byte record {x, y, z, m, h} to LDS.
// After a barrier every wave reads the tile back by broadcast and runs the
// pair kernel against its 64 targets.
//
// Pair kernel.  Separations and the minimum-image choice are made in FP64
// (positions up to a few units, clump separations of 1e-3 and below would
// lose their low bits in FP32), then cast to FP32.  The n = 0 term and the
// images n = +-1..+-n_img are Newtonian rsqrt terms:
//   r_n^2 = rho^2 + (d - nL)^2,   S  = sum_n r_n^-3,
//   U = sum_n n r_n^-3,            Fz = d S - L U = sum_n r_n^-3 (d - nL),
//   P = sum_n r_n^-1.
// For |n| >= 2 the pair of images +-n shares C_n = rho^2 + d^2 + n^2 L^2, so
// r^2_{+-n} = C_n -+ 2 n L d costs 1.5 operations per image; S and U are
// built as suffix sums over descending n (T += r^-3, U += T), which needs
// no explicit r^-3 and no per-image weight.  The x and y components factor
// out of the image sum: a_xy += m_j S (dx, dy).
// Pairs closer than their softening length h_i + h_j (n = 0 inside the
// spline core), coincident pairs, the self pair and pairs with
// h_i + h_j > L/2 (where images could need softening too) take a rare,
// divergent FP64 branch that evaluates every image with the spline law.
//
// Accumulation.  Per target, FP32 partial sums over 32 sources are folded
// into Kahan-compensated totals (or, in plain mode, every pair is added
// straight into an FP32 total).
//
// Short target lists.  When the target blocks alone would leave the device
// idle, the sources are split into chunks too (a grid of target blocks x
// source chunks): each workgroup writes its compensated totals in FP64 to
// the workspace and a second pass adds the chunks in order.  The chunking
// depends only on the list's length and N, so results stay deterministic;
// lists long enough to fill the device take one chunk and the direct write.
#include <algorithm>

#include "common.h"
#include "pair_f64.h"
#include "pair_fp32.h"

namespace steps {

namespace {

constexpr int kBlock = 256;  // targets per workgroup and sources per LDS tile
constexpr int kSub = 32;     // sources per compensated flush

struct ExactArgs {
    const double *x, *y, *z, *m, *h;
    const int64_t *targets;  // null: target k is particle k
    const int *perm;         // list positions in spatial order of their targets, or null
    float *ax, *ay, *az, *pot;
    double *part;            // [chunks][4][n_tgt] chunk totals, or null for one chunk
    double L, invL, halfL;
    ImageConsts c;
    int N, n_tgt;
    int chunk;               // sources per chunk (a multiple of kBlock, or N)
};

template <int NIMG, bool POT, bool COMP>
__global__ __launch_bounds__(kBlock) void forces_exact_kernel(ExactArgs a) {
    __shared__ SrcRec tile[kBlock];
    const int tid = threadIdx.x;
    const int k = blockIdx.x * kBlock + tid;
    const bool active = k < a.n_tgt;
    const int64_t kk = active ? (a.perm ? (int64_t)a.perm[k] : (int64_t)k) : 0;  // position in the list
    const int64_t i = a.targets ? a.targets[kk] : kk;
    const double xi = a.x[i], yi = a.y[i], zi = wrap_z(a.z[i], a.L);
    const float hi = (float)a.h[i];

    float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f;  // totals
    float cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;  // Kahan compensations

    __shared__ float wave_hmax[kBlock / 64];
    const int j0 = blockIdx.y * a.chunk, j1 = min(a.N, j0 + a.chunk);
    for (int base = j0; base < j1; base += kBlock) {
        const int j = base + tid;
        float hj = 0.f;
        if (j < j1) {
            SrcRec r;
            r.x = a.x[j];
            r.y = a.y[j];
            r.z = wrap_z(a.z[j], a.L);
            r.m = (float)a.m[j];
            r.h = (float)a.h[j];
            hj = r.h;
            tile[tid] = r;
        }
        // largest softening in the tile: a per-target bound (h_i + max h_j)^2
        // on r^2 below which a pair may need the spline
        for (int off = 32; off >= 1; off >>= 1) hj = fmaxf(hj, __shfl_xor(hj, off));
        if ((tid & 63) == 0) wave_hmax[tid >> 6] = hj;
        __syncthreads();
        float hmax = wave_hmax[0];
        for (int w = 1; w < kBlock / 64; ++w) hmax = fmaxf(hmax, wave_hmax[w]);
        const float hb = hi + hmax;        // >= h_i + h_j for every source in the tile
        const float thr2 = hb * hb;        // rounding is monotonic: >= (h_i + h_j)^2
        const bool wide = hb > (float)a.halfL;
        const int cnt = min(kBlock, j1 - base);
        for (int s0 = 0; s0 < cnt; s0 += kSub) {
            const int e = min(kSub, cnt - s0);
            float px = 0.f, py = 0.f, pz = 0.f, pp = 0.f;
#pragma unroll 2
            for (int s = 0; s < e; ++s) {
                const SrcRec src = tile[s0 + s];
                const double dx64 = xi - src.x;
                const double dy64 = yi - src.y;
                const double t = zi - src.z;
                const double d64 = min_image(t, a.L, a.invL);
                const float dx = (float)dx64, dy = (float)dy64, d = (float)d64;
                float S, Fz, P = 0.f;
                pair_fast<NIMG, POT>(dx, dy, d, a.c, S, Fz, P);
                const float r2_0 = __builtin_fmaf(d, d, __builtin_fmaf(dx, dx, dy * dy));
                if ((wide || r2_0 < thr2) &&
                    (r2_0 < (hi + src.h) * (hi + src.h) || hi + src.h > (float)a.halfL)) {
                    if ((int64_t)(base + s0 + s) == i) {
                        S = 0.f;
                        Fz = 0.f;
                        P = 0.f;
                    } else {
                        const PairSums g = pair_general_f64(dx64, dy64, d64, (double)hi + (double)src.h,
                                                            a.L, (NIMG >= 0) ? NIMG : a.c.n_img);
                        S = g.S;
                        Fz = g.Fz;
                        P = g.P;
                    }
                }
                const float mS = src.m * S;
                if (COMP) {
                    px = __builtin_fmaf(mS, dx, px);
                    py = __builtin_fmaf(mS, dy, py);
                    pz = __builtin_fmaf(src.m, Fz, pz);
                    if (POT) pp = __builtin_fmaf(src.m, P, pp);
                } else {
                    sx = __builtin_fmaf(mS, dx, sx);
                    sy = __builtin_fmaf(mS, dy, sy);
                    sz = __builtin_fmaf(src.m, Fz, sz);
                    if (POT) sp = __builtin_fmaf(src.m, P, sp);
                }
            }
            if (COMP) {
                kahan_add(sx, cx, px);
                kahan_add(sy, cy, py);
                kahan_add(sz, cz, pz);
                if (POT) kahan_add(sp, cp, pp);
            }
        }
        __syncthreads();
    }
    if (active) {
        // attraction: a = -sum m_j S (x_i - x_j), potential = -sum m_j / r
        const int64_t o = kk;
        if (a.part) {
            double *q = a.part + (int64_t)blockIdx.y * 4 * a.n_tgt + o;
            q[0] = (double)sx - (double)cx;
            q[a.n_tgt] = (double)sy - (double)cy;
            q[2 * (int64_t)a.n_tgt] = (double)sz - (double)cz;
            q[3 * (int64_t)a.n_tgt] = (double)sp - (double)cp;
        } else {
            a.ax[o] = -(sx - cx);
            a.ay[o] = -(sy - cy);
            a.az[o] = -(sz - cz);
            if (POT) a.pot[o] = -(sp - cp);
        }
    }
}

// Chunk totals of a short target list added in chunk order (FP64), negated
// and written as FP32.
__global__ void exact_chunks_kernel(const double *part, int chunks, int n_tgt, float *ax, float *ay, float *az,
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

template <int NIMG, bool POT, bool COMP>
hipError_t launch_t(const ExactArgs &a, hipStream_t stream) {
    const int grid = (a.n_tgt + kBlock - 1) / kBlock;
    const int chunks = (a.N + a.chunk - 1) / a.chunk;
    hipLaunchKernelGGL((forces_exact_kernel<NIMG, POT, COMP>), dim3(grid, chunks), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

template <bool POT, bool COMP>
hipError_t launch_nimg(const ExactArgs &a, hipStream_t stream) {
    switch (a.c.n_img) {
        case 0: return launch_t<0, POT, COMP>(a, stream);
        case 1: return launch_t<1, POT, COMP>(a, stream);
        case 2: return launch_t<2, POT, COMP>(a, stream);
        case 4: return launch_t<4, POT, COMP>(a, stream);
        case 8: return launch_t<8, POT, COMP>(a, stream);
        default: return launch_t<-1, POT, COMP>(a, stream);
    }
}

}  // namespace

// Source chunks of the per-target kernels for n_tgt targets of N sources:
// enough (target block, chunk) pairs for 2048 workgroups, chunks of at least
// 4096 sources; one chunk once the targets fill the device.
int per_target_chunks(int64_t N, int64_t n_tgt, int block) {
    const int64_t tblocks = (n_tgt + block - 1) / block;
    int64_t c = (2048 + tblocks - 1) / tblocks;
    c = std::min<int64_t>(c, (N + 4095) / 4096);
    return (int)std::max<int64_t>(1, c);
}

// Workspace of the per-target exact kernel: the spatial order of a long
// list, and the chunk totals of a short one.
size_t exact_per_target_bytes(int64_t N, int64_t n_tgt) {
    const int chunks = per_target_chunks(N, n_tgt, kBlock);
    return ws_total({per_target_bytes(n_tgt), chunks > 1 ? (size_t)chunks * 4 * n_tgt * sizeof(double) : 0});
}

// Launches the FP32 exact-force kernel; arguments already validated.
int launch_forces_exact(const double *pos, const double *mass, const double *eps, int64_t N,
                        double L, int n_img, const int64_t *targets, int64_t n_tgt, int mode,
                        float *out_acc, float *out_pot, Workspace &ws, hipStream_t stream) {
    ExactArgs a;
    a.x = pos;
    a.y = pos + N;
    a.z = pos + 2 * N;
    a.m = mass;
    a.h = eps;
    a.targets = targets;
    a.ax = out_acc;
    a.ay = out_acc + n_tgt;
    a.az = out_acc + 2 * n_tgt;
    a.pot = out_pot;
    a.L = L;
    a.invL = 1.0 / L;
    a.halfL = 0.5 * L;
    a.c.Lf = (float)L;
    a.c.L2f = (float)(L * L);
    a.c.m2Lf = (float)(-2.0 * L);
    a.c.n_img = n_img;
    a.N = (int)N;
    a.n_tgt = (int)n_tgt;
    a.perm = nullptr;
    // walk the targets in spatial order (keys and order in the workspace)
    int rc = check_workspace(ws, exact_per_target_bytes(N, n_tgt));
    if (rc) return rc;
    if (n_tgt >= kOrderTargetsMin && (rc = order_targets(pos, N, L, targets, n_tgt, stream, ws, &a.perm)))
        return rc;
    const int chunks = per_target_chunks(N, n_tgt, kBlock);
    a.chunk = (int)N;
    a.part = nullptr;
    if (chunks > 1) {
        a.chunk = (int)(((N + chunks - 1) / chunks + kBlock - 1) / kBlock * kBlock);
        a.part = (double *)ws.take((size_t)chunks * 4 * n_tgt * sizeof(double));
        if (!a.part) return fail(STEPS_EINVAL, "workspace too small for the chunk totals");
    }
    hipError_t e;
    const bool comp = (mode == STEPS_SUM_COMPENSATED);
    if (out_pot)
        e = comp ? launch_nimg<true, true>(a, stream) : launch_nimg<true, false>(a, stream);
    else
        e = comp ? launch_nimg<false, true>(a, stream) : launch_nimg<false, false>(a, stream);
    if (e == hipSuccess && a.part) {
        const int nch = (int)((N + a.chunk - 1) / a.chunk);
        hipLaunchKernelGGL(exact_chunks_kernel, dim3((unsigned)((n_tgt + 255) / 256)), dim3(256), 0, stream, a.part,
                           nch, (int)n_tgt, out_acc, out_acc + n_tgt, out_acc + 2 * n_tgt, out_pot);
        e = hipGetLastError();
    }
    return hip_status(e, "forces_exact launch");
}

}  // namespace steps
