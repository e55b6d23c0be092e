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
// 32-byte records {x, y, z wrapped, m, h}, with a bounding box per run of 64
// records.  A part is 64 kR consecutive records (kR = 1 particle per lane);
// a group is S parts (S = 16 up to 2^21 particles, else 8; 8 with a table).
// Each particle has 2S slots of FP64 sums (x, y, z, potential).
//
// Schedule (bitwise deterministic, no atomics).  A first launch pairs every
// group with itself (one-sided, every ordered pair, the self pair skipped)
// and initialises the slots.  Then G' - 1 launches (G' = G rounded up to
// even) follow a round-robin tournament: in round r group G'-1 meets group
// r and, for k = 1 .. G'/2 - 1, group (r + k) mod (G'-1) meets group
// (r - k) mod (G'-1), so every unordered pair of groups meets exactly once
// and no group appears twice in a round.  A meeting of groups a and b takes
// S^2 workgroups of one wave: workgroup (i, j) holds part i of a in
// registers and streams part j of b, adding a's sums into slot j of part i
// and b's reactions into slot S + i of part j.  Within a launch each slot
// has one writer, so every sum is a plain read-modify-write in an order
// fixed by (N, S).  A last pass adds the slots in order and writes FP32
// outputs at the particles' own positions.
//
// Workgroup.  One wave owns its part, kR particles per lane, in registers;
// the part's sources come through LDS as kR sub-tiles of 64: at step s lane
// l takes source (l + s) mod 64 of the sub-tile, so no two lanes meet the
// same source at once.  The reaction on a source is summed in FP64 in an
// LDS slot that the lanes update in turn (64 steps visit every lane).  A
// sub-tile whose bounding box is far from the wave's (no pair closer than
// the sum of the largest softenings, no axial separation near L/2) skips the
// softening and half-period screens and the per-pair minimum image; the pair
// arithmetic is the same either way.  One-wave workgroups need no barrier
// between waves.  Small register sets let several of them share a SIMD,
// which hides the latency of the transcendentals (17 reciprocal square
// roots per pair) and of the LDS traffic behind the other waves' work.
#include <algorithm>

#include "common.h"
#include "pair_f64.h"
#include "pair_fp32.h"
#include "table_pair.h"

namespace steps {

namespace {

constexpr int kThreads = 64;  // one wave
// Particles per lane and waves per SIMD.  The exact pair: one particle per
// lane in at most 96 VGPRs, 5 waves per SIMD.  Measured per call at
// N = 2^20, |n| <= 8 with the potential (ms): 1 per lane at 4, 5, 6 and 8
// waves 1994, 1891, 1895 and 1918; 2 per lane at 2 and 3 waves 2067 and
// 2110; 4 per lane at 2 waves (256 VGPRs) 2182.  The extra VALU work of
// one particle per lane (139 instructions per pair in the far loop against
// 134.5 with four, for the reaction's LDS update and the loop) costs less
// than the latency the extra waves hide.  With a table, one per lane and a
// bound of 4 waves (80-83 VGPRs, so 5-6 waves fit): CIC 1436 and TSC 2042 ms,
// against 1473 and 2200 with 2 per lane at 3 waves and 1441 and 2075 with
// the bound at 6 waves.
constexpr int particles_per_thread(int) { return 1; }
constexpr int waves_per_simd(int torder) { return torder > 0 ? 4 : 5; }
constexpr int kSub = 64;    // sources per sub-tile (one rotation)
constexpr int kBox = 8;     // doubles per 64-record box

struct PairwiseArgs {
    const SrcRec *rec;   // [N] records in spatial order
    const double *box;   // [ceil(N/64)][8] bounding boxes of aligned runs of 64 records
    double *sum;         // [2S][4][N] FP64 sums in spatial order (x, y, z, potential)
    double L, invL, halfL, tie;  // tie: |d| within this of L/2 takes the check
    double far_h;                // largest softening sum for which the fast path is allowed
    float tie32;                 // FP32 screen for it: 0.5 L (1 - 1e-6), below every such |d|
    ImageConsts c;
    TableView tv;  // far-image table (table paths only)
    float invLf, invL2f;
    int N, G, Gp;  // particles, groups, groups rounded up to even
    int S;         // parts per group (1, 2, 4, 8 or 16)
    int round;     // tournament round (launches of the meetings)
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
                             const int *perm, SrcRec *rec) {
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
}

// Bounding box {x_lo, x_hi, y_lo, y_hi, z_lo, z_hi, h_max, 0} of the records
// 64b .. 64b+63 (those below N); one wave per box.
__global__ void box_kernel(const SrcRec *rec, int N, double *box) {
    const int b = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t k = (int64_t)b * 64 + (threadIdx.x & 63);
    if ((int64_t)b * 64 >= N) return;  // whole wave leaves together
    double v[7];
    if (k < N) {
        const SrcRec r = rec[k];
        v[0] = r.x;
        v[1] = -r.x;
        v[2] = r.y;
        v[3] = -r.y;
        v[4] = r.z;
        v[5] = -r.z;
        v[6] = (double)r.h;
    } else {
        for (int c = 0; c < 6; ++c) v[c] = HUGE_VAL;  // neutral for the minima
        v[6] = 0.0;
    }
    // minima of (x, -x, y, -y, z, -z), maximum of h, over the wave
    for (int off = 32; off >= 1; off >>= 1) {
        for (int c = 0; c < 6; ++c) v[c] = fmin(v[c], __shfl_xor(v[c], off));
        v[6] = fmax(v[6], __shfl_xor(v[6], off));
    }
    if ((threadIdx.x & 63) == 0) {
        double *o = box + (int64_t)b * kBox;
        o[0] = v[0];
        o[1] = -v[1];
        o[2] = v[2];
        o[3] = -v[3];
        o[4] = v[4];
        o[5] = -v[5];
        o[6] = v[6];
        o[7] = 0.0;
    }
}

__global__ void finish_kernel(const double *sum, int slots, const int *perm, int N, float *ax, float *ay, float *az,
                              float *pot) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = 0; q < slots; ++q)
        for (int c = 0; c < 4; ++c) s[c] += sum[((int64_t)q * 4 + c) * N + k];
    const int p = perm[k];
    // attraction: a = -sum m_j S (x_i - x_j), potential = -sum m_j / r
    ax[p] = (float)(-s[0]);
    ay[p] = (float)(-s[1]);
    az[p] = (float)(-s[2]);
    if (pot) pot[p] = (float)(-s[3]);
}

template <int kR>
struct Owned {
    double x[kR], y[kR], z[kR];
    float h[kR], m[kR];
    int t[kR];  // record index, or N for an empty slot
};

struct WaveBox {
    double x0, x1, y0, y1, z0, z1, h;
};

// True when no pair between the wave's particles (box w) and the records of
// box b needs the softening or the half-period screen: the boxes are apart by
// more than the sum of their largest softenings (with that sum below L/2, so
// that no image n != 0 is softened either) and no axial separation comes
// near L/2.  Then every axial separation t = z_i - z_j of the two boxes has
// the same minimum image t - kL, returned as kL.  Evaluated alike by every
// lane.
__device__ __forceinline__ bool far_boxes(const PairwiseArgs &a, const WaveBox &w, const double *b, double &kL) {
    const double hs = w.h + b[6];
    if (hs > a.far_h) return false;
    const double gx = fmax(0.0, fmax(w.x0 - b[1], b[0] - w.x1));
    const double gy = fmax(0.0, fmax(w.y0 - b[3], b[2] - w.y1));
    // axial separations t = z_i - z_j lie in [tl, th], inside (-L, L)
    const double tl = w.z0 - b[5], th = w.z1 - b[4];
    double gz;
    if (ceil(tl * a.invL) <= floor(th * a.invL)) {
        gz = 0.0;  // a multiple of L inside: some pair may be axially aligned
    } else {
        const double el = fabs(tl - a.L * rint(tl * a.invL)), eh = fabs(th - a.L * rint(th * a.invL));
        gz = fmin(el, eh);
    }
    // no separation within 1e-5 L of a half period (the screen is 5e-7 L)
    const double m = 1e-5 * a.L;
    if (ceil((tl - m) * a.invL - 0.5) <= floor((th + m) * a.invL - 0.5)) return false;
    kL = a.L * floor(tl * a.invL + 0.5);
    return gx * gx + gy * gy + gz * gz > hs * hs * (1.0 + 1e-4) + 1e-300;
}

// LDS of a workgroup: its part's sources (SoA) and their FP64 reaction slots.
template <int kR>
struct Stage {
    double x[64 * kR], y[64 * kR], z[64 * kR];
    float m[64 * kR], h[64 * kR];
    double r[4][64 * kR];  // reactions, FP64
};

// Reaction on the source from an evaluated pair, in the owned sums'
// orientation (dx = x_i - x_j): the source sees -dx, -dy and -d, except
// where |d| = L/2 up to rounding and its own minimum image has the sign of d.
__device__ __forceinline__ double tie_fz(const PairwiseArgs &a, double zi, double zj, double Fz64) {
    const double d64 = min_image(zi - zj, a.L, a.invL);
    if (__builtin_fabs(__builtin_fabs(d64) - a.halfL) <= a.tie) {
        const double dji = min_image(zj - zi, a.L, a.invL);
        if ((dji < 0.0) == (d64 < 0.0)) return -Fz64;
    }
    return Fz64;
}

// The table's far images of one pair (Sect. 2.2, eq. S1R2EwaldCorrectionTable)
// added to (S, Fz): R_z is odd in d and R_rho even, so the corrected pair
// keeps the symmetry of the exact one.  `self`: the pair of a particle with
// itself (no correction).
template <int TORDER, bool COMPLETE>
__device__ __forceinline__ void table_far(const PairwiseArgs &a, float dx, float dy, float d, bool self, float &S,
                                          float &Fz) {
    const float rho = __builtin_sqrtf(__builtin_fmaf(dx, dx, dy * dy));
    const float rr = rho * a.invLf;
    const float delta = __builtin_fabsf(d) * a.invLf;
    const bool inside = (rr <= a.tv.r_max) && !self;
    float tz, tr;
    lookup<(TORDER > 0 ? TORDER : 1)>(a.tv, delta, inside ? rr : 0.f, tz, tr);
    float Rz = (d > 0.f) ? tz : ((d < 0.f) ? -tz : 0.f);
    float Rr = tr;
    if (!inside) {
        Rz = 0.f;
        Rr = 0.f;
        if (!self) {
            const float ds = d * a.invLf;
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
    S = __builtin_fmaf(-Rr * a.invL2f, rinv, S);
    Fz = __builtin_fmaf(-Rz, a.invL2f, Fz);
}

// One wave's rotation over sub-tile s when far_boxes holds (image shift kL):
// 64 steps, lane l taking source (l + step) mod 64.  The separation is the
// FP64 difference of the positions, with the minimum image's shift kL taken
// off the owned z once per sub-tile, rounded to FP32 (as exact as in
// near_pass, with no per-pair floor).  No softening, no half-period screen.
// FP32 pair terms, FP64 sums and reactions as in near_pass.
template <int NIMG, bool POT, int TORDER, bool COMPLETE, bool REACT, int kR>
__device__ __forceinline__ void far_pass(const PairwiseArgs &a, const Owned<kR> &o, Stage<kR> &st, int s, double kL,
                                         double (*acc)[4]) {
    const int lane = threadIdx.x & 63;
    double zs[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) zs[r] = o.z[r] - kL;
    for (int step = 0; step < kSub; ++step) {
        const int k = (s << 6) | ((lane + step) & 63);
        const double sxj = st.x[k], syj = st.y[k], szj = st.z[k];
        const double ms = (double)st.m[k];
        double jx = 0.0, jy = 0.0, jz = 0.0, jp = 0.0;
        if (REACT && step > 0) {
            // the slot as the previous lane left it
            jx = st.r[0][k];
            jy = st.r[1][k];
            jz = st.r[2][k];
            if (POT) jp = st.r[3][k];
        }
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const double dx64 = o.x[r] - sxj, dy64 = o.y[r] - syj;
            const float dx = (float)dx64, dy = (float)dy64, d = (float)(zs[r] - szj);
            float S, Fz, P = 0.f;
            pair_fast<NIMG, POT>(dx, dy, d, a.c, S, Fz, P);
            if (TORDER > 0) table_far<TORDER, COMPLETE>(a, dx, dy, d, false, S, Fz);
            const double S64 = (double)S, Fz64 = (double)Fz;
            const double mS = ms * S64;
            acc[r][0] = __builtin_fma(mS, dx64, acc[r][0]);
            acc[r][1] = __builtin_fma(mS, dy64, acc[r][1]);
            acc[r][2] = __builtin_fma(ms, Fz64, acc[r][2]);
            if (POT) acc[r][3] = __builtin_fma(ms, (double)P, acc[r][3]);
            if (REACT) {
                const double miS = o.m[r] * S64;
                jx = __builtin_fma(miS, dx64, jx);
                jy = __builtin_fma(miS, dy64, jy);
                jz = __builtin_fma(o.m[r], Fz64, jz);
                if (POT) jp = __builtin_fma(o.m[r], (double)P, jp);
            }
        }
        if (REACT) {
            st.r[0][k] = jx;
            st.r[1][k] = jy;
            st.r[2][k] = jz;
            if (POT) st.r[3][k] = jp;
        }
    }
}

// One wave's rotation over sub-tile s in general position: FP64 separation
// and minimum image, then FP32 pair terms and FP64 sums (the records are in
// spatial order, so a particle's near neighbours arrive together and an FP32
// partial would lose their cancellation).  The n = 0 image of a pair inside
// its softening length takes the spline in FP32 (selected per pair; the
// separation is the FP64 one cast); with a softening sum above L/2 the
// images n != 0 may be softened too and the pair is evaluated in FP64 with
// the spline on every image (rare: one pair per lane and pass).  REACT: the
// sources belong to another group and their reactions are summed in the
// FP64 LDS slots; otherwise (the group against itself) the self pair is
// skipped.
template <int NIMG, bool POT, int TORDER, bool COMPLETE, bool REACT, int kR>
__device__ __forceinline__ void near_pass(const PairwiseArgs &a, const Owned<kR> &o, Stage<kR> &st, int s, int base,
                                          float hmax, double (*acc)[4]) {
    const int lane = threadIdx.x & 63;
    float thr2[kR];
    bool wide[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const float hb = o.h[r] + hmax;  // >= h_i + h_j for every source of the sub-tile
        thr2[r] = hb * hb;
        wide[r] = hb > (float)a.halfL;
    }
    for (int step = 0; step < kSub; ++step) {
        const int k = (s << 6) | ((lane + step) & 63);
        SrcRec src;
        src.x = st.x[k];
        src.y = st.y[k];
        src.z = st.z[k];
        src.m = st.m[k];
        src.h = st.h[k];
        double dx64[kR], dy64[kR];
        float S[kR], Fz[kR], P[kR], dr[kR];
        bool tie[kR];
        unsigned soft64 = 0;  // bit r: the pair (r, src) takes the FP64 spline on every image
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            dx64[r] = o.x[r] - src.x;
            dy64[r] = o.y[r] - src.y;
            const double d64 = min_image(o.z[r] - src.z, a.L, a.invL);
            const float dx = (float)dx64[r], dy = (float)dy64[r], d = (float)d64;
            dr[r] = d;
            const float rho2 = __builtin_fmaf(dx, dx, dy * dy);
            const float r2_0 = __builtin_fmaf(d, d, rho2);
            float T, U, Q;
            pair_images<NIMG, POT>(rho2, d, r2_0, a.c, T, U, Q);
            const float hij = o.h[r] + src.h;
            const bool self = !REACT && base + k == o.t[r];
            const bool near = (wide[r] || r2_0 < thr2[r]) && (r2_0 < hij * hij || hij > (float)a.halfL);
            if (near && hij > (float)a.halfL && !self) soft64 |= 1u << r;
            float s0, p0;
            if (__ballot(near && !self) != 0) {
                float sf, pf;
                spline_n0(r2_0, hij, sf, pf);
                const float ri0 = __builtin_amdgcn_rsqf(r2_0);
                s0 = near ? sf : ri0 * ri0 * ri0;
                p0 = near ? pf : ri0;
            } else {
                const float ri0 = __builtin_amdgcn_rsqf(r2_0);
                s0 = ri0 * ri0 * ri0;
                p0 = ri0;
            }
            S[r] = s0 + T;
            Fz[r] = __builtin_fmaf(d, S[r], -a.c.Lf * U);
            P[r] = p0 + Q;
            if (self) {
                // j == i: no term at all, images included
                S[r] = 0.f;
                Fz[r] = 0.f;
                P[r] = 0.f;
            }
            tie[r] = REACT && __builtin_fabsf(d) >= a.tie32;
        }
        while (soft64) {
            // rare and divergent: one pair per lane and pass, operands picked
            // by selects so that the spline code exists once
            const int rr = __builtin_ctz(soft64);
            soft64 &= soft64 - 1;
            double xr = o.x[0], yr = o.y[0], zr = o.z[0];
            float hr = o.h[0];
#pragma unroll
            for (int q = 1; q < kR; ++q)
                if (rr == q) {
                    xr = o.x[q];
                    yr = o.y[q];
                    zr = o.z[q];
                    hr = o.h[q];
                }
            double gs, gf, gp;
            pair_spline_f64(xr - src.x, yr - src.y, min_image(zr - src.z, a.L, a.invL),
                            (double)hr + (double)src.h, a.L, (NIMG >= 0) ? NIMG : a.c.n_img, gs, gf, gp);
#pragma unroll
            for (int q = 0; q < kR; ++q)
                if (rr == q) {
                    S[q] = (float)gs;
                    Fz[q] = (float)gf;
                    P[q] = (float)gp;
                }
        }
        if (TORDER > 0) {
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const bool self = !REACT && base + k == o.t[r];
                table_far<TORDER, COMPLETE>(a, (float)dx64[r], (float)dy64[r], dr[r], self, S[r], Fz[r]);
            }
        }
        const double ms = (double)src.m;
        double jx = 0.0, jy = 0.0, jz = 0.0, jp = 0.0;
        if (REACT && step > 0) {
            // the slot as the previous lane left it
            jx = st.r[0][k];
            jy = st.r[1][k];
            jz = st.r[2][k];
            if (POT) jp = st.r[3][k];
        }
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const double S64 = (double)S[r], Fz64 = (double)Fz[r];
            const double mS = ms * S64;
            acc[r][0] = __builtin_fma(mS, dx64[r], acc[r][0]);
            acc[r][1] = __builtin_fma(mS, dy64[r], acc[r][1]);
            acc[r][2] = __builtin_fma(ms, Fz64, acc[r][2]);
            if (POT) acc[r][3] = __builtin_fma(ms, (double)P[r], acc[r][3]);
            if (REACT) {
                const double fz = tie[r] ? tie_fz(a, o.z[r], src.z, Fz64) : Fz64;
                const double miS = o.m[r] * S64;
                jx = __builtin_fma(miS, dx64[r], jx);
                jy = __builtin_fma(miS, dy64[r], jy);
                jz = __builtin_fma(o.m[r], fz, jz);
                if (POT) jp = __builtin_fma(o.m[r], (double)P[r], jp);
            }
        }
        if (REACT) {
            st.r[0][k] = jx;
            st.r[1][k] = jy;
            st.r[2][k] = jz;
            if (POT) st.r[3][k] = jp;
        }
    }
}

// Workgroup (i, j) of one meeting (REACT: the groups of tournament round
// a.round) or of one group's meeting with itself: part i of group a against
// part j of group b.
template <int NIMG, bool POT, int TORDER, bool COMPLETE, bool REACT>
__global__ __launch_bounds__(kThreads, waves_per_simd(TORDER)) void forces_pairwise_kernel(PairwiseArgs a) {
    constexpr int kR = particles_per_thread(TORDER);
    constexpr int kPart = 64 * kR;  // particles per part
    __shared__ Stage<kR> st;
    const int lane = threadIdx.x;
    const int S = a.S;
    const int meet = blockIdx.x / (S * S);
    const int pi = (blockIdx.x / S) % S, pj = blockIdx.x % S;
    int ga = meet, gb = meet;
    if (REACT) {
        const int M = a.Gp - 1;
        if (meet == 0) {
            ga = M;
            gb = a.round;
        } else {
            ga = (a.round + meet) % M;
            gb = (a.round - meet + M) % M;
        }
        if (ga >= a.G || gb >= a.G) return;  // the empty group of an odd count
    }
    const int64_t g0 = ((int64_t)ga * S + pi) * kPart;  // first owned record
    if (g0 >= a.N) return;                              // an empty part: nothing owned
    const int64_t b0 = ((int64_t)gb * S + pj) * kPart;  // first source record
    const int cnt = (int)max((int64_t)0, min((int64_t)kPart, (int64_t)a.N - b0));
    if (REACT && cnt == 0) return;                      // no sources: nothing to add

    // the owned particles: records g0 + r*64 + lane; empty slots copy the
    // part's first record with no mass (they sit where a particle is, so
    // every pair distance stays that of a real pair)
    Owned<kR> o;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int64_t t64 = g0 + r * 64 + lane;
        const bool real = t64 < a.N;
        const SrcRec rr = a.rec[real ? t64 : g0];
        o.t[r] = real ? (int)t64 : a.N;
        o.x[r] = rr.x;
        o.y[r] = rr.y;
        o.z[r] = rr.z;
        o.h[r] = rr.h;
        o.m[r] = real ? rr.m : 0.f;
    }
    // the part's bounding box (every lane ends with it)
    WaveBox wb;
    {
        double v[7] = {o.x[0], -o.x[0], o.y[0], -o.y[0], o.z[0], -o.z[0], (double)o.h[0]};
#pragma unroll
        for (int r = 1; r < kR; ++r) {
            v[0] = fmin(v[0], o.x[r]);
            v[1] = fmin(v[1], -o.x[r]);
            v[2] = fmin(v[2], o.y[r]);
            v[3] = fmin(v[3], -o.y[r]);
            v[4] = fmin(v[4], o.z[r]);
            v[5] = fmin(v[5], -o.z[r]);
            v[6] = fmax(v[6], (double)o.h[r]);
        }
        for (int off = 32; off >= 1; off >>= 1) {
            for (int c = 0; c < 6; ++c) v[c] = fmin(v[c], __shfl_xor(v[c], off));
            v[6] = fmax(v[6], __shfl_xor(v[6], off));
        }
        wb.x0 = v[0];
        wb.x1 = -v[1];
        wb.y0 = v[2];
        wb.y1 = -v[3];
        wb.z0 = v[4];
        wb.z1 = -v[5];
        wb.h = v[6];
    }

    double acc[kR][4];
#pragma unroll
    for (int r = 0; r < kR; ++r)
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;

    // stage the sources; a partly filled sub-tile is padded with massless
    // copies of its first record (inside its box)
    const int nsub = (cnt + kSub - 1) / kSub;
    const int base = (int)b0;  // b0 < N <= 2^29 whenever cnt > 0
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int t = r * 64 + lane;
        if (t < nsub * kSub) {
            const bool real = t < cnt;
            const SrcRec rr = a.rec[real ? base + t : base + (t & ~(kSub - 1))];
            st.x[t] = rr.x;
            st.y[t] = rr.y;
            st.z[t] = rr.z;
            st.m[t] = real ? rr.m : 0.f;
            st.h[t] = rr.h;
        }
    }
    __syncthreads();
    for (int s = 0; s < nsub; ++s) {
        const double *b = a.box + (int64_t)((base >> 6) + s) * kBox;  // base is a multiple of 64
        double kL = 0.0;
        const bool far = far_boxes(a, wb, b, kL);
        if (__builtin_amdgcn_readfirstlane((int)far))
            far_pass<NIMG, POT, TORDER, COMPLETE, REACT>(a, o, st, s, kL, acc);
        else
            near_pass<NIMG, POT, TORDER, COMPLETE, REACT>(a, o, st, s, base, (float)b[6], acc);
    }
    __syncthreads();
    if (REACT) {
        // reactions on the sources, in the owned sums' orientation, into
        // slot S + pi of part pj
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int t = r * 64 + lane;
            if (t < cnt) {
                double *p = a.sum + ((int64_t)(S + pi) * 4) * a.N + base + t;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (c == 3 && !POT) continue;
                    const double v = st.r[c][t];
                    p[(int64_t)c * a.N] = (c == 3) ? p[(int64_t)c * a.N] + v : p[(int64_t)c * a.N] - v;
                }
            }
        }
    }
    // the owned particles' sums from part pj: slot pj; the self meeting
    // initialises it and clears the reaction slot S + pj
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        if (o.t[r] < a.N) {
            double *p = a.sum + (int64_t)pj * 4 * a.N + o.t[r];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (REACT) {
                    if (c < 3 || POT) p[(int64_t)c * a.N] += acc[r][c];
                } else {
                    p[(int64_t)c * a.N] = acc[r][c];
                    p[((int64_t)S * 4 + c) * a.N] = 0.0;
                }
            }
        }
    }
}

template <int NIMG, bool POT, int TORDER, bool COMPLETE>
struct Launcher {
    static hipError_t run(PairwiseArgs a, hipStream_t stream) {
        const unsigned per_meeting = (unsigned)(a.S * a.S);
        hipLaunchKernelGGL((forces_pairwise_kernel<NIMG, POT, TORDER, COMPLETE, false>), dim3(a.G * per_meeting),
                           dim3(kThreads), 0, stream, a);
        hipError_t e = hipGetLastError();
        for (int r = 0; e == hipSuccess && r + 1 < a.Gp; ++r) {
            a.round = r;
            hipLaunchKernelGGL((forces_pairwise_kernel<NIMG, POT, TORDER, COMPLETE, true>),
                               dim3(a.Gp / 2 * per_meeting), dim3(kThreads), 0, stream, a);
            e = hipGetLastError();
        }
        return e;
    }
};

// Calls f(Launcher<...>{}) for the kernel instance of (n_img, pot, table order, complete).
template <class F>
auto dispatch(int n_img, bool pot, int order, bool complete, F &&f) {
    if (order == 0) {
        // image counts unrolled at compile time where the unrolled loop fits
        // the register budget; the others (the compiler spills the unrolled
        // 1-, 2- and 4-image forms with the potential and the 4-image form
        // without) take the run-time loop, which fits
        if (pot) {
            switch (n_img) {
                case 0: return f(Launcher<0, true, 0, false>{});
                case 8: return f(Launcher<8, true, 0, false>{});
                default: return f(Launcher<-1, true, 0, false>{});
            }
        }
        switch (n_img) {
            case 0: return f(Launcher<0, false, 0, false>{});
            case 1: return f(Launcher<1, false, 0, false>{});
            case 2: return f(Launcher<2, false, 0, false>{});
            case 8: return f(Launcher<8, false, 0, false>{});
            default: return f(Launcher<-1, false, 0, false>{});
        }
    }
    if (order == 1) {
        if (pot) return complete ? f(Launcher<1, true, 1, true>{}) : f(Launcher<1, true, 1, false>{});
        return complete ? f(Launcher<1, false, 1, true>{}) : f(Launcher<1, false, 1, false>{});
    }
    if (pot) return complete ? f(Launcher<1, true, 2, true>{}) : f(Launcher<1, true, 2, false>{});
    return complete ? f(Launcher<1, false, 2, true>{}) : f(Launcher<1, false, 2, false>{});
}

}  // namespace

// Parts per group of a pairwise call.  More parts make a launch hold more
// workgroups at the price of 2 sum slots (64 B) per particle each.  Measured
// per call at N = 2^20 with parts of 64: S = 16 and 32 took 1891 and 1894 ms
// (exact), S = 8, 16 and 32 CIC 1441, 1461 and 1464 ms and TSC 2075, 2089
// and 2085 ms.  Above 2^21 particles a call has enough meetings with S = 8
// and the slots would grow past 2 GiB.
int pairwise_parts(int64_t N, const steps_cyl_table *table) {
    if (table) return 8;
    return N <= ((int64_t)1 << 21) ? 16 : 8;
}

size_t pairwise_bytes_S(int64_t N, int S) {
    const int64_t nbox = (N + 63) / 64;
    return ws_total({order_targets_bytes(N), (size_t)N * sizeof(SrcRec), (size_t)nbox * kBox * sizeof(double),
                     (size_t)2 * S * 4 * N * sizeof(double)});
}

size_t pairwise_bytes(int64_t N, int, const steps_cyl_table *table, int, bool) {
    return pairwise_bytes_S(N, pairwise_parts(N, table));
}

// Launches the pairwise path for all N particles: exact images |n| <= n_img,
// or (table non-null) images |n| <= 1 plus the table's far images with CIC
// (order 1) or TSC (order 2) interpolation.  Arguments already validated.
// Scratch (spatial order, records, boxes, FP64 sums) comes from `ws`.
int launch_forces_pairwise(const double *pos, const double *mass, const double *eps, int64_t N, double L,
                           int n_img, const steps_cyl_table *table, int order, float *out_acc, float *out_pot,
                           Workspace &ws, hipStream_t stream, int s_cap) {
    int S = pairwise_parts(N, table);
    if (s_cap > 0) S = std::min(S, s_cap);
    int rc = check_workspace(ws, pairwise_bytes_S(N, S));
    if (rc) return rc;
    const int group = 64 * particles_per_thread(table ? 1 : 0) * S;
    PairwiseArgs a;
    a.L = L;
    a.invL = 1.0 / L;
    a.halfL = 0.5 * L;
    a.tie = 1e-12 * L;
    a.far_h = 0.49 * L;
    a.tie32 = (float)(0.5 * L * (1.0 - 1e-6));
    a.c.Lf = (float)L;
    a.c.L2f = (float)(L * L);
    a.c.m2Lf = (float)(-2.0 * L);
    a.c.n_img = table ? 1 : n_img;
    a.invLf = (float)(1.0 / L);
    a.invL2f = (float)(1.0 / (L * L));
    if (table) a.tv = table_view(table);
    a.N = (int)N;
    a.G = (int)((N + group - 1) / group);
    a.Gp = a.G + (a.G & 1);
    a.round = 0;
    a.S = S;
    const int ord = table ? order : 0;
    const bool complete = table && table->complete != 0;

    const int *perm = nullptr;
    if ((rc = order_targets(pos, N, L, nullptr, N, stream, ws, &perm))) return rc;
    const int64_t nbox = (N + 63) / 64;
    SrcRec *rec = (SrcRec *)ws.take((size_t)N * sizeof(SrcRec));
    double *box = (double *)ws.take((size_t)nbox * kBox * sizeof(double));
    double *sum = (double *)ws.take((size_t)2 * S * 4 * N * sizeof(double));
    if (!rec || !box || !sum) return fail(STEPS_EINVAL, "workspace too small for the pairwise path");
    a.rec = rec;
    a.box = box;
    a.sum = sum;
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL(stage_kernel, dim3(nb), dim3(256), 0, stream, pos, mass, eps, (int)N, L, perm, rec);
    hipLaunchKernelGGL(box_kernel, dim3((unsigned)((nbox + 3) / 4)), dim3(256), 0, stream, a.rec, (int)N, box);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = dispatch(a.c.n_img, out_pot != nullptr, ord, complete, [&](auto l) { return l.run(a, stream); });
    if (e == hipSuccess) {
        hipLaunchKernelGGL(finish_kernel, dim3(nb), dim3(256), 0, stream, a.sum, 2 * S, perm, (int)N, out_acc,
                           out_acc + N, out_acc + 2 * N, out_pot);
        e = hipGetLastError();
    }
    return hip_status(e, "forces_pairwise launch");
}

}  // namespace steps
