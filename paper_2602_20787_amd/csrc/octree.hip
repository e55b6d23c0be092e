// Barnes-Hut octree force in the S1 x R2 topology (Sect. 2.4, "Octree"):
// cubic cells, a root cell twice the largest linear size of the volume
// (S0 = 2 max(L, 2 R_dom)), a random shift of the domain along the axis and
// a rotation about it at every call, cell monopoles, and a radial correction
// table measured on the initial load and subtracted from the tree forces.
//
// Build (FP64, all on the GPU, one host synchronisation per level):
//  1. rotate by the given angle, shift and wrap z, and form 63-bit Morton
//     keys of the integer cell coordinates q = floor((p - lo) 2^21 / S0)
//     (x bit above y above z per level); radix-sort (key, index);
//  2. levels 1..21: the particles of still-open cells are "active"; a cell
//     of level l starts where an active particle's key prefix (3 l bits)
//     differs from its predecessor's; scans number the cells; a cell stays a
//     leaf when it holds at most leaf_size particles (or at level 21);
//  3. mass, mass-weighted position and largest softening bottom-up (leaves
//     from their particles, cells from their children);
//  4. depth-first order = sort of (start, level); the "skip" of a cell is
//     the first cell of the order that starts at its end.
//
// Groups: for every cell holding more than 64 particles, its children that
// hold at most 64 are packed greedily, in order, into runs of at most 64
// particles (a leaf holding more is cut into runs of 64); a tree of at most
// 64 particles is one group.  Groups are thus made of whole sibling cells
// and stay compact where 64 consecutive particles in key order would not
// (the key order jumps between distant octants).
//
// Walk: one 64-lane wave per group.  The wave walks the depth-first list
// without a stack: a cell is
// accepted for the whole group when size^2 < theta^2 d^2 and
// d^2 > (h_group + h_cell)^2,
// d the distance (periodic in z) from its centre of mass to the group's
// bounding box; an accepted cell adds its monopole, an opened leaf its
// particles, both through the pair interaction of the tabulated scheme
// (exact images |n| <= 1 plus the table's band).  The decision is
// wave-uniform, so the lanes never diverge.  Accelerations are rotated
// back and written in the caller's particle order.
#include <cmath>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "table_pair.h"

namespace steps {
namespace {

constexpr int kLevels = 21;
constexpr int kBlock = 256;
constexpr int kMaxBins = 256;
constexpr int kGroup = 64;

// one cell in depth-first order (88 B): monopole, and the traceless
// quadrupole about the centre of mass (xx, yy, zz, xy, xz, yz) when enabled
struct CellRec {
    double cx, cy, cz, mass, hmax, size;
    int start, count, skip, leaf;
    float q[6];
};

}  // namespace
}  // namespace steps

struct steps_cyl_tree {
    int leaf_size = 16;
    int quadrupole = 0;
    int64_t cap_n = 0, cap_cells = 0;
    size_t cub_bytes = 0;
    void *cub_tmp = nullptr;
    // particles
    double *tx = nullptr, *ty = nullptr, *tz = nullptr;
    uint64_t *key_in = nullptr, *key_out = nullptr;
    int *idx_in = nullptr, *idx_out = nullptr;
    double *sx = nullptr, *sy = nullptr, *sz = nullptr, *sm = nullptr, *sh = nullptr;
    int *act = nullptr, *fs = nullptr, *fe = nullptr, *ss = nullptr, *se = nullptr;
    // cells, in build order (level by level)
    int *c_start = nullptr, *c_count = nullptr, *c_level = nullptr, *c_leaf = nullptr;
    double *c_m = nullptr, *c_mx = nullptr, *c_my = nullptr, *c_mz = nullptr, *c_h = nullptr;
    double *c_q = nullptr;  // [6][cap_cells] quadrupoles (when enabled)
    uint64_t *c_key_in = nullptr, *c_key_out = nullptr;
    int *c_id_in = nullptr, *c_id_out = nullptr;
    steps::CellRec *cells = nullptr;  // depth-first
    int *cell_level = nullptr;        // depth-first
    int *g_cnt = nullptr, *g_off = nullptr;      // per cell: groups it packs, running total
    int *g_start = nullptr, *g_count = nullptr;  // per group: particle range
    int64_t n_cells = 0, n = 0, n_groups = 0;
    // walk statistics, per wave
    int *wave_cells = nullptr, *wave_parts = nullptr;
    // radial correction
    double *corr = nullptr;
    int n_bins = 0;
    double corr_rdom = 0.0;
    // calibration scratch
    double *bin_sum = nullptr, *bin_cnt = nullptr;
    float *acc_dir = nullptr, *acc_tree = nullptr;
    int64_t cap_cal = 0;
};

namespace steps {
namespace {

template <typename T>
hipError_t grow(T *&p, int64_t n) {
    (void)hipFree(p);
    p = nullptr;
    return hipMalloc(&p, (size_t)std::max<int64_t>(n, 1) * sizeof(T));
}

hipError_t ensure_particles(steps_cyl_tree *t, int64_t n) {
    if (n <= t->cap_n) return hipSuccess;
    const int64_t c = n + n / 4 + 1024;
    hipError_t e = hipSuccess;
#define G(p) \
    if (e == hipSuccess) e = grow(t->p, c);
    G(tx) G(ty) G(tz) G(key_in) G(key_out) G(idx_in) G(idx_out) G(sx) G(sy) G(sz) G(sm) G(sh)
    G(act) G(fs) G(fe) G(ss) G(se) G(wave_cells) G(wave_parts) G(g_start) G(g_count)
#undef G
    if (e != hipSuccess) return e;
    // scratch of the library sort and scan, sized for c items
    size_t b1 = 0, b2 = 0;
    e = rocprim::radix_sort_pairs(nullptr, b1, t->key_in, t->key_out, t->idx_in, t->idx_out, (int)c, 0, 63);
    if (e == hipSuccess) e = rocprim::inclusive_scan(nullptr, b2, t->fs, t->ss, (size_t)c, rocprim::plus<int>(), 0);
    if (e != hipSuccess) return e;
    const size_t need = std::max(b1, b2);
    if (need > t->cub_bytes) {
        (void)hipFree(t->cub_tmp);
        t->cub_tmp = nullptr;
        e = hipMalloc(&t->cub_tmp, need);
        if (e != hipSuccess) return e;
        t->cub_bytes = need;
    }
    t->cap_n = c;
    return hipSuccess;
}

hipError_t ensure_cells(steps_cyl_tree *t, int64_t n, hipStream_t stream) {
    if (n <= t->cap_cells) return hipSuccess;
    const int64_t c = n + n / 2 + 64;
    // keep what is built so far (levels above the current one)
    const int64_t keep = t->cap_cells;
    hipError_t e = hipSuccess;
    auto regrow = [&](auto *&p) {
        using T = std::remove_reference_t<decltype(*p)>;
        if (e != hipSuccess) return;
        T *q = nullptr;
        e = hipMalloc(&q, (size_t)c * sizeof(T));
        if (e == hipSuccess && p && keep) e = hipMemcpyAsync(q, p, (size_t)keep * sizeof(T), hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        (void)hipFree(p);
        p = q;
    };
    regrow(t->c_start);
    regrow(t->c_count);
    regrow(t->c_level);
    regrow(t->c_leaf);
    regrow(t->c_m);
    regrow(t->c_mx);
    regrow(t->c_my);
    regrow(t->c_mz);
    regrow(t->c_h);
    if (e == hipSuccess) {  // filled after the last level: nothing to keep
        (void)hipFree(t->c_q);
        t->c_q = nullptr;
        e = hipMalloc(&t->c_q, (size_t)6 * c * sizeof(double));
    }
    regrow(t->c_key_in);
    regrow(t->c_key_out);
    regrow(t->c_id_in);
    regrow(t->c_id_out);
    regrow(t->cells);
    regrow(t->cell_level);
    regrow(t->g_cnt);
    regrow(t->g_off);
    if (e != hipSuccess) return e;
    t->cap_cells = c;
    // the cell sort's and the cell scan's scratch grow with the cell count
    size_t b = 0, b2 = 0;
    e = rocprim::radix_sort_pairs(nullptr, b, t->c_key_in, t->c_key_out, t->c_id_in, t->c_id_out, (int)c, 0,
                                           37);
    if (e == hipSuccess) e = rocprim::inclusive_scan(nullptr, b2, t->g_cnt, t->g_off, (size_t)c, rocprim::plus<int>(), 0);
    if (e != hipSuccess) return e;
    b = std::max(b, b2);
    if (b > t->cub_bytes) {
        (void)hipFree(t->cub_tmp);
        t->cub_tmp = nullptr;
        e = hipMalloc(&t->cub_tmp, b);
        if (e != hipSuccess) return e;
        t->cub_bytes = b;
    }
    return hipSuccess;
}

struct Frame {
    double c, s, shift, L, lo[3], scale;
};

// rotation, shift and wrap as separately rounded operations (no contraction),
// so that keys and cells do not depend on the compiler's choices
__global__ void keys_kernel(const double *pos, int64_t N, Frame f, double *tx, double *ty, double *tz,
                            uint64_t *key, int *idx) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double X = pos[i], Y = pos[N + i], Z = pos[2 * N + i];
    const double x = f.c * X - f.s * Y;
    const double y = f.s * X + f.c * Y;
    double z = Z + f.shift;
    z = z - f.L * floor(z / f.L);
    if (z >= f.L) z = 0.0;
    tx[i] = x;
    ty[i] = y;
    tz[i] = z;
    const double p[3] = {x, y, z};
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) {
        double v = floor((p[a] - f.lo[a]) * f.scale);
        v = v < 0.0 ? 0.0 : (v > (double)((1 << kLevels) - 1) ? (double)((1 << kLevels) - 1) : v);
        q[a] = (uint64_t)v;
    }
    uint64_t k = 0;
    for (int b = 0; b < kLevels; ++b) {
        k |= ((q[0] >> b) & 1ull) << (3 * b + 2);
        k |= ((q[1] >> b) & 1ull) << (3 * b + 1);
        k |= ((q[2] >> b) & 1ull) << (3 * b);
    }
    key[i] = k;
    idx[i] = (int)i;
}

__global__ void gather_kernel(const int *idx, int N, const double *tx, const double *ty, const double *tz,
                              const double *mass, const double *eps, double *sx, double *sy, double *sz, double *sm,
                              double *sh, int *act, int root_open) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int j = idx[i];
    sx[i] = tx[j];
    sy[i] = ty[j];
    sz[i] = tz[j];
    sm[i] = mass[j];
    sh[i] = eps[j];
    act[i] = root_open;
}

// cell boundaries of one level among the active particles
__global__ void flags_kernel(const uint64_t *key, const int *act, int N, int shift, int *fs, int *fe) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const bool a = act[i] != 0;
    const uint64_t p = key[i] >> shift;
    const bool first = a && (i == 0 || !act[i - 1] || (key[i - 1] >> shift) != p);
    const bool last = a && (i == N - 1 || !act[i + 1] || (key[i + 1] >> shift) != p);
    fs[i] = first;
    fe[i] = last;
}

__global__ void compact_kernel(const int *fs, const int *fe, const int *ss, const int *se, int N, int off, int *c_start,
                               int *c_count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (fs[i]) c_start[off + ss[i] - 1] = i;
    if (fe[i]) c_count[off + se[i] - 1] = i;  // last index for now
}

__global__ void cells_kernel(int off, int n, int level, int leaf_size, int *c_start, int *c_count, int *c_level,
                             int *c_leaf) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int cnt = c_count[off + k] - c_start[off + k] + 1;
    c_count[off + k] = cnt;
    c_level[off + k] = level;
    c_leaf[off + k] = (cnt <= leaf_size || level == kLevels) ? 1 : 0;
}

// particles of open cells stay active one level down
__global__ void activity_kernel(int *act, const int *ss, int N, int off, const int *c_leaf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || !act[i]) return;
    act[i] = c_leaf[off + ss[i] - 1] ? 0 : 1;
}

// geometric centre of a cell from its key prefix (massless cells only)
__device__ void cell_centre(uint64_t key, int level, const Frame &f, double side, double *c) {
    uint64_t q[3] = {0, 0, 0};
    for (int b = 0; b < level; ++b) {
        const uint64_t digit = (key >> (3 * (kLevels - 1 - b))) & 7ull;
        q[0] = 2 * q[0] + ((digit >> 2) & 1);
        q[1] = 2 * q[1] + ((digit >> 1) & 1);
        q[2] = 2 * q[2] + (digit & 1);
    }
    const double h = side / (double)(1ull << level);
    for (int a = 0; a < 3; ++a) c[a] = f.lo[a] + ((double)q[a] + 0.5) * h;
}

// mass, mass-weighted position and largest softening of one level's cells
__global__ void moments_kernel(int off, int n, int child_off, int n_child, const int *c_start, const int *c_count,
                               const int *c_leaf, double *c_m, double *c_mx, double *c_my, double *c_mz, double *c_h,
                               const double *sx, const double *sy, const double *sz, const double *sm,
                               const double *sh) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int c = off + k;
    const int s = c_start[c], e = s + c_count[c];
    double m = 0.0, mx = 0.0, my = 0.0, mz = 0.0, h = 0.0;
    if (c_leaf[c]) {
        for (int j = s; j < e; ++j) {
            m += sm[j];
            mx += sm[j] * sx[j];
            my += sm[j] * sy[j];
            mz += sm[j] * sz[j];
            h = fmax(h, sh[j]);
        }
    } else {
        // first child: the level below's cell that starts here (binary search)
        int lo = 0, hi = n_child - 1;
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (c_start[child_off + mid] < s) lo = mid + 1; else hi = mid;
        }
        for (int q = child_off + lo; q < child_off + n_child && c_start[q] < e; ++q) {
            m += c_m[q];
            mx += c_mx[q];
            my += c_my[q];
            mz += c_mz[q];
            h = fmax(h, c_h[q]);
        }
    }
    c_m[c] = m;
    c_mx[c] = mx;
    c_my[c] = my;
    c_mz[c] = mz;
    c_h[c] = h;
}

// traceless quadrupole about the centre of mass, one level's cells: leaves
// from their particles, cells from their children (parallel-axis shift)
__global__ void quadrupole_kernel(int off, int n, int child_off, int n_child, int cap, const int *c_start,
                                  const int *c_count, const int *c_leaf, const double *c_m, const double *c_mx,
                                  const double *c_my, const double *c_mz, double *c_q, const double *sx,
                                  const double *sy, const double *sz, const double *sm) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int c = off + k;
    const int s = c_start[c], e = s + c_count[c];
    double q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double m = c_m[c];
    if (m > 0.0) {
        const double gx = c_mx[c] / m, gy = c_my[c] / m, gz = c_mz[c] / m;
        auto add = [&](double w, double x, double y, double z) {
            const double r2 = x * x + y * y + z * z;
            q[0] += w * (3.0 * x * x - r2);
            q[1] += w * (3.0 * y * y - r2);
            q[2] += w * (3.0 * z * z - r2);
            q[3] += w * 3.0 * x * y;
            q[4] += w * 3.0 * x * z;
            q[5] += w * 3.0 * y * z;
        };
        if (c_leaf[c]) {
            for (int j = s; j < e; ++j) add(sm[j], sx[j] - gx, sy[j] - gy, sz[j] - gz);
        } else {
            int lo = 0, hi = n_child - 1;
            while (lo < hi) {
                const int mid = (lo + hi) / 2;
                if (c_start[child_off + mid] < s) lo = mid + 1; else hi = mid;
            }
            for (int ch = child_off + lo; ch < child_off + n_child && c_start[ch] < e; ++ch) {
                const double mc = c_m[ch];
                for (int a = 0; a < 6; ++a) q[a] += c_q[(size_t)a * cap + ch];
                if (mc > 0.0) add(mc, c_mx[ch] / mc - gx, c_my[ch] / mc - gy, c_mz[ch] / mc - gz);
            }
        }
    }
    for (int a = 0; a < 6; ++a) c_q[(size_t)a * cap + c] = q[a];
}

__global__ void dfs_keys_kernel(int n, const int *c_start, const int *c_level, uint64_t *key, int *id) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    key[k] = ((uint64_t)c_start[k] << 5) | (uint64_t)c_level[k];
    id[k] = k;
}

__global__ void dfs_cells_kernel(int n, int N, const uint64_t *key, const int *id, const int *c_start,
                                 const int *c_count, const int *c_level, const int *c_leaf, const double *c_m,
                                 const double *c_mx, const double *c_my, const double *c_mz, const double *c_h,
                                 const double *c_q, int cap, int quad, const uint64_t *pkey, Frame f, double side,
                                 CellRec *cells, int *cell_level) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int c = id[p];
    const int end = c_start[c] + c_count[c];
    int skip = n;
    if (end < N) {  // first cell of the order that starts at `end` (the shallowest)
        const uint64_t want = (uint64_t)end << 5;
        int lo = 0, hi = n;
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (key[mid] < want) lo = mid + 1; else hi = mid;
        }
        skip = lo;
    }
    CellRec r;
    const double m = c_m[c];
    if (m > 0.0) {
        r.cx = c_mx[c] / m;
        r.cy = c_my[c] / m;
        r.cz = c_mz[c] / m;
    } else {
        double g[3];
        cell_centre(pkey[c_start[c]], c_level[c], f, side, g);
        r.cx = g[0];
        r.cy = g[1];
        r.cz = g[2];
    }
    r.mass = m;
    r.hmax = c_h[c];
    r.size = side / (double)(1ull << c_level[c]);
    r.start = c_start[c];
    r.count = c_count[c];
    r.skip = skip;
    r.leaf = c_leaf[c];
    for (int a = 0; a < 6; ++a) r.q[a] = quad ? (float)c_q[(size_t)a * cap + c] : 0.f;
    cells[p] = r;
    cell_level[p] = c_level[c];
}

// groups packed by cell c (see the file comment); with out < 0 only counted
__device__ int pack_groups(const CellRec *cells, int c, int *g_start, int *g_count, int out) {
    const CellRec r = cells[c];
    int n = 0;
    auto emit = [&](int s, int k) {
        if (out >= 0) {
            g_start[out + n] = s;
            g_count[out + n] = k;
        }
        ++n;
    };
    if (r.count <= kGroup) {
        if (c == 0) emit(0, r.count);  // the whole tree is one group
        return n;
    }
    if (r.leaf) {
        for (int s = r.start; s < r.start + r.count; s += kGroup) emit(s, min(kGroup, r.start + r.count - s));
        return n;
    }
    int run_s = 0, run_n = 0;
    for (int ch = c + 1; ch < r.skip; ch = cells[ch].skip) {
        const int cc = cells[ch].count;
        if (cc > kGroup) {
            if (run_n) emit(run_s, run_n);
            run_n = 0;
        } else {
            if (run_n + cc > kGroup) {
                emit(run_s, run_n);
                run_n = 0;
            }
            if (run_n == 0) run_s = cells[ch].start;
            run_n += cc;
        }
    }
    if (run_n) emit(run_s, run_n);
    return n;
}

__global__ void group_count_kernel(const CellRec *cells, int n, int *g_cnt) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) g_cnt[c] = pack_groups(cells, c, nullptr, nullptr, -1);
}

__global__ void group_write_kernel(const CellRec *cells, int n, const int *g_cnt, const int *g_off, int *g_start,
                                   int *g_count) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n && g_cnt[c]) pack_groups(cells, c, g_start, g_count, g_off[c] - g_cnt[c]);
}

// ---------------------------------------------------------------- walk
struct WalkArgs {
    const CellRec *cells;
    const double *sx, *sy, *sz, *sm, *sh;
    const int *idx, *g_start, *g_count;
    float *ax, *ay, *az;
    int *wave_cells, *wave_parts;
    const double *corr;
    TableView tv;
    PeriodConsts pc;
    double theta2, c, s, corr_step;
    int N, n_cells, n_groups, n_bins;
};

__device__ __forceinline__ double wave_min(double v) {
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// squared distance from c to the box [lo, hi], periodic along z (no
// contraction, so that the acceptance decisions round as written)
__device__ double box_distance2(double cx, double cy, double cz, const double lo[3], const double hi[3],
                                double L) {
#pragma clang fp contract(off)
    const double dx = fmax(0.0, fmax(lo[0] - cx, cx - hi[0]));
    const double dy = fmax(0.0, fmax(lo[1] - cy, cy - hi[1]));
    double dz = 1e300;
    for (int k = -1; k <= 1; ++k) {
        const double z = cz + k * L;
        dz = fmin(dz, fmax(0.0, fmax(lo[2] - z, z - hi[2])));
    }
    return dx * dx + dy * dy + dz * dz;
}

// size^2 < theta^2 d^2 and d^2 > (h_group + h_cell)^2, compared squared
__device__ bool accept_cell(const CellRec &r, const double lo[3], const double hi[3], double hg, double theta2,
                            double L) {
#pragma clang fp contract(off)
    const double d2 = box_distance2(r.cx, r.cy, r.cz, lo, hi, L);
    const double hs = hg + r.hmax;
    return r.size * r.size < theta2 * d2 && d2 > hs * hs;
}

// quadrupole term of an accepted cell for the images |n| <= 4 about the
// minimum image (beyond, the term falls as 1/n^4), subtracted from the
// partial sums (which carry the opposite sign of the acceleration):
// a += Q s / r^5 - (5/2) (s.Q.s) s / r^7.  Q s_n = Q s_0 - n L Q e_z.
constexpr int kQuadImages = 4;

__device__ __forceinline__ void quadrupole_term(const CellRec &r, double xi, double yi, double zi,
                                                const PeriodConsts &pc, float &px, float &py, float &pz) {
    const float sx = (float)(xi - r.cx), sy = (float)(yi - r.cy);
    const float d = (float)min_image(zi - r.cz, pc.L, pc.invL);
    const float rho2 = __builtin_fmaf(sx, sx, sy * sy);
    const float bx = __builtin_fmaf(r.q[0], sx, __builtin_fmaf(r.q[3], sy, r.q[4] * d));
    const float by = __builtin_fmaf(r.q[3], sx, __builtin_fmaf(r.q[1], sy, r.q[5] * d));
    const float bz = __builtin_fmaf(r.q[4], sx, __builtin_fmaf(r.q[5], sy, r.q[2] * d));
#pragma unroll
    for (int n = -kQuadImages; n <= kQuadImages; ++n) {
        const float nL = (float)n * pc.c.Lf;
        const float sz = d - nL;
        const float qx = __builtin_fmaf(-nL, r.q[4], bx);
        const float qy = __builtin_fmaf(-nL, r.q[5], by);
        const float qz = __builtin_fmaf(-nL, r.q[2], bz);
        const float r2 = __builtin_fmaf(sz, sz, rho2);
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float ri2 = ri * ri;
        const float ri5 = ri2 * ri2 * ri;
        const float sqs = __builtin_fmaf(sx, qx, __builtin_fmaf(sy, qy, sz * qz));
        const float c = -2.5f * sqs * ri2;
        px = __builtin_fmaf(-ri5, __builtin_fmaf(c, sx, qx), px);
        py = __builtin_fmaf(-ri5, __builtin_fmaf(c, sy, qy), py);
        pz = __builtin_fmaf(-ri5, __builtin_fmaf(c, sz, qz), pz);
    }
}

template <int ORDER, bool QUAD, bool COMPLETE>
__global__ __launch_bounds__(kBlock) void tree_walk_kernel(WalkArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = (int)(((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6);
    if (wave >= a.n_groups) return;  // whole wave
    const int g0 = a.g_start[wave];
    const bool active = lane < a.g_count[wave];
    const int i = g0 + lane;
    const int ii = active ? i : g0;
    const double xi = a.sx[ii], yi = a.sy[ii], zi = a.sz[ii];
    const float hi = (float)a.sh[ii];
    double lo[3] = {wave_min(xi), wave_min(yi), wave_min(zi)};
    double up[3] = {wave_max(xi), wave_max(yi), wave_max(zi)};
    const double hg = wave_max(a.sh[ii]);
    float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    float px = 0.f, py = 0.f, pz = 0.f, pp = 0.f;
    int pending = 0, n_cell = 0, n_part = 0;
    int p = 0;
    while (p < a.n_cells) {
        const CellRec r = a.cells[p];
        // every lane evaluates the same FP64 test on the same data
        const int acc = __builtin_amdgcn_readfirstlane(accept_cell(r, lo, up, hg, a.theta2, a.pc.L) ? 1 : 0);
        if (acc) {
            SrcRec src;
            src.x = r.cx;
            src.y = r.cy;
            src.z = r.cz;
            src.m = (float)r.mass;
            src.h = (float)r.hmax;
            table_pair<ORDER, false, COMPLETE>(a.tv, a.pc, xi, yi, zi, hi, src, false, active, px, py, pz, pp);
            if (QUAD) quadrupole_term(r, xi, yi, zi, a.pc, px, py, pz);
            ++n_cell;
            if (++pending == 16) {
                kahan_add(sx, cx, px);
                kahan_add(sy, cy, py);
                kahan_add(sz, cz, pz);
                px = py = pz = 0.f;
                pending = 0;
            }
            p = __builtin_amdgcn_readfirstlane(r.skip);
        } else if (__builtin_amdgcn_readfirstlane(r.leaf)) {
            const int e = r.start + r.count;
            for (int j = r.start; j < e; ++j) {
                SrcRec src;
                src.x = a.sx[j];
                src.y = a.sy[j];
                src.z = a.sz[j];
                src.m = (float)a.sm[j];
                src.h = (float)a.sh[j];
                table_pair<ORDER, false, COMPLETE>(a.tv, a.pc, xi, yi, zi, hi, src, j == i, active, px, py, pz, pp);
            }
            n_part += r.count;
            kahan_add(sx, cx, px);
            kahan_add(sy, cy, py);
            kahan_add(sz, cz, pz);
            px = py = pz = 0.f;
            pending = 0;
            p = __builtin_amdgcn_readfirstlane(r.skip);
        } else {
            ++p;
        }
    }
    kahan_add(sx, cx, px);
    kahan_add(sy, cy, py);
    kahan_add(sz, cz, pz);
    if (lane == 0) {
        a.wave_cells[wave] = n_cell;
        a.wave_parts[wave] = n_part;
    }
    if (!active) return;
    // acceleration in the rotated frame (the sums carry the opposite sign)
    double gx = -(double)(sx - cx), gy = -(double)(sy - cy);
    const float gz = -(sz - cz);
    if (a.n_bins > 0) {  // radial correction, linear between bin centres
        const double rho = sqrt(xi * xi + yi * yi);
        if (rho > 0.0) {
            const double t = rho / a.corr_step - 0.5;
            double dlt;
            if (t <= 0.0) {
                dlt = a.corr[0];
            } else if (t >= a.n_bins - 1) {
                dlt = a.corr[a.n_bins - 1];
            } else {
                const int k = (int)t;
                const double fr = t - k;
                dlt = (1.0 - fr) * a.corr[k] + fr * a.corr[k + 1];
            }
            gx -= dlt * xi / rho;
            gy -= dlt * yi / rho;
        }
    }
    const int o = a.idx[i];
    a.ax[o] = (float)(a.c * gx + a.s * gy);
    a.ay[o] = (float)(-a.s * gx + a.c * gy);
    a.az[o] = gz;
}

// ---------------------------------------------------------------- calibration
// per-bin sum and count of the radial error, one block per bin (fixed order)
__global__ __launch_bounds__(kBlock) void radial_bins_kernel(const double *pos, const float *at, const float *ad,
                                                             int N, double rdom, int n_bins, double *sum,
                                                             double *cnt) {
    __shared__ double s_sum[kBlock], s_cnt[kBlock];
    const int b = blockIdx.x;
    double su = 0.0, cn = 0.0;
    for (int i = threadIdx.x; i < N; i += kBlock) {
        const double x = pos[i], y = pos[N + i];
        const double rho = sqrt(x * x + y * y);
        int k = (int)floor(rho / rdom * n_bins);
        k = k < 0 ? 0 : (k > n_bins - 1 ? n_bins - 1 : k);
        if (k != b) continue;
        if (rho > 0.0) {
            const double ex = (double)at[i] - (double)ad[i], ey = (double)at[N + i] - (double)ad[N + i];
            su += (ex * x + ey * y) / rho;
        }
        cn += 1.0;
    }
    s_sum[threadIdx.x] = su;
    s_cnt[threadIdx.x] = cn;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sum[b] += s_sum[0];
        cnt[b] += s_cnt[0];
    }
}

__global__ void zero_kernel(double *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

#define TRY(x)                                                   \
    do {                                                         \
        hipError_t e_ = (x);                                     \
        if (e_ != hipSuccess) return hip_status(e_, #x);         \
    } while (0)

int build(steps_cyl_tree *t, const double *pos, const double *mass, const double *eps, int64_t N, double L,
          double R_dom, double shift, double angle, hipStream_t stream, Frame &f, double &side) {
    const int n = (int)N;
    TRY(ensure_particles(t, N));
    TRY(ensure_cells(t, N / 2 + 64, stream));
    side = 2.0 * std::fmax(L, 2.0 * R_dom);
    f.c = std::cos(angle);
    f.s = std::sin(angle);
    f.shift = shift;
    f.L = L;
    f.lo[0] = -0.5 * side;
    f.lo[1] = -0.5 * side;
    f.lo[2] = 0.5 * L - 0.5 * side;
    f.scale = (double)(1 << kLevels) / side;
    hipLaunchKernelGGL(keys_kernel, dim3(blocks(N)), dim3(kBlock), 0, stream, pos, N, f, t->tx, t->ty, t->tz,
                       t->key_in, t->idx_in);
    TRY(hipGetLastError());
    size_t bytes = t->cub_bytes;
    TRY(rocprim::radix_sort_pairs(t->cub_tmp, bytes, t->key_in, t->key_out, t->idx_in, t->idx_out, n, 0, 63,
                                           stream));
    const int root_leaf = (n <= t->leaf_size) ? 1 : 0;
    hipLaunchKernelGGL(gather_kernel, dim3(blocks(N)), dim3(kBlock), 0, stream, t->idx_out, n, t->tx, t->ty, t->tz,
                       mass, eps, t->sx, t->sy, t->sz, t->sm, t->sh, t->act, 1 - root_leaf);
    TRY(hipGetLastError());
    // level 0: the root
    const int root[4] = {0, n, 0, root_leaf};
    TRY(hipMemcpyAsync(t->c_start, &root[0], sizeof(int), hipMemcpyHostToDevice, stream));
    TRY(hipMemcpyAsync(t->c_count, &root[1], sizeof(int), hipMemcpyHostToDevice, stream));
    TRY(hipMemcpyAsync(t->c_level, &root[2], sizeof(int), hipMemcpyHostToDevice, stream));
    TRY(hipMemcpyAsync(t->c_leaf, &root[3], sizeof(int), hipMemcpyHostToDevice, stream));
    std::vector<int> off(1, 0), cnt(1, 1);
    int total = 1;
    bool open = !root_leaf;
    for (int level = 1; level <= kLevels && open; ++level) {
        const int sh = 3 * (kLevels - level);
        hipLaunchKernelGGL(flags_kernel, dim3(blocks(N)), dim3(kBlock), 0, stream, t->key_out, t->act, n, sh, t->fs,
                           t->fe);
        TRY(hipGetLastError());
        bytes = t->cub_bytes;
        TRY(rocprim::inclusive_scan(t->cub_tmp, bytes, t->fs, t->ss, (size_t)(n), rocprim::plus<int>(), stream));
        bytes = t->cub_bytes;
        TRY(rocprim::inclusive_scan(t->cub_tmp, bytes, t->fe, t->se, (size_t)(n), rocprim::plus<int>(), stream));
        int m = 0;
        TRY(hipMemcpyAsync(&m, t->ss + (n - 1), sizeof(int), hipMemcpyDeviceToHost, stream));
        TRY(hipStreamSynchronize(stream));
        if (m == 0) break;
        if ((int64_t)total + m > ((int64_t)1 << 30))
            return fail(STEPS_EINVAL, "more than 2^30 tree cells (coincident particles?)");
        TRY(ensure_cells(t, (int64_t)total + m, stream));
        hipLaunchKernelGGL(compact_kernel, dim3(blocks(N)), dim3(kBlock), 0, stream, t->fs, t->fe, t->ss, t->se, n,
                           total, t->c_start, t->c_count);
        hipLaunchKernelGGL(cells_kernel, dim3(blocks(m)), dim3(kBlock), 0, stream, total, m, level, t->leaf_size,
                           t->c_start, t->c_count, t->c_level, t->c_leaf);
        hipLaunchKernelGGL(activity_kernel, dim3(blocks(N)), dim3(kBlock), 0, stream, t->act, t->ss, n, total,
                           t->c_leaf);
        TRY(hipGetLastError());
        off.push_back(total);
        cnt.push_back(m);
        total += m;
        // any cell of this level still open?
        int any = 0;
        if (level < kLevels) {
            bytes = t->cub_bytes;
            TRY(rocprim::inclusive_scan(t->cub_tmp, bytes, t->act, t->fs, (size_t)(n), rocprim::plus<int>(), stream));
            TRY(hipMemcpyAsync(&any, t->fs + (n - 1), sizeof(int), hipMemcpyDeviceToHost, stream));
            TRY(hipStreamSynchronize(stream));
        }
        open = any > 0;
    }
    // moments bottom-up
    const int n_lev = (int)off.size();
    for (int l = n_lev - 1; l >= 0; --l) {
        const int co = (l + 1 < n_lev) ? off[l + 1] : 0, cn = (l + 1 < n_lev) ? cnt[l + 1] : 0;
        hipLaunchKernelGGL(moments_kernel, dim3(blocks(cnt[l])), dim3(kBlock), 0, stream, off[l], cnt[l], co, cn,
                           t->c_start, t->c_count, t->c_leaf, t->c_m, t->c_mx, t->c_my, t->c_mz, t->c_h, t->sx, t->sy,
                           t->sz, t->sm, t->sh);
        TRY(hipGetLastError());
        if (t->quadrupole) {
            hipLaunchKernelGGL(quadrupole_kernel, dim3(blocks(cnt[l])), dim3(kBlock), 0, stream, off[l], cnt[l], co,
                               cn, (int)t->cap_cells, t->c_start, t->c_count, t->c_leaf, t->c_m, t->c_mx, t->c_my,
                               t->c_mz, t->c_q, t->sx, t->sy, t->sz, t->sm);
            TRY(hipGetLastError());
        }
    }
    // depth-first order and skip links
    hipLaunchKernelGGL(dfs_keys_kernel, dim3(blocks(total)), dim3(kBlock), 0, stream, total, t->c_start, t->c_level,
                       t->c_key_in, t->c_id_in);
    TRY(hipGetLastError());
    bytes = t->cub_bytes;
    TRY(rocprim::radix_sort_pairs(t->cub_tmp, bytes, t->c_key_in, t->c_key_out, t->c_id_in, t->c_id_out,
                                           total, 0, 37, stream));
    hipLaunchKernelGGL(dfs_cells_kernel, dim3(blocks(total)), dim3(kBlock), 0, stream, total, n, t->c_key_out,
                       t->c_id_out, t->c_start, t->c_count, t->c_level, t->c_leaf, t->c_m, t->c_mx, t->c_my, t->c_mz,
                       t->c_h, t->c_q, (int)t->cap_cells, t->quadrupole, t->key_out, f, side, t->cells,
                       t->cell_level);
    TRY(hipGetLastError());
    // target groups
    hipLaunchKernelGGL(group_count_kernel, dim3(blocks(total)), dim3(kBlock), 0, stream, t->cells, total, t->g_cnt);
    TRY(hipGetLastError());
    bytes = t->cub_bytes;
    TRY(rocprim::inclusive_scan(t->cub_tmp, bytes, t->g_cnt, t->g_off, (size_t)(total), rocprim::plus<int>(), stream));
    hipLaunchKernelGGL(group_write_kernel, dim3(blocks(total)), dim3(kBlock), 0, stream, t->cells, total, t->g_cnt,
                       t->g_off, t->g_start, t->g_count);
    TRY(hipGetLastError());
    int ng = 0;
    TRY(hipMemcpyAsync(&ng, t->g_off + (total - 1), sizeof(int), hipMemcpyDeviceToHost, stream));
    TRY(hipStreamSynchronize(stream));
    t->n_groups = ng;
    t->n_cells = total;
    t->n = N;
    return STEPS_OK;
}

int walk(steps_cyl_tree *t, const steps_cyl_table *table, int order, double L, double theta, const Frame &f,
         bool correct, float *out_acc, hipStream_t stream) {
    WalkArgs a;
    a.cells = t->cells;
    a.sx = t->sx;
    a.sy = t->sy;
    a.sz = t->sz;
    a.sm = t->sm;
    a.sh = t->sh;
    a.idx = t->idx_out;
    a.g_start = t->g_start;
    a.g_count = t->g_count;
    a.n_groups = (int)t->n_groups;
    a.ax = out_acc;
    a.ay = out_acc + t->n;
    a.az = out_acc + 2 * t->n;
    a.wave_cells = t->wave_cells;
    a.wave_parts = t->wave_parts;
    a.corr = t->corr;
    a.tv = table_view(table);
    a.pc = period_consts(L);
    a.theta2 = theta * theta;
    a.c = f.c;
    a.s = f.s;
    a.n_bins = correct ? t->n_bins : 0;
    a.corr_step = t->n_bins ? t->corr_rdom / t->n_bins : 1.0;
    a.N = (int)t->n;
    a.n_cells = (int)t->n_cells;
    const int64_t threads = t->n_groups * 64;
    const dim3 grid(blocks(threads)), block(kBlock);
    const int variant = (order == 2 ? 4 : 0) + (t->quadrupole ? 2 : 0) + (a.tv.complete ? 1 : 0);
    switch (variant) {
        case 0: hipLaunchKernelGGL((tree_walk_kernel<1, false, false>), grid, block, 0, stream, a); break;
        case 1: hipLaunchKernelGGL((tree_walk_kernel<1, false, true>), grid, block, 0, stream, a); break;
        case 2: hipLaunchKernelGGL((tree_walk_kernel<1, true, false>), grid, block, 0, stream, a); break;
        case 3: hipLaunchKernelGGL((tree_walk_kernel<1, true, true>), grid, block, 0, stream, a); break;
        case 4: hipLaunchKernelGGL((tree_walk_kernel<2, false, false>), grid, block, 0, stream, a); break;
        case 5: hipLaunchKernelGGL((tree_walk_kernel<2, false, true>), grid, block, 0, stream, a); break;
        case 6: hipLaunchKernelGGL((tree_walk_kernel<2, true, false>), grid, block, 0, stream, a); break;
        default: hipLaunchKernelGGL((tree_walk_kernel<2, true, true>), grid, block, 0, stream, a); break;
    }
    return hip_status(hipGetLastError(), "tree walk");
}

int check_common(const double *pos, const double *mass, const double *eps, int64_t N, double L, double R_dom,
                 const steps_cyl_table *table, int order, double theta) {
    if (!pos || !mass || !eps || !table) return fail(STEPS_EINVAL, "pos, mass, eps and table must be non-null");
    if (N < 1 || N > STEPS_MAX_N) return fail(STEPS_EINVAL, "N=%lld outside [1, 2^29]", (long long)N);
    if (!finite_positive(L) || !finite_positive(R_dom)) return fail(STEPS_EINVAL, "L and R_dom must be finite and > 0");
    if (order != 1 && order != 2) return fail(STEPS_EINVAL, "order=%d: 1 (CIC) or 2 (TSC)", order);
    if (!std::isfinite(theta) || theta < 0.0) return fail(STEPS_EINVAL, "theta must be finite and >= 0");
    return STEPS_OK;
}

}  // namespace
}  // namespace steps

using namespace steps;

STEPS_API int steps_cyl_tree_create(int leaf_size, int quadrupole, steps_cyl_tree **out) {
    if (!out) return fail(STEPS_EINVAL, "out must be non-null");
    if (leaf_size < 1 || leaf_size > 64) return fail(STEPS_EINVAL, "leaf_size=%d outside [1, 64]", leaf_size);
    if (quadrupole != 0 && quadrupole != 1) return fail(STEPS_EINVAL, "quadrupole must be 0 or 1");
    clear_error();
    steps_cyl_tree *t = new (std::nothrow) steps_cyl_tree();
    if (!t) return fail(STEPS_ENOMEM, "out of host memory");
    t->leaf_size = leaf_size;
    t->quadrupole = quadrupole;
    *out = t;
    return STEPS_OK;
}

STEPS_API void steps_cyl_tree_destroy(steps_cyl_tree *t) {
    if (!t) return;
    void *ptrs[] = {t->cub_tmp, t->tx, t->ty, t->tz, t->key_in, t->key_out, t->idx_in, t->idx_out, t->sx, t->sy,
                    t->sz, t->sm, t->sh, t->act, t->fs, t->fe, t->ss, t->se, t->c_start, t->c_count, t->c_level,
                    t->c_leaf, t->c_m, t->c_mx, t->c_my, t->c_mz, t->c_h, t->c_q, t->c_key_in, t->c_key_out, t->c_id_in,
                    t->c_id_out, t->cells, t->cell_level, t->wave_cells, t->wave_parts, t->corr, t->bin_sum,
                    t->g_cnt, t->g_off, t->g_start, t->g_count,
                    t->bin_cnt, t->acc_dir, t->acc_tree};
    for (void *p : ptrs) (void)hipFree(p);
    delete t;
}

STEPS_API int steps_cyl_tree_forces(steps_cyl_tree *t, const double *pos, const double *mass, const double *eps,
                                    int64_t N, double L, double R_dom, const steps_cyl_table *table, int order,
                                    double theta, double shift, double angle, int correct, float *out_acc,
                                    hipStream_t stream) {
    if (!t || !out_acc) return fail(STEPS_EINVAL, "tree and out_acc must be non-null");
    int rc = check_common(pos, mass, eps, N, L, R_dom, table, order, theta);
    if (rc) return rc;
    if (!std::isfinite(shift) || !std::isfinite(angle)) return fail(STEPS_EINVAL, "shift and angle must be finite");
    if (correct && t->n_bins == 0) return fail(STEPS_EINVAL, "no radial correction has been set");
    if ((rc = require_device())) return rc;
    clear_error();
    Frame f;
    double side;
    if ((rc = build(t, pos, mass, eps, N, L, R_dom, shift, angle, stream, f, side))) return rc;
    return walk(t, table, order, L, theta, f, correct != 0, out_acc, stream);
}

STEPS_API int steps_cyl_tree_set_correction(steps_cyl_tree *t, const double *corr, int n_bins, double R_dom) {
    if (!t) return fail(STEPS_EINVAL, "tree must be non-null");
    if (n_bins == 0) {
        clear_error();
        t->n_bins = 0;
        return STEPS_OK;
    }
    if (!corr || n_bins < 1 || n_bins > kMaxBins || !finite_positive(R_dom))
        return fail(STEPS_EINVAL, "need corr, 1 <= n_bins <= %d and R_dom > 0", kMaxBins);
    for (int k = 0; k < n_bins; ++k)
        if (!std::isfinite(corr[k])) return fail(STEPS_EINVAL, "non-finite correction");
    int rc = require_device();
    if (rc) return rc;
    clear_error();
    if (!t->corr) STEPS_CHECK_HIP(hipMalloc(&t->corr, kMaxBins * sizeof(double)));
    STEPS_CHECK_HIP(hipMemcpy(t->corr, corr, n_bins * sizeof(double), hipMemcpyHostToDevice));
    t->n_bins = n_bins;
    t->corr_rdom = R_dom;
    return STEPS_OK;
}

STEPS_API int steps_cyl_tree_calibrate(steps_cyl_tree *t, const double *pos, const double *mass, const double *eps,
                                       int64_t N, double L, double R_dom, const steps_cyl_table *table, int order,
                                       double theta, const double *shifts, const double *angles, int n_real,
                                       int n_bins, double *out_corr, hipStream_t stream) {
    if (!t || !shifts || !angles) return fail(STEPS_EINVAL, "tree, shifts and angles must be non-null");
    int rc = check_common(pos, mass, eps, N, L, R_dom, table, order, theta);
    if (rc) return rc;
    if (n_real < 1 || n_real > 1024) return fail(STEPS_EINVAL, "n_real=%d outside [1, 1024]", n_real);
    if (n_bins < 1 || n_bins > kMaxBins) return fail(STEPS_EINVAL, "n_bins=%d outside [1, %d]", n_bins, kMaxBins);
    for (int k = 0; k < n_real; ++k)
        if (!std::isfinite(shifts[k]) || !std::isfinite(angles[k]))
            return fail(STEPS_EINVAL, "shifts and angles must be finite");
    if ((rc = require_device())) return rc;
    clear_error();
    if (N > t->cap_cal) {
        (void)hipFree(t->acc_dir);
        (void)hipFree(t->acc_tree);
        t->acc_dir = t->acc_tree = nullptr;
        t->cap_cal = 0;
        STEPS_CHECK_HIP(hipMalloc(&t->acc_dir, 3 * N * sizeof(float)));
        STEPS_CHECK_HIP(hipMalloc(&t->acc_tree, 3 * N * sizeof(float)));
        t->cap_cal = N;
    }
    if (!t->bin_sum) {
        STEPS_CHECK_HIP(hipMalloc(&t->bin_sum, kMaxBins * sizeof(double)));
        STEPS_CHECK_HIP(hipMalloc(&t->bin_cnt, kMaxBins * sizeof(double)));
    }
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(kBlock), 0, stream, t->bin_sum, kMaxBins);
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(kBlock), 0, stream, t->bin_cnt, kMaxBins);
    STEPS_CHECK_HIP(hipGetLastError());
    rc = steps_cyl_forces_table(pos, mass, eps, N, L, table, order, nullptr, N, t->acc_dir, nullptr, stream);
    if (rc) return rc;
    for (int k = 0; k < n_real; ++k) {
        Frame f;
        double side;
        if ((rc = build(t, pos, mass, eps, N, L, R_dom, shifts[k], angles[k], stream, f, side))) return rc;
        if ((rc = walk(t, table, order, L, theta, f, false, t->acc_tree, stream))) return rc;
        hipLaunchKernelGGL(radial_bins_kernel, dim3(n_bins), dim3(kBlock), 0, stream, pos, t->acc_tree, t->acc_dir,
                           (int)N, R_dom, n_bins, t->bin_sum, t->bin_cnt);
        STEPS_CHECK_HIP(hipGetLastError());
    }
    std::vector<double> s(n_bins), c(n_bins), corr(n_bins);
    STEPS_CHECK_HIP(hipMemcpyAsync(s.data(), t->bin_sum, n_bins * sizeof(double), hipMemcpyDeviceToHost, stream));
    STEPS_CHECK_HIP(hipMemcpyAsync(c.data(), t->bin_cnt, n_bins * sizeof(double), hipMemcpyDeviceToHost, stream));
    STEPS_CHECK_HIP(hipStreamSynchronize(stream));
    for (int k = 0; k < n_bins; ++k) corr[k] = c[k] > 0.0 ? s[k] / c[k] : 0.0;
    if (out_corr)
        for (int k = 0; k < n_bins; ++k) out_corr[k] = corr[k];
    return steps_cyl_tree_set_correction(t, corr.data(), n_bins, R_dom);
}

STEPS_API int steps_cyl_tree_info(const steps_cyl_tree *t, int64_t *n_cells, int64_t *cell_interactions,
                                  int64_t *particle_interactions) {
    if (!t) return fail(STEPS_EINVAL, "tree must be non-null");
    clear_error();
    if (n_cells) *n_cells = t->n_cells;
    if (cell_interactions || particle_interactions) {
        const int64_t waves = t->n_groups;
        std::vector<int> wc(waves), wp(waves), gc(waves);
        if (waves) {
            STEPS_CHECK_HIP(hipMemcpy(wc.data(), t->wave_cells, waves * sizeof(int), hipMemcpyDeviceToHost));
            STEPS_CHECK_HIP(hipMemcpy(wp.data(), t->wave_parts, waves * sizeof(int), hipMemcpyDeviceToHost));
            STEPS_CHECK_HIP(hipMemcpy(gc.data(), t->g_count, waves * sizeof(int), hipMemcpyDeviceToHost));
        }
        int64_t sc = 0, sp = 0;
        for (int64_t w = 0; w < waves; ++w) {
            sc += (int64_t)gc[w] * wc[w];
            sp += (int64_t)gc[w] * wp[w];
        }
        if (cell_interactions) *cell_interactions = sc;
        if (particle_interactions) *particle_interactions = sp;
    }
    return STEPS_OK;
}

STEPS_API int steps_cyl_tree_cells(const steps_cyl_tree *t, int *host_level, int *host_start, int *host_count,
                                   int *host_skip, int *host_leaf, double *host_mass, double *host_com,
                                   int *host_order) {
    if (!t) return fail(STEPS_EINVAL, "tree must be non-null");
    clear_error();
    const int64_t n = t->n_cells;
    std::vector<CellRec> r(n);
    if (n) STEPS_CHECK_HIP(hipMemcpy(r.data(), t->cells, n * sizeof(CellRec), hipMemcpyDeviceToHost));
    if (host_level && n) STEPS_CHECK_HIP(hipMemcpy(host_level, t->cell_level, n * sizeof(int), hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < n; ++k) {
        if (host_start) host_start[k] = r[k].start;
        if (host_count) host_count[k] = r[k].count;
        if (host_skip) host_skip[k] = r[k].skip;
        if (host_leaf) host_leaf[k] = r[k].leaf;
        if (host_mass) host_mass[k] = r[k].mass;
        if (host_com) {
            host_com[k] = r[k].cx;
            host_com[n + k] = r[k].cy;
            host_com[2 * n + k] = r[k].cz;
        }
    }
    if (host_order && t->n)
        STEPS_CHECK_HIP(hipMemcpy(host_order, t->idx_out, t->n * sizeof(int), hipMemcpyDeviceToHost));
    return STEPS_OK;
}
