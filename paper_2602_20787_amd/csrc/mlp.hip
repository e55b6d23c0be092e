// The far-image correction network on gfx950: parameter packing, forward
// evaluation, training-sample generation, a fused forward+backward training
// kernel on BF16 MFMA (FP32 accumulation), a deterministic gradient
// reduction with Adam, and the C entry points of the network handle.
//
// Precision: the network keeps FP32 master weights.  Every evaluation uses
// the weights rounded to BF16; layers 2-4 run on MFMA with BF16 inputs and
// FP32 accumulation; layer 1 on MFMA with its FP32 inputs split exactly into
// three BF16 parts (an FP32 layer); layer 5 and all activations in FP32 on
// the VALU.
// The backward pass feeds MFMA with BF16 copies of the pre-activation
// gradients (dW = dZ X^T, dX = W^T dZ); bias gradients and the layer 1 and 5
// gradients stay FP32.  BF16 roundings are treated as the identity in the
// backward pass.
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.h"
#include "learned_model.h"
#include "mlp_device.h"
#include "pair_f64.h"

struct steps_cyl_mlp {
    float *master = nullptr;           // [kParams] FP32
    float *adam_m = nullptr;           // [kParams]
    float *adam_v = nullptr;           // [kParams]
    steps::mlp::Packed *packed = nullptr;
    steps::mlp::PackedT *packedT = nullptr;
    int64_t adam_t = 0;                // Adam steps taken
    int device = 0;
};

namespace steps {
namespace mlp {

namespace {

// ---------------------------------------------------------------- packing
// One thread per parameter: writes its BF16-rounded copies into the packed
// forward and backward layouts.
// lane half and position of feature r in the D layout: r = 32b + 8(v/4) + 4h + v%4
__device__ __forceinline__ void dpos(int r, int &b, int &v, int &h) {
    b = r >> 5;
    const int rem = r & 31;
    h = (rem >> 2) & 1;
    v = 4 * (rem >> 3) + (rem & 3);
}

// K slot of feature i: i = phi(16t + 8h + e)
__device__ __forceinline__ void kpos(int i, int &t, int &h, int &e) {
    t = i >> 4;
    const int rem = i & 15;
    h = (rem >> 2) & 1;
    e = 4 * (rem >> 3) + (rem & 3);
}

__device__ void pack_one(int p, float w, Packed *P, PackedT *PT) {
    if (p < OFF_B1) {
        // W1[r][c]: row r of the layer-1 A fragment, K slots 3c .. 3c+2
        const int r = p >> 1, c = p & 1;
        __bf16 *q = reinterpret_cast<__bf16 *>(&P->A1[r >> 5][r & 31]);
        q[3 * c] = q[3 * c + 1] = q[3 * c + 2] = (__bf16)w;
    } else if (p < OFF_W[0]) {
        int b, v, h;
        dpos(p - OFF_B1, b, v, h);
        P->Bias1[h][b][v] = w;
    } else if (p < OFF_W5) {
        int k = 0;
        while (k < 2 && p >= OFF_W[k + 1]) ++k;
        const int q = p - OFF_W[k];
        if (q >= 4096) {  // bias of layer k+2
            int b, v, h;
            dpos(q - 4096, b, v, h);
            P->Bias[h][k][b][v] = w;
            return;
        }
        const int o = q / 64, i = q % 64;  // W[o][i]
        {   // forward fragment: row o of M block o/32, K slot with phi = i
            int t, h, e;
            kpos(i, t, h, e);
            const int lane = (o & 31) + 32 * h;
            reinterpret_cast<__bf16 *>(&P->A[k][o >> 5][t][lane])[e] = (__bf16)w;
        }
        {   // backward fragment of W^T: row i of M block i/32, K slot with phi = o
            int t, h, e;
            kpos(o, t, h, e);
            const int lane = (i & 31) + 32 * h;
            reinterpret_cast<__bf16 *>(&PT->AT[k][i >> 5][t][lane])[e] = (__bf16)w;
        }
    } else if (p < OFF_B5) {
        const int c = (p - OFF_W5) / 64, r = (p - OFF_W5) % 64;
        int b, v, h;
        dpos(r, b, v, h);
        reinterpret_cast<float *>(&P->W5[h][b][v])[c] = (float)(__bf16)w;
    } else {
        P->b5[p - OFF_B5] = w;
    }
}

__global__ void pack_kernel(const float *master, Packed *P, PackedT *PT) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kParams) pack_one(p, master[p], P, PT);
    if (p < 2) P->b5[2 + p] = 0.f;
}

// ---------------------------------------------------------------- forward
__global__ __launch_bounds__(256) void forward_kernel(const Packed *__restrict__ Pg,
                                                      const float *__restrict__ in, float *__restrict__ out,
                                                      int64_t B) {
    __shared__ Packed P;
    load_packed(&P, Pg);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t s = ((int64_t)blockIdx.x * 4 + wave) * 32 + (lane & 31);
    const bool ok = s < B;
    const float f1 = ok ? in[s] : 0.f, f2 = ok ? in[B + s] : 0.f;
    float o0, o1;
    forward32<false>(P, f1, f2, o0, o1, nullptr, nullptr);
    if (ok && lane < 32) {
        out[s] = o0;
        out[B + s] = o1;
    }
}

// ---------------------------------------------------------------- training data
// Exact image band 2 <= |n| <= 1024 in FP64 for samples (delta, r) in units
// of L; writes features F[2][n] and targets T[2][n] = (R - baseline) / s.
__device__ __forceinline__ double rsqrt_f64(double x) {
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    y = y * (1.5 - 0.5 * x * y * y);
    y = y * (1.5 - 0.5 * x * y * y);
    return y * (1.5 - 0.5 * x * y * y);
}

__global__ __launch_bounds__(256) void samples_kernel(const double *__restrict__ in, int64_t n,
                                                      float *__restrict__ F, float *__restrict__ T) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double delta = in[k], r = in[n + k];
    double Rz = 0.0, Rr = 0.0;
    const double r2 = r * r;
    for (int q = kFarImages; q >= 2; --q) {  // ascending |n| would add large terms last
        const double up = delta - (double)q, um = delta + (double)q;
        const double ip = rsqrt_f64(up * up + r2), im = rsqrt_f64(um * um + r2);
        const double ip3 = ip * ip * ip, im3 = im * im * im;
        Rz += -up * ip3 - um * im3;
        Rr += -r * (ip3 + im3);
    }
    double bz, br;
    baseline_f64(delta, r, bz, br);
    const double s = (double)kOutScale / (1.0 + r2);
    float f1, f2;
    features_f32((float)delta, (float)r, f1, f2);
    F[k] = f1;
    F[n + k] = f2;
    T[k] = (float)((Rz - bz) / s);
    T[n + k] = (float)((Rr - br) / s);
}

// ---------------------------------------------------------------- training
// Sample index of batch slot k at step `step` of a permuted pass over n
// samples: an affine bijection modulo n (n a power of two, odd multiplier).
__device__ __forceinline__ int64_t batch_index(int64_t k, int64_t base, uint64_t mul, uint64_t add,
                                               int64_t n) {
    const uint64_t pos = (uint64_t)(base + k);
    return (int64_t)((pos * mul + add) & (uint64_t)(n - 1));
}

struct TrainArgs {
    const Packed *P;
    const PackedT *PT;
    const float *F, *T;     // features / targets [2][n]
    int64_t n;              // samples available
    int64_t count;          // samples in this batch
    int64_t base;           // first batch slot (for the permutation)
    uint64_t mul, add;      // permutation; mul = 0 selects identity (slot k -> sample k)
    float *partial;         // [waves][kParams] gradient partials
    float *loss_partial;    // [waves]
};

struct TrainLDS {
    float z[4][64][32];
    __bf16 x[3][64][32];
    float dzf[64][32];
    __bf16 dzb[64][32];
    float dout[2][32];
    float feat[2][32];
};

__global__ __launch_bounds__(64) void train_kernel(TrainArgs A) {
    __shared__ TrainLDS S;
    const Packed &P = *A.P;
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, col = lane & 31;
    const int64_t wave = blockIdx.x;
    const int64_t slot = wave * 32 + col;
    const bool ok = slot < A.count;
    int64_t s = 0;
    if (ok) s = A.mul ? batch_index(slot, A.base, A.mul, A.add, A.n) : slot;
    const float f1 = ok ? A.F[s] : 0.f, f2 = ok ? A.F[A.n + s] : 0.f;
    const float t0 = ok ? A.T[s] : 0.f, t1 = ok ? A.T[A.n + s] : 0.f;
    float o0, o1;
    forward32<true>(P, f1, f2, o0, o1, &S.z[0][0][0], &S.x[0][0][0]);
    // loss = mean of squared errors over both outputs and all samples
    const float inv_count = 1.0f / (float)A.count;
    const float e0 = ok ? (o0 - t0) : 0.f, e1 = ok ? (o1 - t1) : 0.f;
    const float d0 = e0 * inv_count, d1 = e1 * inv_count;  // d loss / d o
    if (h == 0) {
        S.dout[0][col] = d0;
        S.dout[1][col] = d1;
        S.feat[0][col] = f1;
        S.feat[1][col] = f2;
    }
    // loss partial over this wave's samples (lanes of half 0)
    float l = (h == 0) ? (e0 * e0 + e1 * e1) : 0.f;
    for (int off = 32; off >= 1; off >>= 1) l += __shfl_xor(l, off);
    __syncthreads();
    float *G = A.partial + wave * (int64_t)kParams;
    if (lane == 0) A.loss_partial[wave] = l * 0.5f * inv_count;
    // layer 5: dW5[c][r] = sum_j dout_c[j] a4[r][j], db5 = sum_j dout_c[j]
    {
        const int r = lane;
        float g0 = 0.f, g1 = 0.f;
        for (int j = 0; j < 32; ++j) {
            const float a4 = silu(S.z[3][r][j]);
            g0 = __builtin_fmaf(S.dout[0][j], a4, g0);
            g1 = __builtin_fmaf(S.dout[1][j], a4, g1);
        }
        G[OFF_W5 + r] = g0;
        G[OFF_W5 + 64 + r] = g1;
        if (lane < 2) {
            float b = 0.f;
            for (int j = 0; j < 32; ++j) b += S.dout[lane][j];
            G[OFF_B5 + lane] = b;
        }
    }
    // d loss / d z4 in the D layout
    float dz[2][16];
    {
        const float dd0 = S.dout[0][col], dd1 = S.dout[1][col];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = drow(b, v, h);
                const float2 w5 = P.W5[h][b][v];
                const float da = __builtin_fmaf(w5.y, dd1, w5.x * dd0);
                dz[b][v] = da * silu_grad(S.z[3][r][col]);
            }
    }
    for (int k = 2; k >= 0; --k) {  // MFMA layers 4, 3, 2
        __syncthreads();
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = drow(b, v, h);
                S.dzf[r][col] = dz[b][v];
                S.dzb[r][col] = (__bf16)dz[b][v];
            }
        __syncthreads();
        // bias gradient: row r = lane, FP32
        {
            float g = 0.f;
            for (int j = 0; j < 32; ++j) g += S.dzf[lane][j];
            G[OFF_B[k] + lane] = g;
        }
        // dW = bf16(dZ) X^T: M = out rows, N = in rows, K = 32 samples
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
            for (int bn = 0; bn < 2; ++bn) {
                f32x16 acc = (f32x16){0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                                      0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&S.dzb[32 * bm + col][16 * ks + 8 * h]);
                    const bf16x8 bb = *reinterpret_cast<const bf16x8 *>(&S.x[k][32 * bn + col][16 * ks + 8 * h]);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int o = drow(bm, v, h), i = 32 * bn + col;
                    G[OFF_W[k] + o * 64 + i] = acc[v];
                }
            }
        // dX = W^T bf16(dZ) in the D layout of the previous layer, then through SiLU
        bf16x8 xb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int e = 0; e < 8; ++e) xb[t][e] = (__bf16)dz[t >> 1][8 * (t & 1) + e];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            f32x16 acc = (f32x16){0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                                  0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A.PT->AT[k][b][t][lane], xb[t], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = drow(b, v, h);
                dz[b][v] = acc[v] * silu_grad(S.z[k][r][col]);
            }
        }
    }
    // layer 1: dW1[r][c] = sum_j dz1[r][j] f_c[j], db1[r] = sum_j dz1[r][j]
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) S.dzf[drow(b, v, h)][col] = dz[b][v];
    __syncthreads();
    {
        const int r = lane;
        float g0 = 0.f, g1 = 0.f, gb = 0.f;
        for (int j = 0; j < 32; ++j) {
            const float d = S.dzf[r][j];
            g0 = __builtin_fmaf(d, S.feat[0][j], g0);
            g1 = __builtin_fmaf(d, S.feat[1][j], g1);
            gb += d;
        }
        G[OFF_W1 + 2 * r] = g0;
        G[OFF_W1 + 2 * r + 1] = g1;
        G[OFF_B1 + r] = gb;
    }
}

// Sums the per-wave partials in wave order (deterministic).  mode 0: write
// the gradient to `grad`; mode 1: Adam update of master/m/v and repacking.
struct ReduceArgs {
    const float *partial;
    const float *loss_partial;
    int64_t waves;
    float *grad;       // mode 0
    float *loss_out;   // mode 0 and 1 (may be null)
    float *master, *m, *v;
    Packed *P;
    PackedT *PT;
    float lr, beta1, beta2, eps, bc1, bc2;  // bc = 1 - beta^t
    int mode;
};

__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs R) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && R.loss_out) {
        float l = 0.f;
        for (int64_t w = 0; w < R.waves; ++w) l += R.loss_partial[w];
        *R.loss_out = l;
    }
    if (p >= kParams) return;
    float g = 0.f;
    for (int64_t w = 0; w < R.waves; ++w) g += R.partial[w * (int64_t)kParams + p];
    if (R.mode == 0) {
        R.grad[p] = g;
        return;
    }
    const float m = R.beta1 * R.m[p] + (1.0f - R.beta1) * g;
    const float v = R.beta2 * R.v[p] + (1.0f - R.beta2) * g * g;
    R.m[p] = m;
    R.v[p] = v;
    const float mh = m / R.bc1, vh = v / R.bc2;
    const float w = R.master[p] - R.lr * mh / (sqrtf(vh) + R.eps);
    R.master[p] = w;
    pack_one(p, w, R.P, R.PT);
}

__global__ void sumsq_loss_kernel(const float *out, const float *T, int64_t n, float *partial) {
    // per-block partial of sum (o - T)^2 over both outputs
    __shared__ float red[256];
    float acc = 0.f;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const float a = out[k] - T[k], b = out[n + k] - T[n + k];
        acc += a * a + b * b;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------- host helpers
int pack(steps_cyl_mlp *net, hipStream_t stream) {
    hipLaunchKernelGGL(pack_kernel, dim3((kParams + 255) / 256), dim3(256), 0, stream, net->master,
                       net->packed, net->packedT);
    return hip_status(hipGetLastError(), "mlp pack");
}

int launch_train(steps_cyl_mlp *net, const float *F, const float *T, int64_t n, int64_t count,
                 int64_t base, uint64_t mul, uint64_t add, float *partial, float *loss_partial,
                 hipStream_t stream) {
    TrainArgs A;
    A.P = net->packed;
    A.PT = net->packedT;
    A.F = F;
    A.T = T;
    A.n = n;
    A.count = count;
    A.base = base;
    A.mul = mul;
    A.add = add;
    A.partial = partial;
    A.loss_partial = loss_partial;
    const int64_t waves = (count + 31) / 32;
    hipLaunchKernelGGL(train_kernel, dim3((unsigned)waves), dim3(64), 0, stream, A);
    return hip_status(hipGetLastError(), "mlp train kernel");
}

int launch_reduce(steps_cyl_mlp *net, const float *partial, const float *loss_partial, int64_t waves,
                  int mode, float *grad, float *loss_out, float lr, float b1, float b2, float eps,
                  hipStream_t stream) {
    ReduceArgs R;
    R.partial = partial;
    R.loss_partial = loss_partial;
    R.waves = waves;
    R.grad = grad;
    R.loss_out = loss_out;
    R.master = net->master;
    R.m = net->adam_m;
    R.v = net->adam_v;
    R.P = net->packed;
    R.PT = net->packedT;
    R.lr = lr;
    R.beta1 = b1;
    R.beta2 = b2;
    R.eps = eps;
    R.mode = mode;
    if (mode == 1) {
        net->adam_t += 1;
        R.bc1 = (float)(1.0 - std::pow((double)b1, (double)net->adam_t));
        R.bc2 = (float)(1.0 - std::pow((double)b2, (double)net->adam_t));
    } else {
        R.bc1 = R.bc2 = 1.f;
    }
    hipLaunchKernelGGL(reduce_kernel, dim3((kParams + 255) / 256), dim3(256), 0, stream, R);
    return hip_status(hipGetLastError(), "mlp reduce kernel");
}

}  // namespace

int launch_samples(const double *in, int64_t n, float *F, float *T, hipStream_t stream) {
    hipLaunchKernelGGL(samples_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, in, n, F, T);
    return hip_status(hipGetLastError(), "mlp samples kernel");
}

int launch_forward(const steps_cyl_mlp *net, const float *in, float *out, int64_t B, hipStream_t stream) {
    const int64_t blocks = (B + 127) / 128;
    hipLaunchKernelGGL(forward_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, net->packed, in, out, B);
    return hip_status(hipGetLastError(), "mlp forward kernel");
}

const Packed *packed_of(const steps_cyl_mlp *net) { return net->packed; }

// ---------------------------------------------------------------- entry points
namespace {

int alloc_net(steps_cyl_mlp **out) {
    steps_cyl_mlp *net = new (std::nothrow) steps_cyl_mlp();
    if (!net) return fail(STEPS_ENOMEM, "out of host memory");
    hipError_t e;
    if ((e = hipGetDevice(&net->device)) != hipSuccess ||
        (e = hipMalloc(&net->master, kParams * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&net->adam_m, kParams * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&net->adam_v, kParams * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&net->packed, sizeof(Packed))) != hipSuccess ||
        (e = hipMalloc(&net->packedT, sizeof(PackedT))) != hipSuccess) {
        (void)hipFree(net->master);
        (void)hipFree(net->adam_m);
        (void)hipFree(net->adam_v);
        (void)hipFree(net->packed);
        (void)hipFree(net->packedT);
        delete net;
        return fail(STEPS_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    *out = net;
    return STEPS_OK;
}

int upload_params(steps_cyl_mlp *net, const float *host) {
    STEPS_CHECK_HIP(hipMemcpy(net->master, host, kParams * sizeof(float), hipMemcpyHostToDevice));
    STEPS_CHECK_HIP(hipMemset(net->adam_m, 0, kParams * sizeof(float)));
    STEPS_CHECK_HIP(hipMemset(net->adam_v, 0, kParams * sizeof(float)));
    STEPS_CHECK_HIP(hipMemset(net->packed, 0, sizeof(Packed)));
    STEPS_CHECK_HIP(hipMemset(net->packedT, 0, sizeof(PackedT)));
    net->adam_t = 0;
    int rc = pack(net, 0);
    if (rc) return rc;
    STEPS_CHECK_HIP(hipDeviceSynchronize());
    return STEPS_OK;
}

bool finite_params(const float *p) {
    for (int i = 0; i < kParams; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

constexpr char kMagic[8] = {'S', 'C', 'Y', 'L', 'M', 'L', 'P', '1'};
constexpr uint32_t kFormatVersion = 1;

uint64_t fnv1a(const void *data, size_t n) {
    const unsigned char *p = static_cast<const unsigned char *>(data);
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace
}  // namespace mlp
}  // namespace steps

using namespace steps;
using namespace steps::mlp;

STEPS_API int steps_cyl_mlp_create(const float *init_params, steps_cyl_mlp **out) {
    if (!init_params || !out) return fail(STEPS_EINVAL, "init_params and out must be non-null");
    if (!finite_params(init_params)) return fail(STEPS_EINVAL, "init_params holds a non-finite value");
    int rc = require_device();
    if (rc) return rc;
    clear_error();
    steps_cyl_mlp *net = nullptr;
    if ((rc = alloc_net(&net))) return rc;
    if ((rc = upload_params(net, init_params))) {
        steps_cyl_mlp_destroy(net);
        return rc;
    }
    *out = net;
    return STEPS_OK;
}

STEPS_API void steps_cyl_mlp_destroy(steps_cyl_mlp *net) {
    if (!net) return;
    (void)hipFree(net->master);
    (void)hipFree(net->adam_m);
    (void)hipFree(net->adam_v);
    (void)hipFree(net->packed);
    (void)hipFree(net->packedT);
    delete net;
}

STEPS_API int steps_cyl_mlp_get_params(const steps_cyl_mlp *net, float *host_out) {
    if (!net || !host_out) return fail(STEPS_EINVAL, "net and host_out must be non-null");
    clear_error();
    STEPS_CHECK_HIP(hipMemcpy(host_out, net->master, kParams * sizeof(float), hipMemcpyDeviceToHost));
    return STEPS_OK;
}

STEPS_API int steps_cyl_mlp_set_params(steps_cyl_mlp *net, const float *host_params) {
    if (!net || !host_params) return fail(STEPS_EINVAL, "net and host_params must be non-null");
    if (!finite_params(host_params)) return fail(STEPS_EINVAL, "params hold a non-finite value");
    clear_error();
    return upload_params(net, host_params);
}

STEPS_API int steps_cyl_mlp_forward(const steps_cyl_mlp *net, const float *in, float *out, int64_t B,
                                    hipStream_t stream) {
    if (!net || !in || !out) return fail(STEPS_EINVAL, "net, in and out must be non-null");
    if (B < 1 || B > ((int64_t)1 << 40)) return fail(STEPS_EINVAL, "B=%lld out of range", (long long)B);
    clear_error();
    return launch_forward(net, in, out, B, stream);
}

STEPS_API int steps_cyl_mlp_grad(const steps_cyl_mlp *net, const float *in, const float *target, int64_t B,
                                 float *grad_out, float *loss_out, hipStream_t stream) {
    if (!net || !in || !target || !grad_out)
        return fail(STEPS_EINVAL, "net, in, target and grad_out must be non-null");
    if (B < 1 || B > ((int64_t)1 << 24)) return fail(STEPS_EINVAL, "B=%lld outside [1, 2^24]", (long long)B);
    clear_error();
    const int64_t waves = (B + 31) / 32;
    float *partial = nullptr, *lp = nullptr;
    STEPS_CHECK_HIP(hipMalloc(&partial, waves * (int64_t)kParams * sizeof(float)));
    hipError_t e = hipMalloc(&lp, waves * sizeof(float));
    if (e != hipSuccess) {
        (void)hipFree(partial);
        return fail(STEPS_ENOMEM, "device allocation failed");
    }
    steps_cyl_mlp *mnet = const_cast<steps_cyl_mlp *>(net);
    int rc = launch_train(mnet, in, target, B, B, 0, 0, 0, partial, lp, stream);
    if (!rc) rc = launch_reduce(mnet, partial, lp, waves, 0, grad_out, loss_out, 0.f, 0.f, 0.f, 0.f, stream);
    hipError_t se = hipStreamSynchronize(stream);
    (void)hipFree(partial);
    (void)hipFree(lp);
    if (rc) return rc;
    return hip_status(se, "stream synchronize");
}

STEPS_API int steps_cyl_mlp_samples(const double *in, int64_t n, float *features, float *targets,
                                    hipStream_t stream) {
    if (!in || !features || !targets) return fail(STEPS_EINVAL, "in, features and targets must be non-null");
    if (n < 1 || n > ((int64_t)1 << 34)) return fail(STEPS_EINVAL, "n=%lld out of range", (long long)n);
    int rc = require_device();
    if (rc) return rc;
    clear_error();
    return launch_samples(in, n, features, targets, stream);
}

STEPS_API int steps_cyl_mlp_train(steps_cyl_mlp *net, const steps_cyl_train_cfg *cfg, hipStream_t stream) {
    if (!net || !cfg) return fail(STEPS_EINVAL, "net and cfg must be non-null");
    if (!cfg->train_in || cfg->n_train < 32 || (cfg->n_train & (cfg->n_train - 1)))
        return fail(STEPS_EINVAL, "train_in must be non-null and n_train a power of two >= 32");
    if (cfg->batch < 32 || cfg->batch > cfg->n_train || cfg->steps < 0)
        return fail(STEPS_EINVAL, "batch must lie in [32, n_train] and steps >= 0");
    if (!(cfg->lr > 0.f) || !(cfg->lr_min >= 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) ||
        !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) || !(cfg->adam_eps > 0.f))
        return fail(STEPS_EINVAL, "invalid optimiser hyper-parameters");
    if (cfg->val_in && cfg->n_val < 1) return fail(STEPS_EINVAL, "n_val must be >= 1 with val_in");
    if (cfg->eval_every < 0) return fail(STEPS_EINVAL, "eval_every must be >= 0");
    clear_error();
    const int64_t n = cfg->n_train, B = cfg->batch, waves = (B + 31) / 32;
    const int64_t nv = cfg->val_in ? cfg->n_val : 0;
    float *F = nullptr, *T = nullptr, *Fv = nullptr, *Tv = nullptr, *Ov = nullptr, *partial = nullptr,
          *lp = nullptr, *loss = nullptr, *vpart = nullptr;
    const int vblocks = 256;
    auto cleanup = [&]() {
        (void)hipFree(F); (void)hipFree(T); (void)hipFree(Fv); (void)hipFree(Tv); (void)hipFree(Ov);
        (void)hipFree(partial); (void)hipFree(lp); (void)hipFree(loss); (void)hipFree(vpart);
    };
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&F, 2 * n * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&T, 2 * n * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&partial, waves * (int64_t)kParams * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&lp, waves * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&loss, sizeof(float))) != hipSuccess ||
        (nv && ((e = hipMalloc(&Fv, 2 * nv * sizeof(float))) != hipSuccess ||
                (e = hipMalloc(&Tv, 2 * nv * sizeof(float))) != hipSuccess ||
                (e = hipMalloc(&Ov, 2 * nv * sizeof(float))) != hipSuccess ||
                (e = hipMalloc(&vpart, vblocks * sizeof(float))) != hipSuccess))) {
        cleanup();
        return fail(STEPS_ENOMEM, "training scratch allocation failed: %s", hipGetErrorString(e));
    }
    int rc = launch_samples(cfg->train_in, n, F, T, stream);
    if (!rc && nv) rc = launch_samples(cfg->val_in, nv, Fv, Tv, stream);
    int64_t hist = 0;
    const double pi = 3.14159265358979323846;
    uint64_t rng = cfg->seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    auto next = [&]() {  // splitmix64
        uint64_t z = (rng += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    uint64_t mul = next() | 1ull, add = next();
    int64_t consumed = 0;
    for (int64_t s = 0; !rc && s < cfg->steps; ++s) {
        if (consumed + B > n) {  // new pass over the samples, new permutation
            mul = next() | 1ull;
            add = next();
            consumed = 0;
        }
        const double frac = cfg->steps > 1 ? (double)s / (double)(cfg->steps - 1) : 1.0;
        const float lr = (float)(cfg->lr_min + 0.5 * (cfg->lr - cfg->lr_min) * (1.0 + std::cos(pi * frac)));
        rc = launch_train(net, F, T, n, B, consumed, mul, add, partial, lp, stream);
        consumed += B;
        if (!rc)
            rc = launch_reduce(net, partial, lp, waves, 1, nullptr, loss, lr, cfg->beta1, cfg->beta2,
                               cfg->adam_eps, stream);
        const bool eval = cfg->eval_every > 0 && ((s + 1) % cfg->eval_every == 0 || s + 1 == cfg->steps);
        if (!rc && eval && cfg->history && hist < cfg->history_len) {
            float tl = 0.f, vl = 0.f;
            e = hipMemcpyAsync(&tl, loss, sizeof(float), hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess && nv) {
                rc = launch_forward(net, Fv, Ov, nv, stream);
                if (!rc) {
                    hipLaunchKernelGGL(sumsq_loss_kernel, dim3(vblocks), dim3(256), 0, stream, Ov, Tv, nv, vpart);
                    std::vector<float> hv(vblocks);
                    e = hipMemcpyAsync(hv.data(), vpart, vblocks * sizeof(float), hipMemcpyDeviceToHost, stream);
                    if (e == hipSuccess) e = hipStreamSynchronize(stream);
                    double acc = 0.0;
                    for (float x : hv) acc += x;
                    vl = (float)(acc / (2.0 * (double)nv));
                }
            } else if (e == hipSuccess) {
                e = hipStreamSynchronize(stream);
            }
            if (e != hipSuccess) rc = hip_status(e, "training history");
            cfg->history[3 * hist + 0] = (float)(s + 1);
            cfg->history[3 * hist + 1] = tl;
            cfg->history[3 * hist + 2] = vl;
            ++hist;
        }
    }
    if (!rc) rc = hip_status(hipStreamSynchronize(stream), "training synchronize");
    cleanup();
    return rc;
}

STEPS_API int steps_cyl_mlp_save(const steps_cyl_mlp *net, const char *path) {
    if (!net || !path) return fail(STEPS_EINVAL, "net and path must be non-null");
    clear_error();
    std::vector<float> p(kParams);
    STEPS_CHECK_HIP(hipMemcpy(p.data(), net->master, kParams * sizeof(float), hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(STEPS_EIO, "cannot open %s for writing", path);
    const uint32_t ver = kFormatVersion, np = kParams;
    const uint64_t sum = fnv1a(p.data(), p.size() * sizeof(float));
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&ver, 4, 1, f) == 1 &&
              std::fwrite(&np, 4, 1, f) == 1 && std::fwrite(p.data(), sizeof(float), kParams, f) == (size_t)kParams &&
              std::fwrite(&sum, 8, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(STEPS_EIO, "short write to %s", path);
    return STEPS_OK;
}

STEPS_API int steps_cyl_mlp_load(const char *path, steps_cyl_mlp **out) {
    if (!path || !out) return fail(STEPS_EINVAL, "path and out must be non-null");
    clear_error();
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(STEPS_EIO, "cannot open %s", path);
    char magic[8];
    uint32_t ver = 0, np = 0;
    uint64_t sum = 0;
    std::vector<float> p(kParams);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
              std::fread(&ver, 4, 1, f) == 1 && ver == kFormatVersion && std::fread(&np, 4, 1, f) == 1 &&
              np == (uint32_t)kParams && std::fread(p.data(), sizeof(float), kParams, f) == (size_t)kParams &&
              std::fread(&sum, 8, 1, f) == 1;
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;
    std::fclose(f);
    if (!ok) return fail(STEPS_EIO, "%s is not a steps_cyl network file (magic, version, size)", path);
    if (sum != fnv1a(p.data(), p.size() * sizeof(float))) return fail(STEPS_EIO, "%s: checksum mismatch", path);
    if (!finite_params(p.data())) return fail(STEPS_EIO, "%s holds non-finite parameters", path);
    return steps_cyl_mlp_create(p.data(), out);
}
