// Device-side building blocks of the far-image correction network
// (2 -> 64 -> 64 -> 64 -> 64 -> 2, base-2 SiLU): parameter layout, the packed
// MFMA operand layout, and the per-wave forward pass over 32 samples.
// Layers 1-4 run on MFMA (layer 1 on the exact three-part BF16 split of its
// FP32 inputs, so it stays an FP32 layer), layer 5 on the VALU.
//
// MFMA mapping (v_mfma_f32_32x32x16_bf16, FP32 accumulation).  Hidden
// layers 2-4 are computed transposed, Y^T[64 x 32] = W[64 x 64] X^T[64 x 32],
// with the 32 samples of a wave as the N dimension:
//   A (32 x 16, weights):   lane l holds row l%32, k = 8(l/32) + e, e = 0..7
//   B (16 x 32, inputs):    lane l holds column l%32, k = 8(l/32) + e
//   D (32 x 32, outputs):   lane l holds column l%32, rows
//                           8(v/4) + 4(l/32) + v%4 for v = 0..15
// Each lane's D values of one layer are fed unchanged (after bias, SiLU and
// BF16 rounding) as the B operand of the next layer: K step t takes the
// values v = 8(t%2)..8(t%2)+7 of M block t/2.  K slot kappa = 16t + 8h + e
// (h = l/32) therefore holds the physical feature
//   phi(kappa) = 16t + 8(e/4) + 4h + e%4,
// and the weight fragments are packed with their input columns permuted by
// phi.  No data moves between lanes from layer to layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace steps {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kWidth = 64;
constexpr int kParams = 12802;
// offsets in the flat parameter vector: W1 (64x2), b1, W2, b2, W3, b3, W4, b4,
// W5 (2x64), b5; weights (fan_out, fan_in) row-major
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = 128;
constexpr int OFF_W[3] = {192, 4352, 8512};   // W2, W3, W4
constexpr int OFF_B[3] = {4288, 8448, 12608}; // b2, b3, b4
constexpr int OFF_W5 = 12672;
constexpr int OFF_B5 = 12800;

// network domain and model constants (the learned correction, per unit L)
constexpr float kRhoMin = 0.05f;
constexpr float kRhoMax = 20.0f;
constexpr float kOutScale = 0.02f;    // s(r) = 0.02 / (1 + r^2)
constexpr double kRodInner = 1.5;     // rods from 1.5 L
constexpr int kFarImages = 1024;      // ... to 1024.5 L

// Packed inference parameters, laid out so that every lane reads what it
// needs as consecutive 16-byte chunks from one base address per lane half
// h (the kernels copy this block to LDS):
//   A     forward A fragments of layers 2-4 [layer][M block][K step][lane]
//   A1    layer 1 A fragments [M block][lane]: lane l < 32 holds row
//         32b + l as {w0, w0, w0, w1, w1, w1, 0, 0} (W1 BF16-rounded), the
//         other lanes zeros
//   Bias1 b1[drow(b, v, h)] at [h][b][v]
//   Bias  b_{k+2}[drow(b, v, h)] at [h][k][b][v]
//   W5    {W5[0][r], W5[1][r]} for r = drow(b, v, h) at [h][b][v]
//         (BF16-rounded)
struct alignas(16) Packed {
    bf16x8 A[3][2][4][64];
    bf16x8 A1[2][64];
    alignas(16) float Bias1[2][2][16];
    alignas(16) float Bias[2][3][2][16];
    float2 W5[2][2][16];
    float b5[4];  // b5[0], b5[1], unused
};
static_assert(sizeof(Packed) % 16 == 0, "packed parameters must be 16-byte sized");

// Transposed fragments for the backward pass (A = W^T, K permuted by phi).
struct alignas(16) PackedT {
    bf16x8 AT[3][2][4][64];
};

__device__ __forceinline__ int phi(int kappa) {
    const int t = kappa >> 4, h = (kappa >> 3) & 1, e = kappa & 7;
    return 16 * t + 8 * (e >> 2) + 4 * h + (e & 3);
}

// physical output row of D element v of M block b for lane half h
__device__ __forceinline__ int drow(int b, int v, int h) {
    return 32 * b + 8 * (v >> 2) + 4 * h + (v & 3);
}

// Activation s(u) = u / (1 + 2^-u) = SiLU(u ln 2) / ln 2: SiLU with the
// factor ln 2 absorbed into the adjacent weights, so that the hardware exp2
// needs no scaling (two VALU operations and two transcendentals per unit).
__device__ __forceinline__ float silu(float u) {
    return u * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-u));
}

// ds/du = sigma (1 + u ln2 (1 - sigma)), sigma = 1 / (1 + 2^-u)
__device__ __forceinline__ float silu_grad(float u) {
    const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-u));
    return sg * __builtin_fmaf(u * 0.6931471805599453f, 1.0f - sg, 1.0f);
}

// f = hi + mid + lo with each part BF16 (round to nearest even): each
// remainder is exact in FP32, and what the three parts leave is below
// 2^-26 |f|, under FP32 rounding.
__device__ __forceinline__ void split3(float f, __bf16 &hi, __bf16 &mid, __bf16 &lo) {
    hi = (__bf16)f;
    const float r1 = f - (float)hi;
    mid = (__bf16)r1;
    lo = (__bf16)(r1 - (float)mid);
}

// Forward pass for the 32 samples of a wave.  Lanes l and l+32 both carry
// the features (f1, f2) of sample l%32 and both return its outputs (o0, o1).
// With CAPTURE, the pre-activations of layers 1..4 (zc, [4][64][32] FP32) and
// the BF16 inputs of layers 2..4 (xc, [3][64][32]) are stored in
// [feature][sample] layout (sample = column l%32) for the backward pass.
template <bool CAPTURE>
__device__ __forceinline__ void forward32(const Packed &P, float f1, float f2, float &o0, float &o1,
                                          float *zc, __bf16 *xc) {
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, col = lane & 31;
    bf16x8 xb[4];
    const float(*Bias)[2][16] = P.Bias[h];
    const float2(*W5)[16] = P.W5[h];
    // layer 1 on MFMA: K slots 0-5 of lanes 0-31 hold the three-part BF16
    // splits of f1 and f2 (exact products with the BF16 weights, FP32
    // accumulation: layer 1 in FP32), the bias enters as the C operand
    {
        __bf16 p0, p1, p2, q0, q1, q2;
        split3(f1, p0, p1, p2);
        split3(f2, q0, q1, q2);
        const __bf16 zero = (__bf16)0.f;
        bf16x8 xin;
        xin[0] = h ? zero : p0;
        xin[1] = h ? zero : p1;
        xin[2] = h ? zero : p2;
        xin[3] = h ? zero : q0;
        xin[4] = h ? zero : q1;
        xin[5] = h ? zero : q2;
        xin[6] = zero;
        xin[7] = zero;
        f32x16 acc1[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            acc1[b] = *reinterpret_cast<const f32x16 *>(&P.Bias1[h][b][0]);
            acc1[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(P.A1[b][lane], xin, acc1[b], 0, 0, 0);
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = drow(b, v, h);
                const float z = acc1[b][v];
                xb[2 * b + (v >> 3)][v & 7] = (__bf16)silu(z);
                if (CAPTURE) {
                    zc[r * 32 + col] = z;
                    xc[r * 32 + col] = xb[2 * b + (v >> 3)][v & 7];
                }
            }
        }
    }
    float a4[2][16];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        f32x16 acc[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            // the bias enters as the C operand of the first MFMA of the chain
            acc[b] = *reinterpret_cast<const f32x16 *>(&Bias[k][b][0]);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(P.A[k][b][t][lane], xb[t], acc[b], 0, 0, 0);
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = drow(b, v, h);
                const float z = acc[b][v];
                const float a = silu(z);
                if (CAPTURE) zc[(k + 1) * 64 * 32 + r * 32 + col] = z;
                if (k < 2) {
                    xb[2 * b + (v >> 3)][v & 7] = (__bf16)a;
                    if (CAPTURE) xc[(k + 1) * 64 * 32 + r * 32 + col] = xb[2 * b + (v >> 3)][v & 7];
                } else {
                    a4[b][v] = a;
                }
            }
        }
    }
    // layer 5 on the VALU: half-sums over this lane's 32 rows, then the halves
    float p0 = 0.f, p1 = 0.f;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const float2 w = W5[b][v];
            p0 = __builtin_fmaf(w.x, a4[b][v], p0);
            p1 = __builtin_fmaf(w.y, a4[b][v], p1);
        }
    }
    const float q0 = __shfl_xor(p0, 32);
    const float q1 = __shfl_xor(p1, 32);
    // same operand order in both halves so they agree bitwise
    o0 = (h ? (q0 + p0) : (p0 + q0)) + P.b5[0];
    o1 = (h ? (q1 + p1) : (p1 + q1)) + P.b5[1];
}

// Copies the packed parameters into LDS cooperatively (16-byte chunks).
__device__ __forceinline__ void load_packed(Packed *dst, const Packed *src) {
    const int n = (int)(sizeof(Packed) / 16);
    const uint4 *s = reinterpret_cast<const uint4 *>(src);
    uint4 *d = reinterpret_cast<uint4 *>(dst);
    for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
}

}  // namespace mlp
}  // namespace steps
