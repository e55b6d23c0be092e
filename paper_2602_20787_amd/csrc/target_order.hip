// Spatial order of the targets, shared by the force kernels: a 30-bit
// Morton key of (x, y) over the transverse extent and of z over the period,
// radix-sorted together with the targets' positions in the caller's list.  Neighbouring lanes then
// hold neighbouring targets, which keeps data-dependent work (table gathers,
// the softened branch) coherent within a wave.  The order changes no result:
// each target's sum runs over the sources in their own order and is written
// to the target's own position in the list.
#include <rocprim/device/device_radix_sort.hpp>

#include "common.h"
#include "pair_f64.h"

namespace steps {
namespace {

constexpr int kExtentBlocks = 64;

__global__ void extent_kernel(const double *pos, int N, double *partial) {
    __shared__ double m[256];
    double v = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256)
        v = fmax(v, fmax(fabs(pos[i]), fabs(pos[N + i])));
    m[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) m[threadIdx.x] = fmax(m[threadIdx.x], m[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = m[0];
}

__global__ void order_keys_kernel(const double *pos, int N, double L, const double *partial, const int64_t *targets,
                                  int n_tgt, uint32_t *key, int *idx) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_tgt) return;
    const int64_t i = targets ? targets[k] : (int64_t)k;
    double ext = 0.0;
    for (int b = 0; b < kExtentBlocks; ++b) ext = fmax(ext, partial[b]);
    const double sc = ext > 0.0 ? 1024.0 / (2.0 * ext) : 0.0;
    const double zw = wrap_z(pos[2 * N + i], L);
    const uint32_t q[3] = {(uint32_t)fmin(1023.0, fmax(0.0, floor((pos[i] + ext) * sc))),
                           (uint32_t)fmin(1023.0, fmax(0.0, floor((pos[N + i] + ext) * sc))),
                           (uint32_t)fmin(1023.0, fmax(0.0, floor(zw / L * 1024.0)))};
    uint32_t code = 0;
    for (int b = 0; b < 10; ++b)
        code |= (((q[0] >> b) & 1u) << (3 * b + 2)) | (((q[1] >> b) & 1u) << (3 * b + 1)) |
                (((q[2] >> b) & 1u) << (3 * b));
    key[k] = code;
    idx[k] = k;
}

}  // namespace

namespace {

// bytes of rocPRIM's temporary storage for sorting n (key, index) pairs
size_t sort_storage(int n) {
    size_t bytes = 0;
    if (rocprim::radix_sort_pairs(nullptr, bytes, (uint32_t *)nullptr, (uint32_t *)nullptr, (int *)nullptr,
                                  (int *)nullptr, n, 0, 30) != hipSuccess)
        return 0;
    return bytes;
}

}  // namespace

size_t order_targets_bytes(int64_t n_tgt) {
    // partials; keys and indices, twice; the sort's storage
    return ws_total({(size_t)8 * kExtentBlocks, (size_t)16 * n_tgt, sort_storage((int)n_tgt)});
}

int order_targets(const double *pos, int64_t N, double L, const int64_t *targets, int64_t n_tgt, hipStream_t stream,
                  Workspace &ws, const int **perm) {
    *perm = nullptr;
    const int n = (int)n_tgt;
    size_t sort_bytes = 0;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, sort_bytes, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                             (int *)nullptr, (int *)nullptr, n, 0, 30, stream);
    if (e != hipSuccess) return hip_status(e, "target order");
    double *partial = (double *)ws.take((size_t)8 * kExtentBlocks);
    uint32_t *k_in = (uint32_t *)ws.take((size_t)16 * n);
    void *tmp = ws.take(sort_bytes);
    if (!partial || !k_in || (sort_bytes && !tmp))
        return fail(STEPS_EINVAL, "workspace too small for the target order (%zu bytes)", ws.size);
    uint32_t *k_out = k_in + n;
    int *i_in = (int *)(k_out + n), *i_out = i_in + n;
    hipLaunchKernelGGL(extent_kernel, dim3(kExtentBlocks), dim3(256), 0, stream, pos, (int)N, partial);
    hipLaunchKernelGGL(order_keys_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, pos, (int)N, L, partial,
                       targets, n, k_in, i_in);
    e = hipGetLastError();
    if (e == hipSuccess) e = rocprim::radix_sort_pairs(tmp, sort_bytes, k_in, k_out, i_in, i_out, n, 0, 30, stream);
    if (e != hipSuccess) return hip_status(e, "target order");
    *perm = i_out;
    return STEPS_OK;
}

}  // namespace steps
