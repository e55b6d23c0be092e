// steps_cyl_forces_noalloc: the pairwise exact path of steps_cyl_forces for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  Its workspace is
// a fixed array in the library's device image, one copy per device, shared
// by every call on that device.
#include <algorithm>
#include <mutex>

#include "common.h"

namespace steps {
namespace {

// Largest workspace of one call: the pairwise path at N = 2^20 with groups
// of one part (spatial order 16 B, records 32 B and two slots of FP64 sums
// 64 B per particle, boxes, the radix sort's storage) fits with room.
constexpr size_t kScratchBytes = (size_t)128 << 20;

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {nullptr};
std::mutex g_scratch_mutex;

// Device address of `scratch` on the current device, looked up once per
// device (host code never passes the array's own name to a kernel: on the
// host it only stands for the symbol).
int scratch_on_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(STEPS_ENODEV, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(STEPS_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return STEPS_OK;
}

}  // namespace
}  // namespace steps

using namespace steps;

STEPS_API int steps_cyl_forces_noalloc(const double *pos, const double *mass, const double *eps, int64_t N,
                                       double L, int n_img, float *out_acc, float *out_pot, hipStream_t stream) {
    if (!pos || !mass || !eps) return fail(STEPS_EINVAL, "pos, mass and eps must be non-null");
    if (!out_acc) return fail(STEPS_EINVAL, "out_acc must be non-null");
    if (N < 1 || N > STEPS_NOALLOC_MAX_N)
        return fail(STEPS_EINVAL, "N=%lld outside [1, %lld], the static scratch's limit", (long long)N,
                    (long long)STEPS_NOALLOC_MAX_N);
    if (!finite_positive(L)) return fail(STEPS_EINVAL, "L must be finite and > 0");
    if (n_img < 0 || n_img > STEPS_MAX_NIMG)
        return fail(STEPS_EINVAL, "n_img=%d outside [0, %d]", n_img, STEPS_MAX_NIMG);
    int rc = require_device();
    if (rc) return rc;
    clear_error();
    // groups of 16 parts as in steps_cyl_forces, or fewer parts (fewer sum
    // slots) so that the workspace fits the static array
    int S = 16;
    while (S > 1 && pairwise_bytes_S(N, S) > kScratchBytes) S >>= 1;
    if (pairwise_bytes_S(N, S) > kScratchBytes)
        return fail(STEPS_EINVAL, "N=%lld needs %zu bytes of scratch, above the static %zu", (long long)N,
                    pairwise_bytes_S(N, S), kScratchBytes);
    void *p = nullptr;
    if ((rc = scratch_on_device(&p))) return rc;
    Workspace ws;
    ws.base = (char *)p;
    ws.size = kScratchBytes;
    return launch_forces_pairwise(pos, mass, eps, N, L, n_img, nullptr, 0, out_acc, out_pot, ws, stream, S);
}
