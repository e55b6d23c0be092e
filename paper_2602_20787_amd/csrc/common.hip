// Host-side status handling shared by all entry points.
#include "common.h"

#include <cstdarg>
#include <cstring>
#include <mutex>

namespace steps {

namespace {
thread_local char g_last_error[512] = "";

// gfx950 check, cached per device ordinal (0 = unknown, 1 = yes, -1 = no).
constexpr int kMaxDevices = 64;
int g_device_ok[kMaxDevices] = {0};
std::mutex g_device_mutex;
}  // namespace

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_last_error[0] = '\0'; }

const char *last_error() { return g_last_error; }

int hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return STEPS_OK;
    return fail(STEPS_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}

int require_device() {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0)
        return fail(STEPS_ENODEV, "no HIP device available (%s)",
                    e == hipSuccess ? "count is 0" : hipGetErrorString(e));
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(STEPS_ENODEV, "device ordinal %d out of range", dev);
    {
        std::lock_guard<std::mutex> lock(g_device_mutex);
        if (g_device_ok[dev] == 0) {
            hipDeviceProp_t prop;
            e = hipGetDeviceProperties(&prop, dev);
            if (e != hipSuccess) return hip_status(e, "hipGetDeviceProperties");
            g_device_ok[dev] = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : -1;
        }
        if (g_device_ok[dev] < 0) return fail(STEPS_ENODEV, "device %d is not a gfx950", dev);
    }
    return STEPS_OK;
}

int check_workspace(const Workspace &ws, size_t need) {
    if (need > 0 && (!ws.base || ws.size < need))
        return fail(STEPS_EINVAL, "workspace of %zu bytes is smaller than the %zu bytes this call needs", ws.size,
                    need);
    return STEPS_OK;
}

}  // namespace steps

STEPS_API const char *steps_cyl_last_error(void) { return steps::last_error(); }

STEPS_API const char *steps_cyl_version(void) { return "steps_cyl 0.1.0 (gfx950)"; }
