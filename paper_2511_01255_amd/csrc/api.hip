// api.hip -- status strings, per-thread error text, device check.
#include <cstdio>
#include <cstring>

#include "common.hpp"

namespace qpm {

static thread_local char g_last_error[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

void clear_error() { g_last_error[0] = '\0'; }

qpm_status check_device()
{
    int dev = 0;
    QPM_TRY_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    QPM_TRY_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error("device %d is %s; this library is built for gfx950 only", dev, prop.gcnArchName);
        return QPM_ENOTSUP;
    }
    return QPM_OK;
}

}  // namespace qpm

QPM_API const char *qpm_status_string(qpm_status s)
{
    switch (s) {
    case QPM_OK: return "ok";
    case QPM_EINVAL: return "invalid argument";
    case QPM_ERANGE: return "size out of range";
    case QPM_ENOMEM: return "out of device memory";
    case QPM_EHIP: return "HIP runtime error";
    case QPM_ENOTSUP: return "unsupported device";
    default: return "unknown status";
    }
}

QPM_API const char *qpm_last_error(void) { return qpm::g_last_error; }
