// errors.cpp -- status codes and the per-thread last-error message of the
// C ABI (host only).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include "internal.h"

namespace miaug {
namespace {
thread_local char g_err[512] = "";
}

int set_error(int status, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return status;
}

void clear_error() { g_err[0] = 0; }

int hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return MIAUG_OK;
    return set_error(e == hipErrorOutOfMemory ? MIAUG_ENOMEM : MIAUG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace miaug

extern "C" {

int miaug_version(void) { return 10000; }

const char *miaug_status_str(int s) {
    switch (s) {
    case MIAUG_OK: return "ok";
    case MIAUG_EINVAL: return "invalid argument";
    case MIAUG_ESHAPE: return "invalid or unsupported shape";
    case MIAUG_EUNSUPPORTED: return "unsupported";
    case MIAUG_EDEVICE: return "device error";
    case MIAUG_ENOMEM: return "out of memory";
    case MIAUG_ECAPACITY: return "workspace too small";
    default: return "unknown status";
    }
}

const char *miaug_last_error(void) { return miaug::g_err; }

}  // extern "C"
