// Thread-local error messages and the version string of the Bolt library.
#include <cstring>

#include "common.hpp"

namespace {
thread_local char g_msg[512] = "";
}

namespace bolt {

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(BOLT_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return BOLT_OK;
}

}  // namespace bolt

extern "C" const char *bolt_last_error(void) { return g_msg; }

extern "C" const char *bolt_version(void) { return "bolt-gfx950 0.1"; }
