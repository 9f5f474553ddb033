// api.hip -- status strings, per-thread error message, version.
#include <cstdarg>
#include <cstdio>

#include "sad_host.h"

namespace sad {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

}  // namespace sad

extern "C" const char *sad_status_string(sad_status s) {
    switch (s) {
        case SAD_OK: return "ok";
        case SAD_ERR_INVALID_ARGUMENT: return "invalid argument";
        case SAD_ERR_UNSUPPORTED: return "unsupported";
        case SAD_ERR_WORKSPACE: return "workspace too small";
        case SAD_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

extern "C" const char *sad_last_error(void) { return sad::g_err; }

extern "C" const char *sad_version(void) { return "sad-mi355x 0.1 (gfx950)"; }
