// Error reporting and version of the C ABI.
#include <cstdarg>
#include <cstdio>

#include "rpr_internal.hpp"

namespace rpr {

namespace {
thread_local char g_err[512] = "";
}

int set_error(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace rpr

extern "C" const char* last_error(void) { return rpr::g_err; }

extern "C" const char* rpr_version(void) { return "rpr 0.1 gfx950"; }
