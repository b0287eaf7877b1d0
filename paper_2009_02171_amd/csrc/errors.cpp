// Thread-local error text behind csdyn_last_error().
#include <cstdarg>
#include <cstdio>

#include "common.h"

namespace csd {

static thread_local char g_err[512] = {0};

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

}  // namespace csd

extern "C" const char *csdyn_last_error(void) { return csd::g_err; }
