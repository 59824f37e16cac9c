// Error reporting and version query of the C ABI.
#include <cstdarg>
#include <cstdio>
#include <string>

#include "common.hpp"

namespace tbk {

namespace {
thread_local std::string g_last_error;
}

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

tbk_status fail(tbk_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

}  // namespace tbk

extern "C" const char *tbk_last_error(void) { return tbk::g_last_error.c_str(); }

extern "C" int32_t tbk_abi_version(void) { return TBK_ABI_VERSION; }
