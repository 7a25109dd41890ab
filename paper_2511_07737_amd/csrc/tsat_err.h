// tsat_err.h -- error reporting of the C-ABI (thread-local message behind
// tsat_last_error and the status codes of tsat.h).  Free of HIP so that the
// host-only translation units build and run with a plain C++ compiler.
#pragma once

#include <cstdarg>
#include <cstdio>
#include <string>

#include "tsat.h"

namespace tsat_host {

// the message behind tsat_last_error(): one per host thread
inline thread_local std::string g_err;

inline int32_t fail(int32_t code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

} // namespace tsat_host

#define RET(x)                       \
    do {                             \
        int32_t r_ = (x);            \
        if (r_ != TSAT_OK) return r_; \
    } while (0)
