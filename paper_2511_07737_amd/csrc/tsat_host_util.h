// tsat_host_util.h -- device buffers and small helpers shared by the host
// translation units of the library that use the HIP runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "tsat.h"
#include "tsat_err.h"

namespace tsat_host {

// allocation-failure injection for tests of the OOM path: the environment
// variable TSAT_FAIL_ALLOC_AFTER=n makes the (n+1)-th device allocation fail
inline bool inject_alloc_failure()
{
    static int64_t countdown = -2;
    if (countdown == -2) {
        const char* e = getenv("TSAT_FAIL_ALLOC_AFTER");
        countdown = e ? atoll(e) : -1;
    }
    if (countdown < 0) return false;
    if (countdown == 0) return true;
    --countdown;
    return false;
}

// launch-shape knobs, overridable from the environment for tuning sweeps
inline int env_int(const char* name, int dflt)
{
    const char* e = getenv(name);
    return e ? atoi(e) : dflt;
}

struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    int32_t alloc(size_t n, const char* what)
    {
        if (n == bytes && p) return TSAT_OK;
        release();
        if (n == 0) return TSAT_OK;
        if (inject_alloc_failure()) return fail(TSAT_E_OOM, "device allocation of %zu bytes for %s failed (injected)", n, what);
        if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return fail(TSAT_E_OOM, "device allocation of %zu bytes for %s failed", n, what);
        }
        bytes = n;
        return TSAT_OK;
    }
    // grow-only variant for scratch space
    int32_t reserve(size_t n, const char* what) { return (n <= bytes && p) ? TSAT_OK : alloc(n, what); }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

} // namespace tsat_host

#define HIPCHK(x)                                                                                      \
    do {                                                                                               \
        hipError_t e_ = (x);                                                                           \
        if (e_ != hipSuccess) return tsat_host::fail(TSAT_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)
