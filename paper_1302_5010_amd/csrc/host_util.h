// Host-side helpers shared by the C-ABI translation units: the thread-local
// error message behind bmpl_last_error, HIP error mapping and allocation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/bmpl.h"

namespace bmpl {

inline thread_local std::string g_err;

inline bmpl_status fail(bmpl_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

template <class T>
hipError_t dalloc(T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

template <class T>
void dfree(T*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

inline int round_up(int v, int a) { return (v + a - 1) / a * a; }

}  // namespace bmpl

#define HIPC(call)                                                                      \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::bmpl::fail(e_ == hipErrorOutOfMemory ? BMPL_E_NOMEM : BMPL_E_HIP,  \
                                "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),  \
                                __FILE__, __LINE__);                                    \
    } while (0)
