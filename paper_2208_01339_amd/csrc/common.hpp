// Host-side helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdio>
#include <new>
#include <string>

#include "../../include/pp.h"

namespace ppc {

// message of the last failing call on this thread (pp_last_error)
std::string &last_error();

inline pp_status fail(pp_status s, const std::string &msg)
{
    last_error() = msg;
    return s;
}

struct HipError {
    hipError_t e;
    const char *what;
    int line;
};

inline pp_status hip_fail(const HipError &e)
{
    char b[256];
    snprintf(b, sizeof b, "HIP error %s in %s (line %d)", hipGetErrorString(e.e), e.what, e.line);
    return fail(PP_ERR_HIP, b);
}

template <typename T>
T *dalloc(size_t count)
{
    if (count == 0) count = 1;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw std::bad_alloc();
    }
    return (T *)p;
}

template <typename T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

}  // namespace ppc

#define HIPCHK(x)                                                    \
    do {                                                             \
        hipError_t e_ = (x);                                         \
        if (e_ != hipSuccess) throw ppc::HipError{e_, #x, __LINE__}; \
    } while (0)
