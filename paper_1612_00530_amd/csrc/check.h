// Bounds checks of the kernels' gathers and LDS reads, compiled in with
// -DSPMVC_CHECK (a debug build of the library): every gathered column and
// every LDS index goes through in_bounds(i, n), which in a checked build
// records an index outside [0, n) and returns 0 instead, so that a wrong
// index is reported (spmvc_check_violations) rather than read out of bounds.
// In the normal build in_bounds is the identity.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spmvc {

#ifdef SPMVC_CHECK
// one counter per translation unit (each kernel source reads its own)
static __device__ unsigned long long g_bound_violations;

template <class I> __device__ __forceinline__ I in_bounds(I i, I n) {
    const bool ok = !(i < I(0)) && i < n;
    if (!ok) g_bound_violations = 1ull;  // a plain store: every writer writes the same value
    return ok ? i : I(0);
}

// host side: the translation unit's count since the last call, then zero
#define SPMVC_CHECK_READER(NAME)                                                                  \
    unsigned long long NAME() {                                                                   \
        unsigned long long v = 0, z = 0;                                                          \
        SPMVC_HIP(hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_bound_violations), sizeof(v)));             \
        SPMVC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_bound_violations), &z, sizeof(z)));               \
        return v;                                                                                 \
    }
#else
template <class I> __device__ __forceinline__ I in_bounds(I i, I) { return i; }
#define SPMVC_CHECK_READER(NAME) \
    unsigned long long NAME() { return 0; }
#endif

}  // namespace spmvc
