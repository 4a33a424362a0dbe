// Device helpers shared by the kernels that stage x windows in LDS
// (spmv.hip, batched.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "check.h"

namespace spmvc {

// One 16-byte direct global-to-LDS load per lane: the wavefront's 64 chunks
// land contiguously at lds (a wavefront-uniform address).  The builtin exists
// only for the GPU target; the host compilation pass sees an empty body.
__device__ __forceinline__ void lds_load16(const void *g, void *lds) {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
#else
    (void)g;
    (void)lds;
#endif
}

// Window-phased block SpMV, records split into value runs: the sum over one
// run of a (pattern, window) record of the row's x elements for this lane's
// pair of right-hand sides.  ent: the run's window element indices (16-byte
// aligned), xrow: the pair's bytes in window row 0, NRB: bytes per window
// row, lim: the window rows from this row on (indices below it are in the
// window).  Four 16-byte LDS reads in flight per step, added in entry order.
template <int NRB>
__device__ __forceinline__ void win_run_sum(const uint32_t *ent, int cnt, const unsigned char *xrow, uint32_t lim,
                                            double &s0, double &s1) {
    const uint4 *e4 = reinterpret_cast<const uint4 *>(ent);
    int k = 0;
    for (; k + 4 <= cnt; k += 4) {
        const uint4 e = e4[k >> 2];
        const double2 x0 = *reinterpret_cast<const double2 *>(xrow + in_bounds<uint32_t>(e.x, lim) * NRB);
        const double2 x1 = *reinterpret_cast<const double2 *>(xrow + in_bounds<uint32_t>(e.y, lim) * NRB);
        const double2 x2 = *reinterpret_cast<const double2 *>(xrow + in_bounds<uint32_t>(e.z, lim) * NRB);
        const double2 x3 = *reinterpret_cast<const double2 *>(xrow + in_bounds<uint32_t>(e.w, lim) * NRB);
        s0 += x0.x;
        s1 += x0.y;
        s0 += x1.x;
        s1 += x1.y;
        s0 += x2.x;
        s1 += x2.y;
        s0 += x3.x;
        s1 += x3.y;
    }
    for (; k < cnt; ++k) {
        const double2 xv = *reinterpret_cast<const double2 *>(xrow + in_bounds<uint32_t>(ent[k], lim) * NRB);
        s0 += xv.x;
        s1 += xv.y;
    }
}

// The products of one row's entries in the current window from a split
// record (word 0: V[0] run length, word 1: V[1] run length, word 2: slot of
// the V[1] run; entries from word 4): v0 * (sum of the V[0] run) + v1 * (sum
// of the V[1] run) added to (a0, a1).
template <int NRB>
__device__ __forceinline__ void win_row_split(const uint32_t *rec, const unsigned char *xrow, uint32_t lim, double v0,
                                              double v1, double &a0, double &a1) {
    const uint4 h = *reinterpret_cast<const uint4 *>(rec);
    double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
    win_run_sum<NRB>(rec + 4, static_cast<int>(h.x), xrow, lim, s00, s01);
    win_run_sum<NRB>(rec + 4 + h.z, static_cast<int>(h.y), xrow, lim, s10, s11);
    a0 = ::fma(v0, s00, ::fma(v1, s10, a0));
    a1 = ::fma(v0, s01, ::fma(v1, s11, a1));
}

}  // namespace spmvc
