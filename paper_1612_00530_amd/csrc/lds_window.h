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

// Window-phased block SpMV, records split into value runs: the sums over one
// run of a (pattern, window) record of the row's x elements for this lane's
// Q consecutive right-hand sides (Q = 2 or 4: Q / 2 16-byte reads per entry).
// ent: the run's window element indices (16-byte aligned), xrow: the lane's
// first right-hand side in window row 0, NRB: bytes per window row, lim: the
// window rows from this row on (indices below it are in the window).  Four
// entries' reads in flight per step; each sum adds its entries in run order.
template <int NRB, int Q>
__device__ __forceinline__ void win_run_sum(const uint32_t *ent, int cnt, const unsigned char *xrow, uint32_t lim,
                                            double (&s)[Q]) {
    static_assert(Q == 2 || Q == 4, "two or four right-hand sides per lane");
    const uint4 *e4 = reinterpret_cast<const uint4 *>(ent);
    int k = 0;
    for (; k + 4 <= cnt; k += 4) {
        const uint4 e = e4[k >> 2];
        const uint32_t ev[4] = {e.x, e.y, e.z, e.w};
        double2 xv[4][Q / 2];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int h = 0; h < Q / 2; ++h)
                xv[j][h] = *reinterpret_cast<const double2 *>(xrow + in_bounds<uint32_t>(ev[j], lim) * NRB + 16 * h);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int h = 0; h < Q / 2; ++h) {
                s[2 * h] += xv[j][h].x;
                s[2 * h + 1] += xv[j][h].y;
            }
    }
    for (; k < cnt; ++k) {
        const unsigned char *xe = xrow + in_bounds<uint32_t>(ent[k], lim) * NRB;
#pragma unroll
        for (int h = 0; h < Q / 2; ++h) {
            const double2 xv = *reinterpret_cast<const double2 *>(xe + 16 * h);
            s[2 * h] += xv.x;
            s[2 * h + 1] += xv.y;
        }
    }
}

// The products of one row's entries in the current window from a split
// record (word 0: V[0] run length, word 1: V[1] run length, word 2: slot of
// the V[1] run; entries from word 4), for the lane's Q right-hand sides:
// a[q] += v0 * (sum of the V[0] run) + v1 * (sum of the V[1] run).
template <int NRB, int Q>
__device__ __forceinline__ void win_row_split(const uint32_t *rec, const unsigned char *xrow, uint32_t lim, double v0,
                                              double v1, double (&a)[Q]) {
    const uint4 h = *reinterpret_cast<const uint4 *>(rec);
    double s0[Q], s1[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) s0[q] = s1[q] = 0.0;
    win_run_sum<NRB, Q>(rec + 4, static_cast<int>(h.x), xrow, lim, s0);
    win_run_sum<NRB, Q>(rec + 4 + h.z, static_cast<int>(h.y), xrow, lim, s1);
#pragma unroll
    for (int q = 0; q < Q; ++q) a[q] = ::fma(v0, s0[q], ::fma(v1, s1[q], a[q]));
}

}  // namespace spmvc
