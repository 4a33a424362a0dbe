// Fixed-order reductions shared by the kernels (spmv.hip, cg.hip, batched.hip):
// every sum runs in the same order on every launch, so results are bitwise
// reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>

namespace spmvc {

// Sum over the 64 lanes of a wavefront (xor butterfly); the result in every lane.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over a block of NT threads: each wavefront's sum, then the NT / 64
// wavefront sums in wavefront order; the result in every thread.  Every
// thread of the block must call it.  sh: NT / 64 doubles of LDS for the
// wavefront sums -- the caller's (a buffer it is done with: the first barrier
// below orders every earlier access to it before these writes), so that a
// kernel with only dynamic LDS keeps its LDS base at 0.
template <int NT> __device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += sh[i];
    return s;
}

// The same with a static LDS array for the wavefront sums.
template <int NT> __device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[NT / 64];
    return block_sum<NT>(v, sh);
}

}  // namespace spmvc
