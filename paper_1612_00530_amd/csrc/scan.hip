// Device-wide exclusive prefix sum of int64 values (used by the compressor).
#include "internal.h"

namespace spmvc {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Each block scans one tile of kScanTile values and emits the tile total.
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int64_t *in, int64_t *out,
                                                            int64_t *tile_sums, int64_t n) {
    __shared__ int64_t sh[kScanThreads];
    const int tid = threadIdx.x;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + tid * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0;
        s += v[i];
    }
    sh[tid] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int64_t t = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    int64_t run = sh[tid] - s;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (tid == kScanThreads - 1) tile_sums[blockIdx.x] = sh[tid];
}

__global__ void k_scan_add(int64_t *out, const int64_t *tile_off, int64_t n) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] += tile_off[idx / kScanTile];
}

}  // namespace

int64_t exclusive_scan(const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) return 0;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    DevBuf sums;
    sums.alloc(sizeof(int64_t) * static_cast<size_t>(tiles));
    k_scan_tiles<<<static_cast<unsigned>(tiles), kScanThreads, 0, s>>>(in, out, sums.as<int64_t>(), n);
    SPMVC_CHECK_LAUNCH();
    int64_t total = 0;
    if (tiles == 1) {
        SPMVC_HIP(hipMemcpyAsync(&total, sums.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        SPMVC_HIP(hipStreamSynchronize(s));
        return total;
    }
    total = exclusive_scan(sums.as<int64_t>(), sums.as<int64_t>(), tiles, s);
    k_scan_add<<<grid_for(n, 256, 0x7fffffff), 256, 0, s>>>(out, sums.as<int64_t>(), n);
    SPMVC_CHECK_LAUNCH();
    SPMVC_HIP(hipStreamSynchronize(s));
    return total;
}

}  // namespace spmvc
