// Exclusive prefix sum of uint32 counts (reduce, scan of block sums,
// downsweep).  Three launches, no inter-block waiting.  Used for the tile
// counts of every (view, Gaussian) and for the radix-sort digit offsets.
#include "common.h"

namespace xg {

namespace {

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *in, int64_t n,
                                                              uint32_t *sums) {
    __shared__ uint32_t lds[kScanThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t j = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (j < n) acc += in[j];
    }
    uint32_t total;
    block_excl_scan(acc, lds, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block scans the block sums in chunks; writes the grand total and
// raises XG_ECAPACITY when it exceeds `cap`.
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t *sums, int64_t nb, int32_t *total,
                                                   int32_t *status, int64_t cap) {
    __shared__ uint32_t lds[1024 / kWave + 1];
    uint64_t carry = 0;
    for (int64_t c = 0; c < nb; c += blockDim.x) {
        const int64_t j = c + threadIdx.x;
        const uint32_t v = j < nb ? sums[j] : 0u;
        uint32_t t;
        const uint32_t ex = block_excl_scan(v, lds, &t);
        if (j < nb) sums[j] = (uint32_t)(carry + ex);
        carry += t;
    }
    if (threadIdx.x == 0) {
        if (total) *total = (int32_t)(carry > 0x7fffffffull ? 0x7fffffff : carry);
        if (status && (int64_t)carry > cap) *status = XG_ECAPACITY;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t *in, uint32_t *out,
                                                            int64_t n, const uint32_t *sums) {
    __shared__ uint32_t lds[kScanThreads / kWave + 1];
    __shared__ uint32_t tile[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    // coalesced load into LDS, then each thread scans kScanItems consecutive
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t j = base + (int64_t)k * kScanThreads + threadIdx.x;
        tile[k * kScanThreads + threadIdx.x] = j < n ? in[j] : 0u;
    }
    __syncthreads();
    uint32_t loc[kScanItems];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        loc[k] = acc;
        acc += tile[threadIdx.x * kScanItems + k];
    }
    uint32_t total;
    const uint32_t ex = block_excl_scan(acc, lds, &total) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) tile[threadIdx.x * kScanItems + k] = ex + loc[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t j = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (j < n) out[j] = tile[k * kScanThreads + threadIdx.x];
    }
}

}  // namespace

hipError_t launch_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, int32_t *total,
                       int32_t *status, int64_t cap, hipStream_t s) {
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    const unsigned g = (unsigned)(nb > 0 ? nb : 1);
    hipLaunchKernelGGL(k_scan_reduce, dim3(g), dim3(kScanThreads), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, (int64_t)g, total, status, cap);
    hipLaunchKernelGGL(k_scan_down, dim3(g), dim3(kScanThreads), 0, s, in, out, n, tmp);
    return hipGetLastError();
}

}  // namespace xg
