// Exclusive prefix sum of uint32 counts: block sums, then a downsweep that
// adds the sums of the blocks before each block.  Up to kScanSelfBlocks
// blocks, every downsweep block reduces those sums itself (two launches);
// beyond that one block scans them first (three launches), since the
// blocks' own reductions grow with the square of the block count.  No
// inter-block waiting.  Used for the tile counts of the depth-sorted
// (view, Gaussian) items.
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

constexpr int64_t kScanSelfBlocks = 1024;

// SELF: `sums` holds the raw block sums; each block adds those before it
// (in 64 bits) and the last block writes the total and the capacity status.
// Otherwise `sums` holds their exclusive scan (k_scan_top).
template <bool SELF>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t *in, uint32_t *out,
                                                            int64_t n, const uint32_t *sums,
                                                            int32_t *total, int32_t *status,
                                                            int64_t cap) {
    __shared__ uint32_t lds[kScanThreads / kWave + 1];
    __shared__ uint32_t tile[kScanBlock];
    __shared__ uint64_t part[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    // coalesced load into LDS, then each thread scans kScanItems consecutive
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t j = base + (int64_t)k * kScanThreads + threadIdx.x;
        tile[k * kScanThreads + threadIdx.x] = j < n ? in[j] : 0u;
    }
    uint64_t before = 0;
    if (SELF) {
        uint64_t a = 0;
        for (int64_t k = threadIdx.x; k < (int64_t)blockIdx.x; k += kScanThreads) a += sums[k];
        for (int off = kWave / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
        if (lane_id() == 0) part[threadIdx.x / kWave] = a;
    }
    __syncthreads();
    if (SELF) {
#pragma unroll
        for (int w = 0; w < kScanThreads / kWave; ++w) before += part[w];
    } else {
        before = sums[blockIdx.x];
    }
    uint32_t loc[kScanItems];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        loc[k] = acc;
        acc += tile[threadIdx.x * kScanItems + k];
    }
    uint32_t btotal;
    const uint32_t ex = block_excl_scan(acc, lds, &btotal) + (uint32_t)before;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) tile[threadIdx.x * kScanItems + k] = ex + loc[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t j = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (j < n) out[j] = tile[k * kScanThreads + threadIdx.x];
    }
    if (SELF && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const uint64_t all = before + btotal;
        if (total) *total = (int32_t)(all > 0x7fffffffull ? 0x7fffffff : all);
        if (status && (int64_t)all > cap) *status = XG_ECAPACITY;
    }
}

}  // namespace

hipError_t launch_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, int32_t *total,
                       int32_t *status, int64_t cap, hipStream_t s) {
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    const unsigned g = (unsigned)(nb > 0 ? nb : 1);
    hipLaunchKernelGGL(k_scan_reduce, dim3(g), dim3(kScanThreads), 0, s, in, n, tmp);
    if ((int64_t)g <= kScanSelfBlocks) {
        hipLaunchKernelGGL(k_scan_down<true>, dim3(g), dim3(kScanThreads), 0, s, in, out, n, tmp, total,
                           status, cap);
    } else {
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tmp, (int64_t)g, total, status, cap);
        hipLaunchKernelGGL(k_scan_down<false>, dim3(g), dim3(kScanThreads), 0, s, in, out, n, tmp,
                           nullptr, nullptr, cap);
    }
    return hipGetLastError();
}

}  // namespace xg
