// Stage 2 (Sec. 3.2): stable LSD radix sort of the (tile | depth) pairs and
// per-tile ranges.
//
// The 64-bit key (tile << 32 | depth bits) is compacted on the fly to
// (tile << dbits) | (depth - depth_min), where dbits covers only the depth
// bits that vary over the kept Gaussians; only ceil((tile_bits + dbits)/8)
// passes of 8-bit digits are active.  The host enqueues the worst-case
// number of passes; inactive passes return at once, and the header's
// sort_sel records which buffer holds the result, so the launch sequence
// is data independent (graph capturable).
//
// A pass is: per-block digit histograms -> exclusive scan of the
// digit-major histogram matrix (global offsets) -> scatter.  The scatter
// ranks keys stably inside a 4096-key block with wavefront ballots, stages
// them digit-sorted in LDS and writes each digit's run contiguously.
#include "common.h"

namespace xg {

namespace {

struct SortCtl {
    int64_t n;      // pairs to sort (0 if the capacity overflowed)
    uint32_t dmin;
    int dbits;
    int total_bits;
};

__device__ __forceinline__ SortCtl sort_ctl(const Ws &ws) {
    SortCtl c;
    const WsHeader *h = ws.hdr;
    const int64_t np = h->n_pairs;
    c.n = (h->status != XG_OK || np > ws.cap) ? 0 : np;
    c.dmin = h->depth_min;
    const uint32_t dmax = h->depth_max;
    c.dbits = (dmax > c.dmin) ? 32 - __clz((int)(dmax - c.dmin)) : 0;
    c.total_bits = ws.tile_bits + c.dbits;
    return c;
}

__device__ __forceinline__ uint32_t digit_of(uint64_t key, const SortCtl &c, int shift) {
    const uint64_t ck = ((key >> 32) << c.dbits) | (uint64_t)((uint32_t)key - c.dmin);
    return (uint32_t)(ck >> shift) & (kRadix - 1);
}

__global__ __launch_bounds__(kSortThreads) void k_sort_hist(Ws ws, int pass) {
    const SortCtl c = sort_ctl(ws);
    const int shift = pass * kRadixBits;
    if (shift >= c.total_bits) return;
    __shared__ uint32_t hist[kRadix];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t *in = ws.keys[pass & 1];
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
#pragma unroll 4
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t j = base + (int64_t)k * kSortThreads + threadIdx.x;
        if (j < c.n) atomicAdd(&hist[digit_of(in[j], c, shift)], 1u);
    }
    __syncthreads();
    ws.hist[(int64_t)threadIdx.x * ws.hist_blocks + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(Ws ws, int pass) {
    const SortCtl c = sort_ctl(ws);
    const int shift = pass * kRadixBits;
    if (shift >= c.total_bits) return;
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
    if (blockIdx.x == 0 && threadIdx.x == 0) ws.hdr->sort_sel = (pass + 1) & 1;
    if (base >= c.n) return;

    __shared__ uint64_t skeys[kSortBlock];
    __shared__ uint32_t svals[kSortBlock];
    __shared__ uint32_t whist[kSortThreads / kWave][kRadix];
    __shared__ uint32_t bstart[kRadix];
    __shared__ uint32_t goff[kRadix];
    __shared__ uint32_t scan_lds[kSortThreads / kWave + 1];

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    for (int k = 0; k < kSortThreads / kWave; ++k) whist[k][threadIdx.x] = 0;
    __syncthreads();

    const uint64_t *kin = ws.keys[pass & 1];
    const uint32_t *vin = ws.values[pass & 1];
    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rank[kSortItems];
    const int64_t wbase = base + (int64_t)w * (kSortBlock / (kSortThreads / kWave));
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t j = wbase + (int64_t)r * kWave + lane;
        const bool valid = j < c.n;
        key[r] = valid ? kin[j] : 0ull;
        val[r] = valid ? vin[j] : 0u;
        const uint32_t d = digit_of(key[r], c, shift);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        uint32_t old = 0;
        const int leader = __ffsll((unsigned long long)peers) - 1;
        if (valid && lane == leader) old = atomicAdd(&whist[w][d], (uint32_t)__popcll(peers));
        old = (uint32_t)__shfl((int)old, leader < 0 ? 0 : leader, kWave);
        rank[r] = old + (uint32_t)__popcll(peers & lt_mask);
    }
    __syncthreads();
    {
        // per digit: prefix over waves, block-local digit start, global offset
        const int d = threadIdx.x;
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < kSortThreads / kWave; ++k) {
            const uint32_t t = whist[k][d];
            whist[k][d] = acc;
            acc += t;
        }
        uint32_t tot;
        bstart[d] = block_excl_scan(acc, scan_lds, &tot);
        goff[d] = ws.hist[(int64_t)d * ws.hist_blocks + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t j = wbase + (int64_t)r * kWave + lane;
        if (j < c.n) {
            const uint32_t d = digit_of(key[r], c, shift);
            const uint32_t pos = bstart[d] + whist[w][d] + rank[r];
            skeys[pos] = key[r];
            svals[pos] = val[r];
        }
    }
    __syncthreads();
    const int64_t nvalid = min((int64_t)kSortBlock, c.n - base);
    uint64_t *kout = ws.keys[(pass + 1) & 1];
    uint32_t *vout = ws.values[(pass + 1) & 1];
#pragma unroll 4
    for (int k = 0; k < kSortItems; ++k) {
        const int pos = k * kSortThreads + threadIdx.x;
        if (pos < nvalid) {
            const uint64_t kk = skeys[pos];
            const uint32_t d = digit_of(kk, c, shift);
            const uint32_t dst = goff[d] + (uint32_t)pos - bstart[d];
            kout[dst] = kk;
            vout[dst] = svals[pos];
        }
    }
}

// ranges[2g], ranges[2g+1] = [start, end) of tile g in the sorted pairs
// (the array is zero-filled first, so empty tiles read (0, 0)).
__global__ __launch_bounds__(256) void k_ranges(Ws ws) {
    const WsHeader *h = ws.hdr;
    const int64_t np = h->n_pairs;
    const int64_t n = (h->status != XG_OK || np > ws.cap) ? 0 : np;
    const uint64_t *keys = ws.keys[h->sort_sel & 1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t t = (uint32_t)(keys[i] >> 32);
        if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ws.ranges[2 * (int64_t)t] = (uint32_t)i;
        if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) != t) ws.ranges[2 * (int64_t)t + 1] = (uint32_t)(i + 1);
    }
}

// Work order for the persistent blending kernels: tiles bucketed by list
// length on a logarithmic scale (8 buckets per octave), longest first, so
// the heaviest tiles start early and the tail of the launch stays short.
// One workgroup; the order inside a bucket is arbitrary (it only affects
// scheduling, not results).
constexpr int kOrderBuckets = 256;

__global__ __launch_bounds__(1024) void k_tile_order(Ws ws) {
    __shared__ uint32_t hist[kOrderBuckets];
    __shared__ uint32_t scan_lds[1024 / kWave + 1];
    const int64_t nt = ws.total_tiles;
    for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    auto key = [&](int64_t t) -> int {
        const uint32_t len = ws.ranges[2 * t + 1] - ws.ranges[2 * t];
        const int l = (int)(8.0f * __log2f((float)len + 1.0f));
        return kOrderBuckets - 1 - min(l, kOrderBuckets - 1);
    };
    for (int64_t t = threadIdx.x; t < nt; t += blockDim.x) atomicAdd(&hist[key(t)], 1u);
    __syncthreads();
    const uint32_t v = threadIdx.x < kOrderBuckets ? hist[threadIdx.x] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(v, scan_lds, &tot);
    if (threadIdx.x < kOrderBuckets) hist[threadIdx.x] = ex;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < nt; t += blockDim.x) {
        const uint32_t pos = atomicAdd(&hist[key(t)], 1u);
        ws.tile_order[pos] = (int32_t)t;
    }
}

}  // namespace

hipError_t launch_tile_order(const Ws &ws, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, s, ws);
    return hipGetLastError();
}

hipError_t launch_sort(const Ws &ws, hipStream_t s) {
    const int passes = (ws.tile_bits + 32 + kRadixBits - 1) / kRadixBits;
    const unsigned nb = (unsigned)(ws.hist_blocks > 0 ? ws.hist_blocks : 1);
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_sort_hist, dim3(nb), dim3(kSortThreads), 0, s, ws, p);
        hipError_t e = launch_scan(ws.hist, ws.hist, (int64_t)kRadix * ws.hist_blocks, ws.hist_tmp,
                                   nullptr, nullptr, 0, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_sort_scatter, dim3(nb), dim3(kSortThreads), 0, s, ws, p);
    }
    return hipGetLastError();
}

hipError_t launch_ranges(const Ws &ws, hipStream_t s) {
    hipError_t e = launch_fill_u32(ws.ranges, 0u, 2 * ws.total_tiles, s);
    if (e != hipSuccess) return e;
    int64_t nb = (ws.cap + 255) / 256;
    if (nb > 16384) nb = 16384;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(256), 0, s, ws);
    return hipGetLastError();
}

}  // namespace xg
