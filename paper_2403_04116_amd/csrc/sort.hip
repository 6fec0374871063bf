// Stage 2 (Sec. 3.2): the per-tile, depth-ordered Gaussian lists.
//
// Two stable LSD radix sorts replace one sort of (tile | depth) keys:
//   1. items: the (view, Gaussian) records sorted by (view, depth), where
//      the depth part is compacted on the fly to (depth bits - depth_min)
//      over only the bits that vary among kept Gaussians, and culled items
//      go last; equal keys keep (view, Gaussian) index order;
//   2. pairs: the (tile, Gaussian) pairs, emitted in that item order, sorted
//      by tile id only.
// Stability makes every tile's list ordered by (depth, Gaussian index),
// exactly the order of a sort on (tile << 32 | depth bits, index), while
// the bulky pass over pairs moves 8-byte records on tile bits only.
//
// A pass is: per-block digit histograms -> exclusive scan of the
// digit-major histogram matrix (global offsets) -> scatter.  The scatter
// ranks keys stably inside a 4096-key block with wavefront ballots, stages
// them digit-sorted in LDS and writes each digit's run contiguously.
// Item passes beyond the varying bits return at once (the header records
// which buffer holds the result), so launch sequences are data independent.
#include "common.h"

namespace xg {

namespace {

struct Ctl {
    int64_t n;        // elements to sort
    uint32_t dmin;    // items: smallest kept depth bits
    int dbits;        // items: varying depth bits
    int total_bits;   // key bits to sort
};

// (view << 32 | depth bits) keys of the items.
struct ItemSort {
    using Key = uint64_t;
    static __device__ __forceinline__ Ctl ctl(const Ws &ws) {
        Ctl c;
        const WsHeader *h = ws.hdr;
        c.n = ws.n_items;
        c.dmin = h->depth_min;
        const uint32_t dmax = h->depth_max;
        c.dbits = (dmax > c.dmin) ? 32 - __clz((int)(dmax - c.dmin)) : 0;
        c.total_bits = ws.view_bits + c.dbits;
        return c;
    }
    static __device__ __forceinline__ uint32_t digit(Key key, const Ctl &c, int shift) {
        const uint64_t ck = ((key >> 32) << c.dbits) | (uint64_t)((uint32_t)key - c.dmin);
        return (uint32_t)(ck >> shift) & (kRadix - 1);
    }
    static __device__ __forceinline__ Key *keys(const Ws &ws, int b) { return ws.ikeys[b]; }
    static __device__ __forceinline__ uint32_t *vals(const Ws &ws, int b) { return ws.ivals[b]; }
    static __device__ __forceinline__ int blocks(const Ws &ws) { return ws.item_blocks; }
    static __device__ __forceinline__ void done(const Ws &ws, int pass) {
        ws.hdr->item_sel = (pass + 1) & 1;
    }
};

// Global tile ids of the pairs.
struct PairSort {
    using Key = uint32_t;
    static __device__ __forceinline__ Ctl ctl(const Ws &ws) {
        Ctl c;
        const WsHeader *h = ws.hdr;
        const int64_t np = h->n_pairs;
        c.n = (h->status != XG_OK || np > ws.cap) ? 0 : np;
        c.dmin = 0;
        c.dbits = 0;
        c.total_bits = ws.tile_bits;
        return c;
    }
    static __device__ __forceinline__ uint32_t digit(Key key, const Ctl &, int shift) {
        return (key >> shift) & (kRadix - 1);
    }
    static __device__ __forceinline__ Key *keys(const Ws &ws, int b) { return ws.ptile[b]; }
    static __device__ __forceinline__ uint32_t *vals(const Ws &ws, int b) { return ws.pval[b]; }
    static __device__ __forceinline__ int blocks(const Ws &ws) { return ws.pair_blocks; }
    static __device__ __forceinline__ void done(const Ws &, int) {}
};

template <class S>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(Ws ws, int pass) {
    const Ctl c = S::ctl(ws);
    const int shift = pass * kRadixBits;
    if (shift >= c.total_bits) return;
    __shared__ uint32_t hist[kRadix];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const typename S::Key *in = S::keys(ws, pass & 1);
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
#pragma unroll 4
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t j = base + (int64_t)k * kSortThreads + threadIdx.x;
        if (j < c.n) atomicAdd(&hist[S::digit(in[j], c, shift)], 1u);
    }
    __syncthreads();
    ws.hist[(int64_t)threadIdx.x * S::blocks(ws) + blockIdx.x] = hist[threadIdx.x];
}

template <class S>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(Ws ws, int pass) {
    using Key = typename S::Key;
    const Ctl c = S::ctl(ws);
    const int shift = pass * kRadixBits;
    if (shift >= c.total_bits) return;
    const int64_t base = (int64_t)blockIdx.x * kSortBlock;
    if (blockIdx.x == 0 && threadIdx.x == 0) S::done(ws, pass);
    if (base >= c.n) return;

    __shared__ Key skeys[kSortBlock];
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

    const Key *kin = S::keys(ws, pass & 1);
    const uint32_t *vin = S::vals(ws, pass & 1);
    Key key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rank[kSortItems];
    const int64_t wbase = base + (int64_t)w * (kSortBlock / (kSortThreads / kWave));
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t j = wbase + (int64_t)r * kWave + lane;
        const bool valid = j < c.n;
        key[r] = valid ? kin[j] : (Key)0;
        val[r] = valid ? vin[j] : 0u;
        const uint32_t d = S::digit(key[r], c, shift);
        // lanes holding the same digit, via one ballot per digit bit
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
        goff[d] = ws.hist[(int64_t)d * S::blocks(ws) + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t j = wbase + (int64_t)r * kWave + lane;
        if (j < c.n) {
            const uint32_t d = S::digit(key[r], c, shift);
            const uint32_t pos = bstart[d] + whist[w][d] + rank[r];
            skeys[pos] = key[r];
            svals[pos] = val[r];
        }
    }
    __syncthreads();
    const int64_t nvalid = min((int64_t)kSortBlock, c.n - base);
    Key *kout = S::keys(ws, (pass + 1) & 1);
    uint32_t *vout = S::vals(ws, (pass + 1) & 1);
#pragma unroll 4
    for (int k = 0; k < kSortItems; ++k) {
        const int pos = k * kSortThreads + threadIdx.x;
        if (pos < nvalid) {
            const Key kk = skeys[pos];
            const uint32_t d = S::digit(kk, c, shift);
            const uint32_t dst = goff[d] + (uint32_t)pos - bstart[d];
            kout[dst] = kk;
            vout[dst] = svals[pos];
        }
    }
}

// Item keys: (view << 32 | depth bits) for kept items, (n_views << 32 |
// depth_min) for culled ones (they sort last); values = item index.
__global__ __launch_bounds__(256) void k_item_keys(Ws ws) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ws.n_items) return;
    const int v = (int)(idx / ws.n);
    uint64_t key;
    if (ws.counts[idx] > 0)
        key = ((uint64_t)v << 32) | __float_as_uint(ws.rec[idx].b.w);
    else
        key = ((uint64_t)ws.n_views << 32) | ws.hdr->depth_min;
    ws.ikeys[0][idx] = key;
    ws.ivals[0][idx] = (uint32_t)idx;
}

// Tile counts in depth-sorted item order.
__global__ __launch_bounds__(256) void k_gather_counts(Ws ws) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ws.n_items) return;
    ws.icounts[j] = ws.counts[ws.ivals[ws.hdr->item_sel & 1][j]];
}

// ranges[2g], ranges[2g+1] = [start, end) of tile g in the sorted pairs
// (the array is zero-filled first, so empty tiles read (0, 0)).
__global__ __launch_bounds__(256) void k_ranges(Ws ws) {
    const WsHeader *h = ws.hdr;
    const int64_t np = h->n_pairs;
    const int64_t n = (h->status != XG_OK || np > ws.cap) ? 0 : np;
    const uint32_t *tiles = ws.ptile[ws.pair_sel];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t t = tiles[i];
        if (i == 0 || tiles[i - 1] != t) ws.ranges[2 * (int64_t)t] = (uint32_t)i;
        if (i == n - 1 || tiles[i + 1] != t) ws.ranges[2 * (int64_t)t + 1] = (uint32_t)(i + 1);
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

template <class S>
hipError_t radix_passes(const Ws &ws, int passes, int blocks, hipStream_t s) {
    const unsigned nb = (unsigned)(blocks > 0 ? blocks : 1);
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_radix_hist<S>, dim3(nb), dim3(kSortThreads), 0, s, ws, p);
        hipError_t e = launch_scan(ws.hist, ws.hist, (int64_t)kRadix * nb, ws.hist_tmp, nullptr,
                                   nullptr, 0, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter<S>, dim3(nb), dim3(kSortThreads), 0, s, ws, p);
    }
    return hipGetLastError();
}

unsigned grid256(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

}  // namespace

hipError_t launch_sort_items(const Ws &ws, hipStream_t s) {
    hipLaunchKernelGGL(k_item_keys, dim3(grid256(ws.n_items)), dim3(256), 0, s, ws);
    // worst case: view bits + 32 depth bits; passes past the varying bits return at once
    const int passes = (ws.view_bits + 32 + kRadixBits - 1) / kRadixBits;
    return radix_passes<ItemSort>(ws, passes, ws.item_blocks, s);
}

hipError_t launch_gather_counts(const Ws &ws, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_counts, dim3(grid256(ws.n_items)), dim3(256), 0, s, ws);
    return hipGetLastError();
}

hipError_t launch_sort_pairs(const Ws &ws, hipStream_t s) {
    return radix_passes<PairSort>(ws, ws.pair_passes, ws.pair_blocks, s);
}

hipError_t launch_tile_order(const Ws &ws, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, s, ws);
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
