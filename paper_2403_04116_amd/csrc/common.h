// Internal definitions shared by the gfx950 kernels and the host ABI layer.
// Nothing here is part of the public C ABI (include/xg.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xg.h"

namespace xg {

constexpr int kWave = 64;

// Workspace header words (first 256 bytes of the workspace).
struct WsHeader {
    int32_t status;        // XG_OK / XG_ECAPACITY
    int32_t n_pairs;       // pairs requested by the scan (may exceed capacity)
    int32_t item_sel;      // which item key/value buffer holds the depth-sorted items
    uint32_t depth_min;    // min float32 depth bits over kept (view, Gaussian)
    uint32_t depth_max;    // max float32 depth bits
    int32_t queue_fwd;     // persistent forward tile queue head
    int32_t queue_bwd;     // persistent backward tile queue head
    int32_t done_fwd;      // persistent forward workgroups finished
    int32_t done_bwd;      // persistent backward workgroups finished
    int32_t item_passes;   // item-sort passes that moved data
    int32_t pad[54];
};
static_assert(sizeof(WsHeader) == 256, "header is one 256-byte block");

// Render record of one (view, Gaussian), written by the preprocess and read
// by every tile that lists the Gaussian: 64 bytes, one cache line, so a
// staged list entry is a single aligned gather.
//   a: (u_x - floor(u_x), u_y - floor(u_y), qa, qb)
//   b: (qc, -log2(opacity), intensity, float bits of depth)
//   c: (floor(u_x), floor(u_y), x_lo | x_hi << 16, y_lo | y_hi << 16)
//   d: unused
// (qa, qb, qc) factor the inverse 2-D covariance scaled by k = log2(e)/2:
//   k * d^T Sigma''^-1 d = (qa dx + qb dy)^2 + (qc dy)^2
// so that exp(-d^T Sigma''^-1 d / 2) = exp2(-(that)), and the opacity times
// it, the a of Eq. 10, is exp2(-(that - log2 opacity)): the blend kernels
// evaluate one exponential and no product.
struct alignas(64) Record {
    float4 a;
    float4 b;
    int4 c;
    float4 d;
};
static_assert(sizeof(Record) == 64, "one cache line per record");

// Number of XCDs workgroups are dealt to round-robin (MI355X: 8).  Used to
// give each XCD a contiguous range of tiles, so the records its L2 caches
// are shared by the tiles it renders.
constexpr int kXcds = 8;

// Tile of workgroup b in a grid of n tiles such that XCD b % kXcds takes a
// contiguous block of tiles.  A bijection on [0, n) for any n.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int x = b % kXcds, i = b / kXcds;
    const int q = n / kXcds, r = n % kXcds;
    return x * q + min(x, r) + i;
}

// Tile of workgroup b of a one-workgroup-per-tile launch over n tiles: XCD
// b % kXcds walks its contiguous block of tiles in the order the list
// builder left in `order` (longest list first, so the longest tiles start
// early and none is left to run alone at the end of the launch).  An entry
// outside [0, n) (a workspace whose lists were never built) falls back to
// the block's natural order instead of reading out of bounds.
__device__ __forceinline__ int ordered_tile(const int32_t *order, int b, int n) {
    const int i = xcd_tile(b, n);
    const int t = order[i];
    return (unsigned)t < (unsigned)n ? t : i;
}

// Device view of a workspace, resolved on the host from the layout.
struct Ws {
    WsHeader *hdr;
    Record *rec;
    uint32_t *counts;      // tiles per (view, Gaussian), in (view, Gaussian) order
    uint32_t *icounts;     // the same counts in depth-sorted item order
    uint32_t *offsets;     // exclusive scan of icounts
    uint32_t *scan_tmp;
    uint32_t *ikeys[2];    // item sort keys (float32 depth bits; 0xffffffff when culled)
    uint64_t *ivals[2];    // item sort values: (view, Gaussian) index | tile rectangle << 32
    uint32_t *ptile[2];    // pair sort keys (global tile id)
    uint32_t *pval[2];     // pair sort values (Gaussian index)
    uint32_t *ghist;       // radix sort: digit histograms [kMaxPasses][kRadix], one 128-byte line each
    uint32_t *vhist;       // item sort (within each view): digit totals [view][kMaxPasses][kRadix]
    uint32_t *bin_cnt;     // tile lists by counting: [view][partition][local tile] pair counts,
                           // then their exclusive scan down each column
    uint32_t *bin_ptot;    // tile lists by counting: pairs of each [view][partition]
    uint32_t *bin_pstart;  // tile lists by counting: first pair slot of each [view][partition]
    uint32_t *pctr;        // radix sort: partition counters [kMaxPasses]
    uint64_t *lookback[2]; // radix sort: per (partition, digit) aggregate / prefix words
    uint32_t *ranges;
    void *entry_mask;      // per list entry: the 8 x 8 sub-blocks the blending kernels visit
                           // (written by the forward, read by the backward; 1 byte, 2 for 32 x 32 tiles)
    float *grad2d;
    float *ssim;           // loss: three per-pixel SSIM partial-derivative maps, then one
                           // loss share per 48 x 8 loss strip
    int32_t *tile_order;   // persistent queue: tiles in work order
    int32_t *xcd_order;    // one-workgroup-per-tile launches: each XCD's block of tiles, longest list first
    int64_t cap;
    int64_t n_items;       // n_views * n
    int64_t total_tiles;
    int64_t total_pixels;
    int32_t n;
    int32_t n_views;
    int32_t tile_bits;     // bits of the largest global tile id
    int32_t item_blocks;   // radix-sort blocks over the items
    int32_t pair_blocks;   // radix-sort blocks over the pair capacity
    int32_t pair_passes;   // 8-bit passes over the tile id
    int32_t pair_sel;      // buffer holding the tile-sorted pairs (pair_passes & 1)
    // Packed pairs: when the tile id and the Gaussian index fit one word,
    // ptile holds tile << pair_gbits | index and pval is not used
    // (pair_gbits = 0: two arrays).  The blending kernels read the index as
    // pair_vals[p] & pair_gmask.
    int32_t pair_gbits;
    uint32_t pair_gmask;
    const uint32_t *pair_vals;
    // Tile lists by counting (bin_tiles > 0): the row length of bin_cnt (the
    // most tiles of any view) and the partitions of kBinItems items per view.
    // bin_tiles = 0: emission and the radix sort of the pairs by tile.
    int32_t bin_tiles;
    int32_t bin_ppv;
};

// Scalar constants of one rendering.
struct Params {
    float lowpass, alpha_min, alpha_max, t_min, near_z;
    float kappa;           // float32(-2 ln alpha_min): rectangle radius^2
    int32_t tile;
    int32_t lds_batch;
};

constexpr float kLog2eHalf = 0.72134752044448170368f;   // log2(e) / 2
constexpr float kInvLog2eHalf = 1.38629436111989061883f; // 2 ln 2

// Preprocess workgroups: 256 threads, one per (view, Gaussian).
constexpr int kPreThreads = 256;

// The tile rectangle of a (view, Gaussian) item packed in 32 bits and
// carried through the item sort, so the pair emission reads no record:
// first tile column and row (10 bits each), extra columns and rows (5 bits
// each), bit 30 set when the rectangle fits (else the record is read).
__host__ __device__ __forceinline__ uint32_t pack_tile_rect(int tx0, int tx1, int ty0, int ty1) {
    const int dx = tx1 - tx0, dy = ty1 - ty0;
    if (tx0 < 0 || ty0 < 0 || tx0 >= 1024 || ty0 >= 1024 || dx < 0 || dy < 0 || dx >= 32 || dy >= 32)
        return 0u;
    return (1u << 30) | (uint32_t)tx0 | ((uint32_t)ty0 << 10) | ((uint32_t)dx << 20) | ((uint32_t)dy << 25);
}
struct TileRect {
    int tx0, tx1, ty0, ty1;
};
__device__ __forceinline__ bool unpack_tile_rect(uint32_t r, TileRect &t) {
    if (!(r & (1u << 30))) return false;
    t.tx0 = (int)(r & 1023u);
    t.ty0 = (int)((r >> 10) & 1023u);
    t.tx1 = t.tx0 + (int)((r >> 20) & 31u);
    t.ty1 = t.ty0 + (int)((r >> 25) & 31u);
    return true;
}

// Tile rectangle (first/last tile column and row, view-local) of a sorted
// item from its sort value: the packed rectangle, else the record.
__device__ __forceinline__ TileRect item_tile_rect(const Ws &ws, uint64_t val, int tile) {
    TileRect tr;
    if (!unpack_tile_rect((uint32_t)(val >> 32), tr)) {
        const int4 rc = ws.rec[(uint32_t)val].c;
        tr.tx0 = (rc.z & 0xffff) / tile;
        tr.tx1 = (rc.z >> 16) / tile;
        tr.ty0 = (rc.w & 0xffff) / tile;
        tr.ty1 = (rc.w >> 16) / tile;
    }
    return tr;
}

// Lanes of the wavefront whose BITS-bit key equals this lane's (one ballot
// per key bit), restricted to `valid` lanes.
// Per bit: one ballot (a wavefront-uniform mask) and, per half of the
// mask, one XOR with the lane's all-ones-if-clear word and one AND.
template <int BITS>
__device__ __forceinline__ uint64_t match_peers(uint32_t d, bool valid) {
    const uint64_t v = __ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint32_t bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        const uint32_t inv = bit - 1u;   // 0 when the bit is set, all ones when clear
        lo &= (uint32_t)bal ^ inv;
        hi &= (uint32_t)(bal >> 32) ^ inv;
    }
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Tile lists by counting: items per partition (all of one view), pairs per
// LDS window of the ranking kernel, and the most tiles a view may have on
// this path (larger views use emission and the radix sort of the pairs).
constexpr int kBinItems = 2048;
constexpr int kBinWindow = 4096;
constexpr int kBinMaxTiles = 4096;

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;   // 2048 elements

// Radix-sort partitions (keys per workgroup = threads x keys per thread);
// larger partitions shorten the look-back chains, these sizes measured best.
constexpr int kItemSortThreads = 1024, kItemSortItems = 8;    // 8192 items
constexpr int kPairSortThreads = 1024, kPairSortItems = 16;   // 16384 pairs
constexpr int kItemSortBlock = kItemSortThreads * kItemSortItems;
constexpr int kPairSortBlock = kPairSortThreads * kPairSortItems;
// packed pairs move 4-byte keys only, so a partition holds more of them
constexpr int kPackedSortThreads = 1024, kPackedSortItems = 16;
constexpr int kPackedSortBlock = kPackedSortThreads * kPackedSortItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kMaxPasses = 4;                            // 32 depth bits, 8 at a time
constexpr int kGhStride = 32;   // words between histogram bins (spreads their atomics over channels)
constexpr int kSortCtlWords = (kMaxPasses * kRadix + kMaxPasses) * kGhStride;

// ---- launchers (one translation unit per stage) --------------------------
hipError_t launch_preprocess(const Ws &ws, const xg_gaussians &g, const xg_camera *cams,
                             const Params &p, hipStream_t s);
hipError_t launch_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                       int32_t *total, int32_t *status, int64_t cap, hipStream_t s);
hipError_t launch_sort_items(const Ws &ws, hipStream_t s);
hipError_t launch_emit(const Ws &ws, const xg_camera *cams, const Params &p, hipStream_t s);
hipError_t launch_sort_pairs(const Ws &ws, hipStream_t s);
hipError_t launch_ranges(const Ws &ws, bool cleared, hipStream_t s);  // cleared: by the pair sort
hipError_t launch_tile_order(const Ws &ws, hipStream_t s);
hipError_t launch_xcd_order(const Ws &ws, hipStream_t s);
hipError_t launch_bin_lists(const Ws &ws, const xg_camera *cams, const Params &p, hipStream_t s);
hipError_t launch_pair_keys(const Ws &ws, const xg_camera *cams, uint64_t *keys, uint32_t *vals,
                            int64_t cap, hipStream_t s);
// Per-pixel stored transmittances of the stored-list variant: count[tile][px]
// contributors, then t[tile][slot][px] = T before contributor `slot` (the
// first `slots` contributors of each pixel; px = thread index in the tile).
struct TStore {
    float *t;
    int32_t *count;
    int slots;
};

// Optional L1 epilogue of the forward blend: dl[o] = scale * sign(image[o] -
// target[o]) (sign(0) = 0), written with the image (dl null: none).
struct L1Fuse {
    const float *target;
    float *dl;
    float scale;
};
hipError_t launch_render_fwd(const Ws &ws, const xg_camera *cams, const Params &p,
                             float *image, float *final_t, int32_t *n_contrib,
                             int persistent, const TStore &ts, const L1Fuse &l1, hipStream_t s);
hipError_t launch_render_bwd(const Ws &ws, const xg_camera *cams, const Params &p,
                             const float *dl_dimage, const float *final_t,
                             const int32_t *n_contrib, int persistent, const TStore &ts,
                             hipStream_t s);
hipError_t launch_render_counts(const Ws &ws, const xg_camera *cams, const Params &p,
                                int32_t *counts, hipStream_t s);
hipError_t launch_preprocess_bwd(const Ws &ws, const xg_gaussians &g, const xg_camera *cams, bool accumulate,
                                 const Params &p, const xg_grads &gr, hipStream_t s);
hipError_t launch_sh_color(const Ws &ws, const xg_camera *cams_dev, const float *means, const float *sh,
                           int degree, hipStream_t s);
hipError_t launch_render_fwd_rgb(const Ws &ws, const xg_camera *cams, const Params &p, float *image,
                                 float *final_t, int32_t *n_contrib, hipStream_t s);
hipError_t launch_acui_grid(const double size[3], const int32_t grid[3], double d, const int32_t k[3],
                            int64_t count, float *means, hipStream_t s);
int64_t loss_tiles(const xg_camera *cams_host, int n_views);
// this device's address of the static scratch array of xg_loss_grad_static
// (resolved on the first call on each device)
hipError_t static_scratch(float **out);
hipError_t launch_loss_grad(const Ws &ws, const xg_camera *cams_dev, int64_t tiles,
                            const float *image, const float *target, float gamma, float *dl,
                            float *loss, hipStream_t s);
hipError_t launch_l1_grad(const float *image, const float *target, float *out, int64_t n,
                          float scale, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_rirf_fwd(const float *features, const float *weights, int64_t n, int nf,
                           float *intensity, hipStream_t s);
hipError_t launch_rirf_bwd(const float *features, const float *weights, int64_t n, int nf,
                           const float *dl_di, float *grad_f, hipStream_t s);
hipError_t launch_adam(const xg_params &p, const xg_grads &g, float *m, float *v, int32_t *step,
                       const xg_adam &c, float *scales, float *opacity, float *intensity,
                       const int32_t *gate, hipStream_t s);

// ---- device helpers ------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Wave-wide inclusive prefix sum of a uint32 (64 lanes).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t t = __shfl_up(v, o, kWave);
        if (l >= o) v += t;
    }
    return v;
}

// Block-wide exclusive prefix sum over blockDim.x threads (multiple of 64,
// at most 1024).  `lds` must hold blockDim.x / 64 + 1 words.  Returns the
// exclusive prefix of v; *total receives the block sum.  Contains barriers.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *lds, uint32_t *total) {
    const int l = lane_id();
    const int w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    uint32_t inc = wave_incl_scan(v);
    if (l == kWave - 1) lds[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t x = (l < nw) ? lds[l] : 0u;
        uint32_t xi = wave_incl_scan(x);
        if (l < nw) lds[l] = xi - x;
        if (l == nw - 1) lds[nw] = xi;
    }
    __syncthreads();
    uint32_t res = lds[w] + inc - v;
    *total = lds[nw];
    __syncthreads();
    return res;
}

// Work-order buckets of list lengths: eight per octave, longest first.
constexpr int kOrderBuckets = 256;
__device__ __forceinline__ int order_bucket(const Ws &ws, int64_t t) {
    const uint32_t len = ws.ranges[2 * t + 1] - ws.ranges[2 * t];
    const int l = (int)(8.0f * __log2f((float)len + 1.0f));
    return kOrderBuckets - 1 - min(l, kOrderBuckets - 1);
}

// The blend launches' tile order, one XCD's part: the workgroup (at least
// kOrderBuckets threads) orders the contiguous block of tiles that XCD x
// renders (xcd_tile) by list length, longest first, and writes it over the
// same block of xcd_order.  hist: kOrderBuckets words of LDS; scan_lds:
// blockDim.x / 64 + 1 words.
__device__ __forceinline__ void xcd_order_block(const Ws &ws, int x, uint32_t *hist, uint32_t *scan_lds) {
    const int n = (int)ws.total_tiles;
    const int q = n / kXcds, r = n % kXcds;
    const int t0 = x * q + min(x, r), t1 = t0 + q + (x < r ? 1 : 0);
    for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x) atomicAdd(&hist[order_bucket(ws, t)], 1u);
    __syncthreads();
    const uint32_t v = threadIdx.x < kOrderBuckets ? hist[threadIdx.x] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(v, scan_lds, &tot);
    if (threadIdx.x < kOrderBuckets) hist[threadIdx.x] = ex;
    __syncthreads();
    for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x) {
        const uint32_t pos = atomicAdd(&hist[order_bucket(ws, t)], 1u);
        ws.xcd_order[t0 + (int)pos] = (int32_t)t;
    }
}

// Resets the header words of a new frame other than the depth range.
__device__ __forceinline__ void frame_header_reset(WsHeader *h) {
    h->status = XG_OK;
    h->n_pairs = 0;
    h->item_sel = 0;
    h->item_passes = 0;
    h->queue_fwd = 0;
    h->queue_bwd = 0;
    h->done_fwd = 0;
    h->done_bwd = 0;
}

// Folds this workgroup's share of the preprocess's per-block depth partials
// ((min, max) pairs) into the header's depth range, which the preprocess
// set to (0xffffffff, 0).  Called by every thread of the workgroup
// (contains a barrier; at most 1024 threads).
__device__ __forceinline__ void depth_range_fold(WsHeader *h, const uint32_t *part, int64_t nparts) {
    uint32_t dmin = 0xffffffffu, dmax = 0u;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nparts;
         k += (int64_t)gridDim.x * blockDim.x) {
        dmin = min(dmin, part[2 * k]);
        dmax = max(dmax, part[2 * k + 1]);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        dmin = min(dmin, (uint32_t)__shfl_xor((int)dmin, off, kWave));
        dmax = max(dmax, (uint32_t)__shfl_xor((int)dmax, off, kWave));
    }
    __shared__ uint32_t smin[16], smax[16];
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) { smin[w] = dmin; smax[w] = dmax; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x / kWave); ++k) {
            dmin = min(dmin, smin[k]);
            dmax = max(dmax, smax[k]);
        }
        if (dmin != 0xffffffffu) atomicMin(&h->depth_min, dmin);
        if (dmax != 0u) atomicMax(&h->depth_max, dmax);
    }
}

// View index of a global tile id: the last view whose tile_offset <= tile.
__device__ __forceinline__ int view_of_tile(const xg_camera *cams, int n_views, int tile) {
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (cams[mid].tile_offset <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace xg
