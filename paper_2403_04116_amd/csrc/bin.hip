// Stage 2 (Sec. 3.2), the per-tile depth-ordered Gaussian lists, built by
// counting instead of sorting the pairs.
//
// The items (view, Gaussian) are sorted by depth within each view, so the
// items of view v sit in [v n, (v + 1) n) in (depth, Gaussian index)
// order, and their scanned tile counts give every item its pair slots.  A
// tile only lists Gaussians of its own view, in item order.  The lists are
// therefore a stable counting sort of each view's pairs by view-local tile
// id, whose digit range (the view's tiles, at most kBinMaxTiles) is small
// enough to count in LDS:
//   1. k_bin_count: per partition (kBinItems consecutive items of one
//      view), the number of pairs of each tile (LDS atomics over the items'
//      tile rectangles) -> one row of bin_cnt;
//   2. k_bin_columns: down each (view, tile) column of bin_cnt, the
//      exclusive scan over the view's partitions (four segments in parallel),
//      and the tile's total;
//   3. k_bin_starts: per view, the exclusive scan of the tile totals from
//      the view's first pair slot -> the tile ranges [start, end);
//   4. k_bin_scatter: per partition, the pairs in windows of kBinWindow
//      slots: emitted into LDS in slot order, ranked stably within the
//      window (each row of 64 slots matched by tile through an LDS table of
//      lane masks, per-wavefront counters, then a prefix over the
//      wavefronts), reordered in LDS so that each tile's pairs are
//      adjacent, and written at tile start + column prefix + rank (runs of
//      consecutive entries per tile, not one scattered word per pair).
// The result is the same (tile, depth, index) order as the radix sort of
// the pairs, element for element; no pair is read back from memory.
#include "common.h"

namespace xg {

namespace {

struct BinPart {
    int view, q;
    int64_t j0, j1;   // items [j0, j1) of the partition
    int tiles_x, tiles, toff;
};

__device__ __forceinline__ BinPart bin_part(const Ws &ws, const xg_camera *cams, int tile, int part) {
    BinPart b;
    b.view = part / ws.bin_ppv;
    b.q = part - b.view * ws.bin_ppv;
    const int64_t vbase = (int64_t)b.view * ws.n;
    b.j0 = vbase + (int64_t)b.q * kBinItems;
    b.j1 = min(b.j0 + kBinItems, vbase + ws.n);
    const xg_camera &c = cams[b.view];
    b.tiles_x = (c.width + tile - 1) / tile;
    b.tiles = b.tiles_x * ((c.height + tile - 1) / tile);
    b.toff = c.tile_offset;
    return b;
}

constexpr int kCountThreads = 256;
static_assert(kBinItems % kCountThreads == 0, "whole items per thread");

__global__ __launch_bounds__(kCountThreads) void k_bin_count(Ws ws, const xg_camera *cams, int tile) {
    __shared__ uint32_t cnt[kBinMaxTiles];
    const BinPart b = bin_part(ws, cams, tile, blockIdx.x);
    for (int t = threadIdx.x; t < b.tiles; t += kCountThreads) cnt[t] = 0;
    __syncthreads();
    const int sel = ws.hdr->item_sel & 1;
    // every item's count and sort value loaded before any is used
    constexpr int kPer = kBinItems / kCountThreads;
    uint32_t n_t[kPer];
    uint64_t val[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t j = b.j0 + (int64_t)k * kCountThreads + threadIdx.x;
        n_t[k] = j < b.j1 ? ws.icounts[j] : 0u;
        val[k] = j < b.j1 ? ws.ivals[sel][j] : 0ull;
    }
    uint32_t mine = 0;   // this thread's pairs
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (n_t[k] == 0) continue;
        mine += n_t[k];
        const TileRect r = item_tile_rect(ws, val[k], tile);
        for (int ty = r.ty0; ty <= r.ty1; ++ty)
            for (int tx = r.tx0; tx <= r.tx1; ++tx) atomicAdd(&cnt[ty * b.tiles_x + tx], 1u);
    }
    // the partition's pair total (at most kBinItems * kBinMaxTiles)
    __shared__ uint32_t s_tot[kCountThreads / kWave];
    for (int off = kWave / 2; off > 0; off >>= 1) mine += (uint32_t)__shfl_xor((int)mine, off, kWave);
    if (lane_id() == 0) s_tot[threadIdx.x / kWave] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < kCountThreads / kWave; ++w) tot += s_tot[w];
        ws.bin_ptot[blockIdx.x] = tot;
    }
    uint32_t *row = ws.bin_cnt + (int64_t)blockIdx.x * ws.bin_tiles;
    for (int t = threadIdx.x; t < b.tiles; t += kCountThreads) row[t] = cnt[t];
}

// Exclusive scan down each (view, local tile) column of bin_cnt over the
// view's partitions, rewritten in place; the column total goes to the
// tile's range start word until k_bin_starts replaces it.  A workgroup
// takes 64 columns; its four wavefronts split each column's partitions into
// four consecutive segments: each sums its segment, the segment totals are
// scanned through LDS, and each rewrites its segment from its offset.
constexpr int kColTiles = 64;
constexpr int kColSegs = 4;
constexpr int kColThreads = kColTiles * kColSegs;

__global__ __launch_bounds__(kColThreads) void k_bin_columns(Ws ws, const xg_camera *cams, int tile,
                                                             int chunks) {
    __shared__ uint32_t part[kColSegs][kColTiles];
    const int v = blockIdx.x / chunks;
    const int seg = threadIdx.x / kColTiles;
    const int t = (blockIdx.x - v * chunks) * kColTiles + (threadIdx.x % kColTiles);
    const xg_camera &c = cams[v];
    const int tiles = ((c.width + tile - 1) / tile) * ((c.height + tile - 1) / tile);
    const int64_t stride = ws.bin_tiles;
    const int per = (ws.bin_ppv + kColSegs - 1) / kColSegs;
    const int q0 = min(seg * per, ws.bin_ppv), q1 = min(q0 + per, ws.bin_ppv);
    uint32_t *col = ws.bin_cnt + (int64_t)v * ws.bin_ppv * stride + t;
    const bool live = t < tiles;
    uint32_t sum = 0;
    if (live) {
        int q = q0;
        for (; q + 8 <= q1; q += 8) {   // eight loads in flight per step
            uint32_t x[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = col[(int64_t)(q + k) * stride];
#pragma unroll
            for (int k = 0; k < 8; ++k) sum += x[k];
        }
        for (; q < q1; ++q) sum += col[(int64_t)q * stride];
    }
    part[seg][threadIdx.x % kColTiles] = sum;
    __syncthreads();
    if (!live) return;
    uint32_t run = 0, total = 0;
#pragma unroll
    for (int k = 0; k < kColSegs; ++k) {
        const uint32_t x = part[k][threadIdx.x % kColTiles];
        run += k < seg ? x : 0u;
        total += x;
    }
    int q = q0;
    for (; q + 8 <= q1; q += 8) {
        uint32_t x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = col[(int64_t)(q + k) * stride];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            col[(int64_t)(q + k) * stride] = run;
            run += x[k];
        }
    }
    for (; q < q1; ++q) {
        const uint32_t x = col[(int64_t)q * stride];
        col[(int64_t)q * stride] = run;
        run += x;
    }
    if (seg == kColSegs - 1) ws.ranges[2 * ((int64_t)c.tile_offset + t)] = total;
}

// One workgroup per view.  The view's first pair slot is the sum of the
// pair totals of the partitions of the views before it; the pair count of
// the whole frame (every workgroup sums all partitions) is checked against
// the capacity (XG_ECAPACITY, and the pair count, written by the first
// workgroup).  Then the exclusive scan of the view's partition totals
// gives each partition's first slot, and the scan of the tile totals the
// tile ranges.  Empty tiles, and all tiles once the capacity is exceeded,
// read (0, 0).
constexpr int kStartThreads = 1024;

__global__ __launch_bounds__(kStartThreads) void k_bin_starts(Ws ws, const xg_camera *cams, int tile) {
    __shared__ uint32_t lds[kStartThreads / kWave + 1];
    __shared__ uint64_t s_sum[2][kStartThreads / kWave];
    const int v = blockIdx.x;
    const xg_camera &c = cams[v];
    const int tiles = ((c.width + tile - 1) / tile) * ((c.height + tile - 1) / tile);
    const int ppv = ws.bin_ppv;
    const int64_t nparts = (int64_t)ws.n_views * ppv;
    uint64_t before = 0, all = 0;
    for (int64_t k = threadIdx.x; k < nparts; k += kStartThreads) {
        const uint32_t x = ws.bin_ptot[k];
        all += x;
        if (k < (int64_t)v * ppv) before += x;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        before += __shfl_xor(before, off, kWave);
        all += __shfl_xor(all, off, kWave);
    }
    if (lane_id() == 0) {
        s_sum[0][threadIdx.x / kWave] = before;
        s_sum[1][threadIdx.x / kWave] = all;
    }
    __syncthreads();
    before = 0;
    all = 0;
#pragma unroll
    for (int w = 0; w < kStartThreads / kWave; ++w) {
        before += s_sum[0][w];
        all += s_sum[1][w];
    }
    const bool st_ok = ws.hdr->status == XG_OK;   // an item sort that gave up keeps its XG_EHIP
    const bool ok = st_ok && all <= (uint64_t)ws.cap;
    if (v == 0 && threadIdx.x == 0) {
        ws.hdr->n_pairs = (int32_t)(all > 0x7fffffffull ? 0x7fffffffull : all);
        if (st_ok && all > (uint64_t)ws.cap) ws.hdr->status = XG_ECAPACITY;
    }
    // partition starts (below the capacity whenever they are used)
    uint32_t carry = (uint32_t)before;
    for (int q0 = 0; q0 < ppv; q0 += kStartThreads) {
        const int q = q0 + threadIdx.x;
        const uint32_t x = q < ppv ? ws.bin_ptot[(int64_t)v * ppv + q] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(x, lds, &tot);
        if (q < ppv) ws.bin_pstart[(int64_t)v * ppv + q] = carry + ex;
        carry += tot;
    }
    carry = (uint32_t)before;
    uint32_t *rg = ws.ranges + 2 * (int64_t)c.tile_offset;
    for (int t0 = 0; t0 < tiles; t0 += kStartThreads) {
        const int t = t0 + threadIdx.x;
        const uint32_t n = t < tiles ? rg[2 * t] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(n, lds, &tot);
        if (t < tiles) {
            const bool live = ok && n > 0;
            rg[2 * t] = live ? carry + ex : 0u;
            rg[2 * t + 1] = live ? carry + ex + n : 0u;
        }
        carry += tot;
    }
}

// Stable ranking and placement of one partition's pairs.  NW wavefronts;
// LT = the most view-local tiles supported (LB bits).  Per window: the
// pairs of slots [w0, w0 + kBinWindow) are emitted into LDS in slot order;
// wavefront w ranks its kBinWindow / NW consecutive slots, row by row (the
// lanes of a row holding a tile found through the lane-mask table), with a
// 16-bit counter per tile (two per word, LDS atomics from one leader lane
// per tile in a row); a prefix over the wavefronts then turns the counters
// into each wavefront's offset inside the window.  Every pair belongs at
// base[tile] + that offset + its rank, where base[tile] = the tile's start
// + the column prefix of the partition + the window's predecessors; the
// pairs are first permuted in LDS into blocks of one tile each (a
// wavefront scan of the tile totals), so that the stores of a row write
// runs of consecutive list entries.
// (16 wavefronts: at most 64 registers, so that two workgroups share a CU)
template <int LT, int NW>
__global__ __launch_bounds__(NW * kWave, NW == 16 ? 8 : 2) void k_bin_scatter(Ws ws, const xg_camera *cams,
                                                                              int tile) {
    constexpr int NT = NW * kWave;
    constexpr int LB = LT <= 1024 ? 10 : 12;
    constexpr int kRows = kBinWindow / NT;         // rows of 64 slots per wavefront
    constexpr int kMyItems = kBinItems / NT;       // items per thread
    static_assert(LT <= (1 << LB) && kBinWindow % NT == 0 && kBinItems % NT == 0, "shape");
    static_assert(kBinWindow <= 65535, "window offsets and counts fit 16 bits");
    __shared__ uint32_t h16[NW][LT / 2];
    __shared__ uint32_t base[LT];
    __shared__ uint16_t s_lt[kBinWindow];
    __shared__ uint32_t s_gi[kBinWindow];
    // the window's slots in tile order (slot of each window position), and
    // each tile's first window position (two 16-bit starts per word)
    __shared__ uint16_t s_perm[kBinWindow];
    __shared__ uint32_t s_lst[LT / 2];
    __shared__ uint32_t s_alloc;
    // ranking: per wavefront, a 64-bit lane mask for each value of a tile's
    // low kHashBits bits (zero between rows)
    constexpr int kHashBits = 6, kHash = 1 << kHashBits;
    __shared__ uint64_t s_tab[NW][kHash];

    // the first kXcds workgroups write the blend launches' tile order (the
    // ranges are final; every status, since the blends read it even when
    // the lists are empty), in slots the partitions leave idle
    if ((int)blockIdx.x < kXcds) {
        xcd_order_block(ws, blockIdx.x, base, s_lst);
        return;
    }
    const int part = (int)blockIdx.x - kXcds;
    if (ws.hdr->status != XG_OK) return;
    const BinPart b = bin_part(ws, cams, tile, part);
    if (b.j0 >= b.j1) return;
    // the partition's pair slots [S, E)
    const uint32_t S = ws.bin_pstart[part];
    const uint32_t E = S + ws.bin_ptot[part];

    for (int k = threadIdx.x; k < NW * kHash; k += NT) (&s_tab[0][0])[k] = 0ull;
    const uint32_t *colp = ws.bin_cnt + (int64_t)part * ws.bin_tiles;
    for (int t = threadIdx.x; t < b.tiles; t += NT)
        base[t] = ws.ranges[2 * ((int64_t)b.toff + t)] + colp[t];

    // this thread's items: slot range (the exclusive scan of the item
    // counts in item order, from S; also written to offsets), view-local
    // tile rectangle, index
    const int sel = ws.hdr->item_sel & 1;
    // (a view has at most kBinMaxTiles tiles: counts and tile coordinates
    // fit 16 bits)
    uint32_t i_off[kMyItems], i_gi[kMyItems];
    uint32_t i_cy[kMyItems];  // pair count | first tile row << 16
    uint32_t i_x[kMyItems];   // first | last tile column << 16
#pragma unroll
    for (int k = 0; k < kMyItems; ++k) {
        const int64_t j = b.j0 + (int64_t)threadIdx.x * kMyItems + k;
        i_cy[k] = 0;
        i_off[k] = 0;
        i_gi[k] = 0;
        i_x[k] = 0;
        if (j < b.j1) {
            const uint32_t cnt = ws.icounts[j];
            if (cnt > 0) {
                const uint64_t val = ws.ivals[sel][j];
                i_gi[k] = (uint32_t)val - (uint32_t)b.view * (uint32_t)ws.n;
                const TileRect r = item_tile_rect(ws, val, tile);
                i_x[k] = (uint32_t)r.tx0 | ((uint32_t)r.tx1 << 16);
                i_cy[k] = cnt | ((uint32_t)r.ty0 << 16);
            }
        }
    }
    {
        // a thread's items are consecutive (j0 + thread kMyItems + k): one
        // wavefront scan of the thread sums, the wavefront totals through LDS
        __shared__ uint4 s_wt[NW / 4];
        static_assert(NW % 4 == 0, "wavefront totals read four at a time");
        const int wv = threadIdx.x / kWave;
        uint32_t mine = 0;
#pragma unroll
        for (int k = 0; k < kMyItems; ++k) mine += i_cy[k] & 0xffffu;
        const uint32_t inc = wave_incl_scan(mine);
        if (lane_id() == kWave - 1) reinterpret_cast<uint32_t *>(s_wt)[wv] = inc;
        __syncthreads();
        uint32_t run = S + inc - mine;
#pragma unroll
        for (int x4 = 0; x4 < NW / 4; ++x4) {
            const uint4 t = s_wt[x4];
            run += (4 * x4 < wv ? t.x : 0u) + (4 * x4 + 1 < wv ? t.y : 0u) +
                   (4 * x4 + 2 < wv ? t.z : 0u) + (4 * x4 + 3 < wv ? t.w : 0u);
        }
#pragma unroll
        for (int k = 0; k < kMyItems; ++k) {
            i_off[k] = run;
            run += i_cy[k] & 0xffffu;
            const int64_t j = b.j0 + (int64_t)threadIdx.x * kMyItems + k;
            if (j < b.j1) ws.offsets[j] = i_off[k];
        }
    }

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    const int gb = ws.pair_gbits;
    uint32_t *out_t = ws.ptile[ws.pair_sel];
    uint32_t *out_v = ws.pval[ws.pair_sel];

    for (uint32_t w0 = S; w0 < E; w0 += kBinWindow) {
        const uint32_t w1 = min(E, w0 + (uint32_t)kBinWindow);
        const int wn = (int)(w1 - w0);
        for (int k = threadIdx.x; k < NW * (LT / 2); k += NT) (&h16[0][0])[k] = 0u;
        if (threadIdx.x == 0) s_alloc = 0u;
        // emission: each item writes its pairs inside the window, row-major
        // over its rectangle
#pragma unroll
        for (int k = 0; k < kMyItems; ++k) {
            const uint32_t cnt = i_cy[k] & 0xffffu;
            const uint32_t a = max(i_off[k], w0), e = min(i_off[k] + cnt, w1);
            if (cnt == 0 || a >= e) continue;
            const int tx0 = (int)(i_x[k] & 0xffffu), tx1 = (int)(i_x[k] >> 16);
            const uint32_t rw = (uint32_t)(tx1 - tx0 + 1);
            const uint32_t m = a - i_off[k];
            int ty = (int)(i_cy[k] >> 16) + (int)(m / rw);
            int tx = tx0 + (int)(m % rw);
            for (uint32_t s = a; s < e; ++s) {
                s_lt[s - w0] = (uint16_t)(ty * b.tiles_x + tx);
                s_gi[s - w0] = i_gi[k];
                if (++tx > tx1) {
                    tx = tx0;
                    ++ty;
                }
            }
        }
        __syncthreads();
        // ranking: wavefront w owns slots [w kRows 64, (w + 1) kRows 64)
        uint32_t rt[kRows];   // rank in the wavefront | tile << 16 (both below 2^16)
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const int slot = (w * kRows + r) * kWave + lane;
            const bool valid = slot < wn;
            const uint32_t t = valid ? s_lt[slot] : 0u;
            // lanes of the row with this tile: the lanes whose low kHashBits
            // agree (one bit each, OR-ed into this wavefront's table slot,
            // read back, then cleared; a wavefront's LDS operations complete
            // in order) that also agree in the high bits (one ballot each)
            uint64_t *slotp = &s_tab[w][t & (kHash - 1)];
            if (valid) atomicOr(reinterpret_cast<unsigned long long *>(slotp), 1ull << lane);
            const uint64_t same_low = *slotp;
            *slotp = 0ull;
            const uint64_t peers = valid ? same_low & match_peers<LB - kHashBits>(t >> kHashBits, valid) : 0ull;
            const int leader = __ffsll((unsigned long long)peers) - 1;
            uint32_t old = 0;
            if (valid && lane == leader) {
                const uint32_t sh = 16u * (t & 1u);
                old = (atomicAdd(&h16[w][t >> 1], (uint32_t)__popcll(peers) << sh) >> sh) & 0xffffu;
            }
            old = (uint32_t)__shfl((int)old, leader < 0 ? 0 : leader, kWave);
            rt[r] = (old + (uint32_t)__popcll(peers & lt_mask)) | (t << 16);
        }
        __syncthreads();
        // prefix over the wavefronts, two tiles (one word) per step; then each
        // tile's block of window positions: a wavefront scan of the word
        // totals and one allocation per wavefront (blocks in any order, each
        // tile's block contiguous)
        constexpr int kPairsPerThread = (LT / 2 + NT - 1) / NT;
        uint32_t adv[kPairsPerThread];
#pragma unroll
        for (int k = 0; k < kPairsPerThread; ++k) {
            const int tw = k * NT + threadIdx.x;
            uint32_t run = 0;   // two 16-bit sums
            if (tw < LT / 2) {
#pragma unroll
                for (int x = 0; x < NW; ++x) {
                    const uint32_t hcur = h16[x][tw];
                    h16[x][tw] = run;
                    run += hcur;   // neither half exceeds kBinWindow: no carry
                }
            }
            adv[k] = run;
            const uint32_t lo = run & 0xffffu;
            const uint32_t tot = lo + (run >> 16);
            uint32_t incl = tot;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t up = (uint32_t)__shfl_up((int)incl, d, kWave);
                if (lane >= d) incl += up;
            }
            const uint32_t wsum = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
            uint32_t wbase = 0;
            if (lane == 0 && wsum) wbase = atomicAdd(&s_alloc, wsum);
            wbase = (uint32_t)__shfl((int)wbase, 0, kWave);
            const uint32_t st = wbase + incl - tot;
            if (tw < LT / 2 && tot) s_lst[tw] = st | ((st + lo) << 16);
        }
        __syncthreads();
        // each slot's window position: its tile's block, the wavefronts
        // before it, its rank in the wavefront
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const int slot = (w * kRows + r) * kWave + lane;
            if (slot < wn) {
                const uint32_t t = rt[r] >> 16;
                const uint32_t sh = 16u * (t & 1u);
                const uint32_t off = (h16[w][t >> 1] >> sh) & 0xffffu;
                const uint32_t st = (s_lst[t >> 1] >> sh) & 0xffffu;
                s_perm[st + off + (rt[r] & 0xffffu)] = (uint16_t)slot;
            }
        }
        __syncthreads();
        // placement in tile order: consecutive positions of a tile go to
        // consecutive list entries (coalesced stores)
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const int k = (w * kRows + r) * kWave + lane;
            if (k < wn) {
                const int slot = s_perm[k];
                const uint32_t t = s_lt[slot];
                const uint32_t gi = s_gi[slot];
                const uint32_t st = (s_lst[t >> 1] >> (16u * (t & 1u))) & 0xffffu;
                const uint32_t dst = base[t] + ((uint32_t)k - st);
                const uint32_t gt = (uint32_t)b.toff + t;
                if (dst >= (uint64_t)ws.cap) continue;   // never: the counts add up to the slots
                if (gb) {
                    out_t[dst] = (gt << gb) | gi;
                } else {
                    out_t[dst] = gt;
                    out_v[dst] = gi;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPairsPerThread; ++k) {
            const int tw = k * NT + threadIdx.x;
            if (tw < LT / 2) {
                if (2 * tw < b.tiles) base[2 * tw] += adv[k] & 0xffffu;
                if (2 * tw + 1 < b.tiles) base[2 * tw + 1] += adv[k] >> 16;
            }
        }
        // the next window's counters are cleared before its ranking, after
        // the barrier that follows its emission; base is next read after that
    }
}

}  // namespace

hipError_t launch_bin_lists(const Ws &ws, const xg_camera *cams, const Params &p, hipStream_t s) {
    if (ws.bin_tiles <= 0 || ws.bin_tiles > kBinMaxTiles || ws.bin_ppv <= 0) return hipErrorInvalidValue;
    const int64_t parts = (int64_t)ws.n_views * ws.bin_ppv;
    if (parts > 0x7fffffff) return hipErrorInvalidValue;
    const unsigned np = (unsigned)parts;
    hipLaunchKernelGGL(k_bin_count, dim3(np), dim3(kCountThreads), 0, s, ws, cams, p.tile);
    const int chunks = (ws.bin_tiles + kColTiles - 1) / kColTiles;
    hipLaunchKernelGGL(k_bin_columns, dim3((unsigned)(ws.n_views * chunks)), dim3(kColThreads), 0, s, ws,
                       cams, p.tile, chunks);
    hipLaunchKernelGGL(k_bin_starts, dim3((unsigned)ws.n_views), dim3(kStartThreads), 0, s, ws, cams, p.tile);
    // kXcds extra workgroups write the blend launches' tile order
    if (ws.bin_tiles <= 1024)
        hipLaunchKernelGGL((k_bin_scatter<1024, 16>), dim3(np + kXcds), dim3(16 * kWave), 0, s, ws, cams, p.tile);
    else
        hipLaunchKernelGGL((k_bin_scatter<4096, 8>), dim3(np + kXcds), dim3(8 * kWave), 0, s, ws, cams, p.tile);
    return hipGetLastError();
}

}  // namespace xg
