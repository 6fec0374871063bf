// Stage 2 (Sec. 3.2): the per-tile, depth-ordered Gaussian lists.
//
// Two stable LSD radix sorts replace one sort of (tile | depth) keys:
//   1. items: the (view, Gaussian) records of each view sorted by depth
//      bits alone (a segmented sort: view v's items stay in [v n, (v+1) n),
//      every view starts its own partitions, digit totals and look-back
//      chains), compacted on the fly to (depth bits - depth_min) over only
//      the bits that vary among kept Gaussians (culled items carry the
//      largest key); equal keys keep Gaussian index order;
//   2. pairs: the (tile, Gaussian) pairs, emitted in that item order, sorted
//      by tile id only.  When every view has few enough tiles the lists are
//      built by counting instead (bin.hip) and this sort is not used.
// A tile only lists Gaussians of its own view, and those appear in the
// item order by (depth, Gaussian index); stability carries that order into
// every tile's list, exactly the order of a sort on (tile << 32 | depth
// bits, index), while each pass moves 8-byte records.
//
// Each sort is one histogram launch (the digit counts of every pass in one
// read of the keys) and one launch per 8-bit pass, in the single-pass
// ("onesweep") form: a workgroup takes the next partition (8192 items or
// 16384 pairs) from an atomic counter, ranks its keys stably (rows of 64
// keys matched by digit through a per-wavefront LDS table of lane masks,
// or by ballots), publishes its per-digit counts, stages its keys
// digit-sorted in LDS, reads the
// running prefix of the partitions before it from their published words
// (decoupled look-back: a partition waits only on ones that started before
// it, and those publish their counts without waiting, so it always
// finishes) and writes each digit's run contiguously.  Item passes past the varying bits are skipped without
// moving data (the header records which buffer holds the result), so launch
// sequences are data independent.  When the tile id and the Gaussian index
// fit one 32-bit word, the pairs are sorted as single packed keys.
#include "common.h"

namespace xg {

namespace {

struct Ctl {
    int64_t n;        // elements to sort
    uint32_t dmin;    // items: smallest kept depth bits
    uint32_t dmax;    // items: largest kept depth bits
    int dbits;        // items: varying depth bits
    int total_bits;   // key bits to sort
};

// Float32 depth bits of the items (0xffffffff for culled items, which the
// digit clamps to the largest kept depth).
struct ItemSort {
    using Key = uint32_t;
    using Val = uint64_t;   // item index | packed tile rectangle << 32
    static __device__ __forceinline__ Ctl ctl(const Ws &ws) {
        Ctl c;
        const WsHeader *h = ws.hdr;
        c.n = ws.n_items;
        c.dmin = h->depth_min;
        c.dmax = h->depth_max;
        c.dbits = (c.dmax > c.dmin) ? 32 - __clz((int)(c.dmax - c.dmin)) : 0;
        c.total_bits = c.dbits;
        return c;
    }
    static __device__ __forceinline__ uint32_t digit(Key key, const Ctl &c, int shift) {
        return ((min(key, c.dmax) - c.dmin) >> shift) & (kRadix - 1);
    }
    static __device__ __forceinline__ Key *keys(const Ws &ws, int b) { return ws.ikeys[b]; }
    static __device__ __forceinline__ Val *vals(const Ws &ws, int b) { return ws.ivals[b]; }
    // tile count of an item from its value (packed rectangle, else the count array)
    static __device__ __forceinline__ uint32_t count_of(const Ws &ws, Val v) {
        TileRect t;
        if (unpack_tile_rect((uint32_t)(v >> 32), t))
            return (uint32_t)((t.tx1 - t.tx0 + 1) * (t.ty1 - t.ty0 + 1));
        return ws.counts[(uint32_t)v];
    }
    static __device__ __forceinline__ int blocks(const Ws &ws) { return ws.item_blocks; }
    static constexpr int kThreads = kItemSortThreads, kItems = kItemSortItems;
    static constexpr bool kHasVal = true;
    static constexpr bool kTabRank = true;   // LDS lane-mask table for the ranking (see k_onesweep)
    // sorted within each view: the items of view v stay in [v n, (v + 1) n)
    static constexpr bool kSegmented = true;
    static __device__ __forceinline__ int64_t seg_len(const Ws &ws) { return ws.n; }
    // passes whose digit is the same for every key could be skipped, but
    // after the compaction to the varying depth bits that is rare, and
    // finding out costs every partition of every pass four block-wide
    // reductions over the histograms
    static constexpr bool kSkipConstant = false;
    // the last pass that moves data also writes the tile counts in sorted order
    static constexpr bool kGatherCounts = true;
    static constexpr bool kClearRanges = false;
    // the result sits in buffer (passes that moved data) & 1
    static __device__ __forceinline__ void done(const Ws &ws, int nrun) {
        ws.hdr->item_sel = nrun & 1;
        ws.hdr->item_passes = nrun;
    }
};

// Global tile ids of the pairs.
struct PairSort {
    using Key = uint32_t;
    using Val = uint32_t;
    static __device__ __forceinline__ Ctl ctl(const Ws &ws) {
        Ctl c;
        const WsHeader *h = ws.hdr;
        const int64_t np = h->n_pairs;
        c.n = (h->status != XG_OK || np > ws.cap) ? 0 : np;
        c.dmin = 0;
        c.dmax = 0;
        c.dbits = 0;
        c.total_bits = ws.tile_bits;
        return c;
    }
    static __device__ __forceinline__ uint32_t digit(Key key, const Ctl &, int shift) {
        return (key >> shift) & (kRadix - 1);
    }
    static __device__ __forceinline__ Key *keys(const Ws &ws, int b) { return ws.ptile[b]; }
    static __device__ __forceinline__ Val *vals(const Ws &ws, int b) { return ws.pval[b]; }
    static __device__ __forceinline__ uint32_t count_of(const Ws &, Val) { return 0; }
    static __device__ __forceinline__ int blocks(const Ws &ws) { return ws.pair_blocks; }
    static constexpr int kThreads = kPairSortThreads, kItems = kPairSortItems;
    static constexpr bool kHasVal = true;
    static constexpr bool kTabRank = false;  // its keys and values fill the LDS
    static constexpr bool kSegmented = false;
    static __device__ __forceinline__ int64_t seg_len(const Ws &) { return 0; }
    static constexpr bool kGatherCounts = false;
    // the tile ranges are cleared here, ahead of k_ranges
    static constexpr bool kClearRanges = true;
    // every pass runs, so the result buffer (pair_passes & 1) is known on the host
    static constexpr bool kSkipConstant = false;
    static __device__ __forceinline__ void done(const Ws &, int) {}
};

// Packed pairs (tile id << gbits | Gaussian index in one word): the same
// sort on the tile bits above the index, with no value array.
struct PackedPairSort {
    using Key = uint32_t;
    using Val = uint32_t;   // unused
    static __device__ __forceinline__ Ctl ctl(const Ws &ws) {
        Ctl c = PairSort::ctl(ws);
        c.dbits = ws.pair_gbits;   // the index bits below the tile id
        return c;
    }
    static __device__ __forceinline__ uint32_t digit(Key key, const Ctl &c, int shift) {
        return (key >> (c.dbits + shift)) & (kRadix - 1);
    }
    static __device__ __forceinline__ Key *keys(const Ws &ws, int b) { return ws.ptile[b]; }
    static __device__ __forceinline__ Val *vals(const Ws &, int) { return nullptr; }
    static __device__ __forceinline__ uint32_t count_of(const Ws &, Val) { return 0; }
    static __device__ __forceinline__ int blocks(const Ws &ws) { return ws.pair_blocks; }
    static constexpr int kThreads = kPackedSortThreads, kItems = kPackedSortItems;
    static constexpr bool kHasVal = false;
    static constexpr bool kTabRank = true;
    static constexpr bool kSegmented = false;
    static __device__ __forceinline__ int64_t seg_len(const Ws &) { return 0; }
    static constexpr bool kGatherCounts = false;
    static constexpr bool kClearRanges = true;
    static constexpr bool kSkipConstant = false;
    static __device__ __forceinline__ void done(const Ws &, int) {}
};

// Look-back words: flag in bits 62-63, count in the low 32 bits.
constexpr uint64_t kLbAggregate = 1ull << 62;   // this partition's own digit count
constexpr uint64_t kLbPrefix = 2ull << 62;      // inclusive prefix through this partition
// Polls of a predecessor's word before a partition gives up (it never has
// to in a correct launch: predecessors publish before they wait); the sort
// then reports XG_EHIP through the status word instead of hanging.
constexpr uint32_t kSpinLimit = 1u << 20;
constexpr int kLookback = 4;     // predecessors read per look-back step

// Partitions of one sort.  Unsegmented: kBlock consecutive keys each.
// Segmented (the items, sorted within each view): every segment of seg_len
// keys starts a new partition, so partition p belongs to segment p / ppv.
template <class S>
struct Parts {
    int64_t ppv;     // partitions per segment (all of them when unsegmented)
    int64_t parts;   // partitions of the sort
    int64_t seg;     // keys per segment (n when unsegmented)
    __device__ __forceinline__ Parts(const Ws &ws, const Ctl &c) {
        constexpr int64_t kBlock = S::kThreads * S::kItems;
        if constexpr (S::kSegmented) {
            seg = S::seg_len(ws);
            ppv = (seg + kBlock - 1) / kBlock;
            parts = c.n > 0 ? ppv * (c.n / (seg > 0 ? seg : 1)) : 0;
        } else {
            seg = c.n;
            ppv = (c.n + kBlock - 1) / kBlock;
            parts = ppv;
        }
    }
    // first key of partition p's segment, and the end of that segment
    __device__ __forceinline__ int64_t seg_base(int64_t p) const { return S::kSegmented ? (p / ppv) * seg : 0; }
    __device__ __forceinline__ int64_t first_part(int64_t p) const { return S::kSegmented ? (p / ppv) * ppv : 0; }
};

// Digit totals of a sort: one 128-byte line per (pass, digit) bin for the
// unsegmented sorts (their histogram atomics come from many workgroups),
// dense [segment][pass][digit] words for the segmented one.
template <class S>
__device__ __forceinline__ uint32_t *digit_bin(const Ws &ws, int64_t segment, int pass, int d) {
    if constexpr (S::kSegmented)
        return ws.vhist + (segment * kMaxPasses + pass) * kRadix + d;
    else
        return ws.ghist + (pass * kRadix + d) * kGhStride;
}

// Zeroes the digit histograms, partition counters and the first pass's
// look-back words of one sort.  The item sort's (depth_part set) also
// resets the frame header (workgroup 0) and folds the preprocess's depth
// partials into the depth range (every workgroup a share, atomically):
// nothing here depends on those words.
template <class S>
__global__ __launch_bounds__(256) void k_sort_prep(Ws ws, const uint32_t *depth_part, int64_t nparts) {
    if (depth_part != nullptr) {
        if (blockIdx.x == 0 && threadIdx.x == 0) frame_header_reset(ws.hdr);
        depth_range_fold(ws.hdr, depth_part, nparts);
    }
    const Ctl c = S::ctl(ws);
    const int64_t parts = Parts<S>(ws, c).parts;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = i0; i < kSortCtlWords; i += stride) ws.ghist[i] = 0;
    if (S::kSegmented)
        for (int64_t i = i0; i < (int64_t)ws.n_views * kMaxPasses * kRadix; i += stride) ws.vhist[i] = 0;
    for (int64_t i = i0; i < parts * kRadix; i += stride) ws.lookback[0][i] = 0;
    if (S::kClearRanges)
        for (int64_t i = i0; i < 2 * ws.total_tiles; i += stride) ws.ranges[i] = 0;
}

// Digit histograms of every pass in one read of the keys: LDS counters
// (LDS atomics) summed per workgroup into the global bins.  Neighbouring
// keys often share their high digits (the pairs of one item), so each bin
// has kHistCopies interleaved copies and lane l counts into copy l mod
// kHistCopies: lanes with equal digits then hit different banks instead
// of serialising on one word.  A grid of at most one workgroup per CU
// strides over the keys, so each global bin receives few atomics.
constexpr int kHistCopies = 8;

template <class S>
__global__ __launch_bounds__(S::kThreads) void k_sort_hist(Ws ws, int passes) {
    using Key = typename S::Key;
    constexpr int kSortThreads = S::kThreads, kSortItems = S::kItems;
    constexpr int kSortBlock = kSortThreads * kSortItems;
    const Ctl c = S::ctl(ws);
    __shared__ uint32_t hist[kMaxPasses][kRadix][kHistCopies];
    const int copy = lane_id() & (kHistCopies - 1);
    for (int i = threadIdx.x; i < kMaxPasses * kRadix * kHistCopies; i += kSortThreads)
        (&hist[0][0][0])[i] = 0;
    __syncthreads();
    const Key *in = S::keys(ws, 0);
    // unsegmented: the grid strides over all keys; segmented: workgroup p
    // counts the keys of partition p into its segment's bins
    const Parts<S> P(ws, c);
    int64_t first = (int64_t)blockIdx.x * kSortBlock, end = c.n, stride = (int64_t)gridDim.x * kSortBlock;
    int64_t segment = 0;
    if constexpr (S::kSegmented) {
        const int64_t p = blockIdx.x;
        segment = P.ppv > 0 ? p / P.ppv : 0;
        first = P.seg_base(p) + (p - P.first_part(p)) * kSortBlock;
        end = min(P.seg_base(p) + P.seg, c.n);
        stride = c.n;   // one partition
        if (p >= P.parts) end = 0;
    }
    for (int64_t base = first; base < end; base += stride) {
        // all loads first (indices clamped into range), then the counting
        Key key[kSortItems];
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const int64_t j = base + (int64_t)k * kSortThreads + threadIdx.x;
            key[k] = in[j < end ? j : end - 1];
        }
        for (int q = 0; q < passes; ++q) {
            if (q * kRadixBits >= c.total_bits) break;
#pragma unroll
            for (int k = 0; k < kSortItems; ++k) {
                const int64_t j = base + (int64_t)k * kSortThreads + threadIdx.x;
                if (j < end) atomicAdd(&hist[q][S::digit(key[k], c, q * kRadixBits)][copy], 1u);
            }
        }
        if (S::kSegmented) break;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * kRadix; i += kSortThreads) {
        const int q = i / kRadix, d = i % kRadix;
        uint32_t h = 0;
#pragma unroll
        for (int k = 0; k < kHistCopies; ++k) h += hist[q][d][k];
        if (h) atomicAdd(digit_bin<S>(ws, segment, q, d), h);
    }
}

// One stable LSD pass on digit `pass` of `passes` launched.
template <class S>
__global__ __launch_bounds__(S::kThreads) void k_onesweep(Ws ws, int pass, int passes) {
    using Key = typename S::Key;
    constexpr int kSortThreads = S::kThreads, kSortItems = S::kItems;
    constexpr int kSortBlock = kSortThreads * kSortItems;
    const Ctl c = S::ctl(ws);
    const int shift = pass * kRadixBits;
    const Parts<S> PP(ws, c);
    const int64_t parts = PP.parts;

    __shared__ Key skeys[kSortBlock];
    using Val = typename S::Val;
    __shared__ Val svals[S::kHasVal ? kSortBlock : 1];
    __shared__ uint32_t whist[kSortThreads / kWave][kRadix];
    // kTabRank: per wavefront and digit, the 64-bit mask of the row's lanes
    // holding that digit (zero between rows)
    __shared__ uint64_t stab[S::kTabRank ? kSortThreads / kWave : 1][S::kTabRank ? kRadix : 1];
    __shared__ uint32_t bstart[kRadix];
    __shared__ uint32_t goff[kRadix];
    __shared__ uint32_t scan_lds[kSortThreads / kWave + 1];
    __shared__ int s_part;

    // The look-back words of the next pass are cleared here (this pass does
    // not use them; the previous pass, which did, has finished).
    {
        uint64_t *next = ws.lookback[(pass + 1) & 1];
        const int64_t slot = blockIdx.x;
        if (slot < parts && threadIdx.x < kRadix) next[slot * kRadix + threadIdx.x] = 0;
    }

    // Which passes move data: those inside the key's bits, and (items) whose
    // digit is not the same for every key.  Every workgroup derives the same
    // plan from the histograms.
    int nrun_before = 0, nrun_total = 0;
    bool run_this = false;
    for (int q = 0; q < passes; ++q) {
        bool run = q * kRadixBits < c.total_bits && c.n > 0;
        if (run && S::kSkipConstant)
            run = !__syncthreads_or(threadIdx.x < kRadix &&
                                    ws.ghist[(q * kRadix + threadIdx.x) * kGhStride] == (uint32_t)c.n);
        if (run && q < pass) ++nrun_before;
        if (q == pass) run_this = run;
        if (run) ++nrun_total;
    }
    // the item sort always moves its data at least once (its last pass writes
    // the tile counts in sorted order), even when every key is equal
    if (S::kGatherCounts && nrun_total == 0 && c.n > 0) {
        nrun_total = 1;
        run_this = pass == 0;
    }
    const int in_sel = S::kSkipConstant ? (nrun_before & 1) : (pass & 1);
    const bool last_run = nrun_before + 1 == nrun_total;
    if (pass == passes - 1 && blockIdx.x == 0 && threadIdx.x == 0) S::done(ws, nrun_total);
    if (!run_this) return;

    if (threadIdx.x == 0) s_part = (int)atomicAdd(&ws.pctr[pass * kGhStride], 1u);
    for (int i = threadIdx.x; i < (kSortThreads / kWave) * kRadix; i += kSortThreads)
        (&whist[0][0])[i] = 0;
    if constexpr (S::kTabRank)
        for (int i = threadIdx.x; i < (kSortThreads / kWave) * kRadix; i += kSortThreads)
            (&stab[0][0])[i] = 0ull;
    __syncthreads();
    const int64_t part = s_part;
    if (part >= parts) return;
    // this partition's keys [base, base + kSortBlock) inside its segment
    // [sbase, send); its look-back stops at the segment's first partition p0
    const int64_t sbase = PP.seg_base(part);
    const int64_t p0 = PP.first_part(part);
    const int64_t send = S::kSegmented ? min(sbase + PP.seg, c.n) : c.n;
    const int64_t base = sbase + (part - p0) * kSortBlock;
    const int64_t segment = S::kSegmented ? part / PP.ppv : 0;

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    const Key *kin = S::keys(ws, in_sel);
    const Val *vin = S::vals(ws, in_sel);
    Key key[kSortItems];
    Val val[kSortItems];
    uint32_t rank[kSortItems];
    const int64_t wbase = base + (int64_t)w * (kSortBlock / (kSortThreads / kWave));
    // all loads first (indices clamped into range), so they overlap
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t j = wbase + (int64_t)r * kWave + lane;
        const int64_t jc = j < send ? j : send - 1;
        key[r] = kin[jc];
        if constexpr (S::kHasVal) val[r] = vin[jc];
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t j = wbase + (int64_t)r * kWave + lane;
        const bool valid = j < send;
        const uint32_t d = S::digit(key[r], c, shift);
        // lanes of the row with this digit: each valid lane ORs its bit into
        // the digit's slot of this wavefront's table, reads the slot back,
        // and every lane clears its slot (a wavefront's LDS operations
        // complete in order); or one ballot per digit bit
        uint64_t peers;
        if constexpr (S::kTabRank) {
            uint64_t *sp = &stab[w][d];
            if (valid) atomicOr(reinterpret_cast<unsigned long long *>(sp), 1ull << lane);
            const uint64_t got = *sp;
            *sp = 0ull;
            peers = valid ? got : 0ull;
        } else {
            peers = match_peers<kRadixBits>(d, valid);
        }
        uint32_t old = 0;
        const int leader = __ffsll((unsigned long long)peers) - 1;
        if (valid && lane == leader) old = atomicAdd(&whist[w][d], (uint32_t)__popcll(peers));
        old = (uint32_t)__shfl((int)old, leader < 0 ? 0 : leader, kWave);
        rank[r] = old + (uint32_t)__popcll(peers & lt_mask);
    }
    __syncthreads();
    // Threads d < 256 each own digit d.  They turn the per-wave counts into
    // exclusive per-wave offsets and publish the partition's count of the
    // digit at once; the keys are then staged digit-sorted in LDS (their
    // registers free) before the look-back for the global offsets.
    const int d = threadIdx.x;
    const bool dig = d < kRadix;
    uint32_t acc = 0;
    uint64_t *lb = ws.lookback[pass & 1];
    if (dig) {
#pragma unroll
        for (int k = 0; k < kSortThreads / kWave; ++k) {
            const uint32_t t = whist[k][d];
            whist[k][d] = acc;
            acc += t;
        }
        __hip_atomic_store(lb + part * kRadix + d, (part == p0 ? kLbPrefix : kLbAggregate) | acc,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // global start of digit d (keys with smaller digits) and its start in
    // this partition
    uint32_t tot;
    const uint32_t dstart = block_excl_scan(dig ? *digit_bin<S>(ws, segment, pass, d) : 0u, scan_lds, &tot);
    const uint32_t bs = block_excl_scan(acc, scan_lds, &tot);
    if (dig) bstart[d] = bs;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t j = wbase + (int64_t)r * kWave + lane;
        if (j < send) {
            const uint32_t dr = S::digit(key[r], c, shift);
            const uint32_t pos = bstart[dr] + whist[w][dr] + rank[r];
            skeys[pos] = key[r];
            if constexpr (S::kHasVal) svals[pos] = val[r];
        }
    }
    if (dig) {
        // Look back over a window of kLookback predecessors at a time (their
        // words are loaded together): add aggregates until a prefix; a
        // predecessor that has not published yet is polled again.
        uint32_t excl = 0, spins = 0;
        bool failed = false;
        for (int64_t q = part - 1; q >= p0;) {
            uint64_t word[kLookback];
#pragma unroll
            for (int k = 0; k < kLookback; ++k)
                word[k] = (q - k >= p0) ? __hip_atomic_load(lb + (q - k) * kRadix + d, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT)
                                        : kLbPrefix;     // before the segment's first partition: prefix 0
            int used = 0;
            bool stop = false, wait = false;
#pragma unroll
            for (int k = 0; k < kLookback; ++k) {
                if (stop || wait) continue;
                const uint64_t flag = word[k] & (3ull << 62);
                if (flag == 0) {
                    wait = true;
                } else {
                    excl += (uint32_t)word[k];
                    ++used;
                    stop = flag == kLbPrefix;
                }
            }
            if (stop) break;
            q -= used;
            if (wait) {
                if (++spins > kSpinLimit) {
                    failed = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (part != p0)
            __hip_atomic_store(lb + part * kRadix + d, kLbPrefix | (uint32_t)(excl + acc), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (failed) __hip_atomic_store(&ws.hdr->status, (int32_t)XG_EHIP, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        goff[d] = (uint32_t)sbase + dstart + excl;
    }
    __syncthreads();
    const int64_t nvalid = min((int64_t)kSortBlock, send - base);
    Key *kout = S::keys(ws, in_sel ^ 1);
    Val *vout = S::vals(ws, in_sel ^ 1);
#pragma unroll 4
    for (int k = 0; k < kSortItems; ++k) {
        const int pos = k * kSortThreads + threadIdx.x;
        if (pos < nvalid) {
            const Key kk = skeys[pos];
            const uint32_t dk = S::digit(kk, c, shift);
            const uint32_t dst = goff[dk] + (uint32_t)pos - bstart[dk];
            if (dst < (uint64_t)send) {   // always true unless a look-back gave up
                kout[dst] = kk;
                if constexpr (S::kHasVal) {
                    vout[dst] = svals[pos];
                    if (S::kGatherCounts && last_run) ws.icounts[dst] = S::count_of(ws, svals[pos]);
                }
            }
        }
    }
}

// ranges[2g], ranges[2g+1] = [start, end) of tile g in the sorted pairs
// (the array is zero-filled first, so empty tiles read (0, 0)).
// Each thread takes kRangeRun consecutive sorted keys (vector loads when
// the run lies inside the pairs) plus the key before and after the run.
constexpr int kRangeRun = 16;

__global__ __launch_bounds__(256) void k_ranges(Ws ws) {
    const WsHeader *h = ws.hdr;
    const int64_t np = h->n_pairs;
    const int64_t n = (h->status != XG_OK || np > ws.cap) ? 0 : np;
    const uint32_t *tiles = ws.ptile[ws.pair_sel];
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRangeRun;
    if (i0 >= n) return;
    uint32_t t[kRangeRun + 2];
    const int gb = ws.pair_gbits;   // packed pairs: the tile id sits above the index bits
    t[0] = i0 > 0 ? tiles[i0 - 1] >> gb : 0xffffffffu;
    if (i0 + kRangeRun <= n) {
        const uint4 *v = reinterpret_cast<const uint4 *>(tiles + i0);   // 64-byte aligned run
#pragma unroll
        for (int k = 0; k < kRangeRun / 4; ++k) {
            const uint4 q = v[k];
            t[1 + 4 * k] = q.x >> gb;
            t[2 + 4 * k] = q.y >> gb;
            t[3 + 4 * k] = q.z >> gb;
            t[4 + 4 * k] = q.w >> gb;
        }
        t[kRangeRun + 1] = i0 + kRangeRun < n ? tiles[i0 + kRangeRun] >> gb : 0xffffffffu;
    } else {
#pragma unroll
        for (int k = 0; k < kRangeRun + 1; ++k) t[1 + k] = i0 + k < n ? tiles[i0 + k] >> gb : 0xffffffffu;
    }
#pragma unroll
    for (int k = 0; k < kRangeRun; ++k) {
        const int64_t i = i0 + k;
        const uint32_t cur = t[1 + k];
        if (i >= n || cur >= (uint32_t)ws.total_tiles) continue;   // never, for emitted pairs
        if (t[k] != cur) ws.ranges[2 * (int64_t)cur] = (uint32_t)i;
        if (t[k + 2] != cur) ws.ranges[2 * (int64_t)cur + 1] = (uint32_t)(i + 1);
    }
}

// Work order for the persistent blending kernels: tiles bucketed by list
// length on a logarithmic scale (8 buckets per octave), longest first, so
// the heaviest tiles start early and the tail of the launch stays short.
// One workgroup; the order inside a bucket is arbitrary (it only affects
// scheduling, not results).

__global__ __launch_bounds__(1024) void k_tile_order(Ws ws) {
    __shared__ uint32_t hist[kOrderBuckets];
    __shared__ uint32_t scan_lds[1024 / kWave + 1];
    const int64_t nt = ws.total_tiles;
    for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    auto key = [&](int64_t t) -> int { return order_bucket(ws, t); };
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

// The blend launches' tile order as a launch of its own (one workgroup per
// XCD), for the list paths whose last kernel does not write it.
__global__ __launch_bounds__(1024) void k_xcd_order(Ws ws) {
    __shared__ uint32_t hist[kOrderBuckets];
    __shared__ uint32_t scan_lds[1024 / kWave + 1];
    xcd_order_block(ws, blockIdx.x, hist, scan_lds);
}

// 64-bit sort keys of the sorted pairs, for inspection: keys[p] =
// (global tile id << 32) | float32 bits of the camera depth of (view of the
// tile, Gaussian), vals[p] = Gaussian index, for p below the device pair
// count (nothing when the status word is not XG_OK).  Grid-stride over at
// most `cap` pairs.
__global__ __launch_bounds__(256) void k_pair_keys(Ws ws, const xg_camera *cams, uint64_t *keys,
                                                   uint32_t *vals, int64_t cap) {
    const WsHeader *h = ws.hdr;
    const int64_t np = h->n_pairs;
    int64_t n = (h->status != XG_OK || np > ws.cap) ? 0 : np;
    if (n > cap) n = cap;
    const uint32_t *tiles = ws.ptile[ws.pair_sel];
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t word = tiles[p];
        const uint32_t tile = ws.pair_gbits ? word >> ws.pair_gbits : word;
        const uint32_t gi = ws.pair_gbits ? (word & ws.pair_gmask) : ws.pval[ws.pair_sel][p];
        const int view = view_of_tile(cams, ws.n_views, (int)tile);
        const uint32_t depth = __float_as_uint(ws.rec[(int64_t)view * ws.n + gi].b.w);
        keys[p] = ((uint64_t)tile << 32) | depth;
        vals[p] = gi;
    }
}

template <class S>
hipError_t radix_passes(const Ws &ws, int passes, int blocks, hipStream_t s,
                        const uint32_t *depth_part = nullptr, int64_t nparts = 0) {
    const unsigned nb = (unsigned)(blocks > 0 ? blocks : 1);
    unsigned np = (unsigned)(((int64_t)blocks * kRadix + 255) / 256);
    if (np > 2048) np = 2048;
    hipLaunchKernelGGL(k_sort_prep<S>, dim3(np > 0 ? np : 1), dim3(256), 0, s, ws, depth_part, nparts);
    // segmented sorts: one histogram workgroup per partition
    const unsigned nh = S::kSegmented ? nb : (nb < 256 ? nb : 256);
    hipLaunchKernelGGL(k_sort_hist<S>, dim3(nh), dim3(S::kThreads), 0, s, ws, passes);
    for (int p = 0; p < passes; ++p)
        hipLaunchKernelGGL(k_onesweep<S>, dim3(nb), dim3(S::kThreads), 0, s, ws, p, passes);
    return hipGetLastError();
}

unsigned grid256(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

}  // namespace

hipError_t launch_sort_items(const Ws &ws, hipStream_t s) {
    // the keys were written by the preprocess; worst case 32 varying depth
    // bits, passes past the varying bits return at once
    const int passes = (32 + kRadixBits - 1) / kRadixBits;
    if (passes > kMaxPasses) return hipErrorInvalidValue;
    // the preprocess left one depth (min, max) pair per workgroup in scan_tmp
    const int64_t nparts = (ws.n_items + kPreThreads - 1) / kPreThreads;
    return radix_passes<ItemSort>(ws, passes, ws.item_blocks, s, ws.scan_tmp, nparts);
}


hipError_t launch_sort_pairs(const Ws &ws, hipStream_t s) {
    if (ws.pair_passes > kMaxPasses) return hipErrorInvalidValue;
    if (ws.pair_gbits) return radix_passes<PackedPairSort>(ws, ws.pair_passes, ws.pair_blocks, s);
    return radix_passes<PairSort>(ws, ws.pair_passes, ws.pair_blocks, s);
}

hipError_t launch_tile_order(const Ws &ws, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, s, ws);
    return hipGetLastError();
}

hipError_t launch_xcd_order(const Ws &ws, hipStream_t s) {
    hipLaunchKernelGGL(k_xcd_order, dim3(kXcds), dim3(1024), 0, s, ws);
    return hipGetLastError();
}

hipError_t launch_pair_keys(const Ws &ws, const xg_camera *cams, uint64_t *keys, uint32_t *vals,
                            int64_t cap, hipStream_t s) {
    int64_t nb = (cap < ws.cap ? cap : ws.cap);
    nb = (nb + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_pair_keys, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(256), 0, s, ws, cams, keys,
                       vals, cap);
    return hipGetLastError();
}

hipError_t launch_ranges(const Ws &ws, bool cleared, hipStream_t s) {
    if (!cleared) {
        const hipError_t e = launch_fill_u32(ws.ranges, 0u, 2 * ws.total_tiles, s);
        if (e != hipSuccess) return e;
    }
    // one thread per run of kRangeRun keys of the capacity (the pair count is
    // only known on the device)
    const int64_t nb = (ws.cap + 256 * kRangeRun - 1) / (256 * kRangeRun);
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(256), 0, s, ws);
    return hipGetLastError();
}

}  // namespace xg
