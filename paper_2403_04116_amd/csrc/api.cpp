// Host side of the C ABI declared in include/xg.h: argument validation
// (before any HIP call), workspace layout, and the launch sequence of each
// stage on the caller's stream.  Nothing here allocates or synchronises.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include "common.h"

#include <algorithm>
#include <cfloat>
#include <cmath>

using namespace xg;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool valid_settings(const xg_settings &s) {
    if (s.tile != 8 && s.tile != 16 && s.tile != 32) return false;
    if (s.lds_batch != 64 && s.lds_batch != 128 && s.lds_batch != 256) return false;
    if (!(s.lowpass >= 0.0f) || !isfinite(s.lowpass)) return false;
    if (!(s.alpha_min >= 0.0f && s.alpha_min < 1.0f)) return false;
    // the backward recovers the transmittance by dividing by 1 - alpha
    if (!(s.alpha_max > 0.0f && s.alpha_max < 1.0f)) return false;
    if (!(s.alpha_min <= s.alpha_max)) return false;
    if (!(s.t_min >= 0.0f && s.t_min < 1.0f)) return false;
    if (!isfinite(s.near_z)) return false;
    if (s.flags & ~XG_F_PERSISTENT) return false;
    return true;
}

int64_t tiles_of(const xg_camera &c, int tile) {
    return (int64_t)((c.width + tile - 1) / tile) * ((c.height + tile - 1) / tile);
}

// Validates the host-side description of a frame.  Checks the cameras'
// offsets against the layout implied by their order and the tile size.
xg_status check_frame(const xg_frame *f, bool need_ws, int64_t *tot_px, int64_t *tot_tiles) {
    if (!f) return XG_EINVAL;
    if (f->n < 0 || f->n_views < 1 || !f->cams) return XG_EINVAL;
    if (!valid_settings(f->settings)) return XG_EINVAL;
    if (f->pair_capacity <= 0 || f->pair_capacity >= (1ll << 31)) return XG_EINVAL;
    if ((int64_t)f->n * f->n_views >= (1ll << 32)) return XG_EINVAL;
    int64_t px = 0, tl = 0;
    for (int v = 0; v < f->n_views; ++v) {
        const xg_camera &c = f->cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 32767 || c.height > 32767) return XG_EINVAL;
        if (c.pixel_offset != px || c.tile_offset != tl) return XG_EINVAL;
        for (int k = 0; k < 9; ++k)
            if (!isfinite(c.rot[k])) return XG_EINVAL;
        for (int k = 0; k < 3; ++k)
            if (!isfinite(c.trans[k])) return XG_EINVAL;
        if (!isfinite(c.fx) || !isfinite(c.fy) || !isfinite(c.cx) || !isfinite(c.cy)) return XG_EINVAL;
        px += (int64_t)c.width * c.height;
        tl += tiles_of(c, f->settings.tile);
    }
    if (px >= (1ll << 31) || tl >= (1ll << 31)) return XG_EINVAL;
    if (need_ws) {
        if (!f->cams_dev || !f->ws) return XG_EINVAL;
        if (((uintptr_t)f->ws) % kAlign != 0) return XG_EINVAL;
    }
    if (tot_px) *tot_px = px;
    if (tot_tiles) *tot_tiles = tl;
    return XG_OK;
}

struct Plan {
    xg_ws_layout lay;
    size_t icounts, scan_tmp, ikeys[2], ivals[2], ptile[2], pval[2], ghist, vhist, bin_cnt, bin_ptot,
        bin_pstart, lookback[2], tile_order, xcd_order, ssim, entry_mask;
    int64_t total_px, total_tiles, n_items;
    int32_t item_blocks, pair_blocks, tile_bits, pair_passes, pair_gbits, bin_tiles, bin_ppv;
};

int bits_of(int64_t v) { return v <= 0 ? 0 : 64 - __builtin_clzll((unsigned long long)v); }

xg_status make_plan(const xg_frame *f, bool need_ws, Plan &P) {
    xg_status st = check_frame(f, need_ws, &P.total_px, &P.total_tiles);
    if (st != XG_OK) return st;
    const int64_t ni = (int64_t)f->n * f->n_views;
    const int64_t cap = f->pair_capacity;
    P.n_items = ni;
    // the items are sorted within each view: every view starts a partition
    P.item_blocks = (int32_t)((int64_t)f->n_views * (((int64_t)f->n + kItemSortBlock - 1) / kItemSortBlock));
    // tile lists by counting when every view has at most kBinMaxTiles tiles
    int64_t max_view_tiles = 0;
    for (int v = 0; v < f->n_views; ++v) {
        const int64_t t = tiles_of(f->cams[v], f->settings.tile);
        if (t > max_view_tiles) max_view_tiles = t;
    }
    P.bin_tiles = max_view_tiles <= kBinMaxTiles ? (int32_t)max_view_tiles : 0;
    P.bin_ppv = (int32_t)(((int64_t)f->n + kBinItems - 1) / kBinItems);
    P.tile_bits = bits_of(P.total_tiles - 1);
    P.pair_passes = (P.tile_bits + kRadixBits - 1) / kRadixBits;
    // one word per pair when tile id and Gaussian index fit 32 bits together
    const int gb = bits_of((int64_t)f->n - 1) > 0 ? bits_of((int64_t)f->n - 1) : 1;
    P.pair_gbits = P.tile_bits + gb <= 32 ? gb : 0;
    const int64_t pblock = P.pair_gbits ? kPackedSortBlock : kPairSortBlock;
    P.pair_blocks = (int32_t)((cap + pblock - 1) / pblock);
    const int64_t lb_words = (int64_t)kRadix * (P.item_blocks > P.pair_blocks ? P.item_blocks : P.pair_blocks);
    const int64_t scan_words = (ni + kScanBlock - 1) / kScanBlock + 1;
    // depth partials: one pair per preprocess workgroup
    const int64_t part_words = 2 * ((ni + kPreThreads - 1) / kPreThreads) + 2;
    size_t o = 0;
    xg_ws_layout &L = P.lay;
    memset(&L, 0, sizeof(L));
    L.status = 0;
    L.n_pairs = offsetof(WsHeader, n_pairs);
    L.depth_range = offsetof(WsHeader, depth_min);
    o = sizeof(WsHeader);
    L.records = o;            o = align_up(o + sizeof(Record) * (size_t)ni);
    L.counts = o;             o = align_up(o + 4 * (size_t)ni);
    P.icounts = o;            o = align_up(o + 4 * (size_t)ni);
    L.offsets = o;            o = align_up(o + 4 * (size_t)ni);
    P.scan_tmp = o;           o = align_up(o + 4 * (size_t)(scan_words > part_words ? scan_words : part_words));
    for (int b = 0; b < 2; ++b) { P.ikeys[b] = o; o = align_up(o + 4 * (size_t)ni); }
    for (int b = 0; b < 2; ++b) { P.ivals[b] = o; o = align_up(o + 8 * (size_t)ni); }
    for (int b = 0; b < 2; ++b) { P.ptile[b] = o; o = align_up(o + 4 * (size_t)cap); }
    for (int b = 0; b < 2; ++b) {   // not needed for packed pairs
        P.pval[b] = o;
        if (P.pair_gbits == 0) o = align_up(o + 4 * (size_t)cap);
    }
    P.ghist = o;              o = align_up(o + 4 * (size_t)kSortCtlWords);
    P.vhist = o;              o = align_up(o + 4 * (size_t)f->n_views * kMaxPasses * kRadix);
    P.bin_cnt = o;            o = align_up(o + 4 * (size_t)f->n_views * P.bin_ppv * P.bin_tiles);
    P.bin_ptot = o;           o = align_up(o + 4 * (size_t)f->n_views * P.bin_ppv);
    P.bin_pstart = o;         o = align_up(o + 4 * (size_t)f->n_views * P.bin_ppv);
    for (int b = 0; b < 2; ++b) { P.lookback[b] = o; o = align_up(o + 8 * (size_t)lb_words); }
    L.ranges = o;             o = align_up(o + 8 * (size_t)P.total_tiles);
    P.entry_mask = o;         o = align_up(o + (f->settings.tile > 16 ? 2 : 1) * (size_t)cap);
    L.grad2d = o;             o = align_up(o + 32 * (size_t)ni);
    P.tile_order = o;         o = align_up(o + 4 * (size_t)P.total_tiles);
    P.xcd_order = o;          o = align_up(o + 4 * (size_t)P.total_tiles);
    P.ssim = o;               o = align_up(o + 12 * (size_t)P.total_px + 4 * (size_t)loss_tiles(f->cams, f->n_views));
    L.pair_tiles = P.ptile[P.pair_passes & 1];
    L.pair_values = P.pair_gbits ? P.ptile[P.pair_passes & 1] : P.pval[P.pair_passes & 1];
    L.pair_index_bits = (size_t)P.pair_gbits;
    L.total = o;
    if (need_ws && f->ws_bytes < L.total) return XG_EINVAL;
    return XG_OK;
}

Ws resolve(const xg_frame *f, const Plan &P) {
    char *b = (char *)f->ws;
    Ws w;
    w.hdr = (WsHeader *)b;
    w.rec = (Record *)(b + P.lay.records);
    w.counts = (uint32_t *)(b + P.lay.counts);
    w.icounts = (uint32_t *)(b + P.icounts);
    w.offsets = (uint32_t *)(b + P.lay.offsets);
    w.scan_tmp = (uint32_t *)(b + P.scan_tmp);
    for (int k = 0; k < 2; ++k) {
        w.ikeys[k] = (uint32_t *)(b + P.ikeys[k]);
        w.ivals[k] = (uint64_t *)(b + P.ivals[k]);
        w.ptile[k] = (uint32_t *)(b + P.ptile[k]);
        w.pval[k] = (uint32_t *)(b + P.pval[k]);
    }
    w.ghist = (uint32_t *)(b + P.ghist);
    w.vhist = (uint32_t *)(b + P.vhist);
    w.bin_cnt = (uint32_t *)(b + P.bin_cnt);
    w.bin_ptot = (uint32_t *)(b + P.bin_ptot);
    w.bin_pstart = (uint32_t *)(b + P.bin_pstart);
    w.bin_tiles = P.bin_tiles;
    w.bin_ppv = P.bin_ppv;
    w.pctr = w.ghist + kMaxPasses * kRadix * kGhStride;
    w.lookback[0] = (uint64_t *)(b + P.lookback[0]);
    w.lookback[1] = (uint64_t *)(b + P.lookback[1]);
    w.ranges = (uint32_t *)(b + P.lay.ranges);
    w.entry_mask = b + P.entry_mask;
    w.grad2d = (float *)(b + P.lay.grad2d);
    w.tile_order = (int32_t *)(b + P.tile_order);
    w.xcd_order = (int32_t *)(b + P.xcd_order);
    w.ssim = (float *)(b + P.ssim);
    w.cap = f->pair_capacity;
    w.n_items = P.n_items;
    w.total_tiles = P.total_tiles;
    w.total_pixels = P.total_px;
    w.n = f->n;
    w.n_views = f->n_views;
    w.tile_bits = P.tile_bits;
    w.item_blocks = P.item_blocks;
    w.pair_blocks = P.pair_blocks;
    w.pair_passes = P.pair_passes;
    w.pair_sel = P.pair_passes & 1;
    w.pair_gbits = P.pair_gbits;
    w.pair_gmask = P.pair_gbits ? (uint32_t)((1ull << P.pair_gbits) - 1) : 0xffffffffu;
    w.pair_vals = P.pair_gbits ? w.ptile[w.pair_sel] : w.pval[w.pair_sel];
    return w;
}

Params params_of(const xg_settings &s) {
    Params p;
    p.lowpass = s.lowpass;
    p.alpha_min = s.alpha_min;
    p.alpha_max = s.alpha_max;
    // a t_min below the smallest normal float32 acts as that value: the
    // transmittance then stays a normal float, which the recomputing
    // backward divides back contributor by contributor
    p.t_min = std::max(s.t_min, FLT_MIN);
    p.near_z = s.near_z;
    // squared Mahalanobis radius beyond which o * exp(-m^2/2) < alpha_min
    // for any o <= 1; +inf when alpha_min == 0
    p.kappa = (float)(-2.0 * log((double)s.alpha_min));
    p.tile = s.tile;
    p.lds_batch = s.lds_batch;
    return p;
}

bool valid_gaussians(const xg_gaussians *g, int32_t n) {
    if (!g || g->n != n) return false;
    if (n > 0 && (!g->means || !g->scales || !g->quats || !g->opacity || !g->intensity)) return false;
    return true;
}

thread_local hipError_t g_last_error = hipSuccess;

xg_status hip_status(hipError_t e) {
    if (e == hipSuccess) return XG_OK;
    g_last_error = e;
    return XG_EHIP;
}

}  // namespace

extern "C" {

int32_t xg_abi_version(void) { return XG_ABI_VERSION; }

const char *xg_status_string(xg_status s) {
    switch (s) {
        case XG_OK: return "XG_OK";
        case XG_EINVAL: return "XG_EINVAL: invalid argument";
        case XG_ECAPACITY: return "XG_ECAPACITY: pair capacity exceeded";
        case XG_EHIP: return "XG_EHIP: HIP launch failed";
    }
    return "unknown xg_status";
}

const char *xg_last_error(void) {
    static thread_local char buf[256];
    snprintf(buf, sizeof(buf), "%s: %s", hipGetErrorName(g_last_error),
             hipGetErrorString(g_last_error));
    return buf;
}

xg_settings xg_default_settings(void) {
    xg_settings s;
    s.tile = 16;
    s.lds_batch = 256;
    s.lowpass = 0.3f;
    s.alpha_min = 1.0f / 255.0f;
    s.alpha_max = 0.99f;
    s.t_min = 1e-4f;
    s.near_z = 0.2f;
    s.flags = 0;
    return s;
}

xg_status xg_camera_from_scanner(double phi, double l_so, double l_sd, int32_t width, int32_t height,
                                 double det_w, double det_h, xg_camera *out) {
    if (!out || width < 1 || height < 1) return XG_EINVAL;
    if (!(l_so > 0.0) || !(l_sd > 0.0) || !(det_w > 0.0) || !(det_h > 0.0) || !isfinite(phi))
        return XG_EINVAL;
    const double sp = sin(phi), cp = cos(phi);
    const double rot[9] = {-sp, cp, 0.0, 0.0, 0.0, -1.0, -cp, -sp, 0.0};
    memset(out, 0, sizeof(*out));
    for (int k = 0; k < 9; ++k) out->rot[k] = (float)rot[k];
    out->trans[2] = (float)l_so;
    out->fx = (float)((l_sd * (double)width) / det_w);
    out->fy = (float)((l_sd * (double)height) / det_h);
    out->cx = (float)((double)width / 2.0);
    out->cy = (float)((double)height / 2.0);
    out->width = width;
    out->height = height;
    return XG_OK;
}

xg_status xg_layout_views(xg_camera *cams, int32_t n_views, int32_t tile, int64_t *total_pixels,
                          int64_t *total_tiles) {
    if (!cams || n_views < 1 || (tile != 8 && tile != 16 && tile != 32)) return XG_EINVAL;
    int64_t px = 0, tl = 0;
    for (int v = 0; v < n_views; ++v) {
        if (cams[v].width < 1 || cams[v].height < 1) return XG_EINVAL;
        if (px >= (1ll << 31) || tl >= (1ll << 31)) return XG_EINVAL;
        cams[v].pixel_offset = (int32_t)px;
        cams[v].tile_offset = (int32_t)tl;
        px += (int64_t)cams[v].width * cams[v].height;
        tl += tiles_of(cams[v], tile);
    }
    if (total_pixels) *total_pixels = px;
    if (total_tiles) *total_tiles = tl;
    return XG_OK;
}

xg_status xg_ws_layout_of(const xg_frame *f, xg_ws_layout *out) {
    if (!out) return XG_EINVAL;
    Plan P;
    xg_status st = make_plan(f, false, P);
    if (st != XG_OK) return st;
    *out = P.lay;
    return XG_OK;
}

xg_status xg_workspace_size(const xg_frame *f, size_t *bytes) {
    if (!bytes) return XG_EINVAL;
    Plan P;
    xg_status st = make_plan(f, false, P);
    if (st != XG_OK) return st;
    *bytes = P.lay.total;
    return XG_OK;
}

xg_status xg_preprocess(const xg_frame *f, const xg_gaussians *g, void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!valid_gaussians(g, f->n)) return XG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const Ws ws = resolve(f, P);
    const Params p = params_of(f->settings);
    return hip_status(launch_preprocess(ws, *g, f->cams_dev, p, s));
}

xg_status xg_bin_sort(const xg_frame *f, void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const Ws ws = resolve(f, P);
    const Params p = params_of(f->settings);
    hipError_t e = hipSuccess;
    if (ws.n_items > 0) {
        e = launch_sort_items(ws, s);
        if (ws.bin_tiles > 0) {
            // the lists by counting (writes the item offsets, the pair count,
            // the capacity status and every tile range)
            if (e == hipSuccess) e = launch_bin_lists(ws, f->cams_dev, p, s);
        } else {
            if (e == hipSuccess)
                e = launch_scan(ws.icounts, ws.offsets, ws.n_items, ws.scan_tmp, &ws.hdr->n_pairs,
                                &ws.hdr->status, ws.cap, s);
            if (e == hipSuccess) e = launch_emit(ws, f->cams_dev, p, s);
            if (e == hipSuccess) e = launch_sort_pairs(ws, s);
            if (e == hipSuccess) e = launch_ranges(ws, true, s);
            // the blend launches' tile order (the counting path's list
            // scatter writes it)
            if (e == hipSuccess) e = launch_xcd_order(ws, s);
        }
    } else {
        e = launch_ranges(ws, false, s);
        if (e == hipSuccess) e = launch_xcd_order(ws, s);
    }
    return hip_status(e);
}

xg_status xg_preprocess_rgb(const xg_frame *f, const xg_gaussians *g, const float *sh, int32_t degree,
                            void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!valid_gaussians(g, f->n) || !sh || degree < 0 || degree > 3) return XG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const Ws ws = resolve(f, P);
    const Params p = params_of(f->settings);
    hipError_t e = launch_preprocess(ws, *g, f->cams_dev, p, s);
    if (e == hipSuccess) e = launch_sh_color(ws, f->cams_dev, g->means, sh, degree, s);
    return hip_status(e);
}

xg_status xg_render_fwd_rgb(const xg_frame *f, const xg_gaussians *g, float *image, float *final_t,
                            int32_t *n_contrib, void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!valid_gaussians(g, f->n) || !image || !final_t || !n_contrib) return XG_EINVAL;
    if (f->settings.flags & XG_F_PERSISTENT) return XG_EINVAL;
    const Ws ws = resolve(f, P);
    const Params p = params_of(f->settings);
    return hip_status(launch_render_fwd_rgb(ws, f->cams_dev, p, image, final_t, n_contrib,
                                            (hipStream_t)stream));
}

static xg_status render_fwd_common(const xg_frame *f, const xg_gaussians *g, float *image,
                                   float *final_t, int32_t *n_contrib, const L1Fuse &l1,
                                   void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!valid_gaussians(g, f->n) || !image || !final_t || !n_contrib) return XG_EINVAL;
    const Ws ws = resolve(f, P);
    const Params p = params_of(f->settings);
    const bool persistent = (f->settings.flags & XG_F_PERSISTENT) != 0;
    // the persistent queue's work order, from the current tile ranges
    if (persistent) {
        const hipError_t e = launch_tile_order(ws, (hipStream_t)stream);
        if (e != hipSuccess) return hip_status(e);
    }
    return hip_status(launch_render_fwd(ws, f->cams_dev, p, image, final_t, n_contrib, persistent,
                                        TStore{nullptr, nullptr, 0}, l1, (hipStream_t)stream));
}

xg_status xg_render_fwd(const xg_frame *f, const xg_gaussians *g, float *image, float *final_t,
                        int32_t *n_contrib, void *stream) {
    return render_fwd_common(f, g, image, final_t, n_contrib, L1Fuse{nullptr, nullptr, 0.0f}, stream);
}

xg_status xg_render_fwd_l1(const xg_frame *f, const xg_gaussians *g, float *image, float *final_t,
                           int32_t *n_contrib, const float *target, float scale, float *dl_dimage,
                           void *stream) {
    if (!target || !dl_dimage || !std::isfinite(scale)) return XG_EINVAL;
    return render_fwd_common(f, g, image, final_t, n_contrib, L1Fuse{target, dl_dimage, scale}, stream);
}

static bool valid_grads(const xg_grads *grads, int32_t n) {
    if (!grads) return false;
    return n == 0 || (grads->means && grads->scales && grads->quats && grads->opacity &&
                      grads->intensity);
}

static xg_status preprocess_bwd_common(const xg_frame *f, const xg_gaussians *g,
                                       const xg_grads *grads, bool accumulate, void *stream);

xg_status xg_render_bwd_2d(const xg_frame *f, const float *dl_dimage, const float *final_t,
                           const int32_t *n_contrib, void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!dl_dimage || !final_t || !n_contrib) return XG_EINVAL;
    const Ws ws = resolve(f, P);
    const Params p = params_of(f->settings);
    const bool persistent = (f->settings.flags & XG_F_PERSISTENT) != 0;
    if (persistent) {
        const hipError_t e = launch_tile_order(ws, (hipStream_t)stream);
        if (e != hipSuccess) return hip_status(e);
    }
    return hip_status(launch_render_bwd(ws, f->cams_dev, p, dl_dimage, final_t, n_contrib, persistent,
                                        TStore{nullptr, nullptr, 0}, (hipStream_t)stream));
}

// Stored-transmittance buffer: int32 count[tiles][tile^2], then float
// t[tiles][slots][tile^2], each part rounded up to 256 bytes.
static int64_t store_count_bytes(const Plan &P, const xg_settings &s) {
    const int64_t px = (int64_t)P.total_tiles * s.tile * s.tile;
    return (px * 4 + 255) / 256 * 256;
}

static int64_t store_bytes_of(const Plan &P, const xg_settings &s, int32_t slots) {
    const int64_t px = (int64_t)P.total_tiles * s.tile * s.tile;
    return store_count_bytes(P, s) + (px * slots * 4 + 255) / 256 * 256;
}

static xg_status store_of(const xg_frame *f, const Plan &P, const void *store, int32_t slots,
                          int64_t store_bytes, TStore &ts) {
    if (slots < 1 || slots > XG_MAX_STORE_SLOTS) return XG_EINVAL;
    if (!store || ((uintptr_t)store & 255) != 0) return XG_EINVAL;
    if (f->settings.flags & XG_F_PERSISTENT) return XG_EINVAL;
    if (store_bytes < store_bytes_of(P, f->settings, slots)) return XG_EINVAL;
    char *base = (char *)const_cast<void *>(store);
    ts.count = (int32_t *)base;
    ts.t = (float *)(base + store_count_bytes(P, f->settings));
    ts.slots = slots;
    return XG_OK;
}

xg_status xg_store_size(const xg_frame *f, int32_t slots, int64_t *bytes) {
    if (!bytes || slots < 1 || slots > XG_MAX_STORE_SLOTS) return XG_EINVAL;
    Plan P;
    xg_status st = make_plan(f, false, P);
    if (st != XG_OK) return st;
    *bytes = store_bytes_of(P, f->settings, slots);
    return XG_OK;
}

xg_status xg_render_fwd_store(const xg_frame *f, const xg_gaussians *g, float *image, float *final_t,
                              int32_t *n_contrib, void *store, int32_t slots, int64_t store_bytes,
                              void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!valid_gaussians(g, f->n) || !image || !final_t || !n_contrib) return XG_EINVAL;
    TStore ts;
    st = store_of(f, P, store, slots, store_bytes, ts);
    if (st != XG_OK) return st;
    const Ws ws = resolve(f, P);
    const Params p = params_of(f->settings);
    return hip_status(launch_render_fwd(ws, f->cams_dev, p, image, final_t, n_contrib, 0, ts,
                                        L1Fuse{nullptr, nullptr, 0.0f}, (hipStream_t)stream));
}

xg_status xg_render_bwd(const xg_frame *f, const xg_gaussians *g, const float *dl_dimage,
                        const float *final_t, const int32_t *n_contrib, const xg_grads *grads,
                        void *stream) {
    // validate everything before the first launch, so EINVAL enqueues nothing
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!valid_gaussians(g, f->n) || !valid_grads(grads, f->n)) return XG_EINVAL;
    st = xg_render_bwd_2d(f, dl_dimage, final_t, n_contrib, stream);
    if (st != XG_OK) return st;
    return preprocess_bwd_common(f, g, grads, true, stream);
}

xg_status xg_render_bwd_store_2d(const xg_frame *f, const float *dl_dimage, const float *final_t,
                                 const int32_t *n_contrib, const void *store, int32_t slots,
                                 int64_t store_bytes, void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!dl_dimage || !final_t || !n_contrib) return XG_EINVAL;
    TStore ts;
    st = store_of(f, P, store, slots, store_bytes, ts);
    if (st != XG_OK) return st;
    const Ws ws = resolve(f, P);
    const Params p = params_of(f->settings);
    return hip_status(launch_render_bwd(ws, f->cams_dev, p, dl_dimage, final_t, n_contrib, 0, ts,
                                        (hipStream_t)stream));
}

xg_status xg_render_bwd_store(const xg_frame *f, const xg_gaussians *g, const float *dl_dimage,
                              const float *final_t, const int32_t *n_contrib, const void *store,
                              int32_t slots, int64_t store_bytes, const xg_grads *grads,
                              void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!valid_gaussians(g, f->n) || !valid_grads(grads, f->n)) return XG_EINVAL;
    st = xg_render_bwd_store_2d(f, dl_dimage, final_t, n_contrib, store, slots, store_bytes, stream);
    if (st != XG_OK) return st;
    return preprocess_bwd_common(f, g, grads, true, stream);
}

static xg_status preprocess_bwd_common(const xg_frame *f, const xg_gaussians *g,
                                       const xg_grads *grads, bool accumulate, void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!valid_gaussians(g, f->n) || !valid_grads(grads, f->n)) return XG_EINVAL;
    if (f->n == 0) return XG_OK;
    const Ws ws = resolve(f, P);
    const Params p = params_of(f->settings);
    return hip_status(launch_preprocess_bwd(ws, *g, f->cams_dev, accumulate, p, *grads,
                                            (hipStream_t)stream));
}

xg_status xg_preprocess_bwd(const xg_frame *f, const xg_gaussians *g, const xg_grads *grads,
                            void *stream) {
    return preprocess_bwd_common(f, g, grads, true, stream);
}

xg_status xg_preprocess_bwd_write(const xg_frame *f, const xg_gaussians *g, const xg_grads *grads,
                                  void *stream) {
    return preprocess_bwd_common(f, g, grads, false, stream);
}

xg_status xg_ws_inspect(const xg_frame *f, xg_ws_view *out) {
    if (!out) return XG_EINVAL;
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    const char *b = (const char *)f->ws;
    memset(out, 0, sizeof(*out));
    out->status = (const int32_t *)(b + P.lay.status);
    out->n_pairs = (const int32_t *)(b + P.lay.n_pairs);
    out->pair_tiles = (const uint32_t *)(b + P.lay.pair_tiles);
    out->pair_values = (const uint32_t *)(b + P.lay.pair_values);
    out->ranges = (const uint32_t *)(b + P.lay.ranges);
    out->records = (const void *)(b + P.lay.records);
    out->grad2d = (const float *)(b + P.lay.grad2d);
    out->pair_index_bits = (int32_t)P.lay.pair_index_bits;
    out->total_tiles = P.total_tiles;
    out->total_pixels = P.total_px;
    out->tile_order = (const int32_t *)(b + P.xcd_order);
    return XG_OK;
}

xg_status xg_pair_keys(const xg_frame *f, uint64_t *keys, uint32_t *values, int64_t capacity,
                       void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!keys || !values || capacity < 0) return XG_EINVAL;
    if (capacity == 0) return XG_OK;
    const Ws ws = resolve(f, P);
    return hip_status(launch_pair_keys(ws, f->cams_dev, keys, values, capacity, (hipStream_t)stream));
}

xg_status xg_render_counts(const xg_frame *f, int32_t *counts, void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!counts) return XG_EINVAL;
    const Ws ws = resolve(f, P);
    const Params p = params_of(f->settings);
    return hip_status(launch_render_counts(ws, f->cams_dev, p, counts, (hipStream_t)stream));
}

// K_i = [M_i / (2 d)] + 1 and the point count; EINVAL unless every input is
// finite and positive and the count fits a Gaussian count (int32).
static xg_status acui_plan(const double size[3], const int32_t grid[3], double d, int32_t k[3],
                           int64_t *count) {
    if (!size || !grid || !(d > 0.0) || !std::isfinite(d)) return XG_EINVAL;
    double total = 1.0;
    for (int i = 0; i < 3; ++i) {
        if (!(size[i] > 0.0) || !std::isfinite(size[i]) || grid[i] < 1) return XG_EINVAL;
        const double h = std::floor((double)grid[i] / (2.0 * d)) + 1.0;
        if (h > 1.0e6) return XG_EINVAL;
        k[i] = (int32_t)h;
        total *= 2.0 * h + 1.0;
    }
    if (total > (double)INT32_MAX) return XG_EINVAL;
    *count = (int64_t)total;
    return XG_OK;
}

xg_status xg_acui_count(const double size[3], const int32_t grid[3], double d, int64_t *count) {
    int32_t k[3];
    int64_t c = 0;
    const xg_status st = acui_plan(size, grid, d, k, &c);
    if (st != XG_OK) return st;
    if (!count) return XG_EINVAL;
    *count = c;
    return XG_OK;
}

xg_status xg_acui_grid(const double size[3], const int32_t grid[3], double d, float *means,
                       int64_t capacity, void *stream) {
    int32_t k[3];
    int64_t c = 0;
    const xg_status st = acui_plan(size, grid, d, k, &c);
    if (st != XG_OK) return st;
    if (!means || capacity < c) return XG_EINVAL;
    return hip_status(launch_acui_grid(size, grid, d, k, c, means, (hipStream_t)stream));
}

xg_status xg_loss_grad(const xg_frame *f, const float *image, const float *target, float gamma,
                       float *dl_dimage, float *loss, void *stream) {
    Plan P;
    xg_status st = make_plan(f, true, P);
    if (st != XG_OK) return st;
    if (!image || !target || !dl_dimage) return XG_EINVAL;
    if (!(gamma >= 0.0f && gamma <= 1.0f)) return XG_EINVAL;
    const Ws ws = resolve(f, P);
    return hip_status(launch_loss_grad(ws, f->cams_dev, loss_tiles(f->cams, f->n_views), image, target,
                                       gamma, dl_dimage, loss, (hipStream_t)stream));
}

xg_status xg_loss_grad_static(const xg_frame *f, const float *image, const float *target, float gamma,
                              float *dl_dimage, float *loss, void *stream) {
    Plan P;
    xg_status st = make_plan(f, false, P);
    if (st != XG_OK) return st;
    if (!f->cams_dev || !image || !target || !dl_dimage) return XG_EINVAL;
    if (!(gamma >= 0.0f && gamma <= 1.0f)) return XG_EINVAL;
    const int64_t strips = loss_tiles(f->cams, f->n_views);
    if (12 * P.total_px + 4 * strips > (int64_t)XG_STATIC_SCRATCH_BYTES) return XG_ECAPACITY;
    float *scratch = nullptr;
    const hipError_t e = static_scratch(&scratch);
    if (e != hipSuccess) return hip_status(e);
    Ws ws;
    memset(&ws, 0, sizeof(ws));
    ws.ssim = scratch;
    ws.total_pixels = P.total_px;
    ws.n_views = f->n_views;
    return hip_status(launch_loss_grad(ws, f->cams_dev, strips, image, target, gamma, dl_dimage, loss,
                                       (hipStream_t)stream));
}

xg_status xg_rirf_fwd(const float *features, const float *weights, int32_t n, int32_t n_features,
                      float *intensity, void *stream) {
    if (n < 0 || n_features < 1 || n_features > XG_MAX_FEATURES) return XG_EINVAL;
    if (n > 0 && (!features || !weights || !intensity)) return XG_EINVAL;
    return hip_status(launch_rirf_fwd(features, weights, n, n_features, intensity, (hipStream_t)stream));
}

xg_status xg_rirf_bwd(const float *features, const float *weights, int32_t n, int32_t n_features,
                      const float *dl_dintensity, float *grad_features, void *stream) {
    if (n < 0 || n_features < 1 || n_features > XG_MAX_FEATURES) return XG_EINVAL;
    if (n > 0 && (!features || !weights || !dl_dintensity || !grad_features)) return XG_EINVAL;
    return hip_status(launch_rirf_bwd(features, weights, n, n_features, dl_dintensity, grad_features,
                                      (hipStream_t)stream));
}

xg_status xg_adam_step(const xg_params *p, const xg_grads *g, float *m, float *v, int32_t *step,
                       const xg_adam *c, float *scales, float *opacity, float *intensity,
                       const int32_t *gate, void *stream) {
    if (!p || !g || !c || !step || p->n < 0) return XG_EINVAL;
    if (!p->means || !p->log_scales || !p->quats || !p->opacity_logit || !p->features || !p->weights)
        return XG_EINVAL;
    if (p->n_features < 1 || p->n_features > XG_MAX_FEATURES) return XG_EINVAL;
    if (!g->means || !g->scales || !g->quats || !g->opacity || !g->intensity) return XG_EINVAL;
    if (!m || !v || !scales || !opacity || !intensity) return XG_EINVAL;
    if (!(c->beta1 >= 0.0 && c->beta1 < 1.0) || !(c->beta2 >= 0.0 && c->beta2 < 1.0)) return XG_EINVAL;
    if (c->reserved != 0) return XG_EINVAL;
    if (!(c->eps >= 0.0f) || c->lr_means_steps < 1) return XG_EINVAL;
    if (!(c->lr_means_start > 0.0f) || !(c->lr_means_end > 0.0f)) return XG_EINVAL;
    const float lrs[6] = {c->lr_means_start, c->lr_means_end, c->lr_scales, c->lr_quats,
                          c->lr_opacity, c->lr_feature};
    for (float lr : lrs)
        if (!(lr >= 0.0f) || !isfinite(lr)) return XG_EINVAL;
    return hip_status(launch_adam(*p, *g, m, v, step, *c, scales, opacity, intensity, gate,
                                  (hipStream_t)stream));
}

xg_status xg_l1_grad(const float *image, const float *target, float *dl_dimage, int64_t n_pixels,
                     float scale, void *stream) {
    if (!image || !target || !dl_dimage || n_pixels < 0 || !isfinite(scale)) return XG_EINVAL;
    if (n_pixels == 0) return XG_OK;
    return hip_status(launch_l1_grad(image, target, dl_dimage, n_pixels, scale, (hipStream_t)stream));
}

}  // extern "C"
