// Stage 3 and its adjoint: front-to-back blending (Eq. 10) of every pixel
// over its tile's depth-sorted list, and the reverse-order backward.
//
// Work decomposition (gfx950, 64-lane wavefronts): one workgroup per tile
// of T x T pixels (T = 8, 16, 32), one lane per pixel, and each wavefront
// owns an 8 x 8 sub-block of the tile.  Gaussians of the tile's list are
// staged through LDS in batches of B; every wavefront then walks the batch
// with the Gaussian's data broadcast from LDS.  A wavefront skips a
// Gaussian whose bounding rectangle misses its 8 x 8 sub-block (a scalar
// test), leaves the batch as soon as all its lanes have terminated, and the
// workgroup stops staging once every lane is done.
//
// Numerics: positions are relative to the centre of the enclosing 32 x 32
// pixel block (the preprocess stores the centre as integer + fraction), the
// same reference for every tile size, so a pixel's arithmetic does not
// depend on the tiling; and the Mahalanobis form is factored
// (k d^T Sigma''^-1 d = (qa dx + qb dy)^2 + (qc dy)^2) so the exponent has
// no catastrophic cancellation; alpha is computed by one inline function
// shared by both kernels, so the backward recomputes the forward's alpha
// bit for bit and can divide the transmittance back.
#include "common.h"

#include <type_traits>

namespace xg {

namespace {

struct Eval {
    float dx, dy, y1, y2, a, alpha;
};

// alpha of one staged Gaussian at a pixel centre (px, py), both relative
// to the block reference point.  sa = (ux, uy, qa, qb), sb = (qc, -log2 o,
// intensity, rectangle word): a = o G = exp2(-(E - log2 o)), with E the
// scaled Mahalanobis term, so the opacity enters the exponent's sum.
__device__ __forceinline__ Eval splat_eval(const float4 &sa, const float4 &sb, float px, float py,
                                           float amax) {
#pragma clang fp contract(off)
    Eval e;
    e.dx = px - sa.x;
    e.dy = py - sa.y;
    e.y1 = fmaf(sa.w, e.dy, sa.z * e.dx);
    e.y2 = sb.x * e.dy;
    const float E = fmaf(e.y2, e.y2, fmaf(e.y1, e.y1, sb.y));
    e.a = __builtin_amdgcn_exp2f(-E);
    e.alpha = fminf(e.a, amax);
    return e;
}

struct TileGeom {
    int view, x0, y0, W, H, pix_off;
    int rx, ry;   // reference point: centre of the enclosing 32 x 32 block
};

__device__ __forceinline__ TileGeom tile_geom(const xg_camera *cams, int n_views, int tile, int T) {
    TileGeom t;
    t.view = view_of_tile(cams, n_views, tile);
    const xg_camera &c = cams[t.view];
    t.W = c.width;
    t.H = c.height;
    t.pix_off = c.pixel_offset;
    const int txn = (t.W + T - 1) / T;
    const int lt = tile - c.tile_offset;
    const int ty = lt / txn;
    t.x0 = (lt - ty * txn) * T;
    t.y0 = ty * T;
    t.rx = (t.x0 & ~31) + 16;
    t.ry = (t.y0 & ~31) + 16;
    return t;
}

// The tile-local rectangle [xl, xh] x [yl, yh] of a staged entry, in the
// form the blend loops test it.  T <= 16: bit x of the low half and bit y of
// the high half are set for the columns and rows the rectangle covers, and a
// lane at (lx, ly) is inside iff both of its two bits are set: one AND and
// one compare per entry against a per-lane constant.  T = 32 (32 columns do
// not fit a half word): the four bounds as bytes, compared one by one.
template <int T>
__device__ __forceinline__ uint32_t rect_word(int xl, int xh, int yl, int yh) {
    if constexpr (T <= 16) {
        const uint32_t xm = ((2u << xh) - 1u) & ~((1u << xl) - 1u);
        const uint32_t ym = ((2u << yh) - 1u) & ~((1u << yl) - 1u);
        return xm | (ym << 16);
    } else {
        return (uint32_t)xl | ((uint32_t)xh << 8) | ((uint32_t)yl << 16) | ((uint32_t)yh << 24);
    }
}

template <int T>
__device__ __forceinline__ uint32_t rect_lane_key(int lx, int ly) {
    return T <= 16 ? (1u << lx) | (1u << (16 + ly)) : 0u;
}

template <int T>
__device__ __forceinline__ bool in_rect(uint32_t rect, uint32_t key, int lx, int ly) {
    if constexpr (T <= 16) {
        return (rect & key) == key;
    } else {
        const int rxl = rect & 255, rxh = (rect >> 8) & 255;
        const int ryl = (rect >> 16) & 255, ryh = rect >> 24;
        return lx >= rxl && lx <= rxh && ly >= ryl && ly <= ryh;
    }
}

// Bit s of the result: the tile-local rectangle [xl, xh] x [yl, yh] touches
// the 8 x 8 sub-block s (row-major, SB sub-blocks per row).
template <int SB>
__device__ __forceinline__ uint32_t subblock_mask(int xl, int xh, int yl, int yh) {
    const int cx0 = xl >> 3, cx1 = xh >> 3, cy0 = yl >> 3, cy1 = yh >> 3;
    const uint32_t row = ((1u << (cx1 - cx0 + 1)) - 1u) << cx0;
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < SB; ++r)
        if (r >= cy0 && r <= cy1) m |= row << (r * SB);
    return m;
}

// Sub-block culling (in stage below): the smallest value over a box
// [X0, X1] x [Y0, Y1] of the exponent
// E(dx, dy) = (qa dx + qb dy)^2 + (qc dy)^2 (qa > 0, qb^2 + qc^2 > 0), whose
// minimum 0 is at the origin.  For a box point p, the segment from p to the
// origin leaves the box through an edge facing the origin, at a point q
// with E(q) <= E(p) (E is convex); so the minimum lies on the vertical edge
// x = Xn and the horizontal edge y = Yn nearest the origin, Xn and Yn the
// origin's coordinates clamped to the box (a clamped coordinate that the
// box already spans gives a line through the box, whose minimum is no
// smaller, and for a box holding the origin both lines give 0).  Along each
// line E is a one-dimensional quadratic minimised at -rx Yn resp. -ry Xn
// (rx = qb / qa, ry = qa qb / (qb^2 + qc^2)), clamped to the edge.
// (X0 <= X1 and Y0 <= Y1, all finite: each clamp is one median of three)
__device__ __forceinline__ float box_min_exponent(float qa, float qb, float qc, float rx, float ry,
                                                  float X0, float X1, float Y0, float Y1) {
    const float xn = __builtin_amdgcn_fmed3f(0.0f, X0, X1);
    const float yn = __builtin_amdgcn_fmed3f(0.0f, Y0, Y1);
    const float x = __builtin_amdgcn_fmed3f(-rx * yn, X0, X1);
    const float e1 = qa * x + qb * yn, e2 = qc * yn;
    const float y = __builtin_amdgcn_fmed3f(-ry * xn, Y0, Y1);
    const float f1 = qa * xn + qb * y, f2 = qc * y;
    return fminf(e1 * e1 + e2 * e2, f1 * f1 + f2 * f2);
}

// Stages list entries [b0, b0 + cnt) of the tile into LDS, with the mask of
// the 8 x 8 sub-blocks each entry must be visited for.  A sub-block is in
// the mask when the entry's rectangle touches it and (CULL) the entry's
// alpha can reach alpha_min somewhere in that part of the rectangle: the
// smallest exponent over the part, a lower bound of every pixel's, is
// compared with log2(o / alpha_min) plus a margin far above float
// rounding.  Dropping the others skips only evaluations that the
// per-pixel alpha test would skip, so results do not change.
// DUAL (the counting forward): s_mask keeps the rectangle-only mask and
// s_cmask receives the culled one.
// MASKIO: 1 (the blending forward) also writes the culled mask of list
// entry p to the workspace's per-entry mask array; 2 (the backward) reads it
// from there instead of testing the sub-blocks again.  Every entry the
// backward stages was staged by the forward of the same lists (a pixel's
// last contributor lies in a batch the forward staged), and both would
// compute the same mask.
template <int T>
using SubMask = std::conditional_t<(T > 16), uint16_t, uint8_t>;

template <int T, int NT, bool CULL, bool DUAL = false, int MASKIO = 0>
__device__ __forceinline__ void stage(const Ws &ws, const uint32_t *vals, uint32_t b0, int cnt,
                                      const TileGeom &tg, float amin, float4 *s_a, float4 *s_b,
                                      uint16_t *s_mask, uint32_t *s_rid, float4 *s_c = nullptr,
                                      uint16_t *s_cmask = nullptr) {
    constexpr int SB = T / 8;
    static_assert(!(MASKIO && DUAL), "the counting forward neither stores nor loads masks");
    SubMask<T> *gmask = reinterpret_cast<SubMask<T> *>(ws.entry_mask);
    const float lg_amin = -__builtin_amdgcn_logf(amin);   // log2(1 / alpha_min)
    for (int k = threadIdx.x; k < cnt; k += NT) {
        const uint32_t gi = vals[b0 + k] & ws.pair_gmask;   // Gaussian index (packed or not)
        const int64_t rid = (int64_t)tg.view * ws.n + gi;
        const Record &rec = ws.rec[rid];
        const float4 ra = rec.a;
        const float4 rb = rec.b;
        const int4 rc = rec.c;
        const float ux = (float)(rc.x - tg.rx) + ra.x;
        const float uy = (float)(rc.y - tg.ry) + ra.y;
        const int xl = max((rc.z & 0xffff) - tg.x0, 0), xh = min((rc.z >> 16) - tg.x0, T - 1);
        const int yl = max((rc.w & 0xffff) - tg.y0, 0), yh = min((rc.w >> 16) - tg.y0, T - 1);
        const uint32_t rect = rect_word<T>(xl, xh, yl, yh);
        s_a[k] = make_float4(ux, uy, ra.z, ra.w);
        s_b[k] = make_float4(rb.x, rb.y, rb.z, __uint_as_float(rect));
        uint32_t m = subblock_mask<SB>(xl, xh, yl, yh);
        uint32_t mc = m;
        if (MASKIO == 2) {
            m = gmask[b0 + k];
        } else if (CULL || DUAL) {
            const float thr = (lg_amin - rb.y) * 1.00001f + 1e-3f;   // log2(o / alpha_min) + margin
            // the edge minimisers' slopes, with approximate reciprocals: an
            // argmin off by a rounding error raises the minimum by a
            // second-order amount, far inside the margin of thr
            const float qa = ra.z, qb = ra.w, qc = rb.x;
            const float rx = qb * __builtin_amdgcn_rcpf(qa);
            const float ry = qa * qb * __builtin_amdgcn_rcpf(qb * qb + qc * qc);
            // pixel centres relative to the Gaussian centre; the box edges
            // clamp the rectangle's (offset once) to each sub-block's, which
            // rounds the same as offsetting the clamped integer (a rounded
            // sum is monotone in its operands)
            const float ox = (float)(tg.x0 - tg.rx) + 0.5f - ux;
            const float oy = (float)(tg.y0 - tg.ry) + 0.5f - uy;
            const float rxl = ox + (float)xl, rxh = ox + (float)xh;
            const float ryl = oy + (float)yl, ryh = oy + (float)yh;
            // A sub-block the rectangle touches has its edges on the right
            // sides of the rectangle's: each clamp is a median of three (for
            // the others the result is masked off).
            if constexpr (SB > 2) {   // 32 x 32 tiles: one box at a time (registers)
#pragma unroll
                for (int sb = 0; sb < SB * SB; ++sb) {
                    if (!((m >> sb) & 1u)) continue;
                    const int bx = (sb % SB) * 8, by = (sb / SB) * 8;
                    const float X0 = __builtin_amdgcn_fmed3f(rxl, ox + (float)bx, rxh);
                    const float X1 = __builtin_amdgcn_fmed3f(rxl, ox + (float)(bx + 7), rxh);
                    const float Y0 = __builtin_amdgcn_fmed3f(ryl, oy + (float)by, ryh);
                    const float Y1 = __builtin_amdgcn_fmed3f(ryl, oy + (float)(by + 7), ryh);
                    if (box_min_exponent(qa, qb, qc, rx, ry, X0, X1, Y0, Y1) > thr) mc &= ~(1u << sb);
                }
            } else {
            // the same minimum with everything that depends on one coordinate
            // only computed once per sub-block column (x) or row (y)
            float X0[SB], X1[SB], xn[SB], ryxn[SB], qaxn[SB];
            float Y0[SB], Y1[SB], yn[SB], rxyn[SB], qbyn[SB], e2s[SB];
#pragma unroll
            for (int c = 0; c < SB; ++c) {
                X0[c] = __builtin_amdgcn_fmed3f(rxl, ox + (float)(8 * c), rxh);
                X1[c] = __builtin_amdgcn_fmed3f(rxl, ox + (float)(8 * c + 7), rxh);
                xn[c] = __builtin_amdgcn_fmed3f(0.0f, X0[c], X1[c]);
                ryxn[c] = -ry * xn[c];
                qaxn[c] = qa * xn[c];
                Y0[c] = __builtin_amdgcn_fmed3f(ryl, oy + (float)(8 * c), ryh);
                Y1[c] = __builtin_amdgcn_fmed3f(ryl, oy + (float)(8 * c + 7), ryh);
                yn[c] = __builtin_amdgcn_fmed3f(0.0f, Y0[c], Y1[c]);
                rxyn[c] = -rx * yn[c];
                qbyn[c] = qb * yn[c];
                const float e2 = qc * yn[c];
                e2s[c] = e2 * e2;
            }
#pragma unroll
            for (int sb = 0; sb < SB * SB; ++sb) {
                const int c = sb % SB, r = sb / SB;
                // nearest point of the box to the centre along the edge x = x(y)
                // facing it, and along y = y(x)
                const float x = __builtin_amdgcn_fmed3f(rxyn[r], X0[c], X1[c]);
                const float e1 = fmaf(qa, x, qbyn[r]);
                const float E = fmaf(e1, e1, e2s[r]);
                const float y = __builtin_amdgcn_fmed3f(ryxn[c], Y0[r], Y1[r]);
                const float f1 = fmaf(qb, y, qaxn[c]), f2 = qc * y;
                const float F = fmaf(f1, f1, f2 * f2);
                if (fminf(E, F) > thr) mc &= ~(1u << sb);
            }
            }
            if (CULL) m = mc;
            if (DUAL) s_cmask[k] = (uint16_t)mc;
            if (MASKIO == 1) gmask[b0 + k] = (SubMask<T>)m;
        }
        s_mask[k] = (uint16_t)m;
        if (s_rid) s_rid[4 * k] = (uint32_t)rid;   // 16-byte slots, like the records
        if (s_c) s_c[k] = rec.d;   // RGB colour of the view (comparison model)
    }
}

// Compacts, in list order, the staged entries [0, cnt) whose rectangle
// touches this wavefront's sub-block w into list[]; returns their number
// (wavefront-uniform).  An entry k is stored as 16 k, the byte offset of its
// slot in the float4 record arrays (k < B <= 256, so 16 k fits 16 bits), and
// the blend loops read records without scaling the index.
__device__ __forceinline__ int wave_list(const uint16_t *s_mask, int cnt, int w, uint16_t *list) {
    const int lane = lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;
    int n = 0;
    for (int c = 0; c < cnt; c += kWave) {
        const int k = c + lane;
        const bool sel = k < cnt && ((s_mask[k] >> w) & 1u);
        const uint64_t bal = __ballot(sel);
        if (sel) list[n + __popcll(bal & lt)] = (uint16_t)(16 * k);
        n += __popcll(bal);
    }
    return n;
}

// Record slot at byte offset `off` (16 x its index) of a float4 array.
__device__ __forceinline__ float4 slot16(const float4 *base, uint32_t off) {
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + off);
}

// LDS of one blending workgroup (the forward leaves rid and wmax unused;
// c holds the staged RGB colours of the CH = 3 forward, cmask the culled
// sub-block masks of the counting forward).
template <int T, int B, int CH = 1, bool CNT = false>
struct BlendLds {
    static constexpr int NW = T * T / kWave;
    float4 a[B];
    float4 b[B];
    float4 c[CH == 3 ? B : 1];
    uint32_t rid[4 * B];   // record index of entry k at rid[4 k] (read at the entry's byte offset)
    uint16_t mask[B];
    uint16_t cmask[CNT ? B : 1];
    alignas(16) uint16_t list[NW][B];
    int wmax[NW];
    int next;
};

// CH = 1: the radiative intensity of the record (Eq. 10).  CH = 3: the
// three colour channels of the record's fourth slot (the comparison model),
// image planar [3][total pixels]; the blending decisions are the same.
// COUNT: the work counts of xg_render_counts (rows documented there)
// instead of the image.  The walk then covers every list entry whose
// rectangle touches the wavefront's 8 x 8 block (the definition's
// evaluations); the culled mask tells which of them the blending kernels
// visit.
template <int T, int B, bool COUNT, bool STORE, int CH = 1>
__device__ __forceinline__ void fwd_tile(int tile, const Ws &ws, const xg_camera *cams,
                                         const Params &p, float *image, float *final_t,
                                         int32_t *n_contrib, int32_t *counts, const TStore &ts,
                                         const L1Fuse &l1, BlendLds<T, B, CH, COUNT> &sh) {
    static_assert(CH == 1 || (CH == 3 && !COUNT && !STORE), "RGB forward: plain variant only");
    static_assert(B % 8 == 0, "list groups of 8 are read 16 bytes at a time");
    constexpr int NT = T * T;
    constexpr int SB = T / 8;
    float4 *s_a = sh.a;
    float4 *s_b = sh.b;
    uint16_t *s_mask = sh.mask;

    const TileGeom tg = tile_geom(cams, ws.n_views, tile, T);
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int sx = (w % SB) * 8, sy = (w / SB) * 8;
    const int lx = sx + (lane & 7), ly = sy + (lane >> 3);
    const int px = tg.x0 + lx, py = tg.y0 + ly;
    const bool inside = px < tg.W && py < tg.H;
    const float pxr = (float)(px - tg.rx) + 0.5f;
    const float pyr = (float)(py - tg.ry) + 0.5f;
    const uint32_t rkey = rect_lane_key<T>(lx, ly);

    const uint32_t s = ws.ranges[2 * (int64_t)tile];
    const uint32_t e = ws.ranges[2 * (int64_t)tile + 1];
    const uint32_t *vals = ws.pair_vals;
    const float amin = p.alpha_min, amax = p.alpha_max, tmin = p.t_min;
    uint16_t *list = sh.list[w];

    float Tr = 1.0f, C = 0.0f, Cg = 0.0f, Cb = 0.0f;
    int last = 0;
    // counting variant: per lane (rows 0-2, 6, 7) and per wavefront (3-5)
    int n_eval = 0, n_con = 0, n_upto = 0, n_fev = 0, n_bev = 0, bev_run = 0;
    int w_red = 0, w_bvis = 0, w_fvis = 0, w_cvis = 0;
    bool done = !inside;
    int nc = 0;   // contributors so far (stored variant)
    float *tbase = STORE ? ts.t + (int64_t)tile * ts.slots * NT + threadIdx.x : nullptr;
    for (uint32_t b0 = s; b0 < e; b0 += B) {
        const int cnt = (int)min((uint32_t)B, e - b0);
        if (!__syncthreads_or(!done)) break;
        // the counting variant keeps every rectangle evaluation (the work
        // count of the definition), the others skip sub-blocks out of reach
        stage<T, NT, !COUNT, COUNT, (COUNT || CH == 3) ? 0 : 1>(ws, vals, b0, cnt, tg, amin, s_a, s_b, s_mask, nullptr,
                                    CH == 3 ? sh.c : nullptr, COUNT ? sh.cmask : nullptr);
        __syncthreads();
        if (!__any(!done)) continue;
        const int nl = wave_list(s_mask, cnt, w, list);
        int lk = -1;   // 16 x batch index of this lane's last contributor in the batch
        // groups of 8 entries (the group bound is wavefront-uniform); the
        // wavefront leaves the batch after a group once all its lanes have
        // terminated
        for (int j0 = 0; j0 < nl; j0 += 8) {
          // the group's eight indices in one 16-byte read (in the row: j0 is
          // a multiple of 8 and B of 8)
          const uint4 idx8 = *reinterpret_cast<const uint4 *>(list + j0);
          const uint32_t iw[4] = {idx8.x, idx8.y, idx8.z, idx8.w};
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (j0 + u >= nl) break;
            const uint32_t off = (iw[u >> 1] >> (16 * (u & 1))) & 0xffffu;   // 16 x batch index
            const float4 sa = slot16(s_a, off);
            const float4 sb = slot16(s_b, off);
            const bool inr = in_rect<T>(__float_as_uint(sb.w), rkey, lx, ly);
            const bool act = !done && inr;
            const bool live = COUNT && __any(!done);   // before this entry
            const Eval ev = splat_eval(sa, sb, pxr, pyr, amax);
            const bool con = act && ev.alpha >= amin;
            const float Tn = fmaf(-Tr, ev.alpha, Tr);   // T (1 - alpha), one rounding
            const bool term = con && Tn < tmin;
            const bool keep = con != term;   // con and not term (term implies con)
            done = done || term;
            if (STORE) {
                if (keep && nc < ts.slots) tbase[(int64_t)nc * NT] = Tr;
                nc += keep ? 1 : 0;
            }
            if constexpr (CH == 3) {
                const float4 sc = slot16(sh.c, off);
                C = keep ? fmaf(sc.x * ev.alpha, Tr, C) : C;
                Cg = keep ? fmaf(sc.y * ev.alpha, Tr, Cg) : Cg;
                Cb = keep ? fmaf(sc.z * ev.alpha, Tr, Cb) : Cb;
            } else {
                C = keep ? fmaf(sb.z * ev.alpha, Tr, C) : C;
            }
            Tr = keep ? Tn : Tr;
            lk = keep ? (int)off : lk;
            if (COUNT) {
                n_eval += act ? 1 : 0;
                n_con += keep ? 1 : 0;
                n_upto = keep ? n_eval : n_upto;
                const bool any_keep = __any(keep);
                w_red += any_keep ? 1 : 0;
                if ((sh.cmask[off >> 4] >> w) & 1u) {   // an entry the blend kernels visit
                    ++w_cvis;
                    if (live) {
                        ++w_fvis;
                        n_fev += act ? 1 : 0;
                    }
                    bev_run += inr ? 1 : 0;
                    if (any_keep) w_bvis = w_cvis;
                    n_bev = keep ? bev_run : n_bev;
                }
            }
          }
          if (!__any(!done)) break;
        }
        if (lk >= 0) last = (int)(b0 - s) + (lk >> 4) + 1;
    }
    if (STORE) ts.count[(int64_t)tile * NT + threadIdx.x] = nc;
    if (inside) {
        const int64_t o = (int64_t)tg.pix_off + (int64_t)py * tg.W + px;
        if (COUNT) {
            const int64_t tp = ws.total_pixels;
            const bool first = lane == 0;   // the block's first pixel
            counts[o] = n_eval;
            counts[tp + o] = n_con;
            counts[2 * tp + o] = n_upto;
            counts[3 * tp + o] = first ? w_red : 0;
            counts[4 * tp + o] = first ? w_bvis : 0;
            counts[5 * tp + o] = first ? w_fvis : 0;
            counts[6 * tp + o] = n_fev;
            counts[7 * tp + o] = n_bev;
        } else {
            image[o] = C;
            if constexpr (CH == 3) {
                image[ws.total_pixels + o] = Cg;
                image[2 * ws.total_pixels + o] = Cb;
            }
            final_t[o] = Tr;
            n_contrib[o] = last;
            if (l1.dl) {
                const float d = C - l1.target[o];
                l1.dl[o] = d > 0.0f ? l1.scale : (d < 0.0f ? -l1.scale : 0.0f);
            }
        }
    }
}

// Pops the next tile of the heavy-first work order (-1 when exhausted).
template <typename Lds>
__device__ __forceinline__ int pop_tile(const Ws &ws, int32_t *queue, Lds &sh) {
    if (threadIdx.x == 0) {
        const int q = atomicAdd(queue, 1);
        sh.next = q < ws.total_tiles ? ws.tile_order[q] : -1;
    }
    __syncthreads();
    const int t = sh.next;
    __syncthreads();
    return t;
}

// The last workgroup of a persistent launch to finish rewinds the queue, so
// the next launch on this workspace starts from the first tile again.
__device__ __forceinline__ void finish_queue(int32_t *queue, int32_t *done) {
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(done, 1) == (int)gridDim.x - 1) {
            atomicExch(queue, 0);
            atomicExch(done, 0);
        }
    }
}

// COUNT = true: instead of the image, write the per-pixel work counts
// (evaluations, contributors, evaluations up to the last contributor) into
// counts[3][total pixels]; the blending decisions are the same.
// PERSIST = true: a grid sized to the device's resident capacity takes
// tiles from the work queue; otherwise one workgroup per tile.
// STORE = true: also keep the transmittance before each of the first
// ts.slots contributors of every pixel (one workgroup per tile only).
template <int T, int B, bool COUNT, bool PERSIST, bool STORE>
__global__ __launch_bounds__(T * T) void k_render_fwd(Ws ws, const xg_camera *cams, Params p,
                                                      float *image, float *final_t,
                                                      int32_t *n_contrib, int32_t *counts,
                                                      TStore ts, L1Fuse l1) {
    __shared__ BlendLds<T, B, 1, COUNT> sh;
    if (!PERSIST) {
        fwd_tile<T, B, COUNT, STORE>(ordered_tile(ws.xcd_order, blockIdx.x, (int)ws.total_tiles), ws, cams, p, image,
                                     final_t, n_contrib, counts, ts, l1, sh);
        return;
    }
    for (;;) {
        const int tile = pop_tile(ws, &ws.hdr->queue_fwd, sh);
        if (tile < 0) break;
        fwd_tile<T, B, COUNT, false>(tile, ws, cams, p, image, final_t, n_contrib, counts, ts, l1, sh);
    }
    finish_queue(&ws.hdr->queue_fwd, &ws.hdr->done_fwd);
}

// Forward of the comparison model: three colour channels per pixel, one
// workgroup per tile.
template <int T, int B>
__global__ __launch_bounds__(T * T) void k_render_fwd_rgb(Ws ws, const xg_camera *cams, Params p,
                                                          float *image, float *final_t,
                                                          int32_t *n_contrib) {
    __shared__ BlendLds<T, B, 3> sh;
    fwd_tile<T, B, false, false, 3>(ordered_tile(ws.xcd_order, blockIdx.x, (int)ws.total_tiles), ws, cams, p, image,
                                    final_t, n_contrib, nullptr, TStore{nullptr, nullptr, 0},
                                    L1Fuse{nullptr, nullptr, 0.0f}, sh);
}

// DPP lane permutations (row = 16 lanes): quad xor 1, quad xor 2, lane
// i^8 within a row (rotate by 8), and mirror within each half row.  Every
// permutation reads a lane of the same row and all lanes are active, so the
// bound control (a lane with no source reads 0) never applies; it spares
// the compiler materialising the old value.
#define XG_DPP(x, ctrl) __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xf, 0xf, true))
constexpr int kDppQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppRowRor8 = 0x128;   // row_ror:8
constexpr int kDppHalfMirror = 0x141; // row_half_mirror

// Wavefront sums of the 7 gradient terms of 2 list entries (acc[e][q]),
// halving the live values at every step (reduce-scatter).  The steps over
// lane bits 5 and 4 swap wavefront halves and rows (gfx950 permlane swaps:
// one swap and one add per pair of values), the lower bits read a partner
// lane through DPP (two selects and one add per pair).  All VALU, no LDS
// traffic: 33 instructions (one entry alone takes 19).  Afterwards lane
// 32 e + 4 q holds value q of entry e (q < 7); a value without a partner at
// some step is summed in both halves and its upper copy is dropped.
template <int G>
struct RedLanes {
    static_assert(G == 2, "groups of 2 entries");
    __device__ static int entry(int lane) { return lane >> 5; }
    __device__ static int word(int lane) { return (lane >> 2) & 7; }
    __device__ static bool adds(int lane) { return (lane & 3) == 0 && word(lane) < 7; }
};

__device__ __forceinline__ float wave_reduce_group(const float (&acc)[2][7]) {
    const int lane = lane_id();
    float b[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        // lanes 0-31 keep entry 0, lanes 32-63 entry 1: b[q]
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc[0][i]), __float_as_uint(acc[1][i]),
                                                        false, false);
        b[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float c[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // even rows keep q = i, odd rows q = i + 4 (q = 3 twice)
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(b[i]), __float_as_uint(b[i < 3 ? i + 4 : 3]),
                                                        false, false);
        c[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool h3 = lane & 8, h2 = lane & 4;
    float d[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
        d[j] = (h3 ? c[j + 2] : c[j]) + XG_DPP(h3 ? c[j] : c[j + 2], kDppRowRor8);
    float x = (h2 ? d[1] : d[0]) + XG_DPP(h2 ? d[0] : d[1], kDppHalfMirror);
    x += XG_DPP(x, kDppQuadXor2);
    x += XG_DPP(x, kDppQuadXor1);
    return x;
}

// List entries whose gradient terms are summed over the wavefront together.
constexpr int kBwdGroup = 2;

template <int T, int B, bool STORE>
__device__ __forceinline__ void bwd_tile(int tile, const Ws &ws, const xg_camera *cams,
                                         const Params &p, const float *dl_dimage,
                                         const float *final_t, const int32_t *n_contrib,
                                         const TStore &ts, BlendLds<T, B> &sh) {
    constexpr int NT = T * T;
    constexpr int NW = NT / kWave;
    constexpr int SB = T / 8;
    static_assert(B % 8 == 0, "list groups of 8 are read 16 bytes at a time");
    static_assert((B & (B - 1)) == 0 && B <= 256, "list offsets are masked to 16 (B - 1) in 16 bits");
    float4 *s_a = sh.a;
    float4 *s_b = sh.b;
    uint32_t *s_rid = sh.rid;
    uint16_t *s_mask = sh.mask;
    int *s_max = sh.wmax;

    const TileGeom tg = tile_geom(cams, ws.n_views, tile, T);
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int sx = (w % SB) * 8, sy = (w / SB) * 8;
    const int lx = sx + (lane & 7), ly = sy + (lane >> 3);
    const int px = tg.x0 + lx, py = tg.y0 + ly;
    const bool inside = px < tg.W && py < tg.H;
    const float pxr = (float)(px - tg.rx) + 0.5f;
    const float pyr = (float)(py - tg.ry) + 0.5f;
    const uint32_t rkey = rect_lane_key<T>(lx, ly);

    const uint32_t s = ws.ranges[2 * (int64_t)tile];
    const uint32_t *vals = ws.pair_vals;
    const float amin = p.alpha_min, amax = p.alpha_max;
    uint16_t *list = sh.list[w];

    float g = 0.0f, Tr = 1.0f;
    int last = 0;
    if (inside) {
        const int64_t o = (int64_t)tg.pix_off + (int64_t)py * tg.W + px;
        g = dl_dimage[o];
        Tr = final_t[o];
        last = n_contrib[o];
        if (g == 0.0f) last = 0;
    }
    // stored variant: index of the next contributor (counting down) and its
    // stored transmittance, loaded one contributor ahead of its use;
    // contributors past the stored slots divide the transmittance back
    int c = -1;
    float tnext = 0.0f;
    const float *tbase = STORE ? ts.t + (int64_t)tile * ts.slots * NT + threadIdx.x : nullptr;
    if (STORE) {
        c = ts.count[(int64_t)tile * NT + threadIdx.x] - 1;
        if (c >= 0 && c < ts.slots) tnext = tbase[(int64_t)c * NT];
    }
    int wmax = last;
    for (int off = kWave / 2; off > 0; off >>= 1) wmax = max(wmax, __shfl_xor(wmax, off, kWave));
    if (lane == 0) s_max[w] = wmax;
    __syncthreads();
    int bmax = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) bmax = max(bmax, s_max[k]);
    wmax = __builtin_amdgcn_readfirstlane(wmax);

    float R = 0.0f;   // intensity behind, seen from just after the current Gaussian
    // the lanes that add a reduced total: entry e of the group, gradient word q
    constexpr int G = kBwdGroup;
    const int lane_e = RedLanes<G>::entry(lane);
    const int lane_q = RedLanes<G>::word(lane);
    const bool lane_adds = RedLanes<G>::adds(lane);
    const uint32_t lane_q4 = 4u * (uint32_t)lane_q;
    const bool small_rid = ws.n_items < (int64_t)1 << 27;   // 32 B x records below 4 GiB
    const bool adds_lo = lane_adds && lane_e == 0, adds_hi = lane_adds && lane_e == 1;
    for (int end = bmax; end > 0; end -= B) {
        const int b0 = max(end - B, 0);
        const int cnt = end - b0;
        __syncthreads();
        stage<T, NT, true, false, 2>(ws, vals, s + (uint32_t)b0, cnt, tg, amin, s_a, s_b, s_mask, s_rid);
        __syncthreads();
        if (b0 >= wmax) continue;
        const int nl = wave_list(s_mask, min(cnt, wmax - b0), w, list);
        // 16 x batch index of this lane's last contributor (-16: none in the batch)
        const int lastk16 = 16 * max(last - b0 - 1, -1);
        // groups of 8 entries from the back, each group's indices in one
        // 16-byte read (j0 is a multiple of 8 and B of 8, so the read stays in
        // the row); entries past nl are skipped by a wavefront-uniform test
        for (int j0 = (nl - 1) & ~7; j0 >= 0; j0 -= 8) {
          const uint4 idx8 = *reinterpret_cast<const uint4 *>(list + j0);
          const uint32_t iw[4] = {idx8.x, idx8.y, idx8.z, idx8.w};
          // Each entry's record is loaded one entry ahead of its use.  Entries
          // past nl are loaded too (and skipped): the offset is masked to a
          // multiple of 16 below 16 B, which keeps every valid entry and keeps
          // whatever the row holds past nl (earlier batches, or LDS never
          // written) inside the record arrays.
          constexpr uint32_t kOffMask = 16u * (B - 1);
          uint32_t off_n = (iw[3] >> 16) & kOffMask;
          float4 sa_n = slot16(s_a, off_n);
          float4 sb_n = slot16(s_b, off_n);
          // the 7 gradient terms of G consecutive entries, summed over the
          // wavefront together; entries that no lane contributes to add zeros
          // and are left out of the atomics (bit e of live4)
          float acc[G][7];
          uint32_t live4 = 0;
          uint32_t rid = 0;   // Gaussian record of entry lane_e
#pragma unroll
          for (int u = 7; u >= 0; --u) {
            const int e = u & (G - 1);
            const uint32_t off = off_n;   // 16 x batch index
            const float4 sa = sa_n;
            const float4 sb = sb_n;
            if (u > 0) {
                off_n = (iw[(u - 1) >> 1] >> (16 * ((u - 1) & 1))) & kOffMask;
                sa_n = slot16(s_a, off_n);
                sb_n = slot16(s_b, off_n);
            }
            const bool inr = j0 + u < nl && (int)off <= lastk16 &&
                             in_rect<T>(__float_as_uint(sb.w), rkey, lx, ly);
            const Eval ev = splat_eval(sa, sb, pxr, pyr, amax);
            const bool act = inr && ev.alpha >= amin;
            if (__any(act)) {
                // Every lane runs the same arithmetic; a lane that is not a
                // contributor adds exact zeros to the reduction (its alpha
                // taken as 0, its alpha gradient masked) and keeps its
                // transmittance and R.
                const float aact = act ? ev.alpha : 0.0f;
                float gT;   // dL/dI times T before this Gaussian
                if (STORE) {
                    const float om = 1.0f - ev.alpha;
                    const float Tj = act ? (c < ts.slots ? tnext : Tr * __builtin_amdgcn_rcpf(om)) : Tr;
                    const int cn = act ? c - 1 : c;
                    if (act && cn >= 0 && cn < ts.slots) tnext = tbase[(int64_t)cn * NT];
                    c = cn;
                    Tr = Tj;
                    gT = g * Tj;
                } else {
                    // T before this Gaussian = T after it / (1 - alpha); a
                    // lane that is not a contributor divides by 1 - 0 (the
                    // reciprocal of 1 is exact) and keeps its T.  T itself is
                    // carried, not dL/dI x T: T stays a normal float down to
                    // t_min, a product with a small dL/dI might not.
                    const float Tj = Tr * __builtin_amdgcn_rcpf(1.0f - aact);
                    Tr = Tj;
                    gT = g * Tj;
                }
                const float it = sb.z;
                float *v = acc[e];
                v[6] = gT * aact;                              // dL/d intensity
                const float dR = it - R;
                const float galpha = gT * dR;                  // dL/d alpha
                // R after this Gaussian: i alpha + (1 - alpha) R
                R = fmaf(aact, dR, R);
                // no alpha gradient through the clamp, nor for a lane that is
                // not a contributor
                const float ga = (act && ev.a <= amax) ? galpha : 0.0f;
                const float gp = ga * ev.a;                    // dL/d power, power = -d^T Q d / 2
                v[5] = gp;                                     // opacity x dL/d opacity (a = o G)
                // moments of gp over the pixel offsets d = pixel - u; the inverse
                // covariance is applied once per (view, Gaussian)
                v[0] = gp * ev.dx;
                v[1] = gp * ev.dy;
                v[2] = v[0] * ev.dx;
                v[3] = v[0] * ev.dy;
                v[4] = v[1] * ev.dy;
                if (lane_e == e) rid = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(s_rid) + off);
                live4 |= 1u << e;
            } else {
#pragma unroll
                for (int q = 0; q < 7; ++q) acc[e][q] = 0.0f;
            }
            if (e == 0 && live4 != 0) {
                const float x = wave_reduce_group(acc);
                // the adding lanes of the live entries (a wavefront-uniform
                // choice per half: no per-lane test of live4)
                const bool l0 = live4 & 1u, l1 = live4 & 2u;
                if ((l0 && adds_lo) || (l1 && adds_hi)) {
                    if (small_rid) {   // 32-bit byte offset from the array base
                        atomicAdd(reinterpret_cast<float *>(reinterpret_cast<char *>(ws.grad2d) + (rid << 5 | lane_q4)), x);
                    } else {
                        atomicAdd(ws.grad2d + 8 * (int64_t)rid + lane_q, x);
                        __asm__ volatile("" ::: "memory");   // keeps the two atomics apart
                    }
                }
                live4 = 0;
            }
          }
        }
    }
}

template <int T, int B, bool PERSIST, bool STORE>
__global__ __launch_bounds__(T * T) void k_render_bwd(Ws ws, const xg_camera *cams, Params p,
                                                      const float *dl_dimage, const float *final_t,
                                                      const int32_t *n_contrib, TStore ts) {
    __shared__ BlendLds<T, B> sh;
    if (!PERSIST) {
        bwd_tile<T, B, STORE>(ordered_tile(ws.xcd_order, blockIdx.x, (int)ws.total_tiles), ws, cams, p, dl_dimage,
                              final_t, n_contrib, ts, sh);
        return;
    }
    for (;;) {
        const int tile = pop_tile(ws, &ws.hdr->queue_bwd, sh);
        if (tile < 0) break;
        bwd_tile<T, B, false>(tile, ws, cams, p, dl_dimage, final_t, n_contrib, ts, sh);
        __syncthreads();
    }
    finish_queue(&ws.hdr->queue_bwd, &ws.hdr->done_bwd);
}

// Workgroups of `kernel` that fit on the device at once (persistent grid).
template <typename K>
unsigned resident_grid(K kernel, int threads, int64_t work) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess) return 0;
    int64_t g = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
    if (g > work) g = work;
    return (unsigned)(g > 0 ? g : 1);
}

template <int T, int B>
hipError_t fwd_t(const Ws &ws, const xg_camera *cams, const Params &p, float *image, float *final_t,
                 int32_t *n_contrib, int persistent, const TStore &ts, const L1Fuse &l1, hipStream_t st) {
    const unsigned nb = (unsigned)(ws.total_tiles > 0 ? ws.total_tiles : 1);
    if (ts.t) {
        if (persistent) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_render_fwd<T, B, false, false, true>), dim3(nb), dim3(T * T), 0, st, ws,
                           cams, p, image, final_t, n_contrib, nullptr, ts, l1);
    } else if (persistent) {
        const unsigned g = resident_grid(k_render_fwd<T, B, false, true, false>, T * T, ws.total_tiles);
        if (g == 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_render_fwd<T, B, false, true, false>), dim3(g), dim3(T * T), 0, st, ws,
                           cams, p, image, final_t, n_contrib, nullptr, ts, l1);
    } else {
        hipLaunchKernelGGL((k_render_fwd<T, B, false, false, false>), dim3(nb), dim3(T * T), 0, st, ws,
                           cams, p, image, final_t, n_contrib, nullptr, ts, l1);
    }
    return hipGetLastError();
}

template <int T, int B>
hipError_t fwd_rgb_t(const Ws &ws, const xg_camera *cams, const Params &p, float *image,
                     float *final_t, int32_t *n_contrib, hipStream_t st) {
    const unsigned nb = (unsigned)(ws.total_tiles > 0 ? ws.total_tiles : 1);
    hipLaunchKernelGGL((k_render_fwd_rgb<T, B>), dim3(nb), dim3(T * T), 0, st, ws, cams, p, image,
                       final_t, n_contrib);
    return hipGetLastError();
}

template <int T, int B>
hipError_t counts_t(const Ws &ws, const xg_camera *cams, const Params &p, int32_t *counts,
                    hipStream_t st) {
    const unsigned nb = (unsigned)(ws.total_tiles > 0 ? ws.total_tiles : 1);
    hipLaunchKernelGGL((k_render_fwd<T, B, true, false, false>), dim3(nb), dim3(T * T), 0, st, ws,
                       cams, p, nullptr, nullptr, nullptr, counts, TStore{nullptr, nullptr, 0},
                       L1Fuse{nullptr, nullptr, 0.0f});
    return hipGetLastError();
}

template <int T, int B>
hipError_t bwd_t(const Ws &ws, const xg_camera *cams, const Params &p, const float *dl,
                 const float *final_t, const int32_t *n_contrib, int persistent, const TStore &ts,
                 hipStream_t st) {
    const unsigned nb = (unsigned)(ws.total_tiles > 0 ? ws.total_tiles : 1);
    if (ts.t) {
        if (persistent) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_render_bwd<T, B, false, true>), dim3(nb), dim3(T * T), 0, st, ws, cams,
                           p, dl, final_t, n_contrib, ts);
    } else if (persistent) {
        const unsigned g = resident_grid(k_render_bwd<T, B, true, false>, T * T, ws.total_tiles);
        if (g == 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_render_bwd<T, B, true, false>), dim3(g), dim3(T * T), 0, st, ws, cams, p,
                           dl, final_t, n_contrib, ts);
    } else {
        hipLaunchKernelGGL((k_render_bwd<T, B, false, false>), dim3(nb), dim3(T * T), 0, st, ws, cams,
                           p, dl, final_t, n_contrib, ts);
    }
    return hipGetLastError();
}

}  // namespace

#define XG_DISPATCH(FN, ...)                                                   \
    switch (p.tile * 1000 + p.lds_batch) {                                     \
        case 8064: return FN<8, 64>(__VA_ARGS__);                              \
        case 8128: return FN<8, 128>(__VA_ARGS__);                             \
        case 8256: return FN<8, 256>(__VA_ARGS__);                             \
        case 16064: return FN<16, 64>(__VA_ARGS__);                            \
        case 16128: return FN<16, 128>(__VA_ARGS__);                           \
        case 16256: return FN<16, 256>(__VA_ARGS__);                           \
        case 32064: return FN<32, 64>(__VA_ARGS__);                            \
        case 32128: return FN<32, 128>(__VA_ARGS__);                           \
        case 32256: return FN<32, 256>(__VA_ARGS__);                           \
        default: return hipErrorInvalidValue;                                  \
    }

hipError_t launch_render_fwd(const Ws &ws, const xg_camera *cams, const Params &p, float *image,
                             float *final_t, int32_t *n_contrib, int persistent, const TStore &ts,
                             const L1Fuse &l1, hipStream_t s) {
    XG_DISPATCH(fwd_t, ws, cams, p, image, final_t, n_contrib, persistent, ts, l1, s)
}

hipError_t launch_render_fwd_rgb(const Ws &ws, const xg_camera *cams, const Params &p, float *image,
                                 float *final_t, int32_t *n_contrib, hipStream_t s) {
    XG_DISPATCH(fwd_rgb_t, ws, cams, p, image, final_t, n_contrib, s)
}

hipError_t launch_render_bwd(const Ws &ws, const xg_camera *cams, const Params &p,
                             const float *dl_dimage, const float *final_t,
                             const int32_t *n_contrib, int persistent, const TStore &ts,
                             hipStream_t s) {
    XG_DISPATCH(bwd_t, ws, cams, p, dl_dimage, final_t, n_contrib, persistent, ts, s)
}

hipError_t launch_render_counts(const Ws &ws, const xg_camera *cams, const Params &p,
                                int32_t *counts, hipStream_t s) {
    XG_DISPATCH(counts_t, ws, cams, p, counts, s)
}

}  // namespace xg
