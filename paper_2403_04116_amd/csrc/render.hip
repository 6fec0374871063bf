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

namespace xg {

namespace {

struct Eval {
    float dx, dy, y1, y2, G, a, alpha;
};

// alpha of one staged Gaussian at a pixel centre (px, py), both relative
// to the block reference point.  sa = (ux, uy, qa, qb), sb = (qc, o, intensity, rect).
__device__ __forceinline__ Eval splat_eval(const float4 &sa, const float4 &sb, float px, float py,
                                           float amax) {
#pragma clang fp contract(off)
    Eval e;
    e.dx = px - sa.x;
    e.dy = py - sa.y;
    e.y1 = fmaf(sa.w, e.dy, sa.z * e.dx);
    e.y2 = sb.x * e.dy;
    const float E = fmaf(e.y2, e.y2, e.y1 * e.y1);
    e.G = __builtin_amdgcn_exp2f(-E);
    e.a = sb.y * e.G;
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

// Stages list entries [b0, b0 + cnt) of the tile into LDS.
template <int T, int NT>
__device__ __forceinline__ void stage(const Ws &ws, const uint32_t *vals, uint32_t b0, int cnt,
                                      const TileGeom &tg, float4 *s_a, float4 *s_b,
                                      uint32_t *s_rid) {
    for (int k = threadIdx.x; k < cnt; k += NT) {
        const uint32_t gi = vals[b0 + k];
        const int64_t rid = (int64_t)tg.view * ws.n + gi;
        const float4 ra = ws.rec.a[rid];
        const float4 rb = ws.rec.b[rid];
        const int4 rc = ws.rec.c[rid];
        const float ux = (float)(rc.x - tg.rx) + ra.x;
        const float uy = (float)(rc.y - tg.ry) + ra.y;
        const int xl = max((rc.z & 0xffff) - tg.x0, 0), xh = min((rc.z >> 16) - tg.x0, T - 1);
        const int yl = max((rc.w & 0xffff) - tg.y0, 0), yh = min((rc.w >> 16) - tg.y0, T - 1);
        const uint32_t rect = (uint32_t)xl | ((uint32_t)xh << 8) | ((uint32_t)yl << 16) | ((uint32_t)yh << 24);
        s_a[k] = make_float4(ux, uy, ra.z, ra.w);
        s_b[k] = make_float4(rb.x, rb.y, rb.z, __uint_as_float(rect));
        if (s_rid) s_rid[k] = (uint32_t)rid;
    }
}

// COUNT = true: instead of the image, write the per-pixel work counts
// (evaluations, contributors, evaluations up to the last contributor) into
// counts[3][total pixels]; the blending decisions are the same.
template <int T, int B, bool COUNT>
__global__ __launch_bounds__(T * T) void k_render_fwd(Ws ws, const xg_camera *cams, Params p,
                                                      float *image, float *final_t,
                                                      int32_t *n_contrib, int32_t *counts) {
    constexpr int NT = T * T;
    constexpr int SB = T / 8;
    __shared__ float4 s_a[B];
    __shared__ float4 s_b[B];

    const int tile = blockIdx.x;
    const TileGeom tg = tile_geom(cams, ws.n_views, tile, T);
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int sx = (w % SB) * 8, sy = (w / SB) * 8;
    const int lx = sx + (lane & 7), ly = sy + (lane >> 3);
    const int px = tg.x0 + lx, py = tg.y0 + ly;
    const bool inside = px < tg.W && py < tg.H;
    const float pxr = (float)(px - tg.rx) + 0.5f;
    const float pyr = (float)(py - tg.ry) + 0.5f;

    const uint32_t s = ws.ranges[2 * (int64_t)tile];
    const uint32_t e = ws.ranges[2 * (int64_t)tile + 1];
    const uint32_t *vals = ws.values[ws.hdr->sort_sel & 1];
    const float amin = p.alpha_min, amax = p.alpha_max, tmin = p.t_min;

    float Tr = 1.0f, C = 0.0f;
    int last = 0;
    int n_eval = 0, n_con = 0, n_upto = 0;
    bool done = !inside;
    for (uint32_t b0 = s; b0 < e; b0 += B) {
        const int cnt = (int)min((uint32_t)B, e - b0);
        if (!__syncthreads_or(!done)) break;
        stage<T, NT>(ws, vals, b0, cnt, tg, s_a, s_b, nullptr);
        __syncthreads();
        if (__any(!done)) {
            for (int k = 0; k < cnt; ++k) {
                const float4 sa = s_a[k];
                const float4 sb = s_b[k];
                const uint32_t rect = __builtin_amdgcn_readfirstlane(__float_as_uint(sb.w));
                const int rxl = rect & 255, rxh = (rect >> 8) & 255;
                const int ryl = (rect >> 16) & 255, ryh = rect >> 24;
                if (rxh < sx || rxl > sx + 7 || ryh < sy || ryl > sy + 7) continue;
                const bool inr = lx >= rxl && lx <= rxh && ly >= ryl && ly <= ryh;
                if (!done && inr) {
                    const Eval ev = splat_eval(sa, sb, pxr, pyr, amax);
                    if (COUNT) ++n_eval;
                    if (ev.alpha >= amin) {
                        const float Tn = Tr * (1.0f - ev.alpha);
                        if (Tn < tmin) {
                            done = true;
                        } else {
                            C = fmaf(sb.z * ev.alpha, Tr, C);
                            Tr = Tn;
                            last = (int)(b0 - s) + k + 1;
                            if (COUNT) { ++n_con; n_upto = n_eval; }
                        }
                    }
                }
                if (!__any(!done)) break;
            }
        }
    }
    if (inside) {
        const int64_t o = (int64_t)tg.pix_off + (int64_t)py * tg.W + px;
        if (COUNT) {
            counts[o] = n_eval;
            counts[ws.total_pixels + o] = n_con;
            counts[2 * ws.total_pixels + o] = n_upto;
        } else {
            image[o] = C;
            final_t[o] = Tr;
            n_contrib[o] = last;
        }
    }
}

// Sum of 8 per-lane values over the wavefront, transposed: afterwards the
// lanes whose bits 0..2 are zero hold the total of value q = lane >> 3.
__device__ __forceinline__ float wave_reduce8(float v[8]) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool hi = lane & 32;
        const float send = hi ? v[k] : v[k + 4];
        const float keep = hi ? v[k + 4] : v[k];
        v[k] = keep + __shfl_xor(send, 32, kWave);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const bool hi = lane & 16;
        const float send = hi ? v[k] : v[k + 2];
        const float keep = hi ? v[k + 2] : v[k];
        v[k] = keep + __shfl_xor(send, 16, kWave);
    }
    {
        const bool hi = lane & 8;
        const float send = hi ? v[0] : v[1];
        const float keep = hi ? v[1] : v[0];
        v[0] = keep + __shfl_xor(send, 8, kWave);
    }
    float x = v[0];
    x += __shfl_xor(x, 4, kWave);
    x += __shfl_xor(x, 2, kWave);
    x += __shfl_xor(x, 1, kWave);
    return x;
}

template <int T, int B>
__global__ __launch_bounds__(T * T) void k_render_bwd(Ws ws, const xg_camera *cams, Params p,
                                                      const float *dl_dimage, const float *final_t,
                                                      const int32_t *n_contrib) {
    constexpr int NT = T * T;
    constexpr int NW = NT / kWave;
    constexpr int SB = T / 8;
    __shared__ float4 s_a[B];
    __shared__ float4 s_b[B];
    __shared__ uint32_t s_rid[B];
    __shared__ int s_max[NW];

    const int tile = blockIdx.x;
    const TileGeom tg = tile_geom(cams, ws.n_views, tile, T);
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int sx = (w % SB) * 8, sy = (w / SB) * 8;
    const int lx = sx + (lane & 7), ly = sy + (lane >> 3);
    const int px = tg.x0 + lx, py = tg.y0 + ly;
    const bool inside = px < tg.W && py < tg.H;
    const float pxr = (float)(px - tg.rx) + 0.5f;
    const float pyr = (float)(py - tg.ry) + 0.5f;

    const uint32_t s = ws.ranges[2 * (int64_t)tile];
    const uint32_t *vals = ws.values[ws.hdr->sort_sel & 1];
    const float amin = p.alpha_min, amax = p.alpha_max;

    float g = 0.0f, Tr = 1.0f;
    int last = 0;
    if (inside) {
        const int64_t o = (int64_t)tg.pix_off + (int64_t)py * tg.W + px;
        g = dl_dimage[o];
        Tr = final_t[o];
        last = n_contrib[o];
        if (g == 0.0f) last = 0;
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
    float *g2d = ws.grad2d;
    for (int end = bmax; end > 0; end -= B) {
        const int b0 = max(end - B, 0);
        const int cnt = end - b0;
        __syncthreads();
        stage<T, NT>(ws, vals, s + (uint32_t)b0, cnt, tg, s_a, s_b, s_rid);
        __syncthreads();
        if (b0 >= wmax) continue;
        for (int k = min(cnt, wmax - b0) - 1; k >= 0; --k) {
            const int pos1 = b0 + k + 1;
            const float4 sa = s_a[k];
            const float4 sb = s_b[k];
            const uint32_t rect = __builtin_amdgcn_readfirstlane(__float_as_uint(sb.w));
            const int rxl = rect & 255, rxh = (rect >> 8) & 255;
            const int ryl = (rect >> 16) & 255, ryh = rect >> 24;
            if (rxh < sx || rxl > sx + 7 || ryh < sy || ryl > sy + 7) continue;
            const bool inr = lx >= rxl && lx <= rxh && ly >= ryl && ly <= ryh;
            float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            bool act = false;
            if (pos1 <= last && inr) {
                const Eval ev = splat_eval(sa, sb, pxr, pyr, amax);
                if (ev.alpha >= amin) {
                    act = true;
                    const float om = 1.0f - ev.alpha;
                    Tr = Tr / om;                           // transmittance before this Gaussian
                    const float it = sb.z;
                    v[6] = g * ev.alpha * Tr;               // dL/d intensity
                    const float galpha = g * Tr * (it - R); // dL/d alpha
                    R = fmaf(it, ev.alpha, om * R);
                    const float ga = (ev.a > amax) ? 0.0f : galpha;
                    v[5] = ga * ev.G;                       // dL/d opacity
                    const float gp = ga * ev.a;             // dL/d power (natural log)
                    const float gk = gp * kInvLog2eHalf;
                    v[0] = gk * (ev.y1 * sa.z);                      // dL/du_x
                    v[1] = gk * fmaf(ev.y1, sa.w, ev.y2 * sb.x);     // dL/du_y
                    v[2] = -0.5f * gp * ev.dx * ev.dx;               // dL/dA
                    v[3] = -gp * ev.dx * ev.dy;                      // dL/dB
                    v[4] = -0.5f * gp * ev.dy * ev.dy;               // dL/dC
                }
            }
            if (!__any(act)) continue;
            const float x = wave_reduce8(v);
            const int q = lane >> 3;
            if ((lane & 7) == 0 && q < 7) atomicAdd(&g2d[8 * (int64_t)s_rid[k] + q], x);
        }
    }
}

template <int T, int B>
hipError_t fwd_t(const Ws &ws, const xg_camera *cams, const Params &p, float *image, float *final_t,
                 int32_t *n_contrib, hipStream_t st) {
    const unsigned nb = (unsigned)(ws.total_tiles > 0 ? ws.total_tiles : 1);
    hipLaunchKernelGGL((k_render_fwd<T, B, false>), dim3(nb), dim3(T * T), 0, st, ws, cams, p, image,
                       final_t, n_contrib, nullptr);
    return hipGetLastError();
}

template <int T, int B>
hipError_t counts_t(const Ws &ws, const xg_camera *cams, const Params &p, int32_t *counts,
                    hipStream_t st) {
    const unsigned nb = (unsigned)(ws.total_tiles > 0 ? ws.total_tiles : 1);
    hipLaunchKernelGGL((k_render_fwd<T, B, true>), dim3(nb), dim3(T * T), 0, st, ws, cams, p, nullptr,
                       nullptr, nullptr, counts);
    return hipGetLastError();
}

template <int T, int B>
hipError_t bwd_t(const Ws &ws, const xg_camera *cams, const Params &p, const float *dl,
                 const float *final_t, const int32_t *n_contrib, hipStream_t st) {
    const unsigned nb = (unsigned)(ws.total_tiles > 0 ? ws.total_tiles : 1);
    hipLaunchKernelGGL((k_render_bwd<T, B>), dim3(nb), dim3(T * T), 0, st, ws, cams, p, dl, final_t,
                       n_contrib);
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
                             float *final_t, int32_t *n_contrib, int persistent, hipStream_t s) {
    (void)persistent;
    XG_DISPATCH(fwd_t, ws, cams, p, image, final_t, n_contrib, s)
}

hipError_t launch_render_bwd(const Ws &ws, const xg_camera *cams, const Params &p,
                             const float *dl_dimage, const float *final_t,
                             const int32_t *n_contrib, int persistent, hipStream_t s) {
    (void)persistent;
    XG_DISPATCH(bwd_t, ws, cams, p, dl_dimage, final_t, n_contrib, s)
}

hipError_t launch_render_counts(const Ws &ws, const xg_camera *cams, const Params &p,
                                int32_t *counts, hipStream_t s) {
    XG_DISPATCH(counts_t, ws, cams, p, counts, s)
}

}  // namespace xg
