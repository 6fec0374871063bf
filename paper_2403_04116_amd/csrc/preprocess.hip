// Stage 1 and its adjoint: projection of radiative Gaussians through the
// cone-beam camera (Eq. 7-9 and the 2-D covariance of Sec. 3.2), emission
// of (tile | depth) keys, and the chain rule back to the 3-D parameters.
//
// One thread per (view, Gaussian) for the forward, one thread per Gaussian
// (summing over views in registers, no atomics) for the adjoint.  These
// kernels are HBM/latency bound and tiny next to the blending kernels.
#include "common.h"

#include <math.h>

namespace xg {

namespace {

// Key path: depth, culling and integer bounding rectangle as a fixed
// float32 operation sequence.  Every operation rounds once (IEEE RNE);
// contraction into fused multiply-adds is disabled, '/' and sqrtf are the
// correctly rounded forms, so the result is reproducible bit for bit.
struct KeyOut {
    float tz;
    int xl, xh, yl, yh;
    int ok;
};

// The unit quaternion, R and M = R diag(s); false when the quaternion is
// zero (the Gaussian is culled in every view).
__device__ __forceinline__ bool key_gaussian(const float *s, const float *q, float *M) {
#pragma clang fp contract(off)
    float qw = q[0], qx = q[1], qy = q[2], qz = q[3];
    float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    if (!(n2 > 0.0f)) return false;
    float nn = sqrtf(n2);
    float w = qw / nn, x = qx / nn, y = qy / nn, z = qz / nn;
    float R[9];
    R[0] = 1.0f - 2.0f * (y * y + z * z);
    R[1] = 2.0f * (x * y - w * z);
    R[2] = 2.0f * (x * z + w * y);
    R[3] = 2.0f * (x * y + w * z);
    R[4] = 1.0f - 2.0f * (x * x + z * z);
    R[5] = 2.0f * (y * z - w * x);
    R[6] = 2.0f * (x * z - w * y);
    R[7] = 2.0f * (y * z + w * x);
    R[8] = 1.0f - 2.0f * (x * x + y * y);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        M[3 * a + 0] = R[3 * a + 0] * s[0];
        M[3 * a + 1] = R[3 * a + 1] * s[1];
        M[3 * a + 2] = R[3 * a + 2] * s[2];
    }
    return true;
}

// Camera-space centre, culling, Sigma'', rectangle in one view.
__device__ __forceinline__ bool key_view(const float *m, const float *M, float o,
                                         const xg_camera &c, const Params &p, KeyOut &out) {
#pragma clang fp contract(off)
    const float *r = c.rot;
    float mx = m[0], my = m[1], mz = m[2];
    float tx = ((r[0] * mx + r[1] * my) + r[2] * mz) + c.trans[0];
    float ty = ((r[3] * mx + r[4] * my) + r[5] * mz) + c.trans[1];
    float tz = ((r[6] * mx + r[7] * my) + r[8] * mz) + c.trans[2];
    if (!(isfinite(tx) && isfinite(ty) && isfinite(tz))) return false;
    if (!(tz > p.near_z)) return false;
    float tz2 = tz * tz;
    float J00 = c.fx / tz;
    float J11 = c.fy / tz;
    float J02 = -((c.fx * tx) / tz2);
    float J12 = -((c.fy * ty) / tz2);
    float A[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        A[k] = J00 * r[k] + J02 * r[6 + k];
        A[3 + k] = J11 * r[3 + k] + J12 * r[6 + k];
    }
    float B[6];
#pragma unroll
    for (int row = 0; row < 2; ++row)
#pragma unroll
        for (int col = 0; col < 3; ++col)
            B[3 * row + col] = (A[3 * row + 0] * M[col] + A[3 * row + 1] * M[3 + col])
                               + A[3 * row + 2] * M[6 + col];
    float sxx = ((B[0] * B[0] + B[1] * B[1]) + B[2] * B[2]) + p.lowpass;
    float syy = ((B[3] * B[3] + B[4] * B[4]) + B[5] * B[5]) + p.lowpass;
    float sxy = (B[0] * B[3] + B[1] * B[4]) + B[2] * B[5];
    float det = sxx * syy - sxy * sxy;
    if (!(det > 0.0f)) return false;
    if (!(o >= p.alpha_min)) return false;
    float ux = c.fx * (tx / tz) + c.cx;
    float uy = c.fy * (ty / tz) + c.cy;
    float rx = sqrtf(p.kappa * sxx);
    float ry = sqrtf(p.kappa * syy);
    float xl = ceilf((ux - rx) - 0.5f);
    float xh = floorf((ux + rx) - 0.5f);
    float yl = ceilf((uy - ry) - 0.5f);
    float yh = floorf((uy + ry) - 0.5f);
    float wmax = (float)(c.width - 1), hmax = (float)(c.height - 1);
    if (!(xl <= xh) || !(xl <= wmax) || !(xh >= 0.0f)) return false;
    if (!(yl <= yh) || !(yl <= hmax) || !(yh >= 0.0f)) return false;
    out.tz = tz;
    out.xl = (int)fmaxf(xl, 0.0f);
    out.xh = (int)fminf(xh, wmax);
    out.yl = (int)fmaxf(yl, 0.0f);
    out.yh = (int)fminf(yh, hmax);
    return true;
}

// Rotation matrix of a unit quaternion (w, x, y, z), float64.
__device__ __forceinline__ void quat_rot(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

// Float64 per-Gaussian part: the unit quaternion and its rotation matrix.
struct Gauss64 {
    double qn;          // norm of the input quaternion
    double q[4];        // unit quaternion
    double R[9];
};

__device__ __forceinline__ void gauss64(const float *q, Gauss64 &G) {
    double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
    G.qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    // one float64 reciprocal per divisor (the float32 results these feed
    // are rounded once; the extra float64 rounding is far below that)
    const double rqn = 1.0 / G.qn;
    G.q[0] = q0 * rqn; G.q[1] = q1 * rqn; G.q[2] = q2 * rqn; G.q[3] = q3 * rqn;
    quat_rot(G.q, G.R);
}

// Float64 projection of one Gaussian into one view: camera-space centre t,
// the 2x3 matrix B = J W R diag(s) with Sigma'' = B B^T + k I, and Sigma''.
struct Proj64 {
    double t[3];
    double rtz;         // 1 / t_z
    double J[6];        // first two rows of J (Eq. 9)
    double A2[6];       // J W
    double B[6];        // J W R diag(s)
    double sxx, sxy, syy;
};

__device__ __forceinline__ void project64(const float *m, const float *s, const double *R,
                                          const xg_camera &c, double lowpass, Proj64 &P) {
    double r[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) r[k] = (double)c.rot[k];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        P.t[a] = r[3 * a] * m[0] + r[3 * a + 1] * m[1] + r[3 * a + 2] * m[2] + (double)c.trans[a];
    double fx = c.fx, fy = c.fy, tz = P.t[2];
    P.rtz = 1.0 / tz;
    P.J[0] = fx * P.rtz; P.J[1] = 0.0; P.J[2] = -fx * P.t[0] * (P.rtz * P.rtz);
    P.J[3] = 0.0; P.J[4] = fy * P.rtz; P.J[5] = -fy * P.t[1] * (P.rtz * P.rtz);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            P.A2[3 * i + k] = P.J[3 * i] * r[k] + P.J[3 * i + 1] * r[3 + k] + P.J[3 * i + 2] * r[6 + k];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            P.B[3 * i + k] = (P.A2[3 * i] * R[k] + P.A2[3 * i + 1] * R[3 + k]
                              + P.A2[3 * i + 2] * R[6 + k]) * (double)s[k];
    P.sxx = P.B[0] * P.B[0] + P.B[1] * P.B[1] + P.B[2] * P.B[2] + lowpass;
    P.syy = P.B[3] * P.B[3] + P.B[4] * P.B[4] + P.B[5] * P.B[5] + lowpass;
    P.sxy = P.B[0] * P.B[3] + P.B[1] * P.B[4] + P.B[2] * P.B[5];
}

// The key path of one (view, Gaussian).  Its float32 operation sequence is
// fixed by the contraction-off scope of key_gaussian / key_view (IEEE
// operations are not reordered or fused without fast-math flags), so it is
// inlined: an out-of-line call kept the rotation and the result on the
// stack (48 bytes of scratch traffic per item each way).
__device__ __forceinline__ KeyOut key_path(const float *m, const float *s, const float *q, float o,
                                        const xg_camera &c, const Params p) {
    float M[9];
    KeyOut out;
    out.ok = key_gaussian(s, q, M) && key_view(m, M, o, c, p, out);
    return out;
}

// One thread per (view, Gaussian), view-major, so each view's records are
// written contiguously.  (Sharing the per-Gaussian part of the projection
// across a workgroup's views through LDS measured slower: the lower
// occupancy and the serial per-Gaussian phase cost more than the work it
// saves.)
__global__ __launch_bounds__(kPreThreads) void k_preprocess(Ws ws, xg_gaussians g,
                                                            const xg_camera *cams, Params p,
                                                            uint32_t *depth_part) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the frame's depth range starts empty; the item sort's first launch
    // folds the per-block partials written below into it
    if (idx == 0) {
        ws.hdr->depth_min = 0xffffffffu;
        ws.hdr->depth_max = 0u;
    }
    // The workgroup's records (and 2-D gradient accumulators) form one
    // contiguous range; they are staged in LDS (16-byte part k of record t
    // at s_rec[k][t]: conflict-free) and written with whole cache lines.
    __shared__ float4 s_rec[4][kPreThreads];
    float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = ra, rc = ra;
    uint32_t dmin = 0xffffffffu, dmax = 0u;
    if (idx < ws.n_items) {
        const int v = (int)(idx / ws.n);
        const int64_t i = idx - (int64_t)v * ws.n;
        const xg_camera &c = cams[v];
        const float *m = g.means + 3 * i;
        const float *s = g.scales + 3 * i;
        const float *q = g.quats + 4 * i;
        const float o = g.opacity[i];
        uint32_t count = 0;
        uint32_t key = 0xffffffffu;   // item sort key: depth bits, the largest when culled
        uint32_t trect = 0;
        const KeyOut ko = key_path(m, s, q, o, c, p);
        if (ko.ok) {
            Gauss64 G64;
            gauss64(q, G64);
            Proj64 P;
            project64(m, s, G64.R, c, (double)p.lowpass, P);
            double det = P.sxx * P.syy - P.sxy * P.sxy;
            const double k = (double)kLog2eHalf;
            // k d^T Sigma''^-1 d = (qa dx + qb dy)^2 + (qc dy)^2
            const double rdet = 1.0 / det;
            double qa = sqrt(k * P.syy * rdet);
            double qb = -k * P.sxy * rdet / qa;
            double qc = sqrt(k / P.syy);
            double ux = (double)c.fx * P.t[0] * P.rtz + (double)c.cx;
            double uy = (double)c.fy * P.t[1] * P.rtz + (double)c.cy;
            double fx_ = floor(ux), fy_ = floor(uy);
            fx_ = fmin(fmax(fx_, -1073741824.0), 1073741824.0);
            fy_ = fmin(fmax(fy_, -1073741824.0), 1073741824.0);
            uint32_t dbits = __float_as_uint(ko.tz);
            ra = make_float4((float)(ux - fx_), (float)(uy - fy_), (float)qa, (float)qb);
            // -log2(o) (+inf for o = 0: then every a is 0)
            rb = make_float4((float)qc, -log2f(o), g.intensity[i], __uint_as_float(dbits));
            const int4 ci = make_int4((int)fx_, (int)fy_, ko.xl | (ko.xh << 16), ko.yl | (ko.yh << 16));
            rc = make_float4(__int_as_float(ci.x), __int_as_float(ci.y), __int_as_float(ci.z),
                             __int_as_float(ci.w));
            const int T = p.tile;
            count = (uint32_t)((ko.xh / T - ko.xl / T + 1) * (ko.yh / T - ko.yl / T + 1));
            trect = pack_tile_rect(ko.xl / T, ko.xh / T, ko.yl / T, ko.yh / T);
            dmin = dbits;
            dmax = dbits;
            key = dbits;
        }
        ws.counts[idx] = count;
        ws.ikeys[0][idx] = key;
        ws.ivals[0][idx] = (uint64_t)idx | ((uint64_t)trect << 32);
    }
    // records of culled items are written as zeros (never read)
    s_rec[0][threadIdx.x] = ra;
    s_rec[1][threadIdx.x] = rb;
    s_rec[2][threadIdx.x] = rc;
    s_rec[3][threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    {
        const int64_t first = (int64_t)blockIdx.x * kPreThreads;
        const int nrec = (int)min((int64_t)kPreThreads, ws.n_items - first);
        float4 *out = reinterpret_cast<float4 *>(ws.rec + first);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int j = m * kPreThreads + threadIdx.x;   // float4 j of the range: record j/4, part j%4
            if (j / 4 < nrec) out[j] = s_rec[j & 3][j >> 2];
        }
        // clear the 2-D gradient accumulators (32 bytes per item) for the backward
        float4 *g2 = reinterpret_cast<float4 *>(ws.grad2d) + 2 * first;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int j = m * kPreThreads + threadIdx.x;
            if (j / 2 < nrec) g2[j] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    // block min/max of the kept depths -> one partial per block
    for (int off = kWave / 2; off > 0; off >>= 1) {
        dmin = min(dmin, (uint32_t)__shfl_xor((int)dmin, off, kWave));
        dmax = max(dmax, (uint32_t)__shfl_xor((int)dmax, off, kWave));
    }
    __shared__ uint32_t smin[kPreThreads / kWave], smax[kPreThreads / kWave];
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) { smin[w] = dmin; smax[w] = dmax; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kPreThreads / kWave; ++k) {
            dmin = min(dmin, smin[k]);
            dmax = max(dmax, smax[k]);
        }
        depth_part[2 * blockIdx.x] = dmin;
        depth_part[2 * blockIdx.x + 1] = dmax;
    }
}

// Resets the header of a frame with no items (one thread).  With items,
// the preprocess opens the depth range and the item sort's first launch
// resets the rest and folds the depth partials into the range.
__global__ void k_header_reset(WsHeader *h) {
    if (threadIdx.x == 0) {
        frame_header_reset(h);
        h->depth_min = 0xffffffffu;
        h->depth_max = 0u;
    }
}

// Duplicate-with-key, in depth order: item j of the depth-sorted items
// writes one (global tile id, Gaussian index) pair per tile of its
// rectangle at its scanned offset.  A stable sort of these pairs by tile
// then leaves every tile's list in (depth, index) order.  Nothing is
// written once the scan has raised XG_ECAPACITY (the later stages then see
// no pairs), so every offset is below the capacity.
//
// The pairs of a workgroup's 256 consecutive items form one contiguous
// range, assembled in LDS in windows of kEmitStage pairs and written as
// whole lines.
constexpr int kEmitStage = 2048;   // 16 KB of LDS: eight workgroups per CU

__global__ __launch_bounds__(256) void k_emit(Ws ws, const xg_camera *cams, int tile) {
    __shared__ uint32_t s_t[kEmitStage];
    __shared__ uint32_t s_v[kEmitStage];
    __shared__ uint32_t s_range[2];
    const int64_t j0 = (int64_t)blockIdx.x * blockDim.x;
    if (j0 >= ws.n_items || ws.hdr->status != XG_OK) return;
    const int64_t j = j0 + threadIdx.x;
    const int64_t jl = min(j0 + (int64_t)blockDim.x, ws.n_items) - 1;   // last item of the block
    if (threadIdx.x == 0) {
        s_range[0] = ws.offsets[j0];
        s_range[1] = ws.offsets[jl] + ws.icounts[jl];
    }
    uint32_t cnt = 0, off = 0;
    uint64_t val = 0;
    if (j < ws.n_items) {
        cnt = ws.icounts[j];
        off = ws.offsets[j];
        val = ws.ivals[ws.hdr->item_sel & 1][j];
    }
    __syncthreads();
    const uint32_t base = s_range[0];
    const uint32_t total = s_range[1] - base;
    // this item's tile rectangle and the first tile of its view
    int tx0 = 0, tx1 = -1, ty0 = 0, txn = 1, toff = 0;
    uint32_t i = 0;
    if (cnt > 0) {
        const uint32_t idx = (uint32_t)val;
        const int v = (int)(idx / (uint32_t)ws.n);
        i = idx - (uint32_t)v * (uint32_t)ws.n;
        const xg_camera &c = cams[v];
        txn = (c.width + tile - 1) / tile;
        toff = c.tile_offset;
        const TileRect tr = item_tile_rect(ws, val, tile);
        tx0 = tr.tx0;
        tx1 = tr.tx1;
        ty0 = tr.ty0;
    }
    const uint32_t rw = (uint32_t)(tx1 - tx0 + 1);
    const uint32_t lo = off - base;   // this item's first pair, relative to the block's
    // The block's pairs are one contiguous range; it is assembled in LDS in
    // windows of kEmitStage pairs and written with whole lines.  An item
    // writes the pairs of its range that fall in the window, at most cnt
    // (the slots the scan reserved), row-major over its rectangle.
    for (uint32_t w0 = 0; w0 < total; w0 += kEmitStage) {
        const uint32_t w1 = min(total, w0 + (uint32_t)kEmitStage);
        const uint32_t a = max(lo, w0), b = min(lo + cnt, w1);
        if (cnt > 0 && a < b) {
            const uint32_t m = a - lo;
            int ty = ty0 + (int)(m / rw);
            int tx = tx0 + (int)(m % rw);
            for (uint32_t q = a; q < b; ++q) {
                const uint32_t t = (uint32_t)(toff + ty * txn + tx);
                // packed: one word (tile << gbits | index); else two arrays
                s_t[q - w0] = ws.pair_gbits ? (t << ws.pair_gbits) | i : t;
                s_v[q - w0] = i;
                if (++tx > tx1) {
                    tx = tx0;
                    ++ty;
                }
            }
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < w1 - w0; k += blockDim.x) {
            ws.ptile[0][base + w0 + k] = s_t[k];
            if (!ws.pair_gbits) ws.pval[0][base + w0 + k] = s_v[k];
        }
        __syncthreads();
    }
}

// Adjoint of the projection for one Gaussian, summed over views.
// grad2d per (view, Gaussian) holds pixel sums of g_p = dL/dpower_p times
// the offsets d = pixel centre - u:
//   (sum g dx, sum g dy, sum g dx^2, sum g dx dy, sum g dy^2, sum g, dL/di, 0)
// where sum g = o dL/do (alpha = o G before the clamp, which has no
// derivative), so dL/do is that sum over all views divided by the opacity.
// With power = -(A dx^2 + 2 B dx dy + C dy^2) / 2 and [[A, B], [B, C]] the
// inverse 2-D covariance: dL/du = [[A, B], [B, C]] (sum g d),
// dL/dA = -sum g dx^2 / 2, dL/dB = -sum g dx dy, dL/dC = -sum g dy^2 / 2.
// ACCUM: add into the gradients; else write them (zeros for a Gaussian no
// view touched).
template <bool ACCUM>
__global__ __launch_bounds__(256, 3) void k_preprocess_bwd(Ws ws, xg_gaussians g, const xg_camera *cams,
                                                        Params p, xg_grads gr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ws.n) return;
    const float *m = g.means + 3 * (int64_t)i;
    const float *s = g.scales + 3 * (int64_t)i;
    const float *q = g.quats + 4 * (int64_t)i;
    double gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0, gi = 0;
    bool any = false;
    Gauss64 G;
    gauss64(q, G);
    const double rqn = 1.0 / G.qn;
    for (int v = 0; v < ws.n_views; ++v) {
        const int64_t idx = (int64_t)v * ws.n + i;
        if (ws.counts[idx] == 0) continue;
        const float4 g0 = reinterpret_cast<const float4 *>(ws.grad2d)[2 * idx];
        const float4 g1 = reinterpret_cast<const float4 *>(ws.grad2d)[2 * idx + 1];
        any = true;
        go += g1.y;
        gi += g1.z;
        const xg_camera &c = cams[v];
        Proj64 P;
        project64(m, s, G.R, c, (double)p.lowpass, P);
        double r[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) r[k] = (double)c.rot[k];
        const double det = P.sxx * P.syy - P.sxy * P.sxy;
        const double rdet = 1.0 / det;
        const double QA = P.syy * rdet, QB = -P.sxy * rdet, QC = P.sxx * rdet;
        const double gux = QA * (double)g0.x + QB * (double)g0.y;
        const double guy = QB * (double)g0.x + QC * (double)g0.y;
        // dL/dSigma'' = -Q G_Q Q, off-diagonal of G_Q carrying half of dL/dB
        const double gA = -0.5 * (double)g0.z, gB = -0.5 * (double)g0.w, gC = -0.5 * (double)g1.x;
        const double T00 = gA * QA + gB * QB, T01 = gA * QB + gB * QC;
        const double T10 = gB * QA + gC * QB, T11 = gB * QB + gC * QC;
        const double GS00 = -(QA * T00 + QB * T10);
        const double GS01 = -(QA * T01 + QB * T11);
        const double GS10 = -(QB * T00 + QC * T10);
        const double GS11 = -(QB * T01 + QC * T11);
        const double gxx = GS00, gyy = GS11, gxy = GS01 + GS10;
        // Sigma'' = B B^T + k I
        double GB[6];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            GB[k] = 2.0 * gxx * P.B[k] + gxy * P.B[3 + k];
            GB[3 + k] = 2.0 * gyy * P.B[3 + k] + gxy * P.B[k];
        }
        // B = A2 R diag(s): dL/d(R diag s) = A2^T GB, dL/dA2 = GB (R diag s)^T
        double Ms[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) Ms[3 * a + b] = G.R[3 * a + b] * (double)s[b];
        double GA2[6];
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                GA2[3 * ii + a] = GB[3 * ii] * Ms[3 * a] + GB[3 * ii + 1] * Ms[3 * a + 1]
                                  + GB[3 * ii + 2] * Ms[3 * a + 2];
        double GR[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double gmab = P.A2[a] * GB[b] + P.A2[3 + a] * GB[3 + b];
                gs[b] += gmab * G.R[3 * a + b];
                GR[3 * a + b] = gmab * (double)s[b];
            }
        // rotation of the unit quaternion, then its normalisation
        const double w = G.q[0], x = G.q[1], y = G.q[2], z = G.q[3];
        double gw = 2 * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
        double gx = 2 * (y * GR[1] + z * GR[2] + y * GR[3] - 2 * x * GR[4] - w * GR[5]
                         + z * GR[6] + w * GR[7] - 2 * x * GR[8]);
        double gy = 2 * (-2 * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5]
                         - w * GR[6] + z * GR[7] - 2 * y * GR[8]);
        double gz = 2 * (-2 * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2 * z * GR[4]
                         + y * GR[5] + x * GR[6] + y * GR[7]);
        const double dot = w * gw + x * gx + y * gy + z * gz;
        gq[0] += (gw - w * dot) * rqn;
        gq[1] += (gx - x * dot) * rqn;
        gq[2] += (gy - y * dot) * rqn;
        gq[3] += (gz - z * dot) * rqn;
        // A2 = J W: dL/dJ = GA2 W^T (only the non-zero entries of J)
        const double GJ00 = GA2[0] * r[0] + GA2[1] * r[1] + GA2[2] * r[2];
        const double GJ02 = GA2[0] * r[6] + GA2[1] * r[7] + GA2[2] * r[8];
        const double GJ11 = GA2[3] * r[3] + GA2[4] * r[4] + GA2[5] * r[5];
        const double GJ12 = GA2[3] * r[6] + GA2[4] * r[7] + GA2[5] * r[8];
        const double fx = c.fx, fy = c.fy, tx = P.t[0], ty = P.t[1];
        const double r1 = P.rtz, r2 = r1 * r1, r3 = r2 * r1;
        const double gtx = GJ02 * (-fx * r2) + gux * (fx * r1);
        const double gty = GJ12 * (-fy * r2) + guy * (fy * r1);
        const double gtz = GJ00 * (-fx * r2) + GJ02 * (2.0 * fx * tx * r3)
                           + GJ11 * (-fy * r2) + GJ12 * (2.0 * fy * ty * r3)
                           + gux * (-fx * tx * r2) + guy * (-fy * ty * r2);
        // t = W mu + tau
#pragma unroll
        for (int a = 0; a < 3; ++a) gm[a] += r[a] * gtx + r[3 + a] * gty + r[6 + a] * gtz;
    }
    if (ACCUM && !any) return;
    // kept items have opacity >= alpha_min (single precision: the division
    // adds no registers to this double-precision kernel)
    const float gof = any ? (float)go / g.opacity[i] : 0.0f;
    float *om = gr.means + 3 * (int64_t)i;
    float *os = gr.scales + 3 * (int64_t)i;
    float *oq = gr.quats + 4 * (int64_t)i;
    if (ACCUM) {
#pragma unroll
        for (int a = 0; a < 3; ++a) { om[a] += (float)gm[a]; os[a] += (float)gs[a]; }
#pragma unroll
        for (int a = 0; a < 4; ++a) oq[a] += (float)gq[a];
        gr.opacity[i] += gof;
        gr.intensity[i] += (float)gi;
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) { om[a] = (float)gm[a]; os[a] = (float)gs[a]; }
#pragma unroll
        for (int a = 0; a < 4; ++a) oq[a] = (float)gq[a];
        gr.opacity[i] = gof;
        gr.intensity[i] = (float)gi;
    }
}

__global__ __launch_bounds__(256) void k_l1_grad(const float *img, const float *tgt, float *out,
                                                 int64_t n, float scale) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const float d = img[k] - tgt[k];
        out[k] = d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

int grid_for(int64_t n, int threads, int max_blocks = 65536) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

}  // namespace


hipError_t launch_preprocess(const Ws &ws, const xg_gaussians &g, const xg_camera *cams,
                             const Params &p, hipStream_t s) {
    const int64_t nb = (ws.n_items + kPreThreads - 1) / kPreThreads;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    // depth partials live in the scan scratch: the item sort's first launch
    // reduces them into the header (and resets it for the frame) before
    // anything else uses that scratch
    uint32_t *part = ws.scan_tmp;
    if (nb > 0)
        hipLaunchKernelGGL(k_preprocess, dim3((unsigned)nb), dim3(kPreThreads), 0, s, ws, g, cams, p,
                           part);
    else
        hipLaunchKernelGGL(k_header_reset, dim3(1), dim3(64), 0, s, ws.hdr);
    return hipGetLastError();
}

hipError_t launch_emit(const Ws &ws, const xg_camera *cams, const Params &p, hipStream_t s) {
    // one thread per depth-sorted item
    const int64_t nb = (ws.n_items + 255) / 256;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(256), 0, s, ws, cams, p.tile);
    return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const Ws &ws, const xg_gaussians &g, const xg_camera *cams, bool accumulate,
                                 const Params &p, const xg_grads &gr, hipStream_t s) {
    // one thread per Gaussian, summing its views in registers
    const int nb = (ws.n + 255) / 256;
    if (accumulate)
        hipLaunchKernelGGL(k_preprocess_bwd<true>, dim3(nb > 0 ? nb : 1), dim3(256), 0, s, ws, g, cams, p, gr);
    else
        hipLaunchKernelGGL(k_preprocess_bwd<false>, dim3(nb > 0 ? nb : 1), dim3(256), 0, s, ws, g, cams, p, gr);
    return hipGetLastError();
}

hipError_t launch_l1_grad(const float *image, const float *target, float *out, int64_t n,
                          float scale, hipStream_t s) {
    hipLaunchKernelGGL(k_l1_grad, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, image, target, out,
                       n, scale);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace xg
