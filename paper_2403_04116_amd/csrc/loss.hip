// Training objective of Eq. 11: L = (1 - gamma) L1 + gamma (1 - mean SSIM)
// and its gradient with respect to the rendered images, every view in one
// launch pair.  SSIM uses an 11 x 11 separable Gaussian window (standard
// deviation 1.5) with zero padding, C1 = 0.01^2, C2 = 0.03^2.
//
// One wavefront per 48 x 8 pixel strip of a view.  Window sums are separable:
//   vertical pass: lane l owns image column x0 - 5 + l (58 of 64 lanes) and
//     walks the 18 rows y0 - 5 .. y0 + 12 with coalesced row loads, keeping
//     the eight 11-tap sums of every quantity in registers;
//   horizontal pass: the vertical sums go through LDS; lane l = 8 j + m
//     takes the run of 6 output pixels (row j, columns 6m .. 6m + 5), reads
//     the 16 vertical sums it needs once and forms the 6 outputs in
//     registers.
// Row j of a quantity sits at LDS word 64 j + kRowOff[j]: the run starts
// 6m (m < 8) plus these offsets cover all 64 banks, so both passes are free
// of bank conflicts (also with 32 banks per half wave).
//
// Kernel 1 (k_ssim_stats): the five statistics mx, my, E[x^2], E[y^2],
// E[xy], the SSIM map S and its partial derivatives with respect to mx,
// E[x^2] and E[xy] (three per-pixel maps in the workspace), and the strip's
// share of the loss.
// Kernel 2 (k_ssim_grad): the adjoint, i.e. the window sums of the three
// maps (the window is symmetric; zero padding makes the adjoint another
// zero-padded window sum) combined with x and y, plus the L1 subgradient.
// Kernel 3 (k_loss_sum, one workgroup, only when the loss value is asked
// for) adds the strip shares in double in a fixed order: the loss value is
// deterministic.
#include "common.h"

#include <math.h>

#include <mutex>

namespace xg {

namespace {

constexpr int kTW = 48;                  // strip width (output columns)
constexpr int kTH = 8;                   // strip height (output rows)
constexpr int kR = 5;                    // window radius
constexpr int kW = 2 * kR + 1;           // window taps
constexpr int kCols = kTW + 2 * kR;      // 58 columns feed the strip
constexpr int kRows = kTH + 2 * kR;      // 18 rows feed the strip
constexpr int kRun = 6;                  // horizontal outputs per lane
constexpr int kRunIn = kRun + 2 * kR;    // 16 vertical sums feed a run
constexpr int kQStride = 64 * kTH + 64;  // LDS words per quantity
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;
static_assert(kCols <= kWave && (kTW / kRun) * kTH == kWave, "one wave per strip");

__host__ __device__ constexpr int row_base(int j) {
    // 64 j + {0, 1, 16, 17, 32, 33, 48, 49}[j]
    return 64 * j + ((j >> 1) << 4) + (j & 1);
}
static_assert(row_base(kTH - 1) + kCols <= kQStride, "rows of a quantity stay in its LDS range");
static_assert(row_base(kTH - 1) + kRun * 7 + kRunIn <= row_base(kTH - 1) + kCols, "runs read inside the row");

struct Win {
    float w[kW];
};

struct Strip {
    int view, x0, y0, W, H;
    int64_t off;
};

__device__ __forceinline__ int strips_x(int W) { return (W + kTW - 1) / kTW; }
__device__ __forceinline__ int strips_y(int H) { return (H + kTH - 1) / kTH; }

__device__ __forceinline__ Strip strip_of(const xg_camera *cams, int n_views, int t) {
    Strip s{-1, 0, 0, 0, 0, 0};
    for (int v = 0; v < n_views; ++v) {
        const int W = cams[v].width, H = cams[v].height;
        const int sx = strips_x(W), nt = sx * strips_y(H);
        if (t < nt) {
            s.view = v;
            s.x0 = (t % sx) * kTW;
            s.y0 = (t / sx) * kTH;
            s.W = W;
            s.H = H;
            s.off = cams[v].pixel_offset;
            return s;
        }
        t -= nt;
    }
    return s;
}

// Vertical pass of Q quantities for this lane's column.  load(i, v) fills
// the Q values of pixel i of the view (row-major index, below 2^30 as views
// are at most 32767 x 32767).  Every row is loaded from a clamped, in-image
// address and zeroed when it lies outside the image, so no load sits behind
// a branch and all rows are in flight together.  Writes the kTH sums of
// every quantity to LDS.  center(v, in) sees the strip's own rows, in = the
// pixel is in the image and in the strip.
template <int Q, class Load, class Center>
__device__ __forceinline__ void vertical_pass(const Win &win, const Strip &s, float *lds, Load load,
                                              Center center) {
    const int l = lane_id();
    const int col = s.x0 - kR + l;
    const bool col_ok = l < kCols && col >= 0 && col < s.W;
    const int cc = min(max(col, 0), s.W - 1);
    const bool col_in = col_ok && l >= kR && l < kR + kTW;
    float acc[Q][kTH];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int j = 0; j < kTH; ++j) acc[q][j] = 0.0f;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int row = s.y0 - kR + r;
        const bool ok = col_ok && row >= 0 && row < s.H;
        float v[Q];
        load(min(max(row, 0), s.H - 1) * s.W + cc, v);
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] = ok ? v[q] : 0.0f;
        if (r >= kR && r < kR + kTH) center(v, ok && col_in);
#pragma unroll
        for (int j = 0; j < kTH; ++j) {
            const int t = r - j;
            if (t >= 0 && t < kW) {
#pragma unroll
                for (int q = 0; q < Q; ++q) acc[q][j] = fmaf(win.w[t], v[q], acc[q][j]);
            }
        }
    }
    if (l < kCols) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < kTH; ++j) lds[q * kQStride + row_base(j) + l] = acc[q][j];
    }
}

// Horizontal pass: the kRun window sums of Q quantities of this lane's run.
template <int Q>
__device__ __forceinline__ void horizontal_pass(const Win &win, const float *lds, float out[Q][kRun]) {
    const int l = lane_id();
    const int base = row_base(l >> 3) + kRun * (l & 7);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        float in[kRunIn];
#pragma unroll
        for (int k = 0; k < kRunIn; ++k) in[k] = lds[q * kQStride + base + k];
#pragma unroll
        for (int i = 0; i < kRun; ++i) {
            float a = 0.0f;
#pragma unroll
            for (int t = 0; t < kW; ++t) a = fmaf(win.w[t], in[i + t], a);
            out[q][i] = a;
        }
    }
}

__device__ __forceinline__ float wave_sum(float v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__global__ __launch_bounds__(kWave) void k_ssim_stats(Ws ws, const xg_camera *cams, Win win,
                                                      int n_strips, const float *image,
                                                      const float *target, float gamma,
                                                      float *partial) {
    __shared__ float lds[5 * kQStride];
    const int t = xcd_tile(blockIdx.x, n_strips);
    const Strip s = strip_of(cams, ws.n_views, t);
    if (s.view < 0) return;
    float l1 = 0.0f;
    const float *img = image + s.off, *tgt = target + s.off;
    vertical_pass<5>(
        win, s, lds,
        [&](int i, float *v) {
            const float x = img[i], y = tgt[i];
            v[0] = x; v[1] = y; v[2] = x * x; v[3] = y * y; v[4] = x * y;
        },
        [&](const float *v, bool in) { l1 += in ? fabsf(v[0] - v[1]) : 0.0f; });
    __syncthreads();
    float st[5][kRun];
    horizontal_pass<5>(win, lds, st);
    const int l = lane_id();
    const int py = s.y0 + (l >> 3), px0 = s.x0 + kRun * (l & 7);
    const int64_t N = ws.total_pixels;
    float *dm = ws.ssim + s.off, *dxx = dm + N, *dxy = dm + 2 * N;
    float ssum = 0.0f;
#pragma unroll
    for (int i = 0; i < kRun; ++i) {
        const float mx = st[0][i], my = st[1][i];
        const float a1 = 2.0f * mx * my + kC1;
        const float a2 = 2.0f * (st[4][i] - mx * my) + kC2;
        const float b1 = mx * mx + my * my + kC1;
        const float b2 = (st[2][i] - mx * mx) + (st[3][i] - my * my) + kC2;
        // hardware reciprocals (1 ulp): a1, b1 >= C1 and a2, b2 > 0 away from
        // perfectly anti-correlated windows, far from the denormal range
        const float ra1 = __builtin_amdgcn_rcpf(a1), ra2 = __builtin_amdgcn_rcpf(a2);
        const float rb1 = __builtin_amdgcn_rcpf(b1), rb2 = __builtin_amdgcn_rcpf(b2);
        const float S = (a1 * a2) * (rb1 * rb2);
        if (py < s.H && px0 + i < s.W) {
            const int k = py * s.W + px0 + i;
            dm[k] = S * (2.0f * my * (ra1 - ra2) + 2.0f * mx * (rb2 - rb1));
            dxx[k] = -S * rb2;
            dxy[k] = 2.0f * S * ra2;
            ssum += S;
        }
    }
    if (!partial) return;
    const float part = wave_sum((1.0f - gamma) * l1 - gamma * ssum);
    if (l == 0) partial[t] = part;
}

__global__ __launch_bounds__(kWave) void k_ssim_grad(Ws ws, const xg_camera *cams, Win win,
                                                     int n_strips, const float *image,
                                                     const float *target, float gamma, float *dl) {
    __shared__ float lds[3 * kQStride];
    const int64_t N = ws.total_pixels;
    const int t = xcd_tile(blockIdx.x, n_strips);
    const Strip s = strip_of(cams, ws.n_views, t);
    if (s.view < 0) return;
    const float *dm = ws.ssim + s.off, *dxx = dm + N, *dxy = dm + 2 * N;
    vertical_pass<3>(
        win, s, lds,
        [&](int i, float *v) {
            v[0] = dm[i]; v[1] = dxx[i]; v[2] = dxy[i];
        },
        [](const float *, bool) {});
    __syncthreads();
    float c[3][kRun];
    horizontal_pass<3>(win, lds, c);
    const int l = lane_id();
    const int py = s.y0 + (l >> 3), px0 = s.x0 + kRun * (l & 7);
    const float inv_n = 1.0f / (float)N;
    const float *img = image + s.off, *tgt = target + s.off;
    float *out = dl + s.off;
    // the run's pixels, loaded together from clamped (in-image) addresses
    const int row = min(py, s.H - 1) * s.W;
    float xs[kRun], ys[kRun];
#pragma unroll
    for (int i = 0; i < kRun; ++i) {
        const int k = row + min(px0 + i, s.W - 1);
        xs[i] = img[k];
        ys[i] = tgt[k];
    }
#pragma unroll
    for (int i = 0; i < kRun; ++i) {
        const float x = xs[i], y = ys[i], d = x - y;
        const float l1 = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
        const float ds = c[0][i] + 2.0f * x * c[1][i] + y * c[2][i];
        if (py < s.H && px0 + i < s.W) out[row + px0 + i] = ((1.0f - gamma) * l1 - gamma * ds) * inv_n;
    }
}

constexpr int kSumThreads = 1024;
constexpr int kSumUnroll = 8;

// loss = gamma + (sum of the strip shares) / N; every thread adds a fixed
// set of shares in double, then a fixed-shape tree adds the threads.
__global__ __launch_bounds__(kSumThreads) void k_loss_sum(const float *partial, int n, float gamma,
                                                          int64_t n_pixels, float *loss) {
    __shared__ double red[kSumThreads / kWave];
    double a = 0.0;
    for (int k0 = threadIdx.x; k0 < n; k0 += kSumThreads * kSumUnroll) {
        float v[kSumUnroll];
#pragma unroll
        for (int u = 0; u < kSumUnroll; ++u) {
            const int k = k0 + u * kSumThreads;
            v[u] = k < n ? partial[k] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kSumUnroll; ++u) a += (double)v[u];
    }
    for (int o = kWave / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, kWave);
    if (lane_id() == 0) red[threadIdx.x / kWave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kSumThreads / kWave; ++w) t += red[w];
        loss[0] = (float)((double)gamma + t / (double)n_pixels);
    }
}

// Per-device addresses of the scratch array below, resolved on the first
// call on each device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices];

}  // namespace

// Scratch of the allocation-free loss gradient (xg_loss_grad_static): the
// three per-pixel maps and the per-strip loss shares of one call.  Each
// device that loads the library holds its own copy until the process ends.
// Host code never passes this name to a kernel (on the host it is only a
// stand-in for the symbol): it resolves each device's address once, with
// hipGetSymbolAddress, and passes that address.
__device__ __align__(256) float scratch[XG_STATIC_SCRATCH_BYTES / sizeof(float)];

hipError_t static_scratch(float **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

int64_t loss_tiles(const xg_camera *cams, int n_views) {
    int64_t t = 0;
    for (int v = 0; v < n_views; ++v)
        t += (int64_t)((cams[v].width + kTW - 1) / kTW) * ((cams[v].height + kTH - 1) / kTH);
    return t;
}

hipError_t launch_loss_grad(const Ws &ws, const xg_camera *cams_dev, int64_t tiles,
                            const float *image, const float *target, float gamma, float *dl,
                            float *loss, hipStream_t s) {
    Win win;
    double w[kW], sum = 0.0;
    for (int k = 0; k < kW; ++k) {
        const double x = (double)(k - kR);
        w[k] = exp(-x * x / (2.0 * 1.5 * 1.5));
        sum += w[k];
    }
    for (int k = 0; k < kW; ++k) win.w[k] = (float)(w[k] / sum);
    if (tiles <= 0) return hipSuccess;
    if (tiles > INT32_MAX) return hipErrorInvalidValue;
    const int n = (int)tiles;
    float *partial = loss ? ws.ssim + 3 * ws.total_pixels : nullptr;
    hipLaunchKernelGGL(k_ssim_stats, dim3((unsigned)n), dim3(kWave), 0, s, ws, cams_dev, win, n, image,
                       target, gamma, partial);
    hipLaunchKernelGGL(k_ssim_grad, dim3((unsigned)n), dim3(kWave), 0, s, ws, cams_dev, win, n, image,
                       target, gamma, dl);
    if (loss)
        hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(kSumThreads), 0, s, partial, n, gamma,
                           (int64_t)ws.total_pixels, loss);
    return hipGetLastError();
}

}  // namespace xg
