// Radiation intensity response (Eq. 3) and the fused optimiser step.
//
// RIRF: intensity = sigmoid(w . f) per Gaussian, one thread per Gaussian.
//
// Adam: gradients of the activated parameters -> raw gradients (chain rule
// through exp / sigmoid / the response) -> Adam (bias-corrected moments,
// Kingma & Ba Algorithm 1) -> new raw parameters and the activated copies
// the next rendering reads.  One thread per raw scalar for means, scales,
// quaternions and opacity; one lane per feature for the feature vectors
// (the intensity needs all of it).  HBM bound: about 28 bytes read and
// 16-20 written per scalar.
#include "common.h"

#include <math.h>

namespace xg {

namespace {

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

// Weights staged in LDS (at most XG_MAX_FEATURES).
__device__ __forceinline__ void load_weights(const float *w, int nf, float *s_w) {
    for (int k = threadIdx.x; k < nf; k += blockDim.x) s_w[k] = w[k];
    __syncthreads();
}

__device__ __forceinline__ float rirf_dot(const float *f, const float *s_w, int nf) {
    float acc = 0.0f;
    for (int k = 0; k < nf; ++k) acc = fmaf(s_w[k], f[k], acc);
    return acc;
}

__global__ __launch_bounds__(256) void k_rirf_fwd(const float *features, const float *weights,
                                                  int64_t n, int nf, float *intensity) {
    __shared__ float s_w[XG_MAX_FEATURES];
    load_weights(weights, nf, s_w);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    intensity[i] = sigmoidf(rirf_dot(features + i * nf, s_w, nf));
}

__global__ __launch_bounds__(256) void k_rirf_bwd(const float *features, const float *weights,
                                                  int64_t n, int nf, const float *dl_di,
                                                  float *grad_f) {
    __shared__ float s_w[XG_MAX_FEATURES];
    load_weights(weights, nf, s_w);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float s = sigmoidf(rirf_dot(features + i * nf, s_w, nf));
    const float g = dl_di[i] * s * (1.0f - s);
    float *gf = grad_f + i * nf;
    for (int k = 0; k < nf; ++k) gf[k] += g * s_w[k];
}

struct AdamArgs {
    xg_params p;
    xg_grads g;
    float *m, *v;
    const int32_t *step;
    const int32_t *gate;    // nullable: nonzero skips the step
    xg_adam c;
    float b1, c1, b2, c2;   // beta and 1 - beta, each rounded once from double
    float *scales, *opacity, *intensity;
    int64_t n;
};

// Per-block step coefficients (bias corrections, position rate) in double
// from the device step counter; false when the gate skips the step.
__device__ __forceinline__ bool step_coefficients(const AdamArgs &a, float coef[3]) {
    __shared__ float s_coef[3];
    __shared__ int s_skip;
    if (threadIdx.x == 0) {
        s_skip = a.gate != nullptr && *a.gate != 0;
        const int t = *a.step + 1;
        const double f = (double)min(t - 1, a.c.lr_means_steps) / (double)max(a.c.lr_means_steps, 1);
        s_coef[0] = (float)(1.0 - pow(a.c.beta1, (double)t));
        s_coef[1] = (float)(1.0 - pow(a.c.beta2, (double)t));
        s_coef[2] = (float)exp((1.0 - f) * log((double)a.c.lr_means_start) +
                               f * log((double)a.c.lr_means_end));
    }
    __syncthreads();
    coef[0] = s_coef[0];
    coef[1] = s_coef[1];
    coef[2] = s_coef[2];
    return !s_skip;
}

__device__ __forceinline__ float adam_update(const AdamArgs &a, int64_t k, float x, float grad,
                                             float lr, float bias1, float bias2) {
    const float m = a.b1 * a.m[k] + a.c1 * grad;
    const float v = a.b2 * a.v[k] + a.c2 * grad * grad;
    a.m[k] = m;
    a.v[k] = v;
    const float mhat = m / bias1;
    const float vhat = v / bias2;
    return x - lr * mhat / (sqrtf(vhat) + a.c.eps);
}

// Raw scalar k of the concatenated [means 3n | log_scales 3n | quats 4n |
// opacity_logit n] state.
__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
    const int64_t n = a.n;
    const int64_t total = 11 * n;
    float coef[3];
    if (!step_coefficients(a, coef)) return;
    const float bias1 = coef[0], bias2 = coef[1], lr_means = coef[2];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        float *param, grad, lr;
        int kind;        // 0 identity, 1 exp, 2 sigmoid (opacity)
        int64_t e;       // index inside the group
        if (k < 3 * n) {
            e = k; param = a.p.means + e; grad = a.g.means[e]; lr = lr_means; kind = 0;
        } else if (k < 6 * n) {
            e = k - 3 * n; param = a.p.log_scales + e; grad = a.g.scales[e]; lr = a.c.lr_scales; kind = 1;
        } else if (k < 10 * n) {
            e = k - 6 * n; param = a.p.quats + e; grad = a.g.quats[e]; lr = a.c.lr_quats; kind = 0;
        } else {
            e = k - 10 * n; param = a.p.opacity_logit + e; grad = a.g.opacity[e]; lr = a.c.lr_opacity; kind = 2;
        }
        const float x = *param;
        // chain rule at the value the renderer used
        if (kind == 1) {
            grad *= expf(x);
        } else if (kind == 2) {
            const float s = sigmoidf(x);
            grad *= s * (1.0f - s);
        }
        const float xn = adam_update(a, k, x, grad, lr, bias1, bias2);
        *param = xn;
        if (kind == 1) a.scales[e] = expf(xn);
        else if (kind == 2) a.opacity[e] = sigmoidf(xn);
    }
}

// Feature vectors: G lanes per Gaussian (G = the feature count rounded up
// to a power of two, at most 64), lane k owning feature k, so every access
// is coalesced.  The response's chain rule at the current features (the
// inner product summed across the G lanes with shuffles), Adam on each
// feature, then the new intensity from the updated features.
template <int G>
__global__ __launch_bounds__(256) void k_adam_features(AdamArgs a) {
    __shared__ float s_w[XG_MAX_FEATURES];
    const int nf = a.p.n_features;
    load_weights(a.p.weights, nf, s_w);
    float coef[3];
    if (!step_coefficients(a, coef)) return;
    const float bias1 = coef[0], bias2 = coef[1];
    const int k = (int)(threadIdx.x % G);   // the stride is a multiple of G
    const bool own = k < nf;
    const float wk = own ? s_w[k] : 0.0f;
    // grid-stride over the groups (the weights and coefficients are set up
    // once per workgroup); the G lanes of a group stay together
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < a.n * G;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / G;
        float *f = a.p.features + i * nf + k;
        const float x = own ? *f : 0.0f;
        float dot = wk * x;
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) dot += __shfl_xor(dot, o, kWave);
        const float s = sigmoidf(dot);
        const float gs = a.g.intensity[i] * s * (1.0f - s);
        float xn = 0.0f;
        if (own) {
            xn = adam_update(a, 11 * a.n + i * nf + k, x, gs * wk, a.c.lr_feature, bias1, bias2);
            *f = xn;
        }
        float dn = wk * xn;
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) dn += __shfl_xor(dn, o, kWave);
        if (k == 0) a.intensity[i] = sigmoidf(dn);
    }
}

__global__ void k_step_advance(int32_t *step, const int32_t *gate) {
    if (threadIdx.x == 0 && (gate == nullptr || *gate == 0)) *step += 1;
}

// Grid of a grid-stride launch of 256 threads over n work items: at most
// 2048 workgroups (8 per CU on 256 CUs), so the per-workgroup set-up (step
// coefficients in double, the response weights) runs a few thousand times
// rather than once per 256 items.
unsigned grid_of(int64_t n) {
    int64_t nb = (n + 255) / 256;
    if (nb < 1) nb = 1;
    if (nb > 2048) nb = 2048;
    return (unsigned)nb;
}

}  // namespace

hipError_t launch_rirf_fwd(const float *features, const float *weights, int64_t n, int nf,
                           float *intensity, hipStream_t s) {
    const int64_t nb = (n + 255) / 256;
    if (nb > 0)
        hipLaunchKernelGGL(k_rirf_fwd, dim3((unsigned)nb), dim3(256), 0, s, features, weights, n, nf,
                           intensity);
    return hipGetLastError();
}

hipError_t launch_rirf_bwd(const float *features, const float *weights, int64_t n, int nf,
                           const float *dl_di, float *grad_f, hipStream_t s) {
    const int64_t nb = (n + 255) / 256;
    if (nb > 0)
        hipLaunchKernelGGL(k_rirf_bwd, dim3((unsigned)nb), dim3(256), 0, s, features, weights, n, nf,
                           dl_di, grad_f);
    return hipGetLastError();
}

hipError_t launch_adam(const xg_params &p, const xg_grads &g, float *m, float *v, int32_t *step,
                       const xg_adam &c, float *scales, float *opacity, float *intensity,
                       const int32_t *gate, hipStream_t s) {
    AdamArgs a{p, g, m, v, step, gate, c,
               (float)c.beta1, (float)(1.0 - c.beta1), (float)c.beta2, (float)(1.0 - c.beta2),
               scales, opacity, intensity, (int64_t)p.n};
    hipLaunchKernelGGL(k_adam, dim3(grid_of(11 * (int64_t)p.n)), dim3(256), 0, s, a);
    int G = 1;
    while (G < p.n_features) G *= 2;
    const dim3 grid(grid_of((int64_t)p.n * G));
    switch (G) {
        case 1: hipLaunchKernelGGL(k_adam_features<1>, grid, dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_adam_features<2>, grid, dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(k_adam_features<4>, grid, dim3(256), 0, s, a); break;
        case 8: hipLaunchKernelGGL(k_adam_features<8>, grid, dim3(256), 0, s, a); break;
        case 16: hipLaunchKernelGGL(k_adam_features<16>, grid, dim3(256), 0, s, a); break;
        case 32: hipLaunchKernelGGL(k_adam_features<32>, grid, dim3(256), 0, s, a); break;
        case 64: hipLaunchKernelGGL(k_adam_features<64>, grid, dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step, gate);
    return hipGetLastError();
}

}  // namespace xg
