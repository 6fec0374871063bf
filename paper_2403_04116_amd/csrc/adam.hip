// Fused optimiser step: gradients of the activated parameters -> raw
// gradients (chain rule through exp / sigmoid) -> Adam (bias-corrected
// moments, Kingma & Ba Algorithm 1) -> new raw parameters and the
// activated copies the next rendering reads.  One thread per raw scalar;
// purely HBM bound (about 28 bytes read and 16-20 written per scalar).
#include "common.h"

#include <math.h>

namespace xg {

namespace {

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

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

// Raw scalar k of the concatenated [means 3n | log_scales 3n | quats 4n |
// opacity_logit n | feature n] state.
__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
    const int64_t n = a.n;
    const int64_t total = 12 * n;
    // step t = counter + 1: bias corrections and the position rate schedule,
    // in double once per block
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
    if (s_skip) return;
    const float bias1 = s_coef[0], bias2 = s_coef[1], lr_means = s_coef[2];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        float *param, grad, lr;
        int kind;        // 0 identity, 1 exp, 2 sigmoid (opacity), 3 sigmoid(lambda f)
        int64_t e;       // index inside the group
        if (k < 3 * n) {
            e = k; param = a.p.means + e; grad = a.g.means[e]; lr = lr_means; kind = 0;
        } else if (k < 6 * n) {
            e = k - 3 * n; param = a.p.log_scales + e; grad = a.g.scales[e]; lr = a.c.lr_scales; kind = 1;
        } else if (k < 10 * n) {
            e = k - 6 * n; param = a.p.quats + e; grad = a.g.quats[e]; lr = a.c.lr_quats; kind = 0;
        } else if (k < 11 * n) {
            e = k - 10 * n; param = a.p.opacity_logit + e; grad = a.g.opacity[e]; lr = a.c.lr_opacity; kind = 2;
        } else {
            e = k - 11 * n; param = a.p.feature + e; grad = a.g.intensity[e]; lr = a.c.lr_feature; kind = 3;
        }
        const float x = *param;
        // chain rule at the value the renderer used
        if (kind == 1) {
            grad *= expf(x);
        } else if (kind == 2) {
            const float s = sigmoidf(x);
            grad *= s * (1.0f - s);
        } else if (kind == 3) {
            const float s = sigmoidf(a.c.feature_weight * x);
            grad *= a.c.feature_weight * s * (1.0f - s);
        }
        const float m = a.b1 * a.m[k] + a.c1 * grad;
        const float v = a.b2 * a.v[k] + a.c2 * grad * grad;
        a.m[k] = m;
        a.v[k] = v;
        const float mhat = m / bias1;
        const float vhat = v / bias2;
        const float xn = x - lr * mhat / (sqrtf(vhat) + a.c.eps);
        *param = xn;
        if (kind == 1) a.scales[e] = expf(xn);
        else if (kind == 2) a.opacity[e] = sigmoidf(xn);
        else if (kind == 3) a.intensity[e] = sigmoidf(a.c.feature_weight * xn);
    }
}

__global__ void k_step_advance(int32_t *step, const int32_t *gate) {
    if (threadIdx.x == 0 && (gate == nullptr || *gate == 0)) *step += 1;
}

}  // namespace

hipError_t launch_adam(const xg_params &p, const xg_grads &g, float *m, float *v, int32_t *step,
                       const xg_adam &c, float *scales, float *opacity, float *intensity,
                       const int32_t *gate, hipStream_t s) {
    AdamArgs a{p, g, m, v, step, gate, c,
               (float)c.beta1, (float)(1.0 - c.beta1), (float)c.beta2, (float)(1.0 - c.beta2),
               scales, opacity, intensity, (int64_t)p.n};
    const int64_t total = 12 * (int64_t)p.n;
    int64_t nb = (total + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step, gate);
    return hipGetLastError();
}

}  // namespace xg
