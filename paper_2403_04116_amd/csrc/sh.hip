// View-dependent RGB colour of the comparison model (3D Gaussian splatting,
// Sec. 3.1 Eq. 2): c = sum_{l <= L} sum_{|m| <= l} k_l^m Y_l^m(d), taken as
// max(c + 1/2, 0) per channel, where d is the unit direction from the X-ray
// source (-R^T t of the view) to the Gaussian centre and Y_l^m are the real
// spherical harmonics (Condon-Shortley phase; basis index l^2 + l + m).
//
// One thread per Gaussian: its (L+1)^2 x 3 coefficients are read once and
// every view's colour is written into the free fourth slot of that
// (view, Gaussian)'s render record, so the RGB blend stages it with the
// rest of the record (one cache line).
#include "common.h"

#include <math.h>

namespace xg {

namespace {

// Normalisation constants of the real harmonics (closed forms, evaluated on
// the host): y0 = 1/(2 sqrt(pi)); l = 1: sqrt(3/(4 pi)); l = 2: (1/2)
// sqrt(15/pi), (1/4) sqrt(5/pi), (1/4) sqrt(15/pi); l = 3: (1/4)
// sqrt(35/(2 pi)), (1/2) sqrt(105/pi), (1/4) sqrt(21/(2 pi)), (1/4)
// sqrt(7/pi), (1/4) sqrt(105/pi).
struct ShConst {
    float y0, c1, c2a, c2b, c2c, c33, c32, c31, c30, c32b;
};

template <int L>
__device__ __forceinline__ void sh_basis(const ShConst &k, float x, float y, float z, float *Y) {
    Y[0] = k.y0;
    if (L >= 1) {
        Y[1] = -k.c1 * y;
        Y[2] = k.c1 * z;
        Y[3] = -k.c1 * x;
    }
    if (L >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = k.c2a * x * y;
        Y[5] = -k.c2a * y * z;
        Y[6] = k.c2b * (2.0f * zz - xx - yy);
        Y[7] = -k.c2a * x * z;
        Y[8] = k.c2c * (xx - yy);
        if (L >= 3) {
            const float r2 = xx + yy;
            Y[9] = -k.c33 * y * (3.0f * xx - yy);
            Y[10] = k.c32 * x * y * z;
            Y[11] = -k.c31 * y * (4.0f * zz - r2);
            Y[12] = k.c30 * z * (2.0f * zz - 3.0f * r2);
            Y[13] = -k.c31 * x * (4.0f * zz - r2);
            Y[14] = k.c32b * z * (xx - yy);
            Y[15] = -k.c33 * x * (xx - 3.0f * yy);
        }
    }
}

template <int L>
__global__ __launch_bounds__(256) void k_sh_color(Ws ws, const xg_camera *cams, ShConst kc,
                                                  const float *means, const float *sh) {
    constexpr int NB = (L + 1) * (L + 1);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ws.n) return;
    float k[NB * 3];
    const float *src = sh + i * (NB * 3);
#pragma unroll
    for (int j = 0; j < NB * 3; ++j) k[j] = src[j];
    const float mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
    for (int v = 0; v < ws.n_views; ++v) {
        const xg_camera &c = cams[v];
        // source position -R^T t
        const float sx = -(c.rot[0] * c.trans[0] + c.rot[3] * c.trans[1] + c.rot[6] * c.trans[2]);
        const float sy = -(c.rot[1] * c.trans[0] + c.rot[4] * c.trans[1] + c.rot[7] * c.trans[2]);
        const float sz = -(c.rot[2] * c.trans[0] + c.rot[5] * c.trans[1] + c.rot[8] * c.trans[2]);
        const float dx = mx - sx, dy = my - sy, dz = mz - sz;
        const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
        float Y[NB];
        sh_basis<L>(kc, dx * inv, dy * inv, dz * inv, Y);
        float r = 0.0f, g = 0.0f, b = 0.0f;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            r = fmaf(k[3 * j], Y[j], r);
            g = fmaf(k[3 * j + 1], Y[j], g);
            b = fmaf(k[3 * j + 2], Y[j], b);
        }
        ws.rec[(int64_t)v * ws.n + i].d =
            make_float4(fmaxf(r + 0.5f, 0.0f), fmaxf(g + 0.5f, 0.0f), fmaxf(b + 0.5f, 0.0f), 0.0f);
    }
}

}  // namespace

hipError_t launch_sh_color(const Ws &ws, const xg_camera *cams_dev, const float *means, const float *sh,
                           int degree, hipStream_t s) {
    const double pi = 3.14159265358979323846;
    ShConst k;
    k.y0 = (float)(0.5 / sqrt(pi));
    k.c1 = (float)sqrt(3.0 / (4.0 * pi));
    k.c2a = (float)(0.5 * sqrt(15.0 / pi));
    k.c2b = (float)(0.25 * sqrt(5.0 / pi));
    k.c2c = (float)(0.25 * sqrt(15.0 / pi));
    k.c33 = (float)(0.25 * sqrt(35.0 / (2.0 * pi)));
    k.c32 = (float)(0.5 * sqrt(105.0 / pi));
    k.c31 = (float)(0.25 * sqrt(21.0 / (2.0 * pi)));
    k.c30 = (float)(0.25 * sqrt(7.0 / pi));
    k.c32b = (float)(0.25 * sqrt(105.0 / pi));
    if (ws.n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((ws.n + 255) / 256)), block(256);
    switch (degree) {
        case 0: hipLaunchKernelGGL(k_sh_color<0>, grid, block, 0, s, ws, cams_dev, k, means, sh); break;
        case 1: hipLaunchKernelGGL(k_sh_color<1>, grid, block, 0, s, ws, cams_dev, k, means, sh); break;
        case 2: hipLaunchKernelGGL(k_sh_color<2>, grid, block, 0, s, ws, cams_dev, k, means, sh); break;
        case 3: hipLaunchKernelGGL(k_sh_color<3>, grid, block, 0, s, ws, cams_dev, k, means, sh); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace xg
