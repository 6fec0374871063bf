// ACUI point grid (Sec. 3.3, Eq. 13): Gaussian centres at
// (n1 S1 d / M1, n2 S2 d / M2, n3 S3 d / M3) for integers |n_i| <= K_i,
// K_i = [M_i / (2 d)] + 1, listed with n1 slowest and n3 fastest.
//
// One thread per coordinate (3 per point), so the float32 [count][3] array
// is written with fully coalesced stores.  The coordinate is evaluated in
// float64 as ((n * S) * d) / M (two products and an IEEE division: nothing
// for the compiler to contract) and rounded once to float32.
#include "common.h"

namespace xg {

namespace {

struct AcuiArgs {
    double size[3], d;
    int32_t grid[3];
    int32_t k[3];          // K_i
    int32_t side[3];       // 2 K_i + 1
    int64_t n_coords;      // 3 * count
};

__global__ __launch_bounds__(256) void k_acui_grid(AcuiArgs a, float *means) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_coords) return;
    const int axis = (int)(c % 3);
    int64_t p = c / 3;
    // index along this axis: p = (i1 * side2 + i2) * side3 + i3
    int64_t i;
    if (axis == 2) {
        i = p % a.side[2];
    } else {
        p /= a.side[2];
        i = axis == 1 ? p % a.side[1] : p / a.side[1];
    }
    const double n = (double)(i - a.k[axis]);
    means[c] = (float)(((n * a.size[axis]) * a.d) / (double)a.grid[axis]);
}

}  // namespace

hipError_t launch_acui_grid(const double size[3], const int32_t grid[3], double d, const int32_t k[3],
                            int64_t count, float *means, hipStream_t s) {
    AcuiArgs a;
    for (int i = 0; i < 3; ++i) {
        a.size[i] = size[i];
        a.grid[i] = grid[i];
        a.k[i] = k[i];
        a.side[i] = 2 * k[i] + 1;
    }
    a.d = d;
    a.n_coords = 3 * count;
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (a.n_coords + 255) / 256;
    hipLaunchKernelGGL(k_acui_grid, dim3((unsigned)blocks), dim3(256), 0, s, a, means);
    return hipGetLastError();
}

}  // namespace xg
