// On-device microbenchmarks of the three ceilings the DRR kernels are
// measured against: HBM bandwidth (a streaming copy and a streaming read),
// scalar FP32 VALU issue rate (independent FMA chains, no memory), and LDS
// read bandwidth (conflict-free 16-byte reads).  Built as libxgpeaks.so,
// separate from the DRR library; the benchmark times each launch with
// events on the caller's stream.  Every kernel writes a result that
// depends on all of its work, so none of it can be removed by the compiler.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

__global__ __launch_bounds__(256) void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                              int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_read(const float4 *__restrict__ src, int64_t n, float *out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    float acc = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float4 v = src[i];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    // a store only for a value no input produces keeps the reads live
    if (acc == -1.0f) out[0] = acc;
}

// 8 independent FMA chains per lane: each iteration issues 8 v_fma_f32.
__global__ __launch_bounds__(256) void k_valu(float *out, int iters, float a, float b) {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = (float)threadIdx.x * 1e-7f + (float)k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    if (s == -1.0f) out[blockIdx.x] = s;
}

// LDS reads: each lane reads 16 bytes per step from consecutive addresses
// (a wavefront covers 1 KB, every bank once per 256 bytes); one XOR per
// dword keeps the VALU below the LDS rate.
__global__ __launch_bounds__(256) void k_lds(uint32_t *out, int iters) {
    __shared__ uint4 buf[4096];   // 64 KB
    for (int i = threadIdx.x; i < 4096; i += blockDim.x)
        buf[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
    __syncthreads();
    uint4 acc = make_uint4(0, 0, 0, 0);
    int idx = threadIdx.x;
    for (int i = 0; i < iters; ++i) {
        const uint4 v = buf[idx];
        acc.x ^= v.x;
        acc.y ^= v.y;
        acc.z ^= v.z;
        acc.w ^= v.w;
        idx = (idx + 256) & 4095;
    }
    const uint32_t r = acc.x ^ acc.y ^ acc.z ^ acc.w;
    if (r == 0xdeadbeefu) out[blockIdx.x] = r;
}

}  // namespace

extern "C" {

// Copies n16 16-byte elements from src to dst (device pointers).
int xgp_copy(const void *src, void *dst, int64_t n16, int blocks, void *stream) {
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const float4 *)src,
                       (float4 *)dst, n16);
    return (int)hipGetLastError();
}

// Reads n16 16-byte elements of src.
int xgp_read(const void *src, int64_t n16, float *out, int blocks, void *stream) {
    hipLaunchKernelGGL(k_read, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const float4 *)src, n16,
                       out);
    return (int)hipGetLastError();
}

// blocks x 256 lanes x iters x 8 FMA instructions.
int xgp_valu(float *out, int iters, int blocks, void *stream) {
    hipLaunchKernelGGL(k_valu, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, iters, 0.999f,
                       1e-3f);
    return (int)hipGetLastError();
}

// blocks x 256 lanes x iters x 16 bytes read from LDS.
int xgp_lds(uint32_t *out, int iters, int blocks, void *stream) {
    hipLaunchKernelGGL(k_lds, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, iters);
    return (int)hipGetLastError();
}

}  // extern "C"
