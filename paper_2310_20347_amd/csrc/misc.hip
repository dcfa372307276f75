// Small auxiliary kernels: C = beta*C (the alpha == 0 / k == 0 case of the
// BLAS semantics), the split-K reduction and a deterministic operand fill
// used by the tuner.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "registry.hpp"

namespace mg {

__global__ void scale_f32_kernel(float *C, int64_t ldc, int m, int n, float beta)
{
    const int64_t total = (int64_t)m * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t - i * n;
        float *c = C + i * ldc + j;
        *c = beta == 0.0f ? 0.0f : beta * *c;   // beta == 0: C is not read
    }
}

__global__ void scale_i32_kernel(int *C, int64_t ldc, int m, int n, int beta)
{
    const int64_t total = (int64_t)m * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t - i * n;
        int *c = C + i * ldc + j;
        *c = beta == 0 ? 0 : (int)((unsigned)beta * (unsigned)*c);
    }
}

__global__ void scale_f64_kernel(double *C, int64_t ldc, int m, int n, double beta)
{
    const int64_t total = (int64_t)m * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t - i * n;
        double *c = C + i * ldc + j;
        *c = beta == 0.0 ? 0.0 : beta * *c;   // beta == 0: C is not read
    }
}

void launch_scale(void *C, int64_t ldc, int m, int n, double beta, int elem, hipStream_t s)
{
    const int64_t total = (int64_t)m * n;
    const int threads = 256;
    int64_t blocks = (total + threads - 1) / threads;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (elem == 1)
        hipLaunchKernelGGL(scale_i32_kernel, dim3((unsigned)blocks), dim3(threads), 0, s,
                           (int *)C, ldc, m, n, (int)beta);
    else if (elem == 2)
        hipLaunchKernelGGL(scale_f64_kernel, dim3((unsigned)blocks), dim3(threads), 0, s,
                           (double *)C, ldc, m, n, beta);
    else
        hipLaunchKernelGGL(scale_f32_kernel, dim3((unsigned)blocks), dim3(threads), 0, s,
                           (float *)C, ldc, m, n, (float)beta);
}

// Split-K reduction: the S partial tiles (row stride n) summed in slice
// order, then the BLAS epilogue.
__global__ void splitk_reduce_f32(const float *P, int S, float *C, int64_t ldc, int m, int n,
                                  float alpha, float beta)
{
    const int64_t total = (int64_t)m * n, slice = (int64_t)m * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        float acc = P[t];
        for (int s = 1; s < S; ++s) acc += P[s * slice + t];
        const int64_t i = t / n, j = t - i * n;
        float *c = C + i * ldc + j;
        float v = alpha * acc;
        if (beta != 0.0f) v = __builtin_fmaf(beta, *c, v);
        *c = v;
    }
}

__global__ void splitk_reduce_i32(const int *P, int S, int *C, int64_t ldc, int m, int n, int alpha,
                                  int beta)
{
    const int64_t total = (int64_t)m * n, slice = (int64_t)m * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        unsigned acc = (unsigned)P[t];
        for (int s = 1; s < S; ++s) acc += (unsigned)P[s * slice + t];
        const int64_t i = t / n, j = t - i * n;
        int *c = C + i * ldc + j;
        unsigned v = (unsigned)alpha * acc;
        if (beta != 0) v += (unsigned)beta * (unsigned)*c;
        *c = (int)v;
    }
}

void launch_splitk_reduce(const void *P, int S, void *C, int64_t ldc, int m, int n,
                          const GemmArgs &a, bool is_int, hipStream_t s)
{
    const int64_t total = (int64_t)m * n;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (is_int)
        hipLaunchKernelGGL(splitk_reduce_i32, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const int *)P, S, (int *)C, ldc, m, n, a.ialpha, a.ibeta);
    else
        hipLaunchKernelGGL(splitk_reduce_f32, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const float *)P, S, (float *)C, ldc, m, n, a.alpha, a.beta);
}

__device__ __forceinline__ uint32_t mix(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return (uint32_t)x;
}

// Fills `count` elements of `es` bytes with finite values in [-1, 1]
// (float formats) or arbitrary bytes (int8).  kind: 0 f32, 1 bf16, 2 f16,
// 3 e4m3, 4 int8, 5 f64.
__global__ void fill_kernel(void *p, int64_t count, int kind, uint32_t seed)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t h = mix(((uint64_t)seed << 40) ^ (uint64_t)t);
        const float v = (float)((int)(h % 2001u) - 1000) * 1e-3f;
        switch (kind) {
        case 0: ((float *)p)[t] = v; break;
        case 1: ((__bf16 *)p)[t] = (__bf16)v; break;
        case 2: ((_Float16 *)p)[t] = (_Float16)v; break;
        case 3: ((uint8_t *)p)[t] = (uint8_t)(h & 0xB7u); break;  // exponent <= 6: |x| < 2
        case 5: ((double *)p)[t] = (double)v; break;
        default: ((int8_t *)p)[t] = (int8_t)(h & 0xFFu); break;
        }
    }
}

void launch_fill(void *p, int64_t count, int kind, uint32_t seed, hipStream_t s)
{
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, count, kind, seed);
}

}  // namespace mg
