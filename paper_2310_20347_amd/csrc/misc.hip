// Small auxiliary kernels: C = beta*C (the alpha == 0 / k == 0 case of the
// BLAS semantics), the split-K reduction, a deterministic operand fill used
// by the tuner, and the debug mode's sentinel fill and count.
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

// Debug mode: the m x n block of C is filled with a sentinel (a NaN with a
// payload of its own; for int32 C the same bits) before a beta = 0 product,
// and counted after it, so elements the product left unwritten are found.
constexpr unsigned kSentinel32 = 0x7FC0DEADu;
constexpr unsigned long long kSentinel64 = 0x7FF8DEADDEADDEADull;

__global__ void debug_fill_kernel(char *C, int64_t ldc, int64_t m, int64_t n, int es)
{
    const int64_t total = m * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t - i * n;
        if (es == 8) ((unsigned long long *)C)[i * ldc + j] = kSentinel64;
        else ((unsigned *)C)[i * ldc + j] = kSentinel32;
    }
}

__global__ void debug_count_kernel(const char *C, int64_t ldc, int64_t m, int64_t n, int es,
                                   unsigned long long *count)
{
    const int64_t total = m * n;
    unsigned long long found = 0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t - i * n;
        if (es == 8) found += ((const unsigned long long *)C)[i * ldc + j] == kSentinel64;
        else found += ((const unsigned *)C)[i * ldc + j] == kSentinel32;
    }
    if (found) atomicAdd(count, found);
}

static int64_t debug_blocks(int64_t total)
{
    int64_t blocks = (total + 255) / 256;
    return blocks > 4096 ? 4096 : (blocks < 1 ? 1 : blocks);
}

void launch_debug_fill(void *C, int64_t ldc, int64_t m, int64_t n, int es, hipStream_t s)
{
    hipLaunchKernelGGL(debug_fill_kernel, dim3((unsigned)debug_blocks(m * n)), dim3(256), 0, s,
                       (char *)C, ldc, m, n, es);
}

void launch_debug_count(const void *C, int64_t ldc, int64_t m, int64_t n, int es,
                        unsigned long long *count, hipStream_t s)
{
    hipLaunchKernelGGL(debug_count_kernel, dim3((unsigned)debug_blocks(m * n)), dim3(256), 0, s,
                       (const char *)C, ldc, m, n, es, count);
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

// e4m3 byte of a finite float (truncated; below 2^-6 to zero, above 448 to
// 448): test data only.
__device__ __forceinline__ uint8_t e4m3_trunc(float v)
{
    const uint32_t b = __float_as_uint(v);
    const uint8_t sign = (uint8_t)((b >> 24) & 0x80u);
    int e = (int)((b >> 23) & 0xFFu) - 127;
    uint32_t m = (b >> 20) & 7u;
    if (e < -6) return sign;
    if (e > 8 || (e == 8 && m == 7u)) {
        e = 8;
        m = 6;
    }
    return (uint8_t)(sign | ((uint32_t)(e + 7) << 3) | m);
}

// Fills `count` elements with the tuner's operands: approximately N(0, 1)
// values (the sum of four uniforms, scaled to unit variance) in the float
// formats, as the benchmark's precision workload draws them (the
// power-limited low-precision kernels run at a clock that depends on the
// data), and arbitrary bytes for int8, int16 and int32.  kind: 0 f32,
// 1 bf16, 2 f16, 3 e4m3, 4 int8, 5 f64, 6 int16, 7 int32.
__global__ void fill_kernel(void *p, int64_t count, int kind, uint32_t seed)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t h = mix(((uint64_t)seed << 40) ^ (uint64_t)t);
        const uint32_t g = mix(((uint64_t)(seed ^ 0x9E3779B9u) << 40) ^ (uint64_t)t);
        const float u = (float)(h & 0xFFFFu) + (float)(h >> 16) + (float)(g & 0xFFFFu) + (float)(g >> 16);
        const float v = (u * (1.0f / 65536.0f) - 2.0f) * 1.7320508f;
        switch (kind) {
        case 0: ((float *)p)[t] = v; break;
        case 1: ((__bf16 *)p)[t] = (__bf16)v; break;
        case 2: ((_Float16 *)p)[t] = (_Float16)v; break;
        case 3: ((uint8_t *)p)[t] = e4m3_trunc(v); break;
        case 5: ((double *)p)[t] = (double)v; break;
        case 6: ((int16_t *)p)[t] = (int16_t)(h & 0xFFFFu); break;
        case 7: ((int32_t *)p)[t] = (int32_t)(h ^ (g << 16)); break;
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
