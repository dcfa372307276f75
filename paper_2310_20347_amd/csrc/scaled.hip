// Power-of-two scaled low-precision GEMM on FP32 operands (gemm_scaled).
//
// A narrow format (bfloat16, binary16, FP8 E4M3FN) covers a range of
// magnitudes that badly scaled FP32 data overflows or underflows.  Each row
// i of op(A) and each column j of op(B) is scaled by a power of two,
// 2^-e_i and 2^-f_j, chosen to place its largest magnitude M in [2^T,
// 2^(T+1)) (e = floor(log2 M) - T; T = 14 for binary16, 7 for E4M3, 0 for
// bfloat16), and rounded to the format (nearest, ties to even; E4M3
// saturates at 448).  The scalings are exact, so
//     C = alpha * 2^(e_i + f_j) * sum_p qa(i,p) qb(p,j) + beta * C
// with the product formed by the library's GEMM of that format (FP32
// accumulation).  Rows or columns that are all zero or hold a non-finite
// value are not scaled (e = 0).
//
// Passes: exponents of op(A) rows and op(B) columns; quantisation into the
// stream's second workspace (operands kept in their stored layout, leading
// dimensions rounded to 16 bytes so the GEMM takes its vectorised path); the
// GEMM (into C when beta = 0, else into the workspace); the scaling epilogue.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "abi_internal.hpp"
#include "mgemm.h"

namespace mg {
namespace {

constexpr int kT_BF16 = 0, kT_F16 = 14, kT_E4M3 = 7;

__device__ __forceinline__ int exponent_of_max(float mx, bool finite, int T)
{
    if (!finite || mx == 0.0f) return 0;
    int ex;
    (void)frexpf(mx, &ex);   // mx = f * 2^ex, f in [0.5, 1)
    return (ex - 1) - T;
}

// Exponents of R vectors of length K, element p of vector r at X[r*ld + p]:
// one workgroup per vector.
__global__ void __launch_bounds__(256) row_exponents(const float *X, int64_t ld, int K, int T, int *e)
{
    __shared__ float s_max[256];
    __shared__ int s_bad[256];
    const int r = blockIdx.x;
    float mx = 0.0f;
    int bad = 0;
    for (int p = threadIdx.x; p < K; p += 256) {
        const float a = fabsf(X[(int64_t)r * ld + p]);
        if (!(a <= 3.402823466e38f)) bad = 1;   // Inf or NaN
        else mx = fmaxf(mx, a);
    }
    s_max[threadIdx.x] = mx;
    s_bad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_max[threadIdx.x] = fmaxf(s_max[threadIdx.x], s_max[threadIdx.x + w]);
            s_bad[threadIdx.x] |= s_bad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) e[r] = exponent_of_max(s_max[0], !s_bad[0], T);
}

// The same for vectors along the other index (element p of vector r at
// X[p*ld + r]): workgroups of 256 vectors x `rows` values of p, neighbouring
// threads on neighbouring addresses; the partial maxima meet in `part` by
// integer atomic max (a non-negative float orders like its bit pattern;
// Inf/NaN are recorded as 0xFFFFFFFF).  `part` starts at zero.
__global__ void __launch_bounds__(256) col_max(const float *X, int64_t ld, int R, int K, int rows, u32 *part)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= R) return;
    const int p0 = blockIdx.y * rows, p1 = min(K, p0 + rows);
    u32 mx = 0;
    for (int p = p0; p < p1; ++p) {
        const float a = fabsf(X[(int64_t)p * ld + r]);
        const u32 b = (a <= 3.402823466e38f) ? __builtin_bit_cast(u32, a) : 0xFFFFFFFFu;
        mx = b > mx ? b : mx;
    }
    atomicMax(&part[r], mx);
}

__global__ void __launch_bounds__(256) col_exponents(const u32 *part, int R, int T, int *e)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= R) return;
    const u32 b = part[r];
    e[r] = exponent_of_max(__builtin_bit_cast(float, b == 0xFFFFFFFFu ? 0u : b), b != 0xFFFFFFFFu, T);
}

__global__ void fill_zero(u32 *p, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Round-to-nearest-even encoders on the FP32 bit pattern.
__device__ __forceinline__ u32 rne_drop(u32 base, u32 rem, u32 half)
{
    return base + ((rem > half || (rem == half && (base & 1u))) ? 1u : 0u);
}

__device__ __forceinline__ unsigned short enc_f16(float y)
{
    const u32 u = __builtin_bit_cast(u32, y);
    const u32 s = (u >> 16) & 0x8000u, a = u & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return (unsigned short)(s | 0x7E00u);
    const u32 e = a >> 23;
    if (e >= 113) {   // |y| >= 2^-14: binary16 normal range (or overflow)
        const u32 q = rne_drop((a >> 13) - (112u << 10), a & 0x1FFFu, 0x1000u);
        return (unsigned short)(s | (q >= 0x7C00u ? 0x7C00u : q));
    }
    if (e < 102) return (unsigned short)s;   // below half the smallest subnormal
    const u32 m = (a & 0x7FFFFFu) | 0x800000u, sh = 126u - e;   // q = y * 2^24
    return (unsigned short)(s | rne_drop(m >> sh, m & ((1u << sh) - 1u), 1u << (sh - 1u)));
}

__device__ __forceinline__ unsigned char enc_e4m3(float y)
{
    const u32 u = __builtin_bit_cast(u32, y);
    const u32 s = (u >> 24) & 0x80u, a = u & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return (unsigned char)(s | 0x7Fu);
    const u32 e = a >> 23;
    if (e >= 121) {   // |y| >= 2^-6: normal range, saturating at 448 (code 0x7E)
        const u32 q = e >= 136 ? 0x7Fu : rne_drop(((e - 120u) << 3) | ((a >> 20) & 7u), a & 0xFFFFFu, 0x80000u);
        return (unsigned char)(s | (q > 0x7Eu ? 0x7Eu : q));
    }
    if (e < 117) return (unsigned char)s;   // below half of 2^-9
    const u32 m = (a & 0x7FFFFFu) | 0x800000u, sh = 141u - e;   // q = y * 2^9
    return (unsigned char)(s | rne_drop(m >> sh, m & ((1u << sh) - 1u), 1u << (sh - 1u)));
}

// Q = codes of the stored rows x cols matrix X scaled by 2^-e[index], the
// index being the element's row (BY_ROW) or column.
// Grid: x over columns (256 per workgroup), y over rows, both strided.
template <int FMT, bool BY_ROW>
__global__ void __launch_bounds__(256) quantize(const float *X, int64_t ld, int rows, int cols,
                                                const int *e, void *Q, int64_t ldq)
{
    for (int r = blockIdx.y; r < rows; r += gridDim.y)
        for (int c = blockIdx.x * 256 + threadIdx.x; c < cols; c += gridDim.x * 256) {
            const float y = ldexpf(X[(int64_t)r * ld + c], -e[BY_ROW ? r : c]);
            if constexpr (FMT == 0) ((unsigned short *)Q)[(int64_t)r * ldq + c] = (unsigned short)bf16_bits(y);
            else if constexpr (FMT == 1) ((unsigned short *)Q)[(int64_t)r * ldq + c] = enc_f16(y);
            else ((unsigned char *)Q)[(int64_t)r * ldq + c] = enc_e4m3(y);
        }
}

// C = alpha * 2^(e_i + f_j) * P + beta * C (C not read when beta = 0; P may be C).
__global__ void __launch_bounds__(256) scale_epilogue(const float *P, int64_t ldp, float *C,
                                                      int64_t ldc, int m, int n, const int *e,
                                                      const int *f, float alpha, float beta)
{
    for (int i = blockIdx.y; i < m; i += gridDim.y)
        for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
            float v = alpha * ldexpf(P[(int64_t)i * ldp + j], e[i] + f[j]);
            if (beta != 0.0f) v = fmaf(beta, C[(int64_t)i * ldc + j], v);
            C[(int64_t)i * ldc + j] = v;
        }
}

// 2-D grid over a rows x cols matrix: 256 columns per workgroup, one row per
// grid row (both capped; the kernels stride).
dim3 grid2(int64_t rows, int64_t cols)
{
    const int64_t gx = std::min<int64_t>((cols + 255) / 256, 1024);
    const int64_t gy = std::min<int64_t>(rows, 65535);
    return dim3((unsigned)std::max<int64_t>(gx, 1), (unsigned)std::max<int64_t>(gy, 1));
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

bool is_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }

template <int FMT>
void launch_quantize(bool by_row, const float *X, int64_t ld, int rows, int cols, const int *e, void *Q,
                     int64_t ldq, hipStream_t s)
{
    const dim3 g = grid2(rows, cols);
    if (by_row)
        hipLaunchKernelGGL((quantize<FMT, true>), g, dim3(256), 0, s, X, ld, rows, cols, e, Q, ldq);
    else
        hipLaunchKernelGGL((quantize<FMT, false>), g, dim3(256), 0, s, X, ld, rows, cols, e, Q, ldq);
}

// Exponents of the R op-vectors of length K stored in X (contiguous or
// not); `part` holds R words of scratch for the strided case.
void launch_exponents(bool contig, const float *X, int64_t ld, int R, int K, int T, int *e, u32 *part,
                      hipStream_t s)
{
    if (contig) {
        hipLaunchKernelGGL(row_exponents, dim3((unsigned)R), dim3(256), 0, s, X, ld, K, T, e);
        return;
    }
    const unsigned gx = (unsigned)((R + 255) / 256);
    const int rows = std::max(256, (K + 65534) / 65535);   // at most 65535 slices of k
    hipLaunchKernelGGL(fill_zero, dim3(gx), dim3(256), 0, s, part, R);
    hipLaunchKernelGGL(col_max, dim3(gx, (unsigned)((K + rows - 1) / rows)), dim3(256), 0, s, X, ld, R,
                       K, rows, part);
    hipLaunchKernelGGL(col_exponents, dim3(gx), dim3(256), 0, s, part, R, T, e);
}

// Workspace layout of one scaled call: exponents e (m) and f (n), partial
// maxima of the strided exponent reductions, the quantised operands, and the
// FP32 partial product when beta != 0 (else the product goes to C).
struct ScaledLayout {
    int fmt, T, es;
    bool ta, tb;
    int64_t ar, ac, br, bc, ldqa, ldqb;
    int64_t e_bytes, f_bytes, part_bytes, qa_bytes, qb_bytes, p_bytes;
    int64_t total() const { return e_bytes + f_bytes + part_bytes + qa_bytes + qb_bytes + p_bytes; }
};

ScaledLayout scaled_layout(char transA, char transB, int64_t m, int64_t n, int64_t k, double beta,
                           int dtype)
{
    ScaledLayout L;
    L.ta = is_trans(transA);
    L.tb = is_trans(transB);
    L.fmt = dtype == GEMM_BF16 ? 0 : (dtype == GEMM_F16 ? 1 : 2);
    L.T = L.fmt == 0 ? kT_BF16 : (L.fmt == 1 ? kT_F16 : kT_E4M3);
    L.es = L.fmt == 2 ? 1 : 2;
    // stored shapes: A is m x k ('N') or k x m ('T'); B is k x n ('N') or n x k ('T')
    L.ar = L.ta ? k : m;
    L.ac = L.ta ? m : k;
    L.br = L.tb ? n : k;
    L.bc = L.tb ? k : n;
    L.ldqa = round_up(L.ac, 16 / L.es);
    L.ldqb = round_up(L.bc, 16 / L.es);
    L.e_bytes = round_up(m * 4, 256);
    L.f_bytes = round_up(n * 4, 256);
    L.part_bytes = L.e_bytes + L.f_bytes;
    L.qa_bytes = round_up(L.ar * L.ldqa * L.es, 256);
    L.qb_bytes = round_up(L.br * L.ldqb * L.es, 256);
    L.p_bytes = beta != 0.0 ? m * n * 4 : 0;
    return L;
}

// Common argument checks and quick returns of the scaled entry points:
// 1 = proceed, otherwise the return code.
int scaled_check(char transA, char transB, int64_t m, int64_t n, int64_t k, double alpha,
                 const void *A, int64_t lda, const void *B, int64_t ldb, double beta, void *C,
                 int64_t ldc, int dtype)
{
    // FP32 operands and C: the FP32 rules of gemm(), then the format (argument 14)
    const int v = validate(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, GEMM_F32);
    if (v != 0) return v;
    if (dtype != GEMM_BF16 && dtype != GEMM_F16 && dtype != GEMM_F8E4M3) return -14;
    if (m == 0 || n == 0) return GEMM_OK;
    if (alpha == 0.0 || k == 0)
        return gemm(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, GEMM_F32);
    if (m > 0x7FFFFFFF || n > 0x7FFFFFFF || k > 0x7FFFFFFF) return GEMM_E_UNSUPPORTED;
    return 1;
}

// The scaled product's passes on the workspace `ws` (L.total() bytes).
int scaled_run(const ScaledLayout &L, char transA, char transB, int64_t m, int64_t n, int64_t k,
               double alpha, const void *A, int64_t lda, const void *B, int64_t ldb, double beta,
               void *C, int64_t ldc, int dtype, char *ws, hipStream_t s)
{
    int *e = (int *)ws, *f = (int *)(ws + L.e_bytes);
    u32 *part_a = (u32 *)(ws + L.e_bytes + L.f_bytes), *part_b = (u32 *)(ws + 2 * L.e_bytes + L.f_bytes);
    char *qa = ws + L.e_bytes + L.f_bytes + L.part_bytes, *qb = qa + L.qa_bytes;
    float *P = L.p_bytes ? (float *)(qb + L.qb_bytes) : (float *)C;
    const int64_t ldp = L.p_bytes ? n : ldc;
    const bool ta = L.ta, tb = L.tb;
    // op(A) row i: stored row i ('N', contiguous) or stored column i ('T');
    // op(B) column j: stored column j ('N') or stored row j ('T', contiguous)
    launch_exponents(!ta, (const float *)A, lda, (int)m, (int)k, L.T, e, part_a, s);
    launch_exponents(tb, (const float *)B, ldb, (int)n, (int)k, L.T, f, part_b, s);
    switch (L.fmt) {
    case 0:
        launch_quantize<0>(!ta, (const float *)A, lda, (int)L.ar, (int)L.ac, e, qa, L.ldqa, s);
        launch_quantize<0>(tb, (const float *)B, ldb, (int)L.br, (int)L.bc, f, qb, L.ldqb, s);
        break;
    case 1:
        launch_quantize<1>(!ta, (const float *)A, lda, (int)L.ar, (int)L.ac, e, qa, L.ldqa, s);
        launch_quantize<1>(tb, (const float *)B, ldb, (int)L.br, (int)L.bc, f, qb, L.ldqb, s);
        break;
    default:
        launch_quantize<2>(!ta, (const float *)A, lda, (int)L.ar, (int)L.ac, e, qa, L.ldqa, s);
        launch_quantize<2>(tb, (const float *)B, ldb, (int)L.br, (int)L.bc, f, qb, L.ldqb, s);
        break;
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        t_tls.hip_err = (int)err;
        return GEMM_E_HIP;
    }
    const int rc = gemm(transA, transB, m, n, k, 1.0, qa, L.ldqa, qb, L.ldqb, 0.0, P, ldp, dtype);
    if (rc != GEMM_OK) return rc;
    hipLaunchKernelGGL(scale_epilogue, grid2(m, n), dim3(256), 0, s, (const float *)P, ldp,
                       (float *)C, ldc, (int)m, (int)n, e, f, (float)alpha, (float)beta);
    err = hipGetLastError();
    if (err != hipSuccess) {
        t_tls.hip_err = (int)err;
        return GEMM_E_HIP;
    }
    return GEMM_OK;
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" int gemm_scaled(char transA, char transB, int64_t m, int64_t n, int64_t k, double alpha,
                           const void *A, int64_t lda, const void *B, int64_t ldb, double beta, void *C,
                           int64_t ldc, int dtype)
{
    const int c = scaled_check(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (c != 1) return c;
    ensure_registered();
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    hipStream_t s = t_tls.stream;
    const ScaledLayout L = scaled_layout(transA, transB, m, n, k, beta, dtype);
    // the stream's reserved workspace (gemm_init / gemm_reserve_workspace)
    char *ws = (char *)stream_workspace(d, s, (size_t)L.total(), 1);
    if (!ws) return GEMM_E_WORKSPACE;
    return scaled_run(L, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, ws, s);
}

extern "C" int64_t gemm_scaled_workspace_bytes(char transA, char transB, int64_t m, int64_t n,
                                               int64_t k, double beta, int dtype)
{
    if (dtype != GEMM_BF16 && dtype != GEMM_F16 && dtype != GEMM_F8E4M3) return -1;
    if (m < 0 || n < 0 || k < 0) return -1;
    if (m == 0 || n == 0 || k == 0) return 0;
    return scaled_layout(transA, transB, m, n, k, beta, dtype).total();
}
