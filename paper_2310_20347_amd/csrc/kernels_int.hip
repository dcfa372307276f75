// INT16 and INT32 GEMM (the paper's 16- and 32-bit integer routines, data-type
// study of section 8.5).  C is int32 in both: the exact integer value
// alpha * op(A) op(B) + beta * C modulo 2^32.
//
// gfx950 has no 16- or 32-bit integer MFMA.  Two configurations per type:
//
//   0  vector ALUs: a 64x64 tile per workgroup, operands staged through LDS
//      element by element (any alignment and layout), 4x4 outputs per thread
//      accumulated in wrapping 32-bit arithmetic (24-bit multiplies for int16).
//
//   1  digit products on the INT8 MFMA.  Each operand value is cut into int8
//      digits by a packing pass (section 5.3's packing, here into digit
//      planes) and the product is formed from INT8 GEMMs over the planes:
//
//      INT32: balanced base-256 digits a = d0 + 2^8 d1 + 2^16 d2 + 2^24 d3
//      (mod 2^32), each in [-128, 127].  Modulo 2^32 only the digit pairs of
//      weight 2^(8s), s = i + j <= 3, remain: ten products,
//        C = alpha * sum_s 2^(8s) sum_{i+j=s} Di Ej^T + beta * C.
//
//      INT16: a = 256 hi + lo + 128 with hi = a >> 8 and lo = (a & 255) - 128,
//      both in [-128, 127]; with a~ = a - 128 and row sums SA_i = sum_p a_ip,
//      SB_j = sum_p b_pj:
//        sum_p a b = 2^16 Hi Hi' + 2^8 (Hi Lo' + Lo Hi') + Lo Lo'
//                    + 128 SA_i + 128 SB_j - 2^14 k,
//      four products and a rank-two correction.
//
//      The planes of one operand row are laid out side by side along k (kp =
//      k rounded up to 64, zero digits past k), A's in increasing digit order
//      and B's in decreasing order, so every class sum_{i+j=s} Di Ej^T is ONE
//      INT8 GEMM over a contiguous window of (s+1) kp values of k: no extra
//      accumulator, the tuned INT8 tile of that size runs it ('N','T', both
//      operands contiguous along k), and the classes accumulate into C through
//      the INT8 epilogue's wrapping alpha / beta (alpha 2^(8s) alpha, beta 1
//      after the first).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "abi_internal.hpp"
#include "mgemm.h"
#include "tile.hpp"

namespace mg {
namespace {

// ---------------------------------------------------------------------------
// Configuration 0: vector-ALU tile.
// ---------------------------------------------------------------------------
template <class T, bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_int_valu_kernel(GemmArgs p)
{
    __shared__ T As[16][65], Bs[16][65];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    int tm, tn;
    raster((int)blockIdx.x, p.tiles_m, p.tiles_n, p.order, p.group, tm, tn);
    const int m0 = tm * 64, n0 = tn * 64;
    const T *A = (const T *)p.A, *B = (const T *)p.B;
    u32 acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0u;
    const int kend = p.ialpha != 0 ? p.k : 0;
    for (int k0 = 0; k0 < kend; k0 += 16) {
        for (int e = tid; e < 1024; e += 256) {
            // consecutive threads along each operand's contiguous index
            const int i = TA ? (e & 63) : (e >> 4), kk = TA ? (e >> 6) : (e & 15);
            const int gi = m0 + i, gk = k0 + kk;
            As[kk][i] = (gi < p.m && gk < p.k)
                            ? (TA ? A[(int64_t)gk * p.lda + gi] : A[(int64_t)gi * p.lda + gk])
                            : T(0);
            const int j = TB ? (e >> 4) : (e & 63), kb = TB ? (e & 15) : (e >> 6);
            const int gj = n0 + j, gkb = k0 + kb;
            Bs[kb][j] = (gj < p.n && gkb < p.k)
                            ? (TB ? B[(int64_t)gj * p.ldb + gkb] : B[(int64_t)gkb * p.ldb + gj])
                            : T(0);
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            int a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if constexpr (sizeof(T) == 2)
                        acc[r][c] += (u32)__mul24(a[r], b[c]);   // |a b| <= 2^30: exact
                    else
                        acc[r][c] += (u32)a[r] * (u32)b[c];      // low 32 bits
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int row = m0 + ty * 4 + r, col = n0 + tx * 4 + c;
            if (row < p.m && col < p.n) {
                int *cp = (int *)p.C + (int64_t)row * p.ldc + col;
                u32 v = (u32)p.ialpha * acc[r][c];
                if (p.ibeta != 0) v += (u32)p.ibeta * (u32)*cp;
                *cp = (int)v;
            }
        }
}

// ---------------------------------------------------------------------------
// Configuration 1: digit planes + INT8 MFMA GEMMs.
// ---------------------------------------------------------------------------

// Digits of one value (most significant last); zero digits past k.
template <int P>
__device__ __forceinline__ void digits_of(int v, bool valid, int (&d)[P])
{
    if (!valid) {
#pragma unroll
        for (int i = 0; i < P; ++i) d[i] = 0;
        return;
    }
    if constexpr (P == 2) {
        d[0] = (v & 255) - 128;   // lo, offset by 128
        d[1] = v >> 8;            // hi (arithmetic shift)
    } else {
        // balanced base-256 digits; the last is taken modulo 256 (a change of
        // 2^32 in the value)
        int64_t r = v;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int di = (int)(signed char)(unsigned char)(r & 255);
            d[i] = di;
            r = (r - di) >> 8;
        }
    }
}

// Writes the P digit planes of `R` operand rows (rows of op(A), or columns of
// op(B)) as int8 rows of P*KP bytes: plane q of row r at r*P*KP + q'*KP, q' =
// q (A) or P-1-q (B, REV).  KMODE: the operand is contiguous along k.  A
// workgroup converts 64 rows x 64 values of k per step through LDS
// (coalesced reads in either layout, 16-byte writes) and walks the k steps
// kb = blockIdx.y, blockIdx.y + gridDim.y, ...  SUMS: adds each row's sum of
// its (k) values to sums[r] (wrapping; the array starts at zero).
template <class T, int P, bool KMODE, bool REV, bool SUMS>
__global__ void __launch_bounds__(256) pack_digits_kernel(const T *X, int64_t ld, int R, int K,
                                                          int KP, char *out, int *sums)
{
    __shared__ int tile[64][65];
    const int tid = threadIdx.x;
    const int r0 = (int)blockIdx.x * 64;
    const int64_t ostride = (int64_t)P * KP;
    const int wr = tid >> 2, wseg = (tid & 3) * 16;   // this thread writes 16 k of row wr
    u32 rowsum = 0u;
    for (int kb = (int)blockIdx.y; kb * 64 < KP; kb += (int)gridDim.y) {
        const int k0 = kb * 64;
        __syncthreads();
        for (int e = tid; e < 4096; e += 256) {
            const int r = KMODE ? (e >> 6) : (e & 63), kk = KMODE ? (e & 63) : (e >> 6);
            const int gr = r0 + r, gk = k0 + kk;
            int v = 0;
            if (gr < R && gk < K)
                v = KMODE ? (int)X[(int64_t)gr * ld + gk] : (int)X[(int64_t)gk * ld + gr];
            tile[r][kk] = v;
        }
        __syncthreads();
        if (r0 + wr < R) {
            u32 w[P][4];
#pragma unroll
            for (int q = 0; q < P; ++q)
#pragma unroll
                for (int h = 0; h < 4; ++h) w[q][h] = 0u;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int v = tile[wr][wseg + e];
                const bool valid = k0 + wseg + e < K;
                if (SUMS) rowsum += (u32)v;   // zero past k
                int d[P];
                digits_of<P>(v, valid, d);
#pragma unroll
                for (int q = 0; q < P; ++q) w[q][e >> 2] |= ((u32)d[q] & 255u) << (8 * (e & 3));
            }
            char *row = out + (int64_t)(r0 + wr) * ostride + k0 + wseg;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const int plane = REV ? P - 1 - q : q;
                *(u32x4 *)(row + (int64_t)plane * KP) = u32x4{w[q][0], w[q][1], w[q][2], w[q][3]};
            }
        }
    }
    if constexpr (SUMS) {
        // the four threads of a row are adjacent lanes of one wave
        rowsum += (u32)__shfl_xor((int)rowsum, 1);
        rowsum += (u32)__shfl_xor((int)rowsum, 2);
        if ((tid & 3) == 0 && r0 + wr < R) atomicAdd((unsigned *)&sums[r0 + wr], rowsum);
    }
}

__global__ void zero_i32_kernel(int *p, int count)
{
    for (int t = (int)(blockIdx.x * blockDim.x + threadIdx.x); t < count; t += (int)(gridDim.x * blockDim.x))
        p[t] = 0;
}

// INT16's rank-two term: C = beta C + alpha (128 SA_i + 128 SB_j - 2^14 k),
// wrapping; C is not read when beta == 0.
__global__ void int16_correction_kernel(int *C, int64_t ldc, int m, int n, const int *sa,
                                        const int *sb, int k, int alpha, int beta)
{
    const int64_t total = (int64_t)m * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t - i * n;
        const u32 corr = 128u * (u32)sa[i] + 128u * (u32)sb[j] - 16384u * (u32)k;
        int *c = C + i * ldc + j;
        u32 v = (u32)alpha * corr;
        if (beta != 0) v += (u32)beta * (u32)*c;
        *c = (int)v;
    }
}

template <class T, int P, bool REV, bool SUMS>
hipError_t launch_pack(const void *X, int64_t ld, bool kmode, int64_t R, int64_t K, int64_t KP,
                       char *out, int *sums, hipStream_t s)
{
    const int64_t bx = (R + 63) / 64, nkb = KP / 64;
    const int64_t by = std::max<int64_t>(1, std::min<int64_t>(nkb, (2048 + bx - 1) / bx));
    const dim3 grid((unsigned)bx, (unsigned)by);
    if (kmode)
        hipLaunchKernelGGL((pack_digits_kernel<T, P, true, REV, SUMS>), grid, dim3(256), 0, s,
                           (const T *)X, ld, (int)R, (int)K, (int)KP, out, sums);
    else
        hipLaunchKernelGGL((pack_digits_kernel<T, P, false, REV, SUMS>), grid, dim3(256), 0, s,
                           (const T *)X, ld, (int)R, (int)K, (int)KP, out, sums);
    return hipGetLastError();
}

template <class T, bool TA, bool TB>
void fill_valu(KernelCfg &c)
{
    c.func[2 * TA + TB][0] = (const void *)&gemm_int_valu_kernel<T, TA, TB>;
    c.func[2 * TA + TB][1] = (const void *)&gemm_int_valu_kernel<T, TA, TB>;
}

template <class T>
void register_int_class(std::vector<KernelCfg> &out, int kclass)
{
    KernelCfg c;
    c.kclass = kclass;
    c.mc = 64;
    c.nc = 64;
    c.kc = 16;
    c.wm = 16;   // thread grid: 4x4 outputs per thread
    c.wn = 16;
    c.threads = 256;
    c.lds = 2 * 16 * 65 * (int)sizeof(T);
    c.stages = 1;
    c.kind = 0;
    fill_valu<T, false, false>(c);
    fill_valu<T, false, true>(c);
    fill_valu<T, true, false>(c);
    fill_valu<T, true, true>(c);
    out.push_back(c);

    // digit products: the packing pass reads any layout and alignment; the
    // entry marks the layouts (the INT8 tiles are chosen per call)
    KernelCfg d;
    d.kclass = kclass;
    d.mc = 256;
    d.nc = 256;
    d.kc = 128;
    d.wm = 2;
    d.wn = 4;
    d.threads = 256;
    d.lds = 0;
    d.stages = 2;
    d.kind = 7;
    d.direct = true;
    constexpr int P = sizeof(T) == 2 ? 2 : 4;
    constexpr bool S = sizeof(T) == 2;
    const void *marks[4] = {
        (const void *)&pack_digits_kernel<T, P, true, false, S>,
        (const void *)&pack_digits_kernel<T, P, false, false, S>,
        (const void *)&pack_digits_kernel<T, P, true, true, S>,
        (const void *)&pack_digits_kernel<T, P, false, true, S>};
    for (int t = 0; t < 4; ++t) {
        d.func[t][0] = marks[t];
        d.func[t][1] = marks[t];
    }
    out.push_back(d);
}

}  // namespace

void register_int_late(std::vector<KernelCfg> &out)
{
    register_int_class<short>(out, K_I16);
    register_int_class<int>(out, K_I32);
}

int digit_planes(int kclass) { return kclass == K_I16 ? 2 : 4; }

DigitLayout digit_layout(int kclass, int64_t m, int64_t n, int64_t k)
{
    DigitLayout L;
    L.P = digit_planes(kclass);
    L.kp = (k + 63) / 64 * 64;
    L.a_off = 0;
    L.b_off = (m * L.P * L.kp + 255) / 256 * 256;
    L.sums_off = L.b_off + (n * L.P * L.kp + 255) / 256 * 256;
    L.total = L.sums_off + (kclass == K_I16 ? ((m + n) * 4 + 255) / 256 * 256 : 0);
    return L;
}

int launch_digits(const KernelCfg &c, const GemmArgs &a, int trans, hipStream_t s, Workspace w)
{
    const bool i16 = c.kclass == K_I16;
    const DigitLayout L = digit_layout(c.kclass, a.m, a.n, a.k);
    if (!w.ptr || w.bytes < (size_t)L.total) return kPackUnavailable;
    if ((int64_t)L.P * L.kp > 0x7FFFFFFF) return GEMM_E_UNSUPPORTED;
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    char *ws = (char *)w.ptr;
    char *pa = ws + L.a_off, *pb = ws + L.b_off;
    int *sa = (int *)(ws + L.sums_off), *sb = sa + a.m;
    const bool ta = (trans >> 1) != 0, tb = (trans & 1) != 0;
    hipError_t e = hipSuccess;
    if (i16) {
        const int cnt = a.m + a.n;
        hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)std::min(1024, (cnt + 255) / 256)),
                           dim3(256), 0, s, sa, cnt);
        if ((e = hipGetLastError()) == hipSuccess)
            e = launch_pack<short, 2, false, true>(a.A, a.lda, !ta, a.m, a.k, L.kp, pa, sa, s);
        if (e == hipSuccess)
            e = launch_pack<short, 2, true, true>(a.B, a.ldb, tb, a.n, a.k, L.kp, pb, sb, s);
        if (e == hipSuccess) {
            const int64_t total = int64_t(a.m) * a.n;
            const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(65536, (total + 255) / 256));
            hipLaunchKernelGGL(int16_correction_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                               (int *)a.C, a.ldc, a.m, a.n, sa, sb, a.k, a.ialpha, a.ibeta);
            e = hipGetLastError();
        }
    } else {
        e = launch_pack<int, 4, false, false>(a.A, a.lda, !ta, a.m, a.k, L.kp, pa, nullptr, s);
        if (e == hipSuccess)
            e = launch_pack<int, 4, true, false>(a.B, a.ldb, tb, a.n, a.k, L.kp, pb, nullptr, s);
    }
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    // the INT8 GEMM of one weight class: A planes from a_plane, B planes from
    // b_plane, over `planes` * kp values of k; the rest of the workspace is
    // the INT8 configuration's own (it runs unsliced when that is too small)
    Workspace rest;
    rest.ptr = ws + L.total;
    rest.bytes = w.bytes - (size_t)L.total;
    const int64_t ldp = (int64_t)L.P * L.kp;
    auto class_gemm = [&](int a_plane, int b_plane, int planes, int shift, bool first) -> int {
        const u32 al = (u32)a.ialpha << shift;
        const int alpha_s = (int)al;
        const int beta_s = first ? a.ibeta : 1;
        GemmArgs b;
        int tr = 0, cfg = 0, kc8 = 0;
        bool vec = true;
        const int saved = t_tls.force_id[K_I8];
        t_tls.force_id[K_I8] = -1;   // a pin on INT8 calls is not meant for these
        const int reg = plan_gemm(GEMM_I8, 'N', 'T', a.m, a.n, (int64_t)planes * L.kp,
                                  (double)alpha_s, pa + (int64_t)a_plane * L.kp, ldp,
                                  pb + (int64_t)b_plane * L.kp, ldp, (double)beta_s, a.C, a.ldc,
                                  d->cus, b, tr, vec, cfg, kc8);
        t_tls.force_id[K_I8] = saved;
        if (reg < 0) return GEMM_E_UNSUPPORTED;
        return launch_gemm(g_cfgs[reg], tr, vec, b, s, rest);
    };
    if (i16) {
        // planes: A [lo | hi], B [hi | lo]
        if ((rc = class_gemm(1, 0, 1, 16, false)) != GEMM_OK) return rc;   // hi hi'
        if ((rc = class_gemm(0, 0, 2, 8, false)) != GEMM_OK) return rc;    // lo hi' + hi lo'
        return class_gemm(0, 1, 1, 0, false);                              // lo lo'
    }
    // planes: A [d0 d1 d2 d3], B [e3 e2 e1 e0]; class s pairs A planes 0..s
    // with B planes 3-s..3
    if ((rc = class_gemm(0, 0, 4, 24, true)) != GEMM_OK) return rc;
    if ((rc = class_gemm(0, 1, 3, 16, false)) != GEMM_OK) return rc;
    if ((rc = class_gemm(0, 2, 2, 8, false)) != GEMM_OK) return rc;
    return class_gemm(0, 3, 1, 0, false);
}

}  // namespace mg
