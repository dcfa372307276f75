// Packing for the FP32-accurate split product (section 5.3's packing, with
// the split of each FP32 value into bf16 pieces folded in).
//
// op(X) -- R rows (m for A, n for B) by K values of k -- is rewritten as
// k-contiguous bf16 rows of KP = T * 32 * ceil(K / 32) values: every block of
// 32 k values becomes T consecutive blocks of 32, block t holding piece
// code[t] (0 = hi, 1 = mid, 2 = lo) of the same 32 values, zero past K.
// With A's blocks in the order (mid, hi, hi) and B's in (hi, mid, hi) (six
// terms: (lo, hi, mid, mid, hi, hi) and (hi, lo, mid, hi, mid, hi)), the bf16
// product of the packed operands over KP is exactly the split product: each
// 32-block of k contributes the listed piece products, smallest first, in
// the same MFMA order as the fused split tile, so the two give equal bits.
//
// One workgroup packs 64 rows x 32 k.  A k-contiguous source (A 'N', B 'T')
// is read along its rows; an m/n-contiguous one (A 'T', B 'N') is read along
// m/n and transposed through LDS.
#include "abi_internal.hpp"
#include "mgemm.h"

namespace mg {

template <bool KMODE>
__global__ void __launch_bounds__(256) pack_split_kernel(const float *X, int64_t ld, int R, int K,
                                                         unsigned short *out, int64_t ldo, int T,
                                                         u32 code)
{
    __shared__ float tile[32][65];
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * 64, kb = blockIdx.y, k0 = kb * 32;
    const int r = r0 + (tid >> 2), kq = 8 * (tid & 3);
    float v[8];
    if constexpr (KMODE) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + kq + e;
            v[e] = (r < R && k < K) ? X[(int64_t)r * ld + k] : 0.0f;
        }
    } else {
        const int lk = tid >> 3, lr = 8 * (tid & 7);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int rr = r0 + lr + e, k = k0 + lk;
            tile[lk][lr + e] = (rr < R && k < K) ? X[(int64_t)k * ld + rr] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = tile[kq + e][tid >> 2];
    }
    if (r >= R) return;
    // pieces, round-to-nearest-even at each step: hi = bf16(x), mid =
    // bf16(x - hi), lo = bf16(x - hi - mid); two values per dword
    u32 pc[3][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float x0 = v[2 * q], x1 = v[2 * q + 1];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const u32 h0 = bf16_bits(x0), h1 = bf16_bits(x1);
            pc[p][q] = h0 | (h1 << 16);
            x0 -= bf16_val(h0);
            x1 -= bf16_val(h1);
        }
    }
    unsigned short *o = out + (int64_t)r * ldo + (int64_t)kb * T * 32 + kq;
    for (int t = 0; t < T; ++t) {
        const int p = (code >> (4 * t)) & 15;
        const u32x4 w = {pc[p][0], pc[p][1], pc[p][2], pc[p][3]};
        *(u32x4 *)(o + 32 * t) = w;
    }
}

// Piece order of the packed blocks: A side and B side, per term.
static u32 piece_code(int terms, bool a_side)
{
    // three terms: mid*hi, hi*mid, hi*hi; six: lo*hi, hi*lo, mid*mid, then those
    static const int a3[3] = {1, 0, 0}, b3[3] = {0, 1, 0};
    static const int a6[6] = {2, 0, 1, 1, 0, 0}, b6[6] = {0, 2, 1, 0, 1, 0};
    const int *l = terms == 3 ? (a_side ? a3 : b3) : (a_side ? a6 : b6);
    u32 c = 0;
    for (int t = 0; t < terms; ++t) c |= u32(l[t]) << (4 * t);
    return c;
}

int64_t packed_k(int64_t k, int terms)
{
    return int64_t(terms) * 32 * ((k + 31) / 32);
}

// Packs op(X) (rows x k; kmode: X row-major rows x k, else X row-major
// k x rows) into `out` (rows x packed_k bf16).
int launch_split_pack(const float *X, int64_t ld, bool kmode, int64_t rows, int64_t k, int terms,
                      bool a_side, unsigned short *out, hipStream_t s)
{
    const int64_t kp = packed_k(k, terms);
    if ((k + 31) / 32 > 65535 || (rows + 63) / 64 > 0x7FFFFFFF) return GEMM_E_UNSUPPORTED;
    const dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((k + 31) / 32));
    const u32 code = piece_code(terms, a_side);
    if (kmode)
        hipLaunchKernelGGL(pack_split_kernel<true>, grid, dim3(256), 0, s, X, ld, (int)rows, (int)k,
                           out, kp, terms, code);
    else
        hipLaunchKernelGGL(pack_split_kernel<false>, grid, dim3(256), 0, s, X, ld, (int)rows,
                           (int)k, out, kp, terms, code);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    return GEMM_OK;
}

const void *split_pack_entry()
{
    return (const void *)&pack_split_kernel<true>;
}

}  // namespace mg
