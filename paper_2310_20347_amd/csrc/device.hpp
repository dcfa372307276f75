// Device-side building blocks of the blocked GEMM family for gfx950.
//
// Vocabulary follows the paper (section 3): the five loops L1..L5 around a
// micro-kernel, block sizes mc x nc x kc for the packed buffers Ac (mc x kc)
// and Bc (kc x nc), and an mr x nr micro-tile of C held in registers
// (section 4.1).  On CDNA4 the packed buffers are LDS panels filled by the
// whole workgroup, and the micro-tile is a wave's grid of 16x16 MFMA
// accumulator blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mg {

typedef unsigned int u32;
typedef unsigned long long u64;
typedef u32 u32x2 __attribute__((ext_vector_type(2)));
typedef u32 u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Kernel arguments of one GEMM (one problem of a grouped launch has the same
// fields).  Sizes fit int32 (checked on the host); strides are int64.
struct GemmArgs {
    const void *A;
    const void *B;
    void *C;
    int64_t lda, ldb, ldc;
    int m, n, k;
    float alpha, beta;      // float paths
    int ialpha, ibeta;      // INT8 path (wrapping int32 arithmetic)
    int tiles_m, tiles_n;   // ceil(m/mc), ceil(n/nc)
    int order;              // 0: B3A2C0 raster (column panels outer), 1: A3B2C0
    int group;              // raster group width, in tiles
    int terms;              // split-product terms (3 or 6) for the split path
    double dalpha, dbeta;   // FP64 path
};

// --------------------------------------------------------------------------
// Element traits.  For every type:
//   GES    bytes of one element in global memory (input format)
//   LES    bytes of one element in LDS (MFMA operand format)
//   PLANES LDS planes per operand (1, or the bf16 pieces of the split path)
//   FDW    dwords of one MFMA operand fragment per lane
//   KF     k covered by one fragment read: 4 lane groups x FDW*4/LES values
//   KC     k per LDS stage: one 128-byte LDS row per operand row
//   MNV    elements per global vector when the operand is contiguous along
//          m or n (the transposed staging mode)
// --------------------------------------------------------------------------
struct TF32 {
    static constexpr int GES = 4, LES = 4, PLANES = 1, FDW = 4, KF = 16, MNV = 4;
    static constexpr bool INT = false, SPLIT = false;
};
struct TBF16 {
    static constexpr int GES = 2, LES = 2, PLANES = 1, FDW = 4, KF = 32, MNV = 4;
    static constexpr bool INT = false, SPLIT = false, HALF = false;
};
struct TF16 {
    static constexpr int GES = 2, LES = 2, PLANES = 1, FDW = 4, KF = 32, MNV = 4;
    static constexpr bool INT = false, SPLIT = false, HALF = true;
};
struct TI8 {
    static constexpr int GES = 1, LES = 1, PLANES = 1, FDW = 4, KF = 64, MNV = 4;
    static constexpr bool INT = true, SPLIT = false;
};
// FP64: v_mfma_f64_16x16x4f64, one double per lane and k step; a 16-byte
// fragment read holds two k steps.
struct TF64 {
    static constexpr int GES = 8, LES = 8, PLANES = 1, FDW = 4, KF = 8, MNV = 2;
    static constexpr bool INT = false, SPLIT = false;
};
struct TF8 {
    static constexpr int GES = 1, LES = 1, PLANES = 1, FDW = 8, KF = 128, MNV = 4;
    static constexpr bool INT = false, SPLIT = false;
};
// FP32 inputs split on the fly into P bf16 pieces (hi, mid[, lo]).
template <int P>
struct TSplit {
    static constexpr int GES = 4, LES = 2, PLANES = P, FDW = 4, KF = 32, MNV = 4;
    static constexpr bool INT = false, SPLIT = true;
};

template <class DT>
struct Kc {
    static constexpr int value = 128 / DT::LES;
};

template <class DT>
struct AccOf {
    typedef f32x4 type;
};
template <>
struct AccOf<TI8> {
    typedef i32x4 type;
};
template <>
struct AccOf<TF64> {
    typedef f64x4 type;
};

// The BLAS alpha of a tile's arguments is non-zero (the k loop runs).
template <class DT>
__device__ __forceinline__ bool alpha_nonzero(const GemmArgs &p)
{
    if constexpr (DT::INT) return p.ialpha != 0;
    else if constexpr (DT::GES == 8) return p.dalpha != 0.0;
    else return p.alpha != 0.0f;
}

// --------------------------------------------------------------------------
// LDS panel layout.  An operand panel (the packed Ac or Bc of one stage) is
// ROWS rows (of m or n) x kc values, 128 bytes per row, k contiguous inside a
// row.  The 16-byte chunks of a row are XOR-swizzled,
//     physical chunk = logical chunk ^ swz(row),  swz(r) = (r ^ (r / V)) & 7,
// so that 8 consecutive rows read at the same logical chunk (one MFMA
// fragment read) and 8 rows V apart written at the same chunk (transposed
// staging) both touch 8 distinct chunks, i.e. all 32 banks once.
// --------------------------------------------------------------------------
template <int V>
__device__ __forceinline__ int swz(int r)
{
    return (r ^ (r / V)) & 7;
}

template <int V>
__device__ __forceinline__ int lds_off(int row, int byte_in_row)
{
    const int chunk = byte_in_row >> 4;
    return row * 128 + (((chunk & ~7) | ((chunk ^ swz<V>(row)) & 7)) << 4) + (byte_in_row & 15);
}

// Round FP32 to bf16, nearest-even (hardware conversion on gfx950).
__device__ __forceinline__ u32 bf16_bits(float x)
{
    __bf16 h = (__bf16)x;
    return (u32)__builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float bf16_val(u32 b)
{
    return __builtin_bit_cast(float, b << 16);
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// The P bf16 pieces of the pair (x0, x1), round-to-nearest-even at each step
// (the same values as bf16_bits / bf16_val one at a time): piece p of x0 in
// the low half of out[p], of x1 in the high half.  Both values convert in
// one instruction (v_cvt_pk_bf16_f32), and the pieces come back to FP32 as
// a shift and a mask of the packed word.
template <int P>
__device__ __forceinline__ void split_pair(float x0, float x1, u32 (&out)[P])
{
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const f32x2_t v = {x0, x1};
        const u32 h = __builtin_bit_cast(u32, __builtin_convertvector(v, bf16x2_t));
        out[p] = h;
        if (p + 1 < P) {
            x0 -= __builtin_bit_cast(float, h << 16);
            x1 -= __builtin_bit_cast(float, h & 0xFFFF0000u);
        }
    }
}

} // namespace mg
