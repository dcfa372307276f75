// The C-resident tile kernel: loops L1..L5 of the paper's B3A2C0 / A3B2C0
// algorithms (section 3.1, Figure "Baseline (B3A2C0) and A3B2C0 algorithms")
// with packing (section 5.3) and a register-resident micro-tile (section 4.1),
// mapped onto gfx950:
//
//   L1/L3 (jc, ic)  -> one workgroup per mc x nc tile of C; the raster order of
//                      tile ids picks the variant (B3A2C0: consecutive
//                      workgroups share a column panel of B; A3B2C0: a row
//                      panel of A), with XCD-aware placement;
//   L2 (pc)         -> the k loop over stages of kc values (not parallel);
//   pack Ac, Bc     -> each stage's A and B panels are staged global -> LDS by
//                      the whole workgroup, converted to the MFMA operand
//                      format and laid out k-contiguous per row (the analogue
//                      of the unit-stride micro-panels of the paper's packing
//                      figure); loads for stage s+1 are in flight while stage s
//                      is multiplied (the prefetch of section 6.2);
//   L4/L5 (jr, ir)  -> waves: each owns an (mc/WM) x (nc/WN) micro-tile;
//   L6 micro-kernel -> per kc stage, a chain of MFMA instructions over 16x16
//                      accumulator blocks held in registers for the whole k
//                      loop (section 4.1: rank-kf updates instead of rank-1).
#pragma once

#include "device.hpp"

namespace mg {

// ---------------------------------------------------------------------------
// Tile raster: tile id -> (tile row, tile column) in the variant's loop order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void raster(int t, int tiles_m, int tiles_n, int order, int group,
                                       int &tm, int &tn)
{
    if (order == 0) {  // B3A2C0: column panels (jc) outermost, in groups
        const int per = group * tiles_m;
        const int g = t / per, r = t - g * per;
        const int width = min(group, tiles_n - g * group);
        tn = g * group + r % width;
        tm = r / width;
    } else {           // A3B2C0: row panels (ic) outermost, in groups
        const int per = group * tiles_n;
        const int g = t / per, r = t - g * per;
        const int height = min(group, tiles_m - g * group);
        tm = g * group + r % height;
        tn = r / height;
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b%8).
// Renumber so that each XCD receives a contiguous range of tile ids, i.e.
// neighbouring tiles (which share A/B panels) share one XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nblocks)
{
    const int xcd = b & 7, idx = b >> 3;
    const int base = nblocks >> 3, rem = nblocks & 7;
    return (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + idx;
}

// ---------------------------------------------------------------------------
// Element-wise (masked) loads assembled into a 16-byte register vector.
// ---------------------------------------------------------------------------
template <int GES, int N>
__device__ __forceinline__ u32x4 load_elems(const char *p, int valid)
{
    u32x4 v = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int e = 0; e < N; ++e) {
        if (e < valid) {
            if constexpr (GES == 4) {
                v[e] = ((const u32 *)p)[e];
            } else if constexpr (GES == 2) {
                v[e / 2] |= (u32)((const unsigned short *)p)[e] << (16 * (e % 2));
            } else {
                v[e / 4] |= (u32)((const unsigned char *)p)[e] << (8 * (e % 4));
            }
        }
    }
    return v;
}

// ---------------------------------------------------------------------------
// Staging of one operand panel (ROWS rows of m or n, KC values of k).
//
// KMODE (operand contiguous along k: A 'N', B 'T'): each item is one 16-byte
// global vector along k, copied (or split) into its LDS row.
// MN mode (operand contiguous along m/n: A 'T', B 'N'): each item is a block
// of KV k-rows x MNV elements, loaded as KV vectors along m/n and transposed
// in registers into MNV LDS chunks of 16 bytes along k.
// ---------------------------------------------------------------------------
template <class DT, int ROWS, int NT, bool KMODE, bool VEC>
struct Stage {
    static constexpr int KC = Kc<DT>::value;
    static constexpr int GES = DT::GES;
    // K mode
    static constexpr int VK = 16 / GES;            // elements per 16 B global vector
    static constexpr int VPR = KC / VK;            // vectors per panel row
    static constexpr int NVEC = ROWS * VPR;
    // MN mode
    static constexpr int KV = 16 / DT::LES;        // k rows per block = one LDS chunk
    static constexpr int MNV = DT::MNV;            // m/n elements per global vector
    static constexpr int GVB = MNV * GES;          // bytes per global vector
    static constexpr int MB = ROWS / MNV;
    static constexpr int NBLK = (KC / KV) * MB;

    static constexpr int ITEMS = KMODE ? NVEC : NBLK;
    static constexpr int PER = (ITEMS + NT - 1) / NT;   // items per thread
    static constexpr int DW = KMODE ? 4 : (KV * GVB) / 4;  // dwords per item
    static_assert(ROWS % MNV == 0, "panel rows must be a multiple of the vector width");

    u32 reg[PER][DW];

    // A full interior stage (all ROWS rows and all KC columns of the stage in
    // bounds, vectorisable operand): plain vector loads, no checks, no
    // branches, so the loads can be scheduled among the MFMAs.
    __device__ __forceinline__ void load_fast(const char *X, int64_t ld, int row0, int k0,
                                              int tid)
    {
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const int item = tid + it * NT;
            if (ITEMS % NT != 0 && item >= ITEMS) break;
            if constexpr (KMODE) {
                const int row = item / VPR, kv = item % VPR;
                const u32x4 v =
                    *(const u32x4 *)(X + ((int64_t)(row0 + row) * ld + k0 + kv * VK) * GES);
#pragma unroll
                for (int d = 0; d < 4; ++d) reg[it][d] = v[d];
            } else {
                const int mb = item % MB, kb = item / MB;
                const char *p = X + ((int64_t)(k0 + kb * KV) * ld + row0 + mb * MNV) * GES;
                const int64_t step = ld * GES;
#pragma unroll
                for (int r = 0; r < KV; ++r) {
                    const char *q = p + r * step;
                    if constexpr (GVB == 16) {
                        const u32x4 v = *(const u32x4 *)q;
#pragma unroll
                        for (int d = 0; d < 4; ++d) reg[it][r * 4 + d] = v[d];
                    } else if constexpr (GVB == 8) {
                        const u32x2 v = *(const u32x2 *)q;
                        reg[it][r * 2 + 0] = v[0];
                        reg[it][r * 2 + 1] = v[1];
                    } else {
                        reg[it][r] = *(const u32 *)q;
                    }
                }
            }
        }
    }

    // Stage starting at k0: the fast path when `full` (rows and k in bounds)
    // and the operand is vectorisable, the checked path otherwise.
    __device__ __forceinline__ void load_any(bool full, const char *X, int64_t ld, int row0, int R,
                                             int k0, int K, int tid)
    {
        if (VEC && full && k0 + KC <= K)
            load_fast(X, ld, row0, k0, tid);
        else
            load(X, ld, row0, R, k0, K, tid);
    }

    // Load stage starting at k0 from the operand X (row stride ld elements),
    // whose panel starts at row0; R rows and K columns are valid.
    __device__ __forceinline__ void load(const char *X, int64_t ld, int row0, int R, int k0,
                                         int K, int tid)
    {
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const int item = tid + it * NT;
            if (ITEMS % NT != 0 && item >= ITEMS) break;
            if constexpr (KMODE) {
                const int row = item / VPR, kv = item % VPR;
                const int grow = row0 + row, gk = k0 + kv * VK;
                u32x4 v = {0u, 0u, 0u, 0u};
                if (grow < R && gk < K) {
                    const char *p = X + ((int64_t)grow * ld + gk) * GES;
                    if (VEC && gk + VK <= K)
                        v = *(const u32x4 *)p;
                    else
                        v = load_elems<GES, VK>(p, K - gk);
                }
#pragma unroll
                for (int d = 0; d < 4; ++d) reg[it][d] = v[d];
            } else {
                const int mb = item % MB, kb = item / MB;
                const int gmn = row0 + mb * MNV, gk0 = k0 + kb * KV;
#pragma unroll
                for (int r = 0; r < KV; ++r) {
                    const int gk = gk0 + r;
                    u32x4 v = {0u, 0u, 0u, 0u};
                    if (gk < K && gmn < R) {
                        const char *p = X + ((int64_t)gk * ld + gmn) * GES;
                        if (VEC && gmn + MNV <= R) {
                            if constexpr (GVB == 16) {
                                v = *(const u32x4 *)p;
                            } else if constexpr (GVB == 8) {
                                const u32x2 w = *(const u32x2 *)p;
                                v[0] = w[0];
                                v[1] = w[1];
                            } else {
                                v[0] = *(const u32 *)p;
                            }
                        } else {
                            v = load_elems<GES, MNV>(p, R - gmn);
                        }
                    }
#pragma unroll
                    for (int d = 0; d < GVB / 4; ++d) reg[it][r * (GVB / 4) + d] = v[d];
                }
            }
        }
    }

    // Write the loaded stage into LDS: `planes` points at plane 0 of this
    // operand's panel; consecutive planes are plane_bytes apart.
    __device__ __forceinline__ void store(char *planes, int plane_bytes, int tid) const
    {
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const int item = tid + it * NT;
            if (ITEMS % NT != 0 && item >= ITEMS) break;
            if constexpr (KMODE) {
                const int row = item / VPR, kv = item % VPR;
                if constexpr (!DT::SPLIT) {
                    u32x4 v = {reg[it][0], reg[it][1], reg[it][2], reg[it][3]};
                    *(u32x4 *)(planes + lds_off<MNV>(row, kv * 16)) = v;
                } else {
                    // 4 FP32 values -> 4 bf16 per plane (8 bytes per plane)
                    u32 piece[DT::PLANES][4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        float x = __builtin_bit_cast(float, reg[it][e]);
#pragma unroll
                        for (int pl = 0; pl < DT::PLANES; ++pl) {
                            const u32 h = bf16_bits(x);
                            piece[pl][e] = h;
                            x = x - bf16_val(h);
                        }
                    }
#pragma unroll
                    for (int pl = 0; pl < DT::PLANES; ++pl) {
                        u32x2 w = {piece[pl][0] | (piece[pl][1] << 16),
                                   piece[pl][2] | (piece[pl][3] << 16)};
                        *(u32x2 *)(planes + pl * plane_bytes + lds_off<MNV>(row, kv * 8)) = w;
                    }
                }
            } else {
                const int mb = item % MB, kb = item / MB;
#pragma unroll
                for (int e = 0; e < MNV; ++e) {
                    const int row = mb * MNV + e;
                    if constexpr (DT::SPLIT) {
                        // KV=8 k-rows of FP32 -> 8 bf16 per plane = one 16 B chunk
                        u32 piece[DT::PLANES][8];
#pragma unroll
                        for (int r = 0; r < 8; ++r) {
                            float x = __builtin_bit_cast(float, reg[it][r * 4 + e]);
#pragma unroll
                            for (int pl = 0; pl < DT::PLANES; ++pl) {
                                const u32 h = bf16_bits(x);
                                piece[pl][r] = h;
                                x = x - bf16_val(h);
                            }
                        }
#pragma unroll
                        for (int pl = 0; pl < DT::PLANES; ++pl) {
                            u32x4 w = {piece[pl][0] | (piece[pl][1] << 16),
                                       piece[pl][2] | (piece[pl][3] << 16),
                                       piece[pl][4] | (piece[pl][5] << 16),
                                       piece[pl][6] | (piece[pl][7] << 16)};
                            *(u32x4 *)(planes + pl * plane_bytes + lds_off<MNV>(row, kb * 16)) = w;
                        }
                    } else if constexpr (GES == 4) {
                        // 4 k-rows x 4 floats: take element e of each row
                        u32x4 w = {reg[it][0 * 4 + e], reg[it][1 * 4 + e], reg[it][2 * 4 + e],
                                   reg[it][3 * 4 + e]};
                        *(u32x4 *)(planes + lds_off<MNV>(row, kb * 16)) = w;
                    } else if constexpr (GES == 2) {
                        // 8 k-rows x MNV halves: half e of each row, paired into dwords
                        const int d = e / 2, sh = 16 * (e % 2);
                        u32 w4[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const u32 lo = (reg[it][(2 * q) * (GVB / 4) + d] >> sh) & 0xFFFFu;
                            const u32 hi = (reg[it][(2 * q + 1) * (GVB / 4) + d] >> sh) & 0xFFFFu;
                            w4[q] = lo | (hi << 16);
                        }
                        u32x4 w = {w4[0], w4[1], w4[2], w4[3]};
                        *(u32x4 *)(planes + lds_off<MNV>(row, kb * 16)) = w;
                    } else {
                        // 16 k-rows x 4 bytes: byte e of each row, four per dword
                        const int sh = 8 * e;
                        u32 w4[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            w4[q] = ((reg[it][4 * q + 0] >> sh) & 0xFFu) |
                                    (((reg[it][4 * q + 1] >> sh) & 0xFFu) << 8) |
                                    (((reg[it][4 * q + 2] >> sh) & 0xFFu) << 16) |
                                    (((reg[it][4 * q + 3] >> sh) & 0xFFu) << 24);
                        }
                        u32x4 w = {w4[0], w4[1], w4[2], w4[3]};
                        *(u32x4 *)(planes + lds_off<MNV>(row, kb * 16)) = w;
                    }
                }
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Scheduling fence: the compiler may not move instructions across it.  It
// keeps a stage's global loads ahead of the MFMA chain they are meant to
// overlap (left alone, the scheduler sinks them next to their LDS stores,
// which exposes the full memory latency once per stage).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pin_order()
{
    __builtin_amdgcn_sched_barrier(0);
}

// ---------------------------------------------------------------------------
// One MFMA of the micro-kernel.  A fragment chunk covers KF values of k: a
// lane of group g = lane/16 holds the k values g*KF/4 .. g*KF/4 + KF/4-1 of
// its row (A) or column (B); A and B use the same k assignment, so every k of
// the chunk is summed exactly once.  A chunk takes SUB MFMAs per 16x16 block:
// the four k=4 steps of the FP32 instruction, or the piece products of the
// split path, or one instruction otherwise.  Sub-step s of every block is
// issued before sub-step s+1 of any block, so consecutive MFMAs write
// different accumulators; each block still sums its sub-steps in order.
// ---------------------------------------------------------------------------
template <class DT>
struct Sub {
    static constexpr int value =
        DT::SPLIT ? (DT::PLANES == 2 ? 3 : 6) : (DT::GES == 4 ? 4 : (DT::GES == 8 ? 2 : 1));
};

template <class DT>
__device__ __forceinline__ void mma_step(typename AccOf<DT>::type &acc, const u32 (*a)[DT::FDW],
                                         const u32 (*b)[DT::FDW], int s)
{
    if constexpr (DT::SPLIT) {
        // piece products, smallest first; planes: 0 = hi, 1 = mid, 2 = lo
        // three terms: mid*hi, hi*mid, hi*hi; six terms: lo*hi, hi*lo, mid*mid, then those
        constexpr int P = DT::PLANES;
        constexpr int TU[6] = {P == 2 ? 1 : 2, 0, P == 2 ? 0 : 1, 1, 0, 0};
        constexpr int TV[6] = {0, P == 2 ? 1 : 2, P == 2 ? 0 : 1, 0, 1, 0};
        const u32 *x = a[TU[s]], *y = b[TV[s]];
        u32x4 xv = {x[0], x[1], x[2], x[3]}, yv = {y[0], y[1], y[2], y[3]};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, xv),
                                                      __builtin_bit_cast(bf16x8, yv), acc, 0, 0, 0);
    } else if constexpr (DT::GES == 8) {  // FP64: k step s of two
        const u64 x = ((u64)a[0][2 * s + 1] << 32) | a[0][2 * s];
        const u64 y = ((u64)b[0][2 * s + 1] << 32) | b[0][2 * s];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(__builtin_bit_cast(double, x),
                                                   __builtin_bit_cast(double, y), acc, 0, 0, 0);
    } else if constexpr (DT::GES == 4) {  // plain FP32: k step s of four
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__builtin_bit_cast(float, a[0][s]),
                                                  __builtin_bit_cast(float, b[0][s]), acc, 0, 0, 0);
    } else if constexpr (DT::GES == 2) {
        u32x4 xv = {a[0][0], a[0][1], a[0][2], a[0][3]}, yv = {b[0][0], b[0][1], b[0][2], b[0][3]};
        if constexpr (DT::HALF)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, xv),
                                                         __builtin_bit_cast(f16x8, yv), acc, 0, 0, 0);
        else
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, xv),
                                                          __builtin_bit_cast(bf16x8, yv), acc, 0, 0, 0);
    } else if constexpr (DT::INT) {
        i32x4 xv = {(int)a[0][0], (int)a[0][1], (int)a[0][2], (int)a[0][3]};
        i32x4 yv = {(int)b[0][0], (int)b[0][1], (int)b[0][2], (int)b[0][3]};
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(xv, yv, acc, 0, 0, 0);
    } else {  // FP8 e4m3 (format code 0 for both operands), unit E8M0 scales (127)
        i32x8 xv, yv;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            xv[d] = (int)a[0][d];
            yv[d] = (int)b[0][d];
        }
        acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(xv, yv, acc, 0, 0, 0, 127, 0, 127);
    }
}

// Read one MFMA operand fragment (all planes) of the 16-row block at `row`.
template <class DT>
__device__ __forceinline__ void read_frag(const char *planes, int plane_bytes, int row, int chunk,
                                          int lane, u32 (*f)[DT::FDW])
{
    const int r = row + (lane & 15);
    const int byte = chunk * (DT::KF * DT::LES) + (lane >> 4) * (DT::FDW * 4);
#pragma unroll
    for (int pl = 0; pl < DT::PLANES; ++pl) {
#pragma unroll
        for (int h = 0; h < DT::FDW / 4; ++h) {
            const u32x4 v =
                *(const u32x4 *)(planes + pl * plane_bytes + lds_off<DT::MNV>(r, byte + 16 * h));
#pragma unroll
            for (int d = 0; d < 4; ++d) f[pl][4 * h + d] = v[d];
        }
    }
}

// ---------------------------------------------------------------------------
// Epilogue of a wave's FM x FN accumulator blocks whose top-left corner is
// (r0, c0): C = alpha * acc + beta * C (C not read when beta == 0; INT8
// wraps modulo 2^32).  Accumulator layout: lane l, register r -> row
// 4*(l/16)+r (FP64: l/16+4r), column l%16 of the block.
// ---------------------------------------------------------------------------
template <class DT, int FM, int FN>
__device__ __forceinline__ void store_c(const GemmArgs &p, const typename AccOf<DT>::type (*acc)[FN],
                                        int r0, int c0, int lane)
{
    const int rbase = r0 + 4 * (lane >> 4);
    const int cbase = c0 + (lane & 15);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // the FP64 MFMA interleaves its rows: register r of lane l is
                // row l/16 + 4r (measured with identity operands)
                const int row = DT::GES == 8 ? r0 + 16 * i + (lane >> 4) + 4 * r : rbase + 16 * i + r;
                const int col = cbase + 16 * j;
                if (row < p.m && col < p.n) {
                    if constexpr (DT::INT) {
                        int *c = (int *)p.C + (int64_t)row * p.ldc + col;
                        u32 v = (u32)p.ialpha * (u32)acc[i][j][r];
                        if (p.ibeta != 0) v += (u32)p.ibeta * (u32)(*c);
                        *c = (int)v;
                    } else if constexpr (DT::GES == 8) {
                        double *c = (double *)p.C + (int64_t)row * p.ldc + col;
                        double v = p.dalpha * acc[i][j][r];
                        if (p.dbeta != 0.0) v = __builtin_fma(p.dbeta, *c, v);
                        *c = v;
                    } else {
                        float *c = (float *)p.C + (int64_t)row * p.ldc + col;
                        float v = p.alpha * acc[i][j][r];
                        if (p.beta != 0.0f) v = __builtin_fmaf(p.beta, *c, v);
                        *c = v;
                    }
                }
            }
}

// The same epilogue with each row block's C values read before any of them
// is written, so with beta != 0 the loads issue together (a store to C must
// otherwise complete before the next load of C: the two may alias).  Twice
// the code of store_c: used by the large single-GEMM tiles, where beta = 1
// costs 2% of an 8192^3 FP32 product with store_c; in the grouped kernels
// the larger code made every launch slower.
template <class DT, int FM, int FN>
__device__ __forceinline__ void store_c_batched(const GemmArgs &p, const typename AccOf<DT>::type (*acc)[FN],
                                        int r0, int c0, int lane)
{
    typedef typename std::conditional<DT::INT, int, typename std::conditional<DT::GES == 8, double, float>::type>::type CT;
    const int rbase = r0 + 4 * (lane >> 4);
    const int cbase = c0 + (lane & 15);
    const bool read_c = DT::INT ? p.ibeta != 0 : (DT::GES == 8 ? p.dbeta != 0.0 : p.beta != 0.0f);
    CT *const C = (CT *)p.C;
    // the FP64 MFMA interleaves its rows: register r of lane l is row
    // l/16 + 4r (measured with identity operands)
    auto row_of = [&](int i, int r) { return DT::GES == 8 ? r0 + 16 * i + (lane >> 4) + 4 * r : rbase + 16 * i + r; };
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        // this row block's C values are all read before any is written, so
        // the loads issue together (a store to C must otherwise complete
        // before the next load of C: the two may alias)
        CT cv[FN][4];
        if (read_c) {
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = row_of(i, r), col = cbase + 16 * j;
                    cv[j][r] = row < p.m && col < p.n ? C[(int64_t)row * p.ldc + col] : CT(0);
                }
        }
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row_of(i, r), col = cbase + 16 * j;
                if (row < p.m && col < p.n) {
                    CT *c = C + (int64_t)row * p.ldc + col;
                    if constexpr (DT::INT) {
                        u32 v = (u32)p.ialpha * (u32)acc[i][j][r];
                        if (read_c) v += (u32)p.ibeta * (u32)cv[j][r];
                        *c = (int)v;
                    } else if constexpr (DT::GES == 8) {
                        double v = p.dalpha * acc[i][j][r];
                        if (read_c) v = __builtin_fma(p.dbeta, cv[j][r], v);
                        *c = v;
                    } else {
                        float v = p.alpha * acc[i][j][r];
                        if (read_c) v = __builtin_fmaf(p.beta, cv[j][r], v);
                        *c = v;
                    }
                }
            }
    }
}

// ---------------------------------------------------------------------------
// The tile: C[m0:m0+MC, n0:n0+NC] = alpha * op(A) op(B) + beta * C.
// ---------------------------------------------------------------------------
// STAGES: LDS buffers (1 or 2).  PF: stages of global loads in flight in
// registers (1, or 2 with two LDS buffers: the loads of stage s+2 are issued
// while stage s is multiplied, so they have two stages of MFMA work to land).
// PEEL: interior tiles run their full stages in a separate loop with
// unchecked loads held ahead of the MFMA chain by scheduling fences (more
// registers live across the chain; off where that costs occupancy).
template <class DT, int MC, int NC, int WM, int WN, bool TA, bool TB, bool VEC, int STAGES,
          int PF = 1, bool PEEL = true>
struct Tile {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int KC = Kc<DT>::value;
    static constexpr int WTM = MC / WM, WTN = NC / WN;   // wave micro-tile (mr x nr)
    static constexpr int FM = WTM / 16, FN = WTN / 16;   // 16x16 MFMA blocks per wave
    static constexpr int PLANE_A = MC * 128, PLANE_B = NC * 128;
    static constexpr int STAGE_BYTES = DT::PLANES * (PLANE_A + PLANE_B);
    static constexpr int LDS_BYTES = STAGES * STAGE_BYTES;
    static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile must be whole MFMA blocks");
    static_assert(STAGES == 1 || STAGES == 2, "one or two LDS stages");
    static_assert(PF == 1 || (PF == 2 && STAGES == 2), "two stages in flight need two LDS buffers");
    static constexpr int MINB = 1;   // workgroups per CU the registers must allow
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget of one CU");
    typedef typename AccOf<DT>::type Acc;
    typedef Stage<DT, MC, NT, !TA, VEC> StageA;   // A 'N' is contiguous along k
    typedef Stage<DT, NC, NT, TB, VEC> StageB;    // B 'T' is contiguous along k

    static __device__ __forceinline__ void compute(const char *buf, Acc (*acc)[FN], int wm,
                                                   int wn, int lane)
    {
        const char *pa = buf;
        const char *pb = buf + DT::PLANES * PLANE_A;
#pragma unroll
        for (int c = 0; c < KC / DT::KF; ++c) {
            u32 fa[FM][DT::PLANES][DT::FDW];
            u32 fb[FN][DT::PLANES][DT::FDW];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                read_frag<DT>(pa, PLANE_A, wm * WTM + 16 * i, c, lane, fa[i]);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                read_frag<DT>(pb, PLANE_B, wn * WTN + 16 * j, c, lane, fb[j]);
#pragma unroll
            for (int st = 0; st < Sub<DT>::value; ++st)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) mma_step<DT>(acc[i][j], fa[i], fb[j], st);
        }
    }

    // Computes tile (tm, tn) of problem p using `lds` (LDS_BYTES bytes).
    static __device__ __forceinline__ void run(const GemmArgs &p, int tm, int tn, char *lds)
    {
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int wm = wave % WM, wn = wave / WM;
        const int m0 = tm * MC, n0 = tn * NC;

        Acc acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = Acc{0, 0, 0, 0};

        const bool form = p.k > 0 && alpha_nonzero<DT>(p);
        const int nk = form ? (p.k + KC - 1) / KC : 0;
        const char *A = (const char *)p.A;
        const char *B = (const char *)p.B;

        StageA sa;
        StageB sb;
        const bool fullA = m0 + MC <= p.m, fullB = n0 + NC <= p.n;   // panel rows in bounds
        // Stages [0, kfull) of an interior tile take the unchecked vector
        // loads; the main loops below run only those, with no branch between
        // load variants, so each loaded register flows straight to its LDS
        // store and the loads stay in flight across the MFMA chain.  The
        // remaining (partial or edge) stages run the checked loop.
        const int kfull = (PEEL && VEC && fullA && fullB) ? p.k / KC : 0;
        if (nk > 0) {
            sa.load_any(fullA, A, p.lda, m0, p.m, 0, p.k, tid);
            sb.load_any(fullB, B, p.ldb, n0, p.n, 0, p.k, tid);
        }
        int s = 0;
        if constexpr (STAGES == 2 && PF == 2) {
            // registers: set 0 holds even stages, set 1 odd stages
            StageA sa1;
            StageB sb1;
            if (nk > 1) {
                sa1.load_any(fullA, A, p.lda, m0, p.m, KC, p.k, tid);
                sb1.load_any(fullB, B, p.ldb, n0, p.n, KC, p.k, tid);
            }
            char *buf0 = lds, *buf1 = lds + STAGE_BYTES;
            if (nk > 0) {
                sa.store(buf0, PLANE_A, tid);
                sb.store(buf0 + DT::PLANES * PLANE_A, PLANE_B, tid);
            }
            __syncthreads();
            // even stage s is in buf0, stage s+1 in register set 1
            for (; s + 3 < kfull; s += 2) {
                sa.load_fast(A, p.lda, m0, (s + 2) * KC, tid);
                sb.load_fast(B, p.ldb, n0, (s + 2) * KC, tid);
                compute(buf0, acc, wm, wn, lane);
                sa1.store(buf1, PLANE_A, tid);
                sb1.store(buf1 + DT::PLANES * PLANE_A, PLANE_B, tid);
                __syncthreads();
                sa1.load_fast(A, p.lda, m0, (s + 3) * KC, tid);
                sb1.load_fast(B, p.ldb, n0, (s + 3) * KC, tid);
                compute(buf1, acc, wm, wn, lane);
                sa.store(buf0, PLANE_A, tid);
                sb.store(buf0 + DT::PLANES * PLANE_A, PLANE_B, tid);
                __syncthreads();
            }
            for (; s < nk; s += 2) {
                if (s + 2 < nk) {
                    sa.load_any(fullA, A, p.lda, m0, p.m, (s + 2) * KC, p.k, tid);
                    sb.load_any(fullB, B, p.ldb, n0, p.n, (s + 2) * KC, p.k, tid);
                }
                compute(buf0, acc, wm, wn, lane);
                if (s + 1 < nk) {
                    sa1.store(buf1, PLANE_A, tid);
                    sb1.store(buf1 + DT::PLANES * PLANE_A, PLANE_B, tid);
                }
                __syncthreads();
                if (s + 1 >= nk) break;
                // odd stage s+1 is in buf1, stage s+2 in register set 0
                if (s + 3 < nk) {
                    sa1.load_any(fullA, A, p.lda, m0, p.m, (s + 3) * KC, p.k, tid);
                    sb1.load_any(fullB, B, p.ldb, n0, p.n, (s + 3) * KC, p.k, tid);
                }
                compute(buf1, acc, wm, wn, lane);
                if (s + 2 < nk) {
                    sa.store(buf0, PLANE_A, tid);
                    sb.store(buf0 + DT::PLANES * PLANE_A, PLANE_B, tid);
                }
                __syncthreads();
            }
        } else if constexpr (STAGES == 2) {
            if (nk > 0) {
                sa.store(lds, PLANE_A, tid);
                sb.store(lds + DT::PLANES * PLANE_A, PLANE_B, tid);
            }
            __syncthreads();
            for (; s + 1 < kfull; ++s) {
                char *cur = lds + (s & 1) * STAGE_BYTES;
                char *nxt = lds + ((s + 1) & 1) * STAGE_BYTES;
                sa.load_fast(A, p.lda, m0, (s + 1) * KC, tid);
                sb.load_fast(B, p.ldb, n0, (s + 1) * KC, tid);
                pin_order();
                compute(cur, acc, wm, wn, lane);
                pin_order();
                sa.store(nxt, PLANE_A, tid);
                sb.store(nxt + DT::PLANES * PLANE_A, PLANE_B, tid);
                __syncthreads();
            }
            for (; s < nk; ++s) {
                char *cur = lds + (s & 1) * STAGE_BYTES;
                char *nxt = lds + ((s + 1) & 1) * STAGE_BYTES;
                if (s + 1 < nk) {
                    sa.load_any(fullA, A, p.lda, m0, p.m, (s + 1) * KC, p.k, tid);
                    sb.load_any(fullB, B, p.ldb, n0, p.n, (s + 1) * KC, p.k, tid);
                }
                compute(cur, acc, wm, wn, lane);
                if (s + 1 < nk) {
                    sa.store(nxt, PLANE_A, tid);
                    sb.store(nxt + DT::PLANES * PLANE_A, PLANE_B, tid);
                }
                __syncthreads();
            }
        } else {
            for (; s + 1 < kfull; ++s) {
                sa.store(lds, PLANE_A, tid);
                sb.store(lds + DT::PLANES * PLANE_A, PLANE_B, tid);
                __syncthreads();
                sa.load_fast(A, p.lda, m0, (s + 1) * KC, tid);
                sb.load_fast(B, p.ldb, n0, (s + 1) * KC, tid);
                compute(lds, acc, wm, wn, lane);
                __syncthreads();
            }
            for (; s < nk; ++s) {
                sa.store(lds, PLANE_A, tid);
                sb.store(lds + DT::PLANES * PLANE_A, PLANE_B, tid);
                __syncthreads();
                if (s + 1 < nk) {
                    sa.load_any(fullA, A, p.lda, m0, p.m, (s + 1) * KC, p.k, tid);
                    sb.load_any(fullB, B, p.ldb, n0, p.n, (s + 1) * KC, p.k, tid);
                }
                compute(lds, acc, wm, wn, lane);
                __syncthreads();
            }
        }

        store_c<DT, FM, FN>(p, acc, m0 + wm * WTM, n0 + wn * WTN, lane);
    }
};

// Split-K: workgroup b computes tile b % tiles over k slice b / tiles
// (kslice values of k, a multiple of the stage depth so that operand
// pointers keep their alignment) and writes the partial tile, unscaled, to
// slice's m x n block of the workspace P; a separate reduction adds the
// slices in order (the paper's "pc cannot be parallelised" race resolved by
// an explicit, deterministic reduction).
template <class T, int GES, bool TA, bool TB>
__device__ __forceinline__ void run_slice(const GemmArgs &p, int kslice, void *P, char *lds)
{
    const int nblocks = p.tiles_m * p.tiles_n;
    const int b = (int)blockIdx.x;
    const int slice = b / nblocks;
    const int t = xcd_remap(b - slice * nblocks, nblocks);
    int tm, tn;
    raster(t, p.tiles_m, p.tiles_n, p.order, p.group, tm, tn);
    const int k0 = slice * kslice;
    GemmArgs q = p;
    q.k = min(kslice, p.k - k0);
    q.A = (const char *)p.A + (TA ? (int64_t)k0 * p.lda : (int64_t)k0) * GES;
    q.B = (const char *)p.B + (TB ? (int64_t)k0 : (int64_t)k0 * p.ldb) * GES;
    q.C = (char *)P + (int64_t)slice * p.m * p.n * 4;
    q.ldc = p.n;
    q.alpha = 1.0f;
    q.beta = 0.0f;
    q.ialpha = 1;
    q.ibeta = 0;
    T::run(q, tm, tn, lds);
}

template <class T, int GES, bool TA, bool TB>
__global__ void __launch_bounds__(T::NT, T::MINB) gemm_splitk_kernel(GemmArgs p, int kslice, void *P)
{
    __shared__ __attribute__((aligned(16))) char lds[T::LDS_BYTES];
    run_slice<T, GES, TA, TB>(p, kslice, P, lds);
}

// One workgroup per tile.
template <class T>
__global__ void __launch_bounds__(T::NT, T::MINB) gemm_tile_kernel(GemmArgs p)
{
    __shared__ __attribute__((aligned(16))) char lds[T::LDS_BYTES];
    const int nblocks = p.tiles_m * p.tiles_n;
    const int t = xcd_remap(blockIdx.x, nblocks);
    int tm, tn;
    raster(t, p.tiles_m, p.tiles_n, p.order, p.group, tm, tn);
    T::run(p, tm, tn, lds);
}

}  // namespace mg
