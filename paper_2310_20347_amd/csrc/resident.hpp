// The other members of the paper's family (section 3.2, Figure "B3C2A0 and
// A3C2B0 algorithms", and the two C3 variants of section 7.2) with the
// micro-kernels of section 4.2, where an A or a B micro-tile stays in
// registers and the L6 loop walks the C block:
//
//   kind 1  B3C2A0: packed Bc in LDS, C block Cc in LDS ("C2"), an A
//           micro-tile resident in registers; L6 runs over the column blocks
//           of Cc, each step a (16 x kf) x (kf x 16) MFMA that reads and
//           writes one 16x16 block of Cc.
//   kind 2  A3C2B0: packed Ac in LDS, Cc in LDS, a B micro-tile resident;
//           L6 runs over the row blocks of Cc.
//   kind 3  C3A2B0: packed Ac in LDS, the C block kept in global memory
//           ("C3": the outermost cache level, L2 on the GPU) for the whole k
//           loop, a B micro-tile resident.
//   kind 4  C3B2A0: packed Bc in LDS, C block in global memory, an A
//           micro-tile resident.
//
// The resident micro-tile is read straight from global memory (unpacked, as
// in the paper's figures).  The running sums live in Cc / in C, so every
// MFMA of these kernels reads and writes its accumulator block: the lower
// arithmetic intensity the paper attributes to A/B-resident micro-kernels
// (section 4.3).  Each entry of C is summed over the same stages, chunks and
// MFMA sub-steps, in the same order, as in the C-resident tile, so all family
// members produce identical bits.
#pragma once

#include <type_traits>

#include "tile.hpp"

namespace mg {

// Resident fragment of one lane: the KF/4 values of k starting at k0 of one
// row (A) or column (B) `r`, zero outside R x K.  KMODE: contiguous along k.
template <class DT, bool KMODE, bool VEC>
__device__ __forceinline__ void load_resident(const char *X, int64_t ld, int r, int R, int k0,
                                              int K, u32 (*f)[DT::FDW])
{
    constexpr int KE = DT::KF / 4;                    // k values per lane
    constexpr int BYTES = KE * DT::GES;               // 16 or 32 bytes in global memory
    u32 raw[BYTES / 4];
#pragma unroll
    for (int d = 0; d < BYTES / 4; ++d) raw[d] = 0u;
    if (r < R && k0 < K) {
        if (KMODE && VEC && k0 + KE <= K) {
            const char *p = X + ((int64_t)r * ld + k0) * DT::GES;
#pragma unroll
            for (int h = 0; h < BYTES / 16; ++h) {
                const u32x4 v = *(const u32x4 *)(p + 16 * h);
#pragma unroll
                for (int d = 0; d < 4; ++d) raw[4 * h + d] = v[d];
            }
        } else {
#pragma unroll
            for (int e = 0; e < KE; ++e) {
                const int k = k0 + e;
                if (k < K) {
                    const char *p = X + (KMODE ? ((int64_t)r * ld + k) : ((int64_t)k * ld + r)) *
                                            DT::GES;
                    if constexpr (DT::GES == 4) {
                        raw[e] = *(const u32 *)p;
                    } else if constexpr (DT::GES == 2) {
                        raw[e / 2] |= (u32)(*(const unsigned short *)p) << (16 * (e % 2));
                    } else {
                        raw[e / 4] |= (u32)(*(const unsigned char *)p) << (8 * (e % 4));
                    }
                }
            }
        }
    }
    if constexpr (DT::SPLIT) {
        // 8 FP32 values -> 8 bf16 per plane
        u32 piece[DT::PLANES][8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float x = __builtin_bit_cast(float, raw[e]);
#pragma unroll
            for (int pl = 0; pl < DT::PLANES; ++pl) {
                const u32 h = bf16_bits(x);
                piece[pl][e] = h;
                x = x - bf16_val(h);
            }
        }
#pragma unroll
        for (int pl = 0; pl < DT::PLANES; ++pl)
#pragma unroll
            for (int q = 0; q < 4; ++q) f[pl][q] = piece[pl][2 * q] | (piece[pl][2 * q + 1] << 16);
    } else {
#pragma unroll
        for (int d = 0; d < DT::FDW; ++d) f[0][d] = raw[d];
    }
}

template <class DT, int MC, int NC, int KIND, bool TA, bool TB, bool VEC>
struct ResidentTile {
    static constexpr bool AR = (KIND == 1 || KIND == 4);   // A micro-tile resident
    static constexpr bool CL = (KIND == 1 || KIND == 2);   // C block in LDS
    static constexpr int NT = 256, NW = 4;
    static constexpr int KC = Kc<DT>::value;
    static constexpr int PROWS = AR ? NC : MC;             // rows of the packed operand
    static constexpr int PLANE = PROWS * 128;
    static constexpr int STAGE_BYTES = DT::PLANES * PLANE;
    static constexpr int CPAD = NC + 4;                    // Cc row stride (floats)
    static constexpr int C_BYTES = CL ? MC * CPAD * 4 : 0;
    static constexpr int LDS_BYTES = STAGE_BYTES + C_BYTES;
    static constexpr int RB = (AR ? MC : NC) / 16 / NW;    // resident blocks per wave
    static constexpr int OB = (AR ? NC : MC) / 16;         // blocks walked by L6
    static_assert(RB >= 1 && (AR ? MC : NC) % (16 * NW) == 0, "resident blocks per wave");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget of one CU");
    typedef typename AccOf<DT>::type Acc;
    typedef typename std::conditional<DT::INT, int, float>::type E;   // element of C
    // the packed operand: B (contiguous along k when 'T') or A (when 'N')
    typedef Stage<DT, PROWS, NT, AR ? TB : !TA, VEC> StageP;

    // 16x16 accumulator block (bi, bj) of the tile: Cc in LDS or C in global.
    static __device__ __forceinline__ void cload(const GemmArgs &p, char *cc, int m0, int n0,
                                                 int bi, int bj, int lane, Acc &acc)
    {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = bi * 16 + 4 * (lane >> 4) + r, col = bj * 16 + (lane & 15);
            if constexpr (CL) {
                acc[r] = ((const E *)cc)[row * CPAD + col];
            } else {
                if (m0 + row < p.m && n0 + col < p.n)
                    acc[r] = ((const E *)p.C)[(int64_t)(m0 + row) * p.ldc + n0 + col];
            }
        }
    }
    static __device__ __forceinline__ void cstore(const GemmArgs &p, char *cc, int m0, int n0,
                                                  int bi, int bj, int lane, const Acc &acc)
    {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = bi * 16 + 4 * (lane >> 4) + r, col = bj * 16 + (lane & 15);
            if constexpr (CL) {
                ((E *)cc)[row * CPAD + col] = acc[r];
            } else {
                if (m0 + row < p.m && n0 + col < p.n)
                    ((E *)p.C)[(int64_t)(m0 + row) * p.ldc + n0 + col] = acc[r];
            }
        }
    }

    static __device__ __forceinline__ void run(const GemmArgs &p, int tm, int tn, char *lds)
    {
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int m0 = tm * MC, n0 = tn * NC;
        char *pk = lds;                      // packed operand stage
        char *cc = lds + STAGE_BYTES;        // Cc (C2 kinds)
        // accumulator block of (resident block rb, walked block ob)
        auto bi_of = [&](int rb, int ob) { return AR ? wave * RB + rb : ob; };
        auto bj_of = [&](int rb, int ob) { return AR ? ob : wave * RB + rb; };

        // C_old of the C3 kinds stays in registers while C accumulates
        Acc cold[CL ? 1 : RB][CL ? 1 : OB];
        const bool use_beta = DT::INT ? p.ibeta != 0 : p.beta != 0.0f;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int ob = 0; ob < OB; ++ob) {
                Acc z = Acc{0, 0, 0, 0};
                if constexpr (!CL) {
                    cold[rb][ob] = z;
                    if (use_beta) cload(p, cc, m0, n0, bi_of(rb, ob), bj_of(rb, ob), lane, cold[rb][ob]);
                }
                cstore(p, cc, m0, n0, bi_of(rb, ob), bj_of(rb, ob), lane, z);
            }

        const bool form = p.k > 0 && alpha_nonzero<DT>(p);
        const int nk = form ? (p.k + KC - 1) / KC : 0;
        const char *Pm = (const char *)(AR ? p.B : p.A);
        const int64_t pld = AR ? p.ldb : p.lda;
        const int prow0 = AR ? n0 : m0, pR = AR ? p.n : p.m;
        const char *Rm = (const char *)(AR ? p.A : p.B);
        const int64_t rld = AR ? p.lda : p.ldb;
        const int rrow0 = AR ? m0 : n0, rR = AR ? p.m : p.n;
        constexpr bool RKMODE = AR ? !TA : TB;   // resident operand contiguous along k

        StageP sp;
        const bool fullP = prow0 + PROWS <= pR;
        if (nk > 0) sp.load_any(fullP, Pm, pld, prow0, pR, 0, p.k, tid);
        for (int s = 0; s < nk; ++s) {
            sp.store(pk, PLANE, tid);
            __syncthreads();
            if (s + 1 < nk) sp.load_any(fullP, Pm, pld, prow0, pR, (s + 1) * KC, p.k, tid);
#pragma unroll
            for (int c = 0; c < KC / DT::KF; ++c) {
                u32 res[RB][DT::PLANES][DT::FDW];
                const int k0 = s * KC + c * DT::KF + (lane >> 4) * (DT::KF / 4);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    load_resident<DT, RKMODE, VEC>(Rm, rld, rrow0 + (wave * RB + rb) * 16 + (lane & 15),
                                                   rR, k0, p.k, res[rb]);
                // L6: walk the blocks of the C block along the other dimension
                for (int ob = 0; ob < OB; ++ob) {
                    u32 pf[DT::PLANES][DT::FDW];
                    read_frag<DT>(pk, PLANE, ob * 16, c, lane, pf);
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        Acc acc;
                        cload(p, cc, m0, n0, bi_of(rb, ob), bj_of(rb, ob), lane, acc);
#pragma unroll
                        for (int st = 0; st < Sub<DT>::value; ++st) {
                            if constexpr (AR) mma_step<DT>(acc, res[rb], pf, st);
                            else mma_step<DT>(acc, pf, res[rb], st);
                        }
                        cstore(p, cc, m0, n0, bi_of(rb, ob), bj_of(rb, ob), lane, acc);
                    }
                }
            }
            __syncthreads();
        }

        // unpack: C = alpha * sum + beta * C_old (C not read when beta == 0)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
            for (int ob = 0; ob < OB; ++ob) {
                Acc acc = Acc{0, 0, 0, 0};
                cload(p, cc, m0, n0, bi_of(rb, ob), bj_of(rb, ob), lane, acc);
                const int bi = bi_of(rb, ob), bj = bj_of(rb, ob);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + bi * 16 + 4 * (lane >> 4) + r;
                    const int col = n0 + bj * 16 + (lane & 15);
                    if (row < p.m && col < p.n) {
                        if constexpr (DT::INT) {
                            int *c = (int *)p.C + (int64_t)row * p.ldc + col;
                            const int old = CL ? (p.ibeta != 0 ? *c : 0) : (int)cold[CL ? 0 : rb][CL ? 0 : ob][r];
                            u32 v = (u32)p.ialpha * (u32)acc[r];
                            if (p.ibeta != 0) v += (u32)p.ibeta * (u32)old;
                            *c = (int)v;
                        } else {
                            float *c = (float *)p.C + (int64_t)row * p.ldc + col;
                            float v = p.alpha * acc[r];
                            if (p.beta != 0.0f) {
                                const float old = CL ? *c : cold[CL ? 0 : rb][CL ? 0 : ob][r];
                                v = __builtin_fmaf(p.beta, old, v);
                            }
                            *c = v;
                        }
                    }
                }
            }
    }
};

template <class T>
__global__ void __launch_bounds__(256) gemm_resident_kernel(GemmArgs p)
{
    __shared__ __attribute__((aligned(16))) char lds[T::LDS_BYTES];
    const int nblocks = p.tiles_m * p.tiles_n;
    const int t = xcd_remap(blockIdx.x, nblocks);
    int tm, tn;
    raster(t, p.tiles_m, p.tiles_n, p.order, p.group, tm, tn);
    T::run(p, tm, tn, lds);
}

}  // namespace mg
