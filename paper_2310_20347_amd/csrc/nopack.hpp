// Packing configurations (section 5.3's packing and its elimination; the
// experiment of section 8.6 with A packed, B packed, both or neither).
//
// An operand that is not packed skips the LDS panel: each wave loads its own
// MFMA fragments straight from global memory into registers, 16 bytes per
// lane per fragment (32 for FP8), one stage ahead of the MFMAs that use them.
// That needs the operand contiguous along k (A 'N', B 'T'; the fragment of a
// lane is then one aligned vector) and costs reuse: each fragment is loaded
// by every wave that multiplies it instead of once per workgroup.  A packed
// operand goes through the direct-staged LDS panel of direct.hpp.  With
// neither operand packed there is no LDS and no barrier: the waves of a
// workgroup run independently.
#pragma once

#include "direct.hpp"

namespace mg {

// Fragments of F 16-row blocks x NCH chunks of one stage of a k-contiguous
// operand, loaded from global memory.  Block b's rows start at row0 + 16*b;
// rows at or past R and k at or past K read as zero.
template <class DT, int F, int NCH>
struct GFrags {
    u32 v[F][NCH][1][DT::FDW];

    __device__ __forceinline__ void load(const char *X, int64_t ld, int row0, int R, int k0, int K,
                                         int lane)
    {
        constexpr int GES = DT::GES, VE = DT::KF / 4;   // elements per lane per chunk
        const int r = lane & 15, g = lane >> 4;
#pragma unroll
        for (int b = 0; b < F; ++b) {
            const int row = row0 + 16 * b + r;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int k = k0 + c * DT::KF + g * VE;
                const char *p = (row < R && k < K) ? X + ((int64_t)row * ld + k) * GES
                                                   : (const char *)g_zero_vec;
#pragma unroll
                for (int h = 0; h < DT::FDW / 4; ++h) {
                    const u32x4 w = *(const u32x4 *)(p + 16 * h);
#pragma unroll
                    for (int d = 0; d < 4; ++d) v[b][c][0][4 * h + d] = w[d];
                }
            }
        }
    }

    // Zero the elements at k >= K (the stage that holds the end of k, with a
    // lane's vector straddling K: its tail was read whole).
    __device__ __forceinline__ void mask_tail(int k0, int K, int lane)
    {
        constexpr int GES = DT::GES, VE = DT::KF / 4, EPD = 4 / GES;   // elements per dword
        const int g = lane >> 4;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int valid = K - (k0 + c * DT::KF + g * VE);   // elements of this lane in range
#pragma unroll
            for (int d = 0; d < DT::FDW; ++d) {
                const int nb = (valid - d * EPD) * GES;   // bytes of dword d to keep
                const u32 mask = nb >= 4 ? 0xFFFFFFFFu : (nb <= 0 ? 0u : (1u << (8 * nb)) - 1u);
#pragma unroll
                for (int b = 0; b < F; ++b) v[b][c][0][d] &= mask;
            }
        }
    }
};

template <class DT, int MC, int NC, int WM, int WN, bool TA, bool TB, bool PKA, bool PKB>
struct UTile {
    static_assert(PKA || !TA, "an unpacked A must be contiguous along k ('N')");
    static_assert(PKB || TB, "an unpacked B must be contiguous along k ('T')");
    static_assert(DT::LES == DT::GES && DT::PLANES == 1, "the input format is the MFMA's");
    static constexpr int NW = WM * WN, NT = 64 * NW;
    static constexpr int KC = 128 / DT::GES;
    static constexpr int WTM = MC / WM, WTN = NC / WN;
    static constexpr int FM = WTM / 16, FN = WTN / 16;
    static constexpr int NCH = KC / DT::KF;
    static constexpr int NS = 2;
    static constexpr int PANEL_A = PKA ? MC * 128 : 0, PANEL_B = PKB ? NC * 128 : 0;
    static constexpr int STAGE_BYTES = PANEL_A + PANEL_B;
    static constexpr int LDS_BYTES = STAGE_BYTES > 0 ? NS * STAGE_BYTES : 16;
    static constexpr int MINB = 1;
    typedef DPanel<DT, MC, NW, !TA> PA;
    typedef DPanel<DT, NC, NW, TB> PB;
    typedef typename AccOf<DT>::type Acc;

    static __device__ __forceinline__ void compute(const char *buf, Acc (*acc)[FN], int wm, int wn,
                                                   int lane, const GFrags<DT, FM, NCH> &ga,
                                                   const GFrags<DT, FN, NCH> &gb)
    {
        const char *pa = buf, *pb = buf + PANEL_A;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            u32 fa[FM][1][DT::FDW], fb[FN][1][DT::FDW];
            if constexpr (PKA) {
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    if constexpr (!TA) read_frag_k<DT, 128>(pa, wm * WTM + 16 * i, c, lane, fa[i]);
                    else read_frag_tr<DT, MC>(pa, wm * WTM + 16 * i, c, lane, fa[i]);
                }
            }
            if constexpr (PKB) {
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if constexpr (TB) read_frag_k<DT, 128>(pb, wn * WTN + 16 * j, c, lane, fb[j]);
                    else read_frag_tr<DT, NC>(pb, wn * WTN + 16 * j, c, lane, fb[j]);
                }
            }
#pragma unroll
            for (int st = 0; st < Sub<DT>::value; ++st)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        mma_step<DT>(acc[i][j], PKA ? fa[i] : ga.v[i][c], PKB ? fb[j] : gb.v[j][c], st);
        }
    }

    static __device__ __forceinline__ void run(const GemmArgs &p, int tm, int tn, char *lds)
    {
        const int tid = threadIdx.x, lane = tid & 63;
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int wm = wave % WM, wn = wave / WM;
        const int m0 = tm * MC, n0 = tn * NC;

        Acc acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = Acc{0, 0, 0, 0};

        const bool form = p.k > 0 && alpha_nonzero<DT>(p);
        const int nk = form ? (p.k + KC - 1) / KC : 0;
        if (nk > 0) {
            const char *A = (const char *)p.A;
            const char *B = (const char *)p.B;
            PA pa;
            PB pb;
            if constexpr (PKA) pa.init(p.lda, m0, p.m, p.k, wave, lane);
            if constexpr (PKB) pb.init(p.ldb, n0, p.n, p.k, wave, lane);
            const int arow = m0 + wm * WTM, bcol = n0 + wn * WTN;
            // register fragments: set 0 even stages, set 1 odd stages (two
            // named sets: a register array cannot be indexed at run time)
            GFrags<DT, FM, NCH> ga0, ga1;
            GFrags<DT, FN, NCH> gb0, gb1;
            if constexpr (!PKA) ga0.load(A, p.lda, arow, p.m, 0, p.k, lane);
            if constexpr (!PKB) gb0.load(B, p.ldb, bcol, p.n, 0, p.k, lane);
            if constexpr (PKA) pa.issue(A, p.lda, 0, lds, wave);
            if constexpr (PKB) pb.issue(B, p.ldb, 0, lds + PANEL_A, wave);
            const bool ragged = (p.k % (DT::KF / 4)) != 0;
            // stage s from set (cur, buffer cur); stage s+1 loaded into the other set
            auto step = [&](int s, GFrags<DT, FM, NCH> &gac, GFrags<DT, FN, NCH> &gbc,
                            GFrags<DT, FM, NCH> &gan, GFrags<DT, FN, NCH> &gbn, int cur) {
                wait_vm<0>();   // stage s (LDS panels and register fragments) has landed
                if constexpr (STAGE_BYTES > 0) __builtin_amdgcn_s_barrier();
                pin_order();
                char *buf = lds + cur * STAGE_BYTES;
                if (ragged && s == nk - 1) {
                    const int valid_k = p.k - s * KC;
                    if constexpr (PKA && !TA) PA::fix_tail(buf, valid_k, tid, NT);
                    if constexpr (PKB && TB) PB::fix_tail(buf + PANEL_A, valid_k, tid, NT);
                    if constexpr (!PKA) gac.mask_tail(s * KC, p.k, lane);
                    if constexpr (!PKB) gbc.mask_tail(s * KC, p.k, lane);
                    if constexpr (STAGE_BYTES > 0) __syncthreads();
                }
                if (s + 1 < nk) {
                    const int k1 = (s + 1) * KC;
                    if constexpr (!PKA) gan.load(A, p.lda, arow, p.m, k1, p.k, lane);
                    if constexpr (!PKB) gbn.load(B, p.ldb, bcol, p.n, k1, p.k, lane);
                    char *nxt = lds + (cur ^ 1) * STAGE_BYTES;
                    if constexpr (PKA) pa.issue(A, p.lda, k1, nxt, wave);
                    if constexpr (PKB) pb.issue(B, p.ldb, k1, nxt + PANEL_A, wave);
                }
                pin_order();
                compute(buf, acc, wm, wn, lane, gac, gbc);
            };
            for (int s = 0; s < nk; s += 2) {
                step(s, ga0, gb0, ga1, gb1, 0);
                if (s + 1 >= nk) break;
                step(s + 1, ga1, gb1, ga0, gb0, 1);
            }
            wait_vm<0>();
            if constexpr (STAGE_BYTES > 0) __builtin_amdgcn_s_barrier();
        }
        store_c<DT, FM, FN>(p, acc, m0 + wm * WTM, n0 + wn * WTN, lane);
    }
};

// One workgroup per tile.
template <class T>
__global__ void __launch_bounds__(T::NT, T::MINB) gemm_nopack_kernel(GemmArgs p)
{
    __shared__ __attribute__((aligned(16))) char lds[T::LDS_BYTES];
    const int nblocks = p.tiles_m * p.tiles_n;
    const int t = xcd_remap(blockIdx.x, nblocks);
    int tm, tn;
    raster(t, p.tiles_m, p.tiles_n, p.order, p.group, tm, tn);
    T::run(p, tm, tn, lds);
}

}  // namespace mg
