// The fused split product on direct-staged FP32 panels: A and B go from
// global memory to LDS unchanged (direct loads, a ring of stages), and each
// wave splits the FP32 values of its MFMA fragments into bf16 pieces as it
// reads them.  Same pieces, same MFMA order per 32-value block of k as the
// register-staged split tile and the packed split (hence the same bits), with
// no staging registers, no LDS stores and two workgroups per CU at 128x128.
#pragma once

#include "direct.hpp"

namespace mg {

template <int P, int MC, int NC, int WM, int WN, bool TA, bool TB, int NS>
struct SDTile {
    typedef TSplit<P> DT;                     // MFMA side: bf16 pieces, k = 32 per fragment
    static constexpr int NW = WM * WN, NT = 64 * NW;
    static constexpr int KC = 32;             // FP32 values of k per stage (128-byte rows)
    static constexpr int WTM = MC / WM, WTN = NC / WN;
    static constexpr int FM = WTM / 16, FN = WTN / 16;
    static constexpr int PANEL_A = MC * 128, PANEL_B = NC * 128;
    static constexpr int STAGE_BYTES = PANEL_A + PANEL_B;
    static constexpr int LDS_BYTES = NS * STAGE_BYTES;
    static constexpr int MINB = 1;
    typedef DPanel<TF32, MC, NW, !TA, 8> PA;
    typedef DPanel<TF32, NC, NW, TB, 8> PB;
    static constexpr int LOADS = PA::PER + PB::PER;
    static_assert(NS >= 2 && LDS_BYTES <= 160 * 1024, "LDS budget of one CU");
    static_assert((NS - 2) * LOADS < 64, "loads in flight must fit the vmcnt counter");
    typedef f32x4 Acc;

    // The 8 FP32 values k = 8g .. 8g+7 of this stage at row (or column) r.
    template <bool KMODE, int ROWS>
    static __device__ __forceinline__ void read8(const char *panel, int r, int g, float v[8])
    {
        if constexpr (KMODE) {
            const f32x4 x = *(const f32x4 *)(panel + k_off<128>(r, 32 * g));
            const f32x4 y = *(const f32x4 *)(panel + k_off<128>(r, 32 * g + 16));
            v[0] = x.x;
            v[1] = x.y;
            v[2] = x.z;
            v[3] = x.w;
            v[4] = y.x;
            v[5] = y.y;
            v[6] = y.z;
            v[7] = y.w;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                v[e] = *(const float *)(panel + mn_off<8, ROWS * 4, 8>(8 * g + e, r * 4));
        }
    }

    // bf16 pieces of 8 values, round-to-nearest-even at each step; dword q
    // of piece p holds values 2q, 2q+1.
    static __device__ __forceinline__ void split8(const float v[8], u32 (*pc)[4])
    {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            u32 w[P];
            split_pair<P>(v[2 * q], v[2 * q + 1], w);
#pragma unroll
            for (int p = 0; p < P; ++p) pc[p][q] = w[p];
        }
    }

    static __device__ __forceinline__ void compute(const char *buf, Acc (*acc)[FN], int wm, int wn,
                                                   int lane)
    {
        const char *pa = buf, *pb = buf + PANEL_A;
        const int g = lane >> 4, r = lane & 15;
        u32 fa[FM][P][4], fb[FN][P][4];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            float v[8];
            read8<!TA, MC>(pa, wm * WTM + 16 * i + r, g, v);
            split8(v, fa[i]);
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            float v[8];
            read8<TB, NC>(pb, wn * WTN + 16 * j + r, g, v);
            split8(v, fb[j]);
        }
#pragma unroll
        for (int st = 0; st < Sub<DT>::value; ++st)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) mma_step<DT>(acc[i][j], fa[i], fb[j], st);
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

        const int nk = (p.k > 0 && p.alpha != 0.0f) ? (p.k + KC - 1) / KC : 0;
        if (nk > 0) {
            const char *A = (const char *)p.A;
            const char *B = (const char *)p.B;
            PA pa;
            PB pb;
            pa.init(p.lda, m0, p.m, p.k, wave, lane);
            pb.init(p.ldb, n0, p.n, p.k, wave, lane);
#pragma unroll
            for (int t = 0; t < NS - 1; ++t) {
                char *buf = lds + t * STAGE_BYTES;
                pa.issue(A, p.lda, t * KC, buf, wave);
                pb.issue(B, p.ldb, t * KC, buf + PANEL_A, wave);
            }
            const bool ragged = (!TA || TB) && (p.k % PA::VK) != 0;
            int rd = 0, wr = NS - 1;
            for (int s = 0; s < nk; ++s) {
                wait_vm<(NS - 2) * LOADS>();
                __builtin_amdgcn_s_barrier();
                pin_order();
                char *cur = lds + rd * STAGE_BYTES;
                if (ragged && s == nk - 1) {
                    const int valid_k = p.k - s * KC;
                    if constexpr (!TA) PA::fix_tail(cur, valid_k, tid, NT);
                    if constexpr (TB) PB::fix_tail(cur + PANEL_A, valid_k, tid, NT);
                    __syncthreads();
                }
                char *nxt = lds + wr * STAGE_BYTES;
                pa.issue(A, p.lda, (s + NS - 1) * KC, nxt, wave);
                pb.issue(B, p.ldb, (s + NS - 1) * KC, nxt + PANEL_A, wave);
                pin_order();
                compute(cur, acc, wm, wn, lane);
                rd = rd + 1 == NS ? 0 : rd + 1;
                wr = wr + 1 == NS ? 0 : wr + 1;
            }
            wait_vm<0>();
            __builtin_amdgcn_s_barrier();
        }
        store_c<DT, FM, FN>(p, acc, m0 + wm * WTM, n0 + wn * WTN, lane);
    }
};

}  // namespace mg
