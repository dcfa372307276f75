// Autotuner: the paper's search over micro-kernel shapes (section 8.4, "In
// search of the best micro-kernel": a two-dimensional (mr, nr) space that
// takes a few dozen experiments and can be automated), here over the
// compiled tile configurations x raster order (B3A2C0 / A3B2C0) x raster
// group, with analytical pruning (the role the paper gives to the cache
// model of section 8.2): configurations whose kernels use scratch (spills;
// section 8.10 shows a spilling micro-kernel losing half its speed) are
// rejected, and so are configurations whose staged panels do not fit LDS.
// A second phase re-times the few fastest candidates of each shape in
// interleaved rounds: the MFMA-dense kernels run under a power limit whose
// clock drifts by 10-15% between bursts, which decides close calls when each
// candidate is timed in one burst.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "abi_internal.hpp"
#include "mgemm.h"


using namespace mg;

static int fill_kind(int kclass)
{
    switch (kclass) {
    case K_F32: case K_SPLIT2: case K_SPLIT3: return 0;
    case K_BF16: return 1;
    case K_F16: return 2;
    case K_F8: return 3;
    case K_F64: return 5;
    case K_I16: return 6;
    case K_I32: return 7;
    default: return 4;
    }
}

extern "C" double gemm_panel_occupancy(int64_t rows, int64_t cols, int64_t elem_bytes,
                                       int64_t capacity_bytes)
{
    if (rows < 0 || cols < 0 || elem_bytes <= 0 || capacity_bytes <= 0) return -1.0;
    return double(rows) * double(cols) * double(elem_bytes) / double(capacity_bytes);
}

extern "C" int gemm_tune_layouts(int dtype, int64_t count, const int64_t *shapes, int reps,
                                 const char *out_path, int model_keep, int trans_mask)
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -1;
    if (count < 0) return -2;
    if (count > 0 && !shapes) return -3;
    if (reps < 1) return -4;
    if (model_keep < 0) return -6;
    if (trans_mask < 1 || trans_mask > 15) return -7;
    ensure_registered();
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;

    // scratch operands sized for the largest shape
    size_t maxA = 0, maxB = 0, maxC = 0;
    for (int64_t i = 0; i < count; ++i) {
        const int64_t m = shapes[3 * i], n = shapes[3 * i + 1], k = shapes[3 * i + 2];
        if (m <= 0 || n <= 0 || k <= 0 || m > 0x7FFFFFFF || n > 0x7FFFFFFF || k > 0x7FFFFFFF)
            return -3;
        const int es = elem_bytes(kclass_of(dtype, k));
        maxA = std::max(maxA, size_t(m * k * es));
        maxB = std::max(maxB, size_t(k * n * es));
        maxC = std::max(maxC, size_t(m * n * (dtype == GEMM_F64 ? 8 : 4)));   // C elements
    }
    void *A = nullptr, *B = nullptr, *C = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto fail = [&](hipError_t e) {
        t_tls.hip_err = (int)e;
        if (s) release_workspaces(d, s);
        if (A) (void)hipFree(A);
        if (B) (void)hipFree(B);
        if (C) (void)hipFree(C);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
        return GEMM_E_HIP;
    };
    hipError_t e;
    if ((e = hipMalloc(&A, std::max<size_t>(maxA, 16))) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&B, std::max<size_t>(maxB, 16))) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&C, std::max<size_t>(maxC, 16))) != hipSuccess) return fail(e);
    if ((e = hipStreamCreate(&s)) != hipSuccess) return fail(e);
    if ((e = hipEventCreate(&e0)) != hipSuccess) return fail(e);
    if ((e = hipEventCreate(&e1)) != hipSuccess) return fail(e);

    // the tuner's private stream gets the workspace its candidates need
    // (tuning allocates; the reservation is released at the end)
    auto reserve_for = [&](const KernelCfg &c, const GemmArgs &a) -> bool {
        const size_t need = workspace_need(c, a, d->cus);
        return need == 0 || reserve_workspace(d, s, need, 0) == GEMM_OK;
    };
    static const int kGroups[3] = {4, 8, 16};
    for (int64_t i = 0; i < count; ++i)
    for (int tr = 0; tr < 4; ++tr) {
        if (!((trans_mask >> tr) & 1)) continue;
        const int64_t m = shapes[3 * i], n = shapes[3 * i + 1], k = shapes[3 * i + 2];
        const int kclass = kclass_of(dtype, k);
        // layout tr = 2*(A is 'T') + (B is 'T'): A stored m x k or k x m, B k x n or n x k
        const char ta = (tr >> 1) ? 'T' : 'N', tb = (tr & 1) ? 'T' : 'N';
        const int64_t lda = (tr >> 1) ? m : k, ldb = (tr & 1) ? k : n;
        launch_fill(A, m * k, fill_kind(kclass), 1u, s);
        launch_fill(B, k * n, fill_kind(kclass), 2u, s);
        struct Cand {
            double us;
            TuneVal v;
            int reg, trans;
            bool vec;
            GemmArgs a;
        };
        std::vector<Cand> cands;
        const std::vector<int> &ids = g_by_class[kclass];
        // model pruning: only the model_keep configurations it ranks first
        std::vector<bool> keep(ids.size(), true);
        if (model_keep > 0 && (size_t)model_keep < ids.size()) {
            std::vector<std::pair<double, size_t>> r;
            for (size_t id = 0; id < ids.size(); ++id)
                r.push_back({model_cycles(g_cfgs[ids[id]], kclass, m, n, k, d->cus), id});
            std::sort(r.begin(), r.end());
            keep.assign(ids.size(), false);
            for (int i = 0; i < model_keep; ++i) keep[r[(size_t)i].second] = true;
        }
        for (size_t id = 0; id < ids.size(); ++id) {
            const KernelCfg &c = g_cfgs[ids[id]];
            if (!c.func[tr][1] || !keep[id]) continue;
            hipFuncAttributes attr;
            if (hipFuncGetAttributes(&attr, c.func[tr][1]) == hipSuccess && attr.localSizeBytes > 0)
                continue;   // spills: rejected
            if (gemm_panel_occupancy(1, c.lds, 1, 160 * 1024) > 1.0)
                continue;   // staged panels exceed one CU's LDS
            for (int order = 0; order < 2; ++order) {
                for (int gi = 0; gi < 3; ++gi) {
                    GemmArgs a;
                    int trans = 0, cfg = 0, kc2 = 0;
                    bool vec = true;
                    const int saved = t_tls.force_id[kclass];
                    const int saved_o = t_tls.force_order[kclass];
                    t_tls.force_id[kclass] = (int)id;
                    t_tls.force_order[kclass] = order;
                    t_tls.force_group = kGroups[gi];
                    const int reg = plan_gemm(dtype, ta, tb, m, n, k, 1.0, A, lda, B, ldb, 0.0, C, n,
                                              d->cus, a, trans, vec, cfg, kc2);
                    t_tls.force_id[kclass] = saved;
                    t_tls.force_order[kclass] = saved_o;
                    t_tls.force_group = 0;
                    if (reg < 0 || cfg != (int)id || !reserve_for(g_cfgs[reg], a)) continue;
                    std::vector<float> ms;
                    for (int r = 0; r < reps + 2; ++r) {
                        (void)hipEventRecord(e0, s);
                        if (launch_gemm(g_cfgs[reg], trans, vec, a, s, stream_reservation(d, s)) != GEMM_OK)
                            break;
                        (void)hipEventRecord(e1, s);
                        if ((e = hipEventSynchronize(e1)) != hipSuccess) return fail(e);
                        float t = 0;
                        (void)hipEventElapsedTime(&t, e0, e1);
                        if (r >= 2) ms.push_back(t);
                    }
                    if ((int)ms.size() != reps) continue;
                    std::sort(ms.begin(), ms.end());
                    const double us = 1e3 * ms[ms.size() / 2];
                    cands.push_back(Cand{us, TuneVal{(int)id, order, kGroups[gi], us}, reg, trans,
                                         vec, a});
                    if (c.kind != 0) break;   // raster group is irrelevant to these
                }
            }
        }
        if (cands.empty()) continue;
        std::sort(cands.begin(), cands.end(),
                  [](const Cand &x, const Cand &y) { return x.us < y.us; });
        // phase two: the fastest candidates (those within 25% of the best),
        // interleaved over rounds, median of all their launches
        static constexpr int kFinal = 4, kRounds = 4;
        size_t nf = 1;
        while (nf < cands.size() && nf < (size_t)kFinal && cands[nf].us < 1.25 * cands[0].us) ++nf;
        TuneVal best = cands[0].v;
        if (nf > 1) {
            std::vector<std::vector<float>> ms(nf);
            for (int round = 0; round < kRounds; ++round) {
                for (size_t q = 0; q < nf; ++q) {
                    const Cand &c = cands[q];
                    for (int r = 0; r < reps; ++r) {
                        (void)hipEventRecord(e0, s);
                        if (launch_gemm(g_cfgs[c.reg], c.trans, c.vec, c.a, s, stream_reservation(d, s)) !=
                            GEMM_OK)
                            break;
                        (void)hipEventRecord(e1, s);
                        if ((e = hipEventSynchronize(e1)) != hipSuccess) return fail(e);
                        float t = 0;
                        (void)hipEventElapsedTime(&t, e0, e1);
                        ms[q].push_back(t);
                    }
                }
            }
            double best_us = 1e300;
            for (size_t q = 0; q < nf; ++q) {
                if (ms[q].empty()) continue;
                std::sort(ms[q].begin(), ms[q].end());
                const double us = 1e3 * ms[q][ms[q].size() / 2];
                if (us < best_us) {
                    best_us = us;
                    best = cands[q].v;
                    best.us = us;
                }
            }
        }
        {
            std::lock_guard<std::mutex> g(g_mu);
            g_table[TuneKey{kclass, tr, bucket(m), bucket(n), bucket(k)}] = best;
        }
    }
    release_workspaces(d, s);
    (void)hipFree(A);
    (void)hipFree(B);
    (void)hipFree(C);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    rebuild_lut();
    if (out_path && *out_path) return save_table(out_path);
    return GEMM_OK;
}

extern "C" int gemm_tune_pruned(int dtype, int64_t count, const int64_t *shapes, int reps,
                                const char *out_path, int model_keep)
{
    return gemm_tune_layouts(dtype, count, shapes, reps, out_path, model_keep, 15);
}

extern "C" int gemm_tune(int dtype, int64_t count, const int64_t *shapes, int reps, const char *out_path)
{
    return gemm_tune_layouts(dtype, count, shapes, reps, out_path, 0, 15);
}
