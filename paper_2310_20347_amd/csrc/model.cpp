// Analytical model of a tile configuration's time on one GPU: the role the
// paper gives to its analytical model of the memory hierarchy (choosing the
// block sizes from cache and register capacities instead of searching), with
// the GPU's capacities: 160 KiB of LDS and 512 VGPRs per lane per SIMD
// bound how many workgroups share a compute unit; the grid is dealt to the
// compute units in rounds; a tile's time is the largest of its MFMA time,
// its L2->LDS operand traffic and its LDS fragment reads (each shared with
// the other workgroups on the unit), plus the load latency a stage ring of
// its depth leaves exposed, plus its epilogue.  The model ranks
// configurations; its absolute times are rough.  Uses: the dispatch
// fallback when the tuning table has no entry, and pruning the tuner's
// search to the model's best candidates (gemm_tune_pruned).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "abi_internal.hpp"
#include "mgemm.h"

namespace mg {

namespace {

constexpr double kClockGHz = 2.1;      // sustained clock under MFMA load
constexpr double kL2BytesPerClk = 64;  // L2 -> compute unit, per compute unit
constexpr double kLdsBytesPerClk = 128;
constexpr double kHbmBytesPerClk = 8e12 / (kClockGHz * 1e9);   // whole device
constexpr double kLoadLatency = 2000;  // cycles from issue to data in LDS, under load
constexpr int kLdsBytes = 160 * 1024, kVgprs = 512, kWavesPerSimd = 8;

// MFMA FLOP per clock per compute unit, FP32-equivalent for the split
// product.
double rate_per_cu(int kclass)
{
    switch (kclass) {
    case K_F32: return 256;
    case K_SPLIT2: return 4096.0 / 3;
    case K_SPLIT3: return 4096.0 / 6;
    case K_BF16: case K_F16: return 4096;
    case K_F8: case K_I8: return 8192;
    case K_F64: return 128;
    // INT16 / INT32 on the vector ALUs (configuration 0): a 24-bit
    // multiply-add per int16 product, a quarter-rate 32-bit multiply and an
    // add per int32 product, each value read from LDS
    case K_I16: return 64;
    case K_I32: return 24;
    default: return 256;
    }
}

// Bytes of one operand element in LDS (the split product keeps 2 or 3 bf16
// planes per FP32 value when staged through registers).
double lds_elem_bytes(int kclass, const KernelCfg &c)
{
    if ((kclass == K_SPLIT2 || kclass == K_SPLIT3) && !c.direct) return kclass == K_SPLIT2 ? 4 : 6;
    return elem_bytes(kclass);
}

// VGPRs per lane: the kernel's own count when the runtime reports it, else
// the accumulators plus a fixed allowance.
int vgprs_of(const KernelCfg &c, int kclass)
{
    const void *f = c.func[0][1] ? c.func[0][1] : c.func[0][0];
    if (!f) f = c.func[1][1];
    if (f) {
        hipFuncAttributes attr;
        if (hipFuncGetAttributes(&attr, f) == hipSuccess && attr.numRegs > 0) return attr.numRegs;
        (void)hipGetLastError();
    }
    const int waves = std::max(1, c.threads / 64);
    const double acc_bytes = kclass == K_F64 ? 8 : 4;
    const double acc = double(c.mc) * c.nc * acc_bytes / 4 / (64.0 * waves);
    return std::min(kVgprs, int(acc) + 64);
}

}  // namespace

double model_cycles(const KernelCfg &c, int kclass, int64_t m, int64_t n, int64_t k, int cus)
{
    if (m <= 0 || n <= 0 || k <= 0 || c.mc <= 0 || c.nc <= 0 || c.kc <= 0 || cus <= 0) return 0;
    if (c.kind == 7) {
        // digit products: INT8 GEMMs over products x k (at about half the
        // INT8 MFMA rate), the packing pass (operands read, digit planes
        // written) and one pass over C per weight class
        const double products = kclass == K_I16 ? 4 : 10, classes = kclass == K_I16 ? 4 : 4;
        const double P = kclass == K_I16 ? 2 : 4;
        const double t_mma = 2.0 * m * n * k * products / (rate_per_cu(K_I8) * 0.5 * cus);
        const double bytes = double(m + n) * k * (elem_bytes(kclass) + P) + classes * 8.0 * m * n;
        return t_mma + bytes / kHbmBytesPerClk + classes * kLoadLatency * 2;
    }
    const int waves = std::max(1, c.threads / 64);
    // workgroups per compute unit
    const int occ_lds = c.lds > 0 ? kLdsBytes / c.lds : 8;
    const int v = std::max(8, (vgprs_of(c, kclass) + 7) / 8 * 8);
    const int occ_vgpr = (4 * std::min(kWavesPerSimd, kVgprs / v)) / waves;
    const int occ = std::max(1, std::min({occ_lds, occ_vgpr, 4 * kWavesPerSimd / waves}));
    const int64_t nk = (k + c.kc - 1) / c.kc;
    double tiles = double((m + c.mc - 1) / c.mc) * double((n + c.nc - 1) / c.nc);
    double slices = 1, extra = 0;
    if (c.kind == 6 && nk >= 4) {
        // split-K: about two workgroups per compute unit, slices of at least two stages
        slices = std::max(1.0, std::min({16.0, double(nk / 2), std::floor(2.0 * cus / tiles)}));
        extra = slices * double(m) * n * 4 * 2 / kHbmBytesPerClk;   // partial tiles out and back
    }
    if (c.kind == 5) {
        // packed split: the packing pass reads FP32 and writes terms bf16 pieces
        const double terms = kclass == K_SPLIT3 ? 6 : 3;
        extra = double(m + n) * k * (4 + 2 * terms) / kHbmBytesPerClk;
    }
    const double work = tiles * slices;
    const double rounds = std::ceil(work / (double(cus) * occ));
    const double conc = std::min<double>(occ, std::ceil(work / cus));
    const double keff = double(nk) * c.kc / slices;
    const double es = elem_bytes(kclass), les = lds_elem_bytes(kclass, c);
    const double wm = std::max(1, c.wm), wn = std::max(1, c.wn);
    // an operand loaded straight to registers (packing configurations) is
    // not read from LDS but is fetched by each wave that uses it
    const bool ua = (c.unpacked & 1) != 0, ub = (c.unpacked & 2) != 0;
    // FP64's element-wise kernel (configuration 0) reads each operand value
    // from LDS for every FMA on the vector ALUs: about a third of the MFMA
    // tiles' rate (measured)
    const double rate = rate_per_cu(kclass) / (kclass == K_F64 && !c.direct ? 3.0 : 1.0);
    const double t_mfma = 2.0 * c.mc * c.nc * keff / rate * conc;
    const double t_l2 = (double(c.mc) * (ua ? wn : 1) + double(c.nc) * (ub ? wm : 1)) * keff * es /
                        kL2BytesPerClk * conc;
    // fragment reads, plus the LDS stores of register staging
    const double lds_rows = waves * ((ua ? 0 : c.mc / wm) + (ub ? 0 : c.nc / wn));
    const double lds_writes = c.direct ? 0.0 : (ua ? 0 : c.mc) + (ub ? 0 : c.nc);
    const double t_lds = (lds_rows + lds_writes) * keff * les / kLdsBytesPerClk * conc;
    const double stages = std::max(1, c.stages);
    const double per_stage = t_mfma / std::max<double>(1.0, double(nk) / slices);
    const double window = (stages - (c.direct ? 1 : 0)) * per_stage + (conc - 1) * per_stage;
    const double exposed = std::max(0.0, kLoadLatency - window) * (double(nk) / slices);
    const double epilogue = double(c.mc) * c.nc * (kclass == K_F64 ? 8 : 4) / kL2BytesPerClk;
    const double t_tile = std::max({t_mfma, t_l2, t_lds}) + exposed + kLoadLatency + epilogue;
    return rounds * t_tile + extra;
}

double model_us(const KernelCfg &c, int kclass, int64_t m, int64_t n, int64_t k, int cus)
{
    return model_cycles(c, kclass, m, n, k, cus) / (kClockGHz * 1e3);
}

// The configuration of class kclass with the lowest modelled time among
// those with a kernel for this layout and staging.
int model_best(int kclass, int trans, bool vec, int64_t m, int64_t n, int64_t k, int cus)
{
    const std::vector<int> &ids = g_by_class[kclass];
    int best = 0;
    double best_t = 1e300;
    for (size_t i = 0; i < ids.size(); ++i) {
        const KernelCfg &c = g_cfgs[ids[i]];
        if (!c.func[trans][vec ? 1 : 0]) continue;
        const double t = model_cycles(c, kclass, m, n, k, cus);
        if (t < best_t * 0.999) {
            best_t = t;
            best = (int)i;
        }
    }
    return best;
}

}  // namespace mg

using namespace mg;

extern "C" double gemm_model_us(int dtype, int id, int64_t m, int64_t n, int64_t k, int cus)
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES || m <= 0 || n <= 0 || k <= 0 || cus <= 0) return -1.0;
    ensure_registered();
    const int kclass = kclass_of(dtype, k);
    if (id < 0 || id >= (int)g_by_class[kclass].size()) return -1.0;
    return model_us(g_cfgs[g_by_class[kclass][id]], kclass, m, n, k, cus);
}
