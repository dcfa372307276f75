// Helpers that instantiate the tile kernel for one configuration.
#pragma once

#include "direct.hpp"
#include "nopack.hpp"
#include "splitdirect.hpp"
#include "registry.hpp"
#include "resident.hpp"
#include "tile.hpp"

namespace mg {

template <class DT, int MC, int NC, int WM, int WN, int ST, bool TA, bool TB, bool VEC, int PF,
          bool PEEL, bool SPLITK = false>
static void fill_one(KernelCfg &c)
{
    typedef Tile<DT, MC, NC, WM, WN, TA, TB, VEC, ST, PF, PEEL> T;
    c.func[2 * TA + TB][VEC] = (const void *)&gemm_tile_kernel<T>;
    if constexpr (SPLITK) c.splitk[2 * TA + TB][VEC] = (const void *)&gemm_splitk_kernel<T, DT::GES, TA, TB>;
}

// Adds configuration (MC, NC, WM, WN, ST) of dtype DT; the element-wise
// (unaligned) staging variant is compiled only when WITH_SCALAR is set.
template <class DT, int MC, int NC, int WM, int WN, int ST, bool WITH_SCALAR, int PF = 1,
          bool PEEL = true, bool SPLITK = false>
static void add_cfg(std::vector<KernelCfg> &out, int kclass)
{
    typedef Tile<DT, MC, NC, WM, WN, false, false, true, ST, PF, PEEL> T;
    KernelCfg c;
    c.kclass = kclass;
    c.mc = MC;
    c.nc = NC;
    c.kc = T::KC;
    c.wm = WM;
    c.wn = WN;
    c.threads = T::NT;
    c.lds = T::LDS_BYTES;
    c.stages = ST;
    c.kind = 0;
    fill_one<DT, MC, NC, WM, WN, ST, false, false, true, PF, PEEL, SPLITK>(c);
    fill_one<DT, MC, NC, WM, WN, ST, false, true, true, PF, PEEL, SPLITK>(c);
    fill_one<DT, MC, NC, WM, WN, ST, true, false, true, PF, PEEL, SPLITK>(c);
    fill_one<DT, MC, NC, WM, WN, ST, true, true, true, PF, PEEL, SPLITK>(c);
    if constexpr (WITH_SCALAR) {
        fill_one<DT, MC, NC, WM, WN, ST, false, false, false, PF, PEEL, SPLITK>(c);
        fill_one<DT, MC, NC, WM, WN, ST, false, true, false, PF, PEEL, SPLITK>(c);
        fill_one<DT, MC, NC, WM, WN, ST, true, false, false, PF, PEEL, SPLITK>(c);
        fill_one<DT, MC, NC, WM, WN, ST, true, true, false, PF, PEEL, SPLITK>(c);
    }
    out.push_back(c);
}

// Adds an A/B-resident family member (kind 1..4, see resident.hpp); only
// the vectorised staging variant is compiled (unaligned operands fall back to
// the class's C-resident configuration 0).
template <class DT, int MC, int NC, int KIND, bool TA, bool TB>
static void fill_resident(KernelCfg &c)
{
    typedef ResidentTile<DT, MC, NC, KIND, TA, TB, true> T;
    c.func[2 * TA + TB][1] = (const void *)&gemm_resident_kernel<T>;
}

template <class DT, int MC, int NC, int KIND>
static void add_resident(std::vector<KernelCfg> &out, int kclass)
{
    typedef ResidentTile<DT, MC, NC, KIND, false, false, true> T;
    KernelCfg c;
    c.kclass = kclass;
    c.mc = MC;
    c.nc = NC;
    c.kc = T::KC;
    const bool ar = (KIND == 1 || KIND == 4);
    c.wm = ar ? 4 : 1;   // A resident: each wave owns mc/4 rows and walks all nc columns
    c.wn = ar ? 1 : 4;
    c.threads = T::NT;
    c.lds = T::LDS_BYTES;
    c.stages = 1;
    c.kind = KIND;
    fill_resident<DT, MC, NC, KIND, false, false>(c);
    fill_resident<DT, MC, NC, KIND, false, true>(c);
    fill_resident<DT, MC, NC, KIND, true, false>(c);
    fill_resident<DT, MC, NC, KIND, true, true>(c);
    out.push_back(c);
}

template <class DT>
static void add_resident_family(std::vector<KernelCfg> &out, int kclass)
{
    add_resident<DT, 64, 64, 1>(out, kclass);   // B3C2A0
    add_resident<DT, 64, 64, 2>(out, kclass);   // A3C2B0
    add_resident<DT, 64, 64, 3>(out, kclass);   // C3A2B0
    add_resident<DT, 64, 64, 4>(out, kclass);   // C3B2A0
}

// Adds a direct-staged configuration (NS-deep LDS ring, direct.hpp): the
// vectorised variant of all four transpositions; unaligned operands fall
// back to the class's configuration 0.
template <class DT, int MC, int NC, int WM, int WN, int NS, bool TA, bool TB, bool SPLITK, int KB,
          bool OVL = false, int MB = 16>
static void fill_direct(KernelCfg &c)
{
    typedef DTile<DT, MC, NC, WM, WN, TA, TB, NS, KB, OVL, MB> T;
    c.func[2 * TA + TB][1] = (const void *)&gemm_direct_kernel<T>;
    if constexpr (SPLITK) c.splitk[2 * TA + TB][1] = (const void *)&gemm_splitk_kernel<T, DT::GES, TA, TB>;
}

template <class DT, int MC, int NC, int WM, int WN, int NS, bool SPLITK = false, int KB = 128,
          bool OVL = false, int MB = 16>
static void add_direct(std::vector<KernelCfg> &out, int kclass)
{
    typedef DTile<DT, MC, NC, WM, WN, false, false, NS, KB, OVL, MB> T;
    KernelCfg c;
    c.kclass = kclass;
    c.mc = MC;
    c.nc = NC;
    c.kc = T::KC;
    c.wm = WM;
    c.wn = WN;
    c.threads = T::NT;
    c.lds = T::LDS_BYTES;
    c.stages = NS;
    c.kind = 0;
    c.direct = true;
    c.mfma = MB;
    fill_direct<DT, MC, NC, WM, WN, NS, false, false, SPLITK, KB, OVL, MB>(c);
    fill_direct<DT, MC, NC, WM, WN, NS, false, true, SPLITK, KB, OVL, MB>(c);
    fill_direct<DT, MC, NC, WM, WN, NS, true, false, SPLITK, KB, OVL, MB>(c);
    fill_direct<DT, MC, NC, WM, WN, NS, true, true, SPLITK, KB, OVL, MB>(c);
    out.push_back(c);
}

// Adds a packing configuration: A and/or B skip the LDS panel (nopack.hpp).
// Only the layouts in which every unpacked operand is contiguous along k are
// compiled (A unpacked: A 'N'; B unpacked: B 'T'); other layouts, and
// unaligned operands, fall back to the class's configuration 0.
template <class DT, int MC, int NC, int WM, int WN, bool PKA, bool PKB, bool TA, bool TB>
static void fill_nopack(KernelCfg &c)
{
    if constexpr ((PKA || !TA) && (PKB || TB)) {
        typedef UTile<DT, MC, NC, WM, WN, TA, TB, PKA, PKB> T;
        c.func[2 * TA + TB][1] = (const void *)&gemm_nopack_kernel<T>;
    }
}

template <class DT, int MC, int NC, int WM, int WN, bool PKA, bool PKB>
static void add_nopack(std::vector<KernelCfg> &out, int kclass)
{
    typedef UTile<DT, MC, NC, WM, WN, false, true, PKA, PKB> T;
    KernelCfg c;
    c.kclass = kclass;
    c.mc = MC;
    c.nc = NC;
    c.kc = T::KC;
    c.wm = WM;
    c.wn = WN;
    c.threads = T::NT;
    c.lds = T::LDS_BYTES;
    c.stages = T::NS;
    c.kind = 0;
    c.direct = true;
    c.unpacked = (PKA ? 0 : 1) | (PKB ? 0 : 2);
    fill_nopack<DT, MC, NC, WM, WN, PKA, PKB, false, false>(c);
    fill_nopack<DT, MC, NC, WM, WN, PKA, PKB, false, true>(c);
    fill_nopack<DT, MC, NC, WM, WN, PKA, PKB, true, false>(c);
    fill_nopack<DT, MC, NC, WM, WN, PKA, PKB, true, true>(c);
    out.push_back(c);
}

// Adds a split-product configuration on direct-staged FP32 panels (the
// pieces formed as fragments are read, splitdirect.hpp).
template <int P, int MC, int NC, int WM, int WN, int NS, bool TA, bool TB>
static void fill_splitdirect(KernelCfg &c)
{
    typedef SDTile<P, MC, NC, WM, WN, TA, TB, NS> T;
    c.func[2 * TA + TB][1] = (const void *)&gemm_direct_kernel<T>;
}

template <int P, int MC, int NC, int WM, int WN, int NS>
static void add_splitdirect(std::vector<KernelCfg> &out, int kclass)
{
    typedef SDTile<P, MC, NC, WM, WN, false, false, NS> T;
    KernelCfg c;
    c.kclass = kclass;
    c.mc = MC;
    c.nc = NC;
    c.kc = T::KC;
    c.wm = WM;
    c.wn = WN;
    c.threads = T::NT;
    c.lds = T::LDS_BYTES;
    c.stages = NS;
    c.kind = 0;
    c.direct = true;
    fill_splitdirect<P, MC, NC, WM, WN, NS, false, false>(c);
    fill_splitdirect<P, MC, NC, WM, WN, NS, false, true>(c);
    fill_splitdirect<P, MC, NC, WM, WN, NS, true, false>(c);
    fill_splitdirect<P, MC, NC, WM, WN, NS, true, true>(c);
    out.push_back(c);
}

}  // namespace mg
