// Helpers that instantiate the tile kernel for one configuration.
#pragma once

#include "registry.hpp"
#include "tile.hpp"

namespace mg {

template <class DT, int MC, int NC, int WM, int WN, int ST, bool TA, bool TB, bool VEC>
static void fill_one(KernelCfg &c)
{
    typedef Tile<DT, MC, NC, WM, WN, TA, TB, VEC, ST> T;
    c.func[2 * TA + TB][VEC] = (const void *)&gemm_tile_kernel<T>;
}

// Adds configuration (MC, NC, WM, WN, ST) of dtype DT; the element-wise
// (unaligned) staging variant is compiled only when WITH_SCALAR is set.
template <class DT, int MC, int NC, int WM, int WN, int ST, bool WITH_SCALAR>
static void add_cfg(std::vector<KernelCfg> &out, int kclass)
{
    typedef Tile<DT, MC, NC, WM, WN, false, false, true, ST> T;
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
    fill_one<DT, MC, NC, WM, WN, ST, false, false, true>(c);
    fill_one<DT, MC, NC, WM, WN, ST, false, true, true>(c);
    fill_one<DT, MC, NC, WM, WN, ST, true, false, true>(c);
    fill_one<DT, MC, NC, WM, WN, ST, true, true, true>(c);
    if constexpr (WITH_SCALAR) {
        fill_one<DT, MC, NC, WM, WN, ST, false, false, false>(c);
        fill_one<DT, MC, NC, WM, WN, ST, false, true, false>(c);
        fill_one<DT, MC, NC, WM, WN, ST, true, false, false>(c);
        fill_one<DT, MC, NC, WM, WN, ST, true, true, false>(c);
    }
    out.push_back(c);
}

}  // namespace mg
