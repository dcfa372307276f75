// Packing configurations (A, B or neither staged in LDS) for FP32 and BF16.
#include "instantiate.hpp"

namespace mg {
template <class DT>
static void add_nopack_family(std::vector<KernelCfg> &out, int kclass)
{
    add_nopack<DT, 64, 64, 2, 2, false, true>(out, kclass);     // A unpacked
    add_nopack<DT, 64, 64, 2, 2, true, false>(out, kclass);     // B unpacked
    add_nopack<DT, 64, 64, 2, 2, false, false>(out, kclass);    // neither: no LDS
    add_nopack<DT, 128, 128, 2, 2, false, true>(out, kclass);   // A unpacked
}

void register_nopack(std::vector<KernelCfg> &out)
{
    add_nopack_family<TF32>(out, K_F32);
    add_nopack_family<TBF16>(out, K_BF16);
}
}  // namespace mg
