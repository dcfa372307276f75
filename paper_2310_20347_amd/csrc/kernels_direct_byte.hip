// FP8 e4m3 / INT8 direct-staged family (global -> LDS loads, NS-deep stage ring).
#include "instantiate.hpp"

namespace mg {
template <class DT>
static void add_byte_direct(std::vector<KernelCfg> &out, int kclass)
{
    add_direct<DT, 256, 256, 2, 4, 2>(out, kclass);   // 8 waves of 128x64
    add_direct<DT, 256, 128, 2, 2, 3>(out, kclass);
    add_direct<DT, 128, 128, 2, 2, 4>(out, kclass);
    add_direct<DT, 128, 128, 2, 2, 2, true>(out, kclass);   // two workgroups per CU; also split-K
}

void register_direct_byte(std::vector<KernelCfg> &out)
{
    add_byte_direct<TF8>(out, K_F8);
    add_byte_direct<TI8>(out, K_I8);
    // INT8 fragments cover 64 bytes of k, so INT8 also has 64-byte stages: a
    // deeper ring in the same LDS (FP8 fragments need all 128 bytes)
    add_direct<TI8, 256, 256, 2, 4, 4, false, 64>(out, K_I8);
    add_direct<TI8, 256, 256, 2, 4, 5, false, 64>(out, K_I8);
}

// Registered after every other family (configuration numbers above stay):
// each stage's last MFMAs deferred past the next barrier (INT8 only: an FP8
// stage is a single fragment chunk, nothing to overlap with).
void register_direct_byte_late(std::vector<KernelCfg> &out)
{
    add_direct<TI8, 256, 256, 2, 4, 2, false, 128, true>(out, K_I8);
    add_direct<TI8, 256, 128, 2, 2, 3, false, 128, true>(out, K_I8);
}
}  // namespace mg
