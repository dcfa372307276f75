// Plain FP32 direct-staged family (global -> LDS loads, NS-deep stage ring).
#include "instantiate.hpp"

namespace mg {
void register_direct_f32(std::vector<KernelCfg> &out)
{
    add_direct<TF32, 128, 128, 2, 2, 2, true>(out, K_F32);   // two workgroups per CU; also split-K
    add_direct<TF32, 128, 128, 2, 2, 4>(out, K_F32);
    add_direct<TF32, 256, 128, 2, 2, 3>(out, K_F32);
    add_direct<TF32, 256, 256, 2, 4, 2>(out, K_F32);   // 8 waves of 128x64
}

// Registered after every other family, so the configuration numbers above
// (and the tuning tables that name them) stay as they were.
void register_direct_f32_late(std::vector<KernelCfg> &out)
{
    // one wave per SIMD (128x128 wave tiles, accumulators in the AGPRs) with
    // each stage's last MFMAs deferred past the next barrier (the 8-wave tile
    // would spill with the deferral)
    add_direct<TF32, 256, 256, 2, 2, 2, false, 128, true>(out, K_F32);
    add_direct<TF32, 256, 128, 2, 2, 3, false, 128, true>(out, K_F32);
}
}  // namespace mg
