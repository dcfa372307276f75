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
}  // namespace mg
