// Plain FP32 family: FP32 MFMA (16x16x4) micro-kernels, kc = 32.
#include "instantiate.hpp"

namespace mg {
void register_f32(std::vector<KernelCfg> &out)
{
    // config 0 is also the element-wise (unaligned operands) fallback
    add_cfg<TF32, 64, 64, 2, 2, 2, true, 1, true, true>(out, K_F32);   // also split-K
    add_cfg<TF32, 128, 128, 2, 2, 2, false, 1, false>(out, K_F32);   // two workgroups per CU
    add_cfg<TF32, 128, 64, 2, 2, 2, false>(out, K_F32);
    add_cfg<TF32, 256, 128, 2, 2, 2, false>(out, K_F32);
    add_cfg<TF32, 256, 256, 2, 2, 2, false, 1, false>(out, K_F32);
}
}  // namespace mg
