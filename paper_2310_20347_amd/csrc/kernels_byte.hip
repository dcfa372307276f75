// 8-bit input families: FP8 e4m3 (16x16x128 f8f6f4 MFMA, unit scales) and
// INT8 (16x16x64 i8 MFMA, int32 accumulate), kc = 128.
#include "instantiate.hpp"

namespace mg {
void register_byte(std::vector<KernelCfg> &out)
{
    add_cfg<TF8, 64, 64, 2, 2, 2, true, 1, true, true>(out, K_F8);   // also split-K
    add_cfg<TF8, 128, 128, 2, 2, 2, false>(out, K_F8);
    add_cfg<TF8, 256, 128, 2, 2, 2, false>(out, K_F8);
    add_cfg<TI8, 64, 64, 2, 2, 2, true, 1, true, true>(out, K_I8);   // also split-K
    add_cfg<TI8, 128, 128, 2, 2, 2, false>(out, K_I8);
    add_cfg<TI8, 256, 128, 2, 2, 2, false>(out, K_I8);
}
}  // namespace mg
