// 16-bit input families: bf16 and fp16 MFMA (16x16x32), kc = 64.
#include "instantiate.hpp"

namespace mg {
void register_half(std::vector<KernelCfg> &out)
{
    add_cfg<TBF16, 64, 64, 2, 2, 2, true, 1, true, true>(out, K_BF16);   // also split-K
    add_cfg<TBF16, 128, 128, 2, 2, 2, false>(out, K_BF16);
    add_cfg<TBF16, 256, 128, 2, 2, 2, false>(out, K_BF16);
    add_cfg<TBF16, 256, 256, 2, 2, 2, false, 1, false>(out, K_BF16);
    add_cfg<TBF16, 256, 256, 2, 4, 2, false>(out, K_BF16);   // 8 waves, 128x64 each
    add_cfg<TF16, 64, 64, 2, 2, 2, true, 1, true, true>(out, K_F16);   // also split-K
    add_cfg<TF16, 128, 128, 2, 2, 2, false>(out, K_F16);
    add_cfg<TF16, 256, 128, 2, 2, 2, false>(out, K_F16);
    add_cfg<TF16, 256, 256, 2, 2, 2, false, 1, false>(out, K_F16);
    add_cfg<TF16, 256, 256, 2, 4, 2, false>(out, K_F16);   // 8 waves, 128x64 each
}
}  // namespace mg
