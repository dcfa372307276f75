// Direct-staged tiles of 32x32 MFMA blocks (BF16, FP16, FP8 e4m3, INT8):
// v_mfma_f32_32x32x16_bf16 / _f16, v_mfma_scale_f32_32x32x64_f8f6f4 and
// v_mfma_i32_32x32x32_i8.  A 32x32 block does twice the multiply-adds of a
// 16x16 one per instruction, so a wave tile issues half as many MFMAs for
// the same fragment bytes; the FP8 stage splits into two fragment chunks,
// which lets its last chunk be deferred past the next barrier (OVL).
#include "instantiate.hpp"

namespace mg {
template <class DT>
static void add_w32(std::vector<KernelCfg> &out, int kclass)
{
    add_direct<DT, 256, 256, 2, 4, 2, false, 128, true, 32>(out, kclass);   // 8 waves of 128x64
    add_direct<DT, 256, 256, 2, 2, 2, false, 128, true, 32>(out, kclass);   // 4 waves of 128x128
    add_direct<DT, 256, 128, 2, 2, 3, false, 128, true, 32>(out, kclass);
    add_direct<DT, 128, 128, 2, 2, 4, false, 128, false, 32>(out, kclass);
}

// Registered after every other family (configuration numbers above stay).
void register_direct_w32_late(std::vector<KernelCfg> &out)
{
    add_w32<TBF16>(out, K_BF16);
    add_w32<TF16>(out, K_F16);
    add_w32<TF8>(out, K_F8);
    add_w32<TI8>(out, K_I8);
}
}  // namespace mg
