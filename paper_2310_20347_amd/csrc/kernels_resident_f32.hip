// A-resident / B-resident family members (B3C2A0, A3C2B0, C3A2B0, C3B2A0)
// of the f32 classes, 64x64 tiles.
#include "instantiate.hpp"

namespace mg {
void register_resident_f32(std::vector<KernelCfg> &out)
{
    add_resident_family<TF32>(out, K_F32);
}
}  // namespace mg
