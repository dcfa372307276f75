// A-resident / B-resident family members (B3C2A0, A3C2B0, C3A2B0, C3B2A0)
// of the half classes, 64x64 tiles.
#include "instantiate.hpp"

namespace mg {
void register_resident_half(std::vector<KernelCfg> &out)
{
    add_resident_family<TBF16>(out, K_BF16);
    add_resident_family<TF16>(out, K_F16);
}
}  // namespace mg
