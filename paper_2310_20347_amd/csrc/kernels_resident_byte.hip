// A-resident / B-resident family members (B3C2A0, A3C2B0, C3A2B0, C3B2A0)
// of the byte classes, 64x64 tiles.
#include "instantiate.hpp"

namespace mg {
void register_resident_byte(std::vector<KernelCfg> &out)
{
    add_resident_family<TF8>(out, K_F8);
    add_resident_family<TI8>(out, K_I8);
}
}  // namespace mg
