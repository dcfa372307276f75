// A-resident / B-resident family members (B3C2A0, A3C2B0, C3A2B0, C3B2A0)
// of the split classes, 64x64 tiles.
#include "instantiate.hpp"

namespace mg {
void register_resident_split(std::vector<KernelCfg> &out)
{
    add_resident_family<TSplit<2>>(out, K_SPLIT2);
    add_resident_family<TSplit<3>>(out, K_SPLIT3);
}
}  // namespace mg
