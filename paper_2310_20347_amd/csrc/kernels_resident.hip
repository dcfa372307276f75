// A-resident / B-resident micro-kernel variants (placeholder).
#include "instantiate.hpp"

namespace mg {
void register_resident(std::vector<KernelCfg> &) {}
}  // namespace mg
