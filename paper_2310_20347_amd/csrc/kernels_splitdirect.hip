// Split-product family on direct-staged FP32 panels (three- and six-term).
#include "instantiate.hpp"

namespace mg {
void register_splitdirect(std::vector<KernelCfg> &out)
{
    add_splitdirect<2, 128, 128, 2, 2, 2>(out, K_SPLIT2);   // two workgroups per CU
    add_splitdirect<2, 256, 128, 2, 2, 3>(out, K_SPLIT2);
    add_splitdirect<3, 128, 128, 2, 2, 2>(out, K_SPLIT3);
    add_splitdirect<3, 64, 64, 2, 2, 2>(out, K_SPLIT3);
}
}  // namespace mg
