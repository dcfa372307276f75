// FP32-accurate split-product family: FP32 operands split into 2 (x3 terms)
// or 3 (x6 terms) bf16 pieces while staged, bf16 MFMA (16x16x32), kc = 64.
#include "instantiate.hpp"

namespace mg {
void register_split(std::vector<KernelCfg> &out)
{
    add_cfg<TSplit<2>, 64, 64, 2, 2, 2, true, 1, true, true>(out, K_SPLIT2);   // also split-K
    add_cfg<TSplit<2>, 128, 128, 2, 2, 2, false>(out, K_SPLIT2);
    add_cfg<TSplit<2>, 128, 64, 2, 2, 2, false>(out, K_SPLIT2);
    add_cfg<TSplit<2>, 256, 128, 2, 2, 1, false>(out, K_SPLIT2);
    add_cfg<TSplit<2>, 128, 128, 2, 2, 2, false, 2>(out, K_SPLIT2);   // two stages in flight
    add_cfg<TSplit<3>, 64, 64, 2, 2, 1, true, 1, true, true>(out, K_SPLIT3);   // also split-K
    add_cfg<TSplit<3>, 128, 128, 2, 2, 1, false>(out, K_SPLIT3);
}
}  // namespace mg
