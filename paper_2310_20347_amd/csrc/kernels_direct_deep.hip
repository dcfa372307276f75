// Deep rings of 64-byte stages with the deferred schedule (BF16, FP16,
// INT8): a 64-byte stage of these types is a single fragment chunk, so the
// whole stage's MFMAs run after the next barrier, while that stage's
// fragments are read; 3 or 4 stages of loads are in flight (the 128-byte
// two-stage ring has one).
#include "instantiate.hpp"

namespace mg {
template <class DT>
static void add_deep(std::vector<KernelCfg> &out, int kclass)
{
    add_direct<DT, 256, 256, 2, 4, 4, false, 64, true>(out, kclass);
    add_direct<DT, 256, 256, 2, 4, 5, false, 64, true>(out, kclass);
}

// Registered after every other family (configuration numbers above stay).
void register_direct_deep_late(std::vector<KernelCfg> &out)
{
    add_deep<TBF16>(out, K_BF16);
    add_deep<TF16>(out, K_F16);
    add_deep<TI8>(out, K_I8);
}
}  // namespace mg
