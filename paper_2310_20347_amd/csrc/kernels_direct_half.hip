// BF16 / FP16 direct-staged family (global -> LDS loads, NS-deep stage ring).
#include "instantiate.hpp"

namespace mg {
template <class DT>
static void add_half_direct(std::vector<KernelCfg> &out, int kclass)
{
    add_direct<DT, 256, 256, 2, 4, 2>(out, kclass);   // 8 waves of 128x64
    add_direct<DT, 256, 256, 2, 2, 2>(out, kclass);   // 4 waves of 128x128
    add_direct<DT, 256, 128, 2, 2, 3>(out, kclass);
    add_direct<DT, 128, 128, 2, 2, 4>(out, kclass);
    add_direct<DT, 128, 128, 2, 2, 2, true>(out, kclass);   // two workgroups per CU; also split-K
    // 64-byte stages: a deeper ring (more loads in flight) in the same LDS
    add_direct<DT, 256, 256, 2, 4, 4, false, 64>(out, kclass);
    add_direct<DT, 256, 256, 2, 4, 5, false, 64>(out, kclass);
}

void register_direct_half(std::vector<KernelCfg> &out)
{
    add_half_direct<TBF16>(out, K_BF16);
    add_half_direct<TF16>(out, K_F16);
}

template <class DT>
static void add_half_late(std::vector<KernelCfg> &out, int kclass)
{
    add_direct<DT, 256, 256, 2, 4, 2, false, 128, true>(out, kclass);
    add_direct<DT, 256, 256, 2, 2, 2, false, 128, true>(out, kclass);
    add_direct<DT, 256, 128, 2, 2, 3, false, 128, true>(out, kclass);
}

// Registered after every other family (configuration numbers above stay):
// each stage's last MFMAs deferred past the next barrier (64-byte stages are
// a single fragment chunk: nothing to overlap with).
void register_direct_half_late(std::vector<KernelCfg> &out)
{
    add_half_late<TBF16>(out, K_BF16);
    add_half_late<TF16>(out, K_F16);
}
}  // namespace mg
