// Grouped persistent kernels of the split family (see grouped.hpp).
// Full kernel: shape 0 is a 64x64 tile with element-wise variants for
// unaligned operands, shape 1 a 128x64 tile; shape 2 is the six-term split at 64x64; all four
// transpositions.  Lean kernel: the split product on direct-staged FP32 panels, 128x128
// (plus the six-term form at 64x64 for k < 64), two workgroups per CU.
#include "grouped.hpp"

namespace mg {
GroupedFamily grouped_family_split()
{
    return make_family<Shape<TSplit<2>, 64, 64, 2>, Shape<TSplit<2>, 128, 64, 2>, Shape<TSplit<3>, 64, 64, 1>, 1,
                       SDShape<2, 128, 128, 2>, SDShape<3, 64, 64, 2>, 2>();
}
}  // namespace mg
