// Grouped persistent kernels of the split family (see grouped.hpp). Full
// kernel: shape 0 is a 64x64 tile with element-wise variants for unaligned
// operands, shape 1 a 128x64 tile; shape 2 is the six-term split at 64x64;
// all four transpositions. Lean kernel ('N','N', aligned operands; the body
// is chosen per problem): the split product on direct-staged FP32 panels:
// three terms at 128x128, 64x64, 64x128 and 128x64, and the six-term form at
// 64x64 (k < 64).
#include "grouped.hpp"

namespace mg {
GroupedFamily grouped_family_split()
{
    return make_family<Shape<TSplit<2>, 64, 64, 2>, Shape<TSplit<2>, 128, 64, 2>, Shape<TSplit<3>, 64, 64, 1>, 1,
                       LeanBodies<2, SDShape<2, 128, 128, 2>, SDShape<3, 64, 64, 2>, SDShape<2, 64, 64, 2>,
                                  SDShape<2, 64, 128, 2>, SDShape<2, 128, 64, 2>>>();
}
}  // namespace mg
