// Grouped persistent kernels of the f32 family (see grouped.hpp). Full
// kernel: shape 0 is a 64x64 tile with element-wise variants for unaligned
// operands, shape 1 a 128x64 tile; all four transpositions. Lean kernel
// ('N','N', aligned operands; the body is chosen per problem): direct-staged
// 128x128, 64x64, 64x128 and 128x64.
#include "grouped.hpp"

namespace mg {
GroupedFamily grouped_family_f32()
{
    return make_family<Shape<TF32, 64, 64, 2>, Shape<TF32, 128, 64, 2>, NoShape, 2,
                       LeanBodies<2, DShape<TF32, 128, 128, 2>, DShape<TF32, 64, 64, 2>, DShape<TF32, 64, 128, 2>,
                                  DShape<TF32, 128, 64, 2>>>();
}
}  // namespace mg
