// Grouped persistent kernels of the f8 family (see grouped.hpp). Full kernel:
// shape 0 is a 64x64 tile with element-wise variants for unaligned operands,
// shape 1 a 128x64 tile; all four transpositions. Lean kernel ('N','N',
// aligned operands; the body is chosen per problem): direct-staged 128x128
// and 64x128 (an 8-bit B panel is stored n-contiguous, so its tile is at
// least 128 wide).
#include "grouped.hpp"

namespace mg {
GroupedFamily grouped_family_f8()
{
    return make_family<Shape<TF8, 64, 64, 2>, Shape<TF8, 128, 64, 2>, NoShape, 1,
                       LeanBodies<2, DShape<TF8, 128, 128, 2>, DShape<TF8, 64, 128, 2>>>();
}
}  // namespace mg
