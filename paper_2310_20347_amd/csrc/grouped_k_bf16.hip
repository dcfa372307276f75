// Grouped persistent kernels of the bf16 family (see grouped.hpp).
// Full kernel: shape 0 is a 64x64 tile with element-wise variants for
// unaligned operands, shape 1 a 128x64 tile; all four
// transpositions.  Lean kernel: one 128x128 'N','N' body, direct-staged
// (global -> LDS loads into a two-stage ring).
#include "grouped.hpp"

namespace mg {
GroupedFamily grouped_family_bf16()
{
    return make_family<Shape<TBF16, 64, 64, 2>, Shape<TBF16, 128, 64, 2>, NoShape, 2,
                       DShape<TBF16, 128, 128, 2>, NoShape, 2>();
}
}  // namespace mg
