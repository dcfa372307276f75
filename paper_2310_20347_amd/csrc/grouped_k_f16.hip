// Grouped persistent kernel of the f16 family (see grouped.hpp).  Shape 0 is
// a 64x64 tile with element-wise variants for unaligned operands, shape 1 a
// 128x128 tile.
#include "grouped.hpp"

namespace mg {
GroupedFamily grouped_family_f16()
{
    return make_family<Shape<TF16, 64, 64, 2>, Shape<TF16, 128, 128, 2>, NoShape>();
}
}  // namespace mg
