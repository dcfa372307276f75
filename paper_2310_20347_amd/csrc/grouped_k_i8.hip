// Grouped persistent kernels of the i8 family (see grouped.hpp). Full kernel:
// shape 0 is a 64x64 tile with element-wise variants for unaligned operands,
// shape 1 a 128x64 tile; all four transpositions. Lean kernel ('N','N',
// aligned operands; the body is chosen per problem): direct-staged 128x128
// and 256x128 (64-byte stages).  Measured on the 512-GEMM batch (m, n, k
// log-uniform on [16, 4096]): one launch takes 0.735 ms with the 128x128 body
// alone, 0.727 ms with these two, 0.728 ms with 128x128 and 64x128, and 0.77
// ms with four bodies (adding 64x128 and 32x128; the kernel's code is then
// four times the one-body kernel's).  (An 8-bit B panel is stored
// n-contiguous, so its tile is at least 128 wide.)
#include "grouped.hpp"

namespace mg {
GroupedFamily grouped_family_i8()
{
    return make_family<Shape<TI8, 64, 64, 2>, Shape<TI8, 128, 64, 2>, NoShape, 1,
                       LeanBodies<2, DShape<TI8, 128, 128, 2>, DShape<TI8, 256, 128, 2, 64>>>();
}
}  // namespace mg
