// FP64 family (the paper's double-precision routine).  Direct-staged tiles
// with the FP64 MFMA (v_mfma_f64_16x16x4f64: 16 values of k per 128-byte
// stage), and, as configuration 0, an element-wise LDS-tiled kernel on the
// vector ALUs for operands the direct loads cannot take (any alignment and
// leading dimension).
#include "instantiate.hpp"

namespace mg {
namespace {

// A 64x64 tile per workgroup of 16x16 threads, 4x4 outputs per thread; k in
// slices of 16 staged through LDS with element-wise loads (zero outside the
// operands), FP64 fused multiply-adds in k order.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_f64_simple_kernel(GemmArgs p)
{
    __shared__ double As[16][65], Bs[16][65];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    int tm, tn;
    raster((int)blockIdx.x, p.tiles_m, p.tiles_n, p.order, p.group, tm, tn);
    const int m0 = tm * 64, n0 = tn * 64;
    const double *A = (const double *)p.A, *B = (const double *)p.B;
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
    const int kend = alpha_nonzero<TF64>(p) ? p.k : 0;
    for (int k0 = 0; k0 < kend; k0 += 16) {
        for (int e = tid; e < 1024; e += 256) {
            // op(A)[m0 + i][k0 + kk], consecutive threads along A's contiguous index
            const int i = TA ? (e & 63) : (e >> 4), kk = TA ? (e >> 6) : (e & 15);
            const int gi = m0 + i, gk = k0 + kk;
            As[kk][i] = (gi < p.m && gk < p.k) ? (TA ? A[(int64_t)gk * p.lda + gi]
                                                     : A[(int64_t)gi * p.lda + gk])
                                               : 0.0;
            // op(B)[k0 + kb][n0 + j]
            const int j = TB ? (e >> 4) : (e & 63), kb = TB ? (e & 15) : (e >> 6);
            const int gj = n0 + j, gkb = k0 + kb;
            Bs[kb][j] = (gj < p.n && gkb < p.k) ? (TB ? B[(int64_t)gj * p.ldb + gkb]
                                                      : B[(int64_t)gkb * p.ldb + gj])
                                                : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = __builtin_fma(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int row = m0 + ty * 4 + r, col = n0 + tx * 4 + c;
            if (row < p.m && col < p.n) {
                double *cp = (double *)p.C + (int64_t)row * p.ldc + col;
                double v = p.dalpha * acc[r][c];
                if (p.dbeta != 0.0) v = __builtin_fma(p.dbeta, *cp, v);
                *cp = v;
            }
        }
}

template <bool TA, bool TB>
void fill_simple(KernelCfg &c)
{
    c.func[2 * TA + TB][0] = (const void *)&gemm_f64_simple_kernel<TA, TB>;
    c.func[2 * TA + TB][1] = (const void *)&gemm_f64_simple_kernel<TA, TB>;
}

}  // namespace

void register_f64(std::vector<KernelCfg> &out)
{
    KernelCfg c;
    c.kclass = K_F64;
    c.mc = 64;
    c.nc = 64;
    c.kc = 16;
    c.wm = 16;   // thread grid: 4x4 outputs per thread
    c.wn = 16;
    c.threads = 256;
    c.lds = 2 * 16 * 65 * 8;
    c.stages = 1;
    c.kind = 0;
    fill_simple<false, false>(c);
    fill_simple<false, true>(c);
    fill_simple<true, false>(c);
    fill_simple<true, true>(c);
    out.push_back(c);
    add_direct<TF64, 128, 128, 2, 2, 2>(out, K_F64);
    add_direct<TF64, 128, 128, 2, 2, 4>(out, K_F64);
    add_direct<TF64, 64, 64, 2, 2, 2>(out, K_F64);
    add_direct<TF64, 64, 64, 2, 2, 4>(out, K_F64);
    add_direct<TF64, 128, 64, 2, 2, 2>(out, K_F64);
    add_direct<TF64, 64, 128, 2, 2, 2>(out, K_F64);
    add_direct<TF64, 64, 64, 2, 2, 3>(out, K_F64);
}

// Registered after every other family, so the configuration numbers above
// (and the tuning tables that name them) stay as they were: each stage's last
// MFMAs deferred past the next barrier (a stage holds 16 values of k, so the
// barrier and the first fragment reads weigh more than in the 16-bit tiles).
void register_f64_late(std::vector<KernelCfg> &out)
{
    add_direct<TF64, 64, 64, 2, 2, 2, false, 128, true>(out, K_F64);
    add_direct<TF64, 64, 64, 2, 2, 3, false, 128, true>(out, K_F64);
    add_direct<TF64, 128, 64, 2, 2, 2, false, 128, true>(out, K_F64);
    add_direct<TF64, 128, 128, 2, 2, 2, false, 128, true>(out, K_F64);
}

}  // namespace mg
