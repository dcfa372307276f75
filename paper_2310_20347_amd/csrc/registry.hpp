// Registry of the compiled kernel family: one entry per (kernel dtype class,
// tile configuration), each holding launchers for the four transposition
// combinations and for the vectorised / element-wise staging variants.
//
// The family mirrors the paper's generator parameters (section 5,
// "P0. Parameter list": m, n, k, mc, nc, kc, mr, nr, lanesize, dtype): here a
// configuration fixes mc x nc (workgroup tile), the wave grid (hence the
// micro-tile mr x nr), kc (one 128-byte LDS row per operand row) and the
// number of LDS stages; the loop-order variant is a launch-time argument.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "device.hpp"

namespace mg {

// Kernel dtype classes (the ABI's split dtype maps to SPLIT2 or SPLIT3).
enum KClass { K_F32 = 0, K_SPLIT2, K_SPLIT3, K_BF16, K_F16, K_F8, K_I8, K_F64, K_I16, K_I32, K_NUM };

struct KernelCfg {
    int kclass = 0;
    int mc = 0, nc = 0, kc = 0;
    int wm = 0, wn = 0;     // waves along m and n
    int threads = 0;
    int lds = 0;            // bytes of LDS per workgroup
    int stages = 0;
    int kind = 0;           // 0: C resident; 1..4: operand resident; 5: packed split; 6: split-K;
                            // 7: digit products (INT16 / INT32 on the INT8 tiles)
    bool direct = false;    // stages fed by direct global -> LDS loads
    int mfma = 16;          // MFMA block of the wave tile: 16 (16x16 MFMAs) or 32 (32x32)
    int packed = -1;        // packed split: registry index of the bf16 tile run on the packed operands
    int base = -1;          // split-K: registry index of the tile it slices
    int unpacked = 0;       // packing configuration: bit 0 A, bit 1 B loaded straight to registers
    // kernel entry per [trans index = 2*transA + transB][vectorised staging]
    const void *func[4][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr},
                              {nullptr, nullptr}};
    // split-K form of the same tile (k sliced over workgroups, partial tiles
    // to a workspace, then an ordered reduction); null when not compiled
    const void *splitk[4][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr},
                                {nullptr, nullptr}};
};

// Each instantiation unit appends its configurations.
void register_f32(std::vector<KernelCfg> &out);
void register_split(std::vector<KernelCfg> &out);
void register_half(std::vector<KernelCfg> &out);
void register_byte(std::vector<KernelCfg> &out);
void register_resident_f32(std::vector<KernelCfg> &out);
void register_resident_split(std::vector<KernelCfg> &out);
void register_resident_half(std::vector<KernelCfg> &out);
void register_resident_byte(std::vector<KernelCfg> &out);
void register_direct_f32(std::vector<KernelCfg> &out);
// appended after every family, so earlier configuration numbers stay
void register_direct_f32_late(std::vector<KernelCfg> &out);
void register_direct_half_late(std::vector<KernelCfg> &out);
void register_direct_byte_late(std::vector<KernelCfg> &out);
void register_f64_late(std::vector<KernelCfg> &out);
void register_int_late(std::vector<KernelCfg> &out);
void register_direct_w32_late(std::vector<KernelCfg> &out);
void register_direct_deep_late(std::vector<KernelCfg> &out);
void register_direct_half(std::vector<KernelCfg> &out);
void register_direct_byte(std::vector<KernelCfg> &out);
void register_nopack(std::vector<KernelCfg> &out);
void register_splitdirect(std::vector<KernelCfg> &out);
void register_f64(std::vector<KernelCfg> &out);

// Plain C = beta * C (alpha == 0 or k == 0); elem: 0 float, 1 int32, 2 double.
void launch_scale(void *C, int64_t ldc, int m, int n, double beta, int elem, hipStream_t s);

// Debug mode: fill the m x n block of C with the sentinel (es: element bytes,
// 4 or 8), and add the number of sentinel elements of the block to *count.
void launch_debug_fill(void *C, int64_t ldc, int64_t m, int64_t n, int es, hipStream_t s);
void launch_debug_count(const void *C, int64_t ldc, int64_t m, int64_t n, int es,
                        unsigned long long *count, hipStream_t s);

// Split-K reduction: C = alpha * sum_{s < S} P[s] + beta * C, slices summed in
// order (P: S partial m x n tiles, row stride n, float or int32).
void launch_splitk_reduce(const void *P, int S, void *C, int64_t ldc, int m, int n,
                          const GemmArgs &a, bool is_int, hipStream_t s);

}  // namespace mg
