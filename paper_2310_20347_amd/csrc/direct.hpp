// Direct-staged tile: the packing step (section 5.3) done by the memory
// system.  On gfx950 a global load can write its 16 bytes per lane straight
// into LDS (lane l -> LDS base + 16*l of a 1 KiB block), so a stage of the
// A and B panels costs no VGPRs and no LDS store instructions, and a ring of
// NS stage buffers keeps NS-1 stages of loads in flight while one stage is
// multiplied: the prefetching of section 6.2 with a depth set by LDS size
// instead of register count.
//
// Used for the input formats that the MFMA consumes as stored (fp32, bf16,
// fp16, fp8, int8).  The XOR swizzle of the panels is applied on the global side:
// each lane fetches the vector that belongs at the LDS slot it writes.
//
// Panel layouts (one stage, KB = 128 or 64 bytes of k per panel row):
//   k-contiguous operand (A 'N', B 'T'): rows of m (or n), KB bytes each,
//     16-byte chunks swizzled (kslot); fragments are read with ds_read_b128.
//   m/n-contiguous operand (A 'T', B 'N'): kc rows of k, each holding the
//     panel's m (or n) values, chunks swizzled (mn_chunk); fragments are read
//     with the gfx950 transposing LDS reads (ds_read_b64_tr_b16 / _b8; lane
//     mapping at read_frag_tr).
// 64-byte stages halve the LDS of a stage, so the same LDS holds a ring
// twice as deep: more loads in flight for the MFMA-dense 16- and 8-bit
// types, whose 128-byte stage is consumed in about a microsecond.
//
// Edges: a lane whose vector lies wholly outside the operand reads a zero
// vector instead; a vector that starts inside and ends outside is read whole
// (it cannot cross a page: it is 16-byte aligned and its first byte is
// valid).  Its out-of-range part only reaches discarded outputs when it runs
// past m or n; when it runs past k (a k-contiguous operand with k not a
// multiple of the vector) the last stage zeroes it in LDS before use.
#pragma once

#include <limits.h>

#include "tile.hpp"

namespace mg {

typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) char lds_char;
typedef __attribute__((address_space(3))) i16x4 lds_i16x4;
typedef __attribute__((address_space(3))) i32x2 lds_i32x2;

// Thirty-two zero bytes: the source of every vector outside the operand.
static __device__ __attribute__((aligned(16))) u32 g_zero_vec[8];

// One direct global -> LDS load of 16 bytes per lane into the 1 KiB LDS
// block at `lds_block` (M0 holds its LDS address).  Written as an asm
// statement rather than the compiler builtin: the compiler does not track
// which LDS bytes a builtin direct load writes, so it would wait for every
// load in flight before each transposing LDS read, which defeats the stage
// ring.  The statement has no register outputs (the data goes to LDS); the
// ordering against LDS reads is explicit here: wait_vm + s_barrier before a
// stage is read, and wait_vm<0> before the LDS is reused or released.
__device__ __forceinline__ void dma16(const void *src, char *lds_block)
{
    const u32 m0 = (u32)(uintptr_t)(lds_char *)lds_block;
    asm volatile("global_load_lds_dwordx4 %0, off" : : "v"(src), "{m0}"(m0) : "memory");
}

// Wait until at most N of this wave's vector-memory operations (direct loads
// included) are outstanding.
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit counter");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Chunk swizzle of an m/n-contiguous panel: the physical 16-byte chunk of
// logical chunk lc in k row kr (RB-byte rows).  gfx950's LDS has 64 banks
// (256 bytes per line).  A 32-bit read serves 32 lanes per pass; a
// transposing 64-bit read serves two 16-lane groups per pass, so the rows
// read by lane groups g and g+1 must fill the two 128-byte halves of a bank
// line without overlap (measured: with only the 16-lane groups spread, half
// of the LDS cycles of those reads were bank conflicts).
//   SK 4: FP32 MFMA fragment, 32-bit reads; group g reads 64 bytes of row 4g+d.
//   SK 8: FP32 read of the split product; group g reads 64 bytes of row 8g+e.
//   SK 9: FP64 MFMA fragment, 64-bit reads; group g reads 128 bytes of row
//         2g+e, so the pair served together reads rows kr and kr+2 (rows of
//         512 bytes or more: row bit 1 picks the half line).
//   SK 2: 16-bit transposing read; group g reads 4 rows (8g + 4h + 0..3) of
//         32 bytes, groups GS = 8 rows apart.
//   SK 1: 8-bit transposing read; group g reads 8 rows (GS*g + 8h + 0..7) of
//         16 bytes, groups GS = KF/4 rows apart.
// Rows of 256 bytes or more start on a bank line, so the 128-byte half is
// chunk bit 3 and the swizzle may flip it; 128-byte rows share a line with
// their neighbour (row parity picks the half) and are spread within it.
//   SK 66: 16-bit transposing read of the 32x32 MFMAs: the two 16-lane groups
//          served together read the same 4 k rows (kr0 .. kr0+3), 64 bytes of
//          each, so each row's 64 bytes take their own quarter of the bank
//          line (rows of 256 bytes or more) or of the row's half line.
//   SK 65: 8-bit transposing read of the 32x32 MFMAs: the pair reads 8 k rows
//          of 32 bytes each, spread over the eighths of the bank line (or of
//          the half line).
template <int SK, int RB, int GS>
__device__ __forceinline__ int mn_chunk(int kr, int lc)
{
    static_assert((GS & (GS - 1)) == 0 && RB >= 128, "power-of-two group stride, rows >= 128 B");
    int x, mask = 7;
    if constexpr (SK == 66) {
        if constexpr (RB >= 256) {
            x = 4 * (kr & 3);
            mask = 15;
        } else {
            x = 4 * ((kr >> 1) & 1);
        }
    } else if constexpr (SK == 65) {
        if constexpr (RB >= 256) {
            x = 2 * (kr & 7);
            mask = 15;
        } else {
            x = 2 * ((kr >> 1) & 3);
        }
    } else if constexpr (SK == 9) {
        static_assert(RB >= 256, "FP64 panels have rows of 256 bytes or more");
        x = 8 * ((kr >> 1) & 1);
        mask = 15;
    } else if constexpr (SK == 8) {
        x = 4 * ((kr >> 3) & 1);
    } else if constexpr (SK == 4) {
        x = 4 * ((kr >> 2) & 1);
    } else if constexpr (SK == 2) {
        if constexpr (RB >= 256) {
            x = 2 * (kr & 3) | 8 * ((kr / GS) & 1);
            mask = 15;
        } else {
            x = 2 * (((kr >> 1) & 1) | (((kr / GS) & 1) << 1));
        }
    } else {
        if constexpr (RB >= 256) {
            x = (kr & 7) | 8 * ((kr / GS) & 1);
            mask = 15;
        } else {
            x = ((kr >> 1) & 3) | (((kr / GS) & 1) << 2);
        }
    }
    return (lc & ~mask) | ((lc ^ x) & mask);
}

template <int SK, int RB, int GS>
__device__ __forceinline__ int mn_off(int kr, int byte)
{
    return kr * RB + (mn_chunk<SK, RB, GS>(kr, byte >> 4) << 4) + (byte & 15);
}

// Chunk swizzle of a k-contiguous panel with KB-byte rows (KB = 128: 8
// chunks; 64: 4 chunks): physical slot of logical chunk lc in row r.  A
// 128-bit read serves 16 lanes per pass, rows r0..r0+7 of two lane groups
// whose logical chunks differ by 1 (16- and 32-bit and INT8 fragments) or 2
// (FP8 fragments, the split product's 32-byte reads).
//   KB 128: two rows per 256-byte bank line, so the four even rows of a
//     pass share one half line.  Their swizzles are {0, 3, 5, 6} (odd rows:
//     {1, 2, 4, 7}); either set XOR 1 or 2 is the other set, so the two
//     groups' chunks fill the half line exactly once.
//   KB 64: four rows per line, rows r and r+4 share a quarter line; their
//     swizzles differ by 3, so {c, c^3, c^1, c^2} (or c^2, c^1) are distinct.
//   R32 (the 32x32 MFMAs' fragments, KB 128): a pass reads rows r0 .. r0+7
//     and r0+16 .. r0+23 at the same logical chunk; rows 16 apart share a
//     half line, so bit 4 of the row flips the set ({0, 3, 5, 6} <-> {1, 2,
//     4, 7}).  Passes of the 16-row pattern read 8 rows that agree in bit 4,
//     so they stay conflict-free.
template <int KB, bool R32 = false>
__device__ __forceinline__ int kslot(int r, int lc)
{
    static_assert(!R32 || KB == 128, "32-row fragments use 128-byte rows");
    if constexpr (KB == 128)
        return lc ^ ((r & 7) ^ (((r >> 1) ^ (r >> 2)) & 1)) ^ (R32 ? ((r >> 4) & 1) : 0);
    else
        return lc ^ (3 * ((r >> 2) & 1));
}

template <int KB, bool R32 = false>
__device__ __forceinline__ int k_off(int row, int byte)
{
    return row * KB + (kslot<KB, R32>(row, byte >> 4) << 4) + (byte & 15);
}

// Fragment of the 16-row block at panel row r0 and chunk c of a k-contiguous
// panel: lane l holds row r0 + l%16, k = c*KF + (l/16)*KF/4 .. +KF/4-1.
template <class DT, int KB>
__device__ __forceinline__ void read_frag_k(const char *panel, int r0, int c, int lane,
                                            u32 (*f)[DT::FDW])
{
    const int r = r0 + (lane & 15);
    const int byte = c * (DT::KF * DT::LES) + (lane >> 4) * (DT::FDW * 4);
#pragma unroll
    for (int h = 0; h < DT::FDW / 4; ++h) {
        const u32x4 v = *(const u32x4 *)(panel + k_off<KB>(r, byte + 16 * h));
#pragma unroll
        for (int d = 0; d < 4; ++d) f[0][4 * h + d] = v[d];
    }
}

// Fragment of the 32-row block at panel row r0 and MFMA chunk c of a
// k-contiguous panel, for the 32x32 MFMAs: lane l holds row r0 + l%32 and
// the FDW*4 bytes of k that start at chunk c's lane half l/32.
template <class DT, int KB>
__device__ __forceinline__ void read_frag_k32(const char *panel, int r0, int c, int lane,
                                              u32 (*f)[DT::FDW])
{
    const int r = r0 + (lane & 31);
    const int byte = c * (2 * DT::FDW * 4) + (lane >> 5) * (DT::FDW * 4);
#pragma unroll
    for (int h = 0; h < DT::FDW / 4; ++h) {
        const u32x4 v = *(const u32x4 *)(panel + k_off<KB, true>(r, byte + 16 * h));
#pragma unroll
        for (int d = 0; d < 4; ++d) f[0][4 * h + d] = v[d];
    }
}

// ---------------------------------------------------------------------------
// One operand panel of a stage: ROWS rows of m (or n) x KC values of k
// (KB bytes of k per row), ROWS*KB/1024 blocks of 1 KiB, PER blocks loaded
// by each of NW waves.
// ---------------------------------------------------------------------------
template <class DT, int ROWS, int NW, bool KMODE, int SK = DT::GES, int KB = 128, bool R32 = false>
struct DPanel {
    static constexpr int GES = DT::GES, KC = KB / GES, VK = 16 / GES;
    static constexpr int NB = ROWS * KB / 1024; // 1 KiB blocks per panel
    static constexpr int CPK = KB / 16;         // k mode: chunks per row
    static constexpr int PER = NB / NW;         // blocks per wave
    static constexpr int RB = ROWS * GES;       // m/n mode: bytes per k row
    static constexpr int CPR = RB / 16;         // m/n mode: chunks per k row
    static constexpr int GS = GES == 1 ? DT::KF / 4 : 8;   // m/n mode: rows between lane groups
    static_assert(NB % NW == 0, "panel blocks must divide among the waves");
    static_assert(KMODE || (RB >= 128 && 64 % CPR == 0), "m/n panel rows of 128..1024 bytes");

    int64_t off[PER];   // lane's byte offset in the operand for the stage at k0 = 0
    int lim[PER];       // the lane's vector is inside the operand iff k0 < lim

    __device__ __forceinline__ void init(int64_t ld, int row0, int R, int K, int wave, int lane)
    {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int b = wave * PER + q;
            if constexpr (KMODE) {
                const int r = (64 / CPK) * b + lane / CPK;
                const int lc = kslot<KB, R32>(r, lane % CPK);
                const int grow = row0 + r, kof = lc * VK;
                off[q] = ((int64_t)grow * ld + kof) * GES;
                lim[q] = grow < R ? K - kof : INT_MIN;
            } else {
                const int kr = (64 / CPR) * b + lane / CPR, pc = lane % CPR;
                const int lc = mn_chunk<SK, RB, GS>(kr, pc);
                const int gcol = row0 + lc * VK;
                off[q] = ((int64_t)kr * ld + gcol) * GES;
                lim[q] = gcol < R ? K - kr : INT_MIN;
            }
        }
    }

    // Issue this wave's loads of the stage starting at k0 into `panel`.
    __device__ __forceinline__ void issue(const char *X, int64_t ld, int k0, char *panel,
                                          int wave) const
    {
        const int64_t kstep = KMODE ? (int64_t)k0 * GES : (int64_t)k0 * ld * GES;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const char *src = k0 < lim[q] ? X + off[q] + kstep : (const char *)g_zero_vec;
            dma16(src, panel + (wave * PER + q) * 1024);
        }
    }

    // k-contiguous panel of the last stage, K - k0 values valid with the
    // chunk at K straddling: zero its values at k >= K.
    static __device__ __forceinline__ void fix_tail(char *panel, int valid_k, int tid, int nt)
    {
        const int lc = valid_k / VK;
        const int keep = (valid_k % VK) * GES;   // bytes of the chunk to keep, 1..15
        for (int r = tid; r < ROWS; r += nt) {
            u32x4 *p = (u32x4 *)(panel + k_off<KB, R32>(r, lc * 16));
            u32x4 v = *p;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int nb = keep - 4 * d;
                const u32 mask = nb >= 4 ? 0xFFFFFFFFu : (nb <= 0 ? 0u : (1u << (8 * nb)) - 1u);
                v[d] &= mask;
            }
            *p = v;
        }
    }
};

// Fragment of the 16-row block at panel offset r0 (m or n) and chunk c of an
// m/n-contiguous panel, in the same per-lane k assignment as read_frag: lane
// group g holds k = c*KF + g*KF/4 .. +KF/4-1, in order.  Lane mapping of a
// transposing read (measured on gfx950): every lane addresses an 8-byte
// segment of E elements (E = 4 for 16-bit, 8 for 8-bit); within each group of
// 16 lanes, value j (j < E) returned to lane i is element i mod E of the
// segment addressed by lane (16/E)*j + i/E.  So lanes (16/E)*j .. +16/E-1
// address consecutive segments of k row j, and lane i receives column i of
// E consecutive k rows.  FP32 has no transposing read: one 32-bit read per k
// row (a 16-lane group reads 64 contiguous bytes of one row; the row swizzle
// puts the two groups served together on different banks).
template <class DT, int ROWS>
__device__ __forceinline__ void read_frag_tr(const char *panel, int r0, int c, int lane,
                                             u32 (*f)[DT::FDW])
{
    constexpr int GES = DT::GES, RB = ROWS * GES;
    const int g = lane >> 4, s = lane & 15;
    if constexpr (GES == 4) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int kr = c * DT::KF + 4 * g + d;
            f[0][d] = *(const u32 *)(panel + mn_off<4, RB, 8>(kr, (r0 + s) * 4));
        }
    } else if constexpr (GES == 8) {
        // FP64: lane group g holds k rows c*KF + 2g and 2g+1, one 64-bit read each
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int kr = c * DT::KF + 2 * g + e;
            const u32x2 v = *(const u32x2 *)(panel + mn_off<9, RB, 8>(kr, (r0 + s) * 8));
            f[0][2 * e] = v[0];
            f[0][2 * e + 1] = v[1];
        }
    } else if constexpr (GES == 2) {
        // two reads of 4 k values: lane s addresses k row 4h + s/4, elements 4*(s%4)..+3
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int kr = c * DT::KF + 8 * g + 4 * h + (s >> 2);
            const int byte = (r0 + 4 * (s & 3)) * 2;
            const i16x4 v =
                __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4 *)(panel + mn_off<2, RB, 8>(kr, byte)));
            const u32x2 w = __builtin_bit_cast(u32x2, v);
            f[0][2 * h] = w[0];
            f[0][2 * h + 1] = w[1];
        }
    } else {
        // KF/32 reads of 8 k values: lane s addresses k row 8h + s/2, bytes 8*(s%2)..+7
#pragma unroll
        for (int h = 0; h < DT::KF / 32; ++h) {
            const int kr = c * DT::KF + (DT::KF / 4) * g + 8 * h + (s >> 1);
            const int byte = r0 + 8 * (s & 1);
            const i32x2 v =
                __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_i32x2 *)(panel + mn_off<1, RB, DT::KF / 4>(kr, byte)));
            f[0][2 * h] = (u32)v[0];
            f[0][2 * h + 1] = (u32)v[1];
        }
    }
}

// Fragment of the 32-column block at panel offset r0 (m or n) and MFMA chunk
// c of an m/n-contiguous panel, for the 32x32 MFMAs: lane l holds column
// r0 + l%32 and the k values of chunk c's lane half l/32, in order.  Each
// 16-lane group q reads 16 columns (r0 + 16 (q%2) ..) of its k rows with the
// transposing reads (lane mapping at read_frag_tr): 16-bit, two reads of 4 k
// rows; 8-bit, FDW/2 reads of 8 k rows.
template <class DT, int ROWS>
__device__ __forceinline__ void read_frag_tr32(const char *panel, int r0, int c, int lane,
                                               u32 (*f)[DT::FDW])
{
    constexpr int GES = DT::GES, RB = ROWS * GES, KF32 = DT::KF / 2;
    const int q = lane >> 4, s = lane & 15;
    const int col0 = r0 + 16 * (q & 1);
    if constexpr (GES == 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int kr = c * KF32 + 8 * (q >> 1) + 4 * h + (s >> 2);
            const int byte = (col0 + 4 * (s & 3)) * 2;
            const i16x4 v =
                __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4 *)(panel + mn_off<66, RB, 8>(kr, byte)));
            const u32x2 w = __builtin_bit_cast(u32x2, v);
            f[0][2 * h] = w[0];
            f[0][2 * h + 1] = w[1];
        }
    } else {
        static_assert(GES == 1, "transposing 32-column reads of 8- and 16-bit panels");
#pragma unroll
        for (int h = 0; h < DT::FDW / 2; ++h) {
            const int kr = c * KF32 + (KF32 / 2) * (q >> 1) + 8 * h + (s >> 1);
            const int byte = col0 + 8 * (s & 1);
            const i32x2 v =
                __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_i32x2 *)(panel + mn_off<65, RB, 8>(kr, byte)));
            f[0][2 * h] = (u32)v[0];
            f[0][2 * h + 1] = (u32)v[1];
        }
    }
}

// 32x32 MFMA accumulators: 16 values per lane; register r of lane l holds
// row 8 (r/4) + 4 (l/32) + r%4 and column l%32 of the block.
template <class DT>
struct Acc32Of {
    typedef f32x16 type;
};
template <>
struct Acc32Of<TI8> {
    typedef i32x16 type;
};

// One 32x32 MFMA step over fragments of KF/2 values of k per lane half
// (sub-step s of Sub<DT>: FP32 takes one value per lane and step).
template <class DT>
__device__ __forceinline__ void mma32(typename Acc32Of<DT>::type &acc, const u32 (*a)[DT::FDW],
                                      const u32 (*b)[DT::FDW], int s)
{
    if constexpr (DT::GES == 4 && !DT::SPLIT) {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(float, a[0][s]),
                                                   __builtin_bit_cast(float, b[0][s]), acc, 0, 0, 0);
    } else if constexpr (DT::GES == 2) {
        u32x4 xv = {a[0][0], a[0][1], a[0][2], a[0][3]}, yv = {b[0][0], b[0][1], b[0][2], b[0][3]};
        if constexpr (DT::HALF)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, xv),
                                                         __builtin_bit_cast(f16x8, yv), acc, 0, 0, 0);
        else
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, xv),
                                                          __builtin_bit_cast(bf16x8, yv), acc, 0, 0, 0);
    } else if constexpr (DT::INT) {
        i32x4 xv = {(int)a[0][0], (int)a[0][1], (int)a[0][2], (int)a[0][3]};
        i32x4 yv = {(int)b[0][0], (int)b[0][1], (int)b[0][2], (int)b[0][3]};
        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(xv, yv, acc, 0, 0, 0);
    } else {
        static_assert(DT::GES == 1 && DT::FDW == 8, "FP8: 32 bytes of k per lane");
        i32x8 xv, yv;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            xv[d] = (int)a[0][d];
            yv[d] = (int)b[0][d];
        }
        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(xv, yv, acc, 0, 0, 0, 127, 0, 127);
    }
}

template <class DT, int FM, int FN>
__device__ __forceinline__ void store_c32(const GemmArgs &p, const typename Acc32Of<DT>::type (*acc)[FN],
                                          int r0, int c0, int lane)
{
    typedef typename std::conditional<DT::INT, int, float>::type CT;
    const int col_l = lane & 31, row_l = 4 * (lane >> 5);
    const bool read_c = DT::INT ? p.ibeta != 0 : p.beta != 0.0f;
    CT *const C = (CT *)p.C;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            // the block's C values are all read before any is written (as in store_c)
            CT cv[16];
            if (read_c) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = r0 + 32 * i + 8 * (r >> 2) + row_l + (r & 3);
                    const int col = c0 + 32 * j + col_l;
                    cv[r] = row < p.m && col < p.n ? C[(int64_t)row * p.ldc + col] : CT(0);
                }
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = r0 + 32 * i + 8 * (r >> 2) + row_l + (r & 3);
                const int col = c0 + 32 * j + col_l;
                if (row < p.m && col < p.n) {
                    CT *c = C + (int64_t)row * p.ldc + col;
                    if constexpr (DT::INT) {
                        u32 v = (u32)p.ialpha * (u32)acc[i][j][r];
                        if (read_c) v += (u32)p.ibeta * (u32)cv[r];
                        *c = (int)v;
                    } else {
                        float v = p.alpha * acc[i][j][r];
                        if (read_c) v = __builtin_fmaf(p.beta, cv[r], v);
                        *c = v;
                    }
                }
            }
        }
}

// ---------------------------------------------------------------------------
// The direct-staged tile: C[m0:m0+MC, n0:n0+NC] = alpha op(A) op(B) + beta C
// with an NS-deep ring of LDS stages.  Requires 16-byte aligned operands and
// leading dimensions (the vectorised case).
// ---------------------------------------------------------------------------
// OVL: the MFMAs of each stage's last fragment chunk are deferred past the
// next stage's barrier, where they run while the first fragments of that
// stage are read from LDS (otherwise every wave waits for those reads after
// each barrier with no MFMA to issue).  The deferred fragments are already in
// registers; each wave waits for its LDS reads to land before the barrier,
// so no load of the next stage can overwrite LDS that is still being read.
// MB: the MFMA block, 16 (16x16 MFMAs) or 32 (32x32 MFMAs: twice the
// multiply-adds per fragment byte read from LDS, 16 accumulators per lane
// and block; 128-byte stages, 8- and 16-bit types).
template <class DT, int MC, int NC, int WM, int WN, bool TA, bool TB, int NS, int KB = 128,
          bool OVL = false, int MB = 16>
struct DTile {
    static constexpr int NW = WM * WN, NT = 64 * NW;
    static constexpr int KC = KB / DT::GES;
    static constexpr int WTM = MC / WM, WTN = NC / WN;
    static constexpr int FM = WTM / MB, FN = WTN / MB;
    static constexpr int PANEL_A = MC * KB, PANEL_B = NC * KB;
    static constexpr int STAGE_BYTES = PANEL_A + PANEL_B;
    static constexpr int LDS_BYTES = NS * STAGE_BYTES;
    static constexpr int MINB = 1;
    static constexpr int KF = MB == 16 ? DT::KF : DT::KF / 2;   // k of one fragment chunk
    static constexpr int NCH = KC / KF;                         // fragment chunks per stage
    static constexpr bool W32 = MB == 32;
    // m/n panel read pattern (the swizzle of mn_chunk)
    static constexpr int SKX = W32 ? 64 + DT::GES : (DT::GES == 8 ? 9 : DT::GES);
    typedef DPanel<DT, MC, NW, !TA, SKX, KB, W32> PA;   // A 'N' is contiguous along k
    typedef DPanel<DT, NC, NW, TB, SKX, KB, W32> PB;    // B 'T' is contiguous along k
    static_assert(KC % KF == 0, "a stage holds whole fragments");
    static_assert(MB == 16 || (MB == 32 && KB == 128 && (DT::GES == 1 || DT::GES == 2)),
                  "32x32 MFMA tiles: 8- and 16-bit types, 128-byte stages");
    static constexpr int LOADS = PA::PER + PB::PER;
    static_assert(DT::LES == DT::GES && DT::PLANES == 1, "direct staging keeps the input format");
    static_assert(NS >= 2 && LDS_BYTES <= 160 * 1024, "LDS budget of one CU");
    static_assert((NS - 2) * LOADS < 64, "loads in flight must fit the vmcnt counter");
    static_assert(WTM % MB == 0 && WTN % MB == 0, "wave tile must be whole MFMA blocks");
    typedef typename std::conditional<W32, typename Acc32Of<DT>::type, typename AccOf<DT>::type>::type Acc;

    static __device__ __forceinline__ void read_chunk(const char *buf, int c, int wm, int wn,
                                                      int lane, u32 (*fa)[1][DT::FDW],
                                                      u32 (*fb)[1][DT::FDW])
    {
        const char *pa = buf, *pb = buf + PANEL_A;
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            if constexpr (W32) {
                if constexpr (!TA) read_frag_k32<DT, KB>(pa, wm * WTM + MB * i, c, lane, fa[i]);
                else read_frag_tr32<DT, MC>(pa, wm * WTM + MB * i, c, lane, fa[i]);
            } else {
                if constexpr (!TA) read_frag_k<DT, KB>(pa, wm * WTM + 16 * i, c, lane, fa[i]);
                else read_frag_tr<DT, MC>(pa, wm * WTM + 16 * i, c, lane, fa[i]);
            }
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            if constexpr (W32) {
                if constexpr (TB) read_frag_k32<DT, KB>(pb, wn * WTN + MB * j, c, lane, fb[j]);
                else read_frag_tr32<DT, NC>(pb, wn * WTN + MB * j, c, lane, fb[j]);
            } else {
                if constexpr (TB) read_frag_k<DT, KB>(pb, wn * WTN + 16 * j, c, lane, fb[j]);
                else read_frag_tr<DT, NC>(pb, wn * WTN + 16 * j, c, lane, fb[j]);
            }
        }
    }

    static __device__ __forceinline__ void mma(Acc &acc, const u32 (*fa)[DT::FDW],
                                               const u32 (*fb)[DT::FDW], int st)
    {
        if constexpr (W32) mma32<DT>(acc, fa, fb, st);
        else mma_step<DT>(acc, fa, fb, st);
    }

    // Scheduling hint for a chunk's fragment reads issued with the previous
    // chunk's MFMAs: alternate one LDS read with an even share of the MFMAs,
    // so the reads spread over the MFMA chain instead of bunching at its start
    // (the instruction order only; every accumulator sees the same MFMAs in
    // the same order).  Given to tiles of one wave per SIMD, which have no
    // second wave to issue MFMAs while one waits for its reads; in the 8-wave
    // tiles it gained 1-2% and made some layouts spill.
    static __device__ __forceinline__ void interleave_reads()
    {
        if constexpr (NW != 4) return;
        constexpr int RK = DT::FDW / 4 > 0 ? DT::FDW / 4 : 1;   // 128-bit reads per k-contiguous fragment
        constexpr int RT = W32 || DT::GES <= 2 ? (DT::GES == 2 ? 2 : DT::FDW / 2)
                                               : (DT::GES == 8 ? 2 : 4);   // reads per m/n fragment
        constexpr int R = FM * (TA ? RT : RK) + FN * (TB ? RK : RT);
        constexpr int M = FM * FN * Sub<DT>::value;
        constexpr int PER = M / R > 0 ? M / R : 1;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);     // one LDS read
            __builtin_amdgcn_sched_group_barrier(0x008, PER, 0);   // then PER MFMAs
        }
    }

    static __device__ __forceinline__ void mfma_chunk(Acc (*acc)[FN], const u32 (*fa)[1][DT::FDW],
                                                      const u32 (*fb)[1][DT::FDW])
    {
#pragma unroll
        for (int st = 0; st < Sub<DT>::value; ++st)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) mma(acc[i][j], fa[i], fb[j], st);
    }

    // The micro-kernel over one stage; the fragments of chunk c+1 are read
    // while the MFMAs of chunk c run.
    static __device__ __forceinline__ void compute(const char *buf, Acc (*acc)[FN], int wm, int wn,
                                                   int lane)
    {
        u32 fa[2][FM][1][DT::FDW], fb[2][FN][1][DT::FDW];
        read_chunk(buf, 0, wm, wn, lane, fa[0], fb[0]);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (c + 1 < NCH) read_chunk(buf, c + 1, wm, wn, lane, fa[(c + 1) & 1], fb[(c + 1) & 1]);
#pragma unroll
            for (int st = 0; st < Sub<DT>::value; ++st)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        mma(acc[i][j], fa[c & 1][i], fb[c & 1][j], st);
        }
    }

    static __device__ __forceinline__ void run(const GemmArgs &p, int tm, int tn, char *lds)
    {
        const int tid = threadIdx.x, lane = tid & 63;
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int wm = wave % WM, wn = wave / WM;
        const int m0 = tm * MC, n0 = tn * NC;

        Acc acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = Acc{};

        const bool form = p.k > 0 && alpha_nonzero<DT>(p);
        const int nk = form ? (p.k + KC - 1) / KC : 0;
        if (nk > 0) {
            const char *A = (const char *)p.A;
            const char *B = (const char *)p.B;
            PA pa;
            PB pb;
            pa.init(p.lda, m0, p.m, p.k, wave, lane);
            pb.init(p.ldb, n0, p.n, p.k, wave, lane);
            // stages 0 .. NS-2 in flight; stages past the end load zeros, so
            // every iteration issues the same number of loads
#pragma unroll
            for (int t = 0; t < NS - 1; ++t) {
                char *buf = lds + t * STAGE_BYTES;
                pa.issue(A, p.lda, t * KC, buf, wave);
                pb.issue(B, p.ldb, t * KC, buf + PANEL_A, wave);
            }
            const bool ragged = (!TA || TB) && (p.k % PA::VK) != 0;
            int rd = 0, wr = NS - 1;   // ring buffers: stage being read, stage being loaded
            if constexpr (OVL) {
                // Fragment buffers alternate by chunk: with an even number of
                // chunks per stage every stage starts in buffer 0 and its
                // last chunk is in buffer 1; with one chunk per stage the
                // deferred chunk is the whole previous stage, and stages
                // alternate buffers (the loop runs stages in pairs, so every
                // buffer index is a compile-time constant).
                static_assert(NCH % 2 == 0 || NCH == 1, "the deferred chunk and the next stage's "
                                                        "first chunk use different fragment buffers");
                u32 fa[2][FM][1][DT::FDW], fb[2][FN][1][DT::FDW];
                auto stage = [&](int s, auto parity) __attribute__((always_inline)) {
                    constexpr int P = decltype(parity)::value;
                    // this wave's loads of stage s have landed and its reads of
                    // stage s-1 (the deferred fragments) are in registers ...
                    __builtin_amdgcn_s_waitcnt(((NS - 2) * LOADS & 15) | (((NS - 2) * LOADS >> 4) << 14) |
                                               (7 << 4));
                    __builtin_amdgcn_s_barrier();   // ... and every wave's
                    pin_order();
                    char *cur = lds + rd * STAGE_BYTES;
                    if (ragged && s == nk - 1) {
                        const int valid_k = p.k - s * KC;
                        if constexpr (!TA) PA::fix_tail(cur, valid_k, tid, NT);
                        if constexpr (TB) PB::fix_tail(cur + PANEL_A, valid_k, tid, NT);
                        __syncthreads();
                    }
                    char *nxt = lds + wr * STAGE_BYTES;
                    pa.issue(A, p.lda, (s + NS - 1) * KC, nxt, wave);
                    pb.issue(B, p.ldb, (s + NS - 1) * KC, nxt + PANEL_A, wave);
                    pin_order();
                    read_chunk(cur, 0, wm, wn, lane, fa[P], fb[P]);
                    if (s > 0) mfma_chunk(acc, fa[1 - P], fb[1 - P]);   // stage s-1's last chunk
#pragma unroll
                    for (int c = 0; c + 1 < NCH; ++c) {
                        read_chunk(cur, c + 1, wm, wn, lane, fa[(c + 1) & 1], fb[(c + 1) & 1]);
                        mfma_chunk(acc, fa[c & 1], fb[c & 1]);
                        interleave_reads();
                    }
                    rd = rd + 1 == NS ? 0 : rd + 1;
                    wr = wr + 1 == NS ? 0 : wr + 1;
                };
                if constexpr (NCH == 1) {
                    // the first stage's parity is chosen so that the last
                    // stage is read into buffer 1
                    int s = 0;
                    if (nk & 1) stage(s++, std::integral_constant<int, 1>());
                    for (; s < nk; s += 2) {
                        stage(s, std::integral_constant<int, 0>());
                        stage(s + 1, std::integral_constant<int, 1>());
                    }
                    mfma_chunk(acc, fa[1], fb[1]);   // the last stage
                } else {
                    for (int s = 0; s < nk; ++s) stage(s, std::integral_constant<int, 0>());
                    mfma_chunk(acc, fa[1], fb[1]);   // the last stage's last chunk
                }
            } else
            for (int s = 0; s < nk; ++s) {
                wait_vm<(NS - 2) * LOADS>();   // this wave's loads of stage s have landed
                __builtin_amdgcn_s_barrier();  // ... and every wave's; stage s-1 is consumed
                pin_order();
                char *cur = lds + rd * STAGE_BYTES;
                if (ragged && s == nk - 1) {
                    const int valid_k = p.k - s * KC;
                    if constexpr (!TA) PA::fix_tail(cur, valid_k, tid, NT);
                    if constexpr (TB) PB::fix_tail(cur + PANEL_A, valid_k, tid, NT);
                    __syncthreads();
                }
                char *nxt = lds + wr * STAGE_BYTES;
                pa.issue(A, p.lda, (s + NS - 1) * KC, nxt, wave);
                pb.issue(B, p.ldb, (s + NS - 1) * KC, nxt + PANEL_A, wave);
                pin_order();
                compute(cur, acc, wm, wn, lane);
                rd = rd + 1 == NS ? 0 : rd + 1;
                wr = wr + 1 == NS ? 0 : wr + 1;
            }
            // no load may still be writing this workgroup's LDS when it is
            // reused (next tile of a persistent launch) or released
            wait_vm<0>();
            __builtin_amdgcn_s_barrier();
        }
        if constexpr (W32) store_c32<DT, FM, FN>(p, acc, m0 + wm * WTM, n0 + wn * WTN, lane);
        else if constexpr (NW == 8) store_c_batched<DT, FM, FN>(p, acc, m0 + wm * WTM, n0 + wn * WTN, lane);
        else store_c<DT, FM, FN>(p, acc, m0 + wm * WTM, n0 + wn * WTN, lane);
    }
};

// One workgroup per tile.
template <class T>
__global__ void __launch_bounds__(T::NT, T::MINB) gemm_direct_kernel(GemmArgs p)
{
    __shared__ __attribute__((aligned(16))) char lds[T::LDS_BYTES];
    const int nblocks = p.tiles_m * p.tiles_n;
    const int t = xcd_remap(blockIdx.x, nblocks);
    int tm, tn;
    raster(t, p.tiles_m, p.tiles_n, p.order, p.group, tm, tn);
    T::run(p, tm, tn, lds);
}

}  // namespace mg
