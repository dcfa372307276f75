// Grouped persistent kernel: many independent GEMMs of uneven shapes in one
// launch.  The host writes a descriptor table (one GemmArgs per problem plus
// the compiled tile body to use and the problem's first global tile id).
// Each workgroup repeatedly takes a global tile id, finds its problem by
// search over the tile prefix, maps the local id through that problem's
// raster order and runs the tile body (the same C-resident tile as the
// single-GEMM kernel).  Tile ids beyond each workgroup's first come from
// atomic counters (one per XCD group), each claimed at the start of the tile
// before it; a workgroup whose group has run out of tiles takes them from the
// other groups' counters.  The last workgroup to finish resets the counters
// to zero, so a launch leaves them ready for the next one (no memset node is
// needed, which keeps the launch capturable in a graph).
#pragma once

#include "direct.hpp"
#include "splitdirect.hpp"
#include "tile.hpp"

namespace mg {

struct GHeader {
    int count;        // problems in the table
    int total_tiles;  // sum of tiles over problems
    int family;       // dtype family the table was built for
    int ts_offset;    // byte offset of the int tile_start[count] array
    int pad[12];
};

struct GDesc {
    GemmArgs a;
    int body;         // shape * 8 + trans * 2 + vec
    int tile_start;   // first global tile id of this problem
    int pad[2];
};
static_assert(sizeof(GHeader) == 64, "header is 64 bytes");
static_assert(sizeof(GDesc) % 16 == 0, "descriptors are 16-byte aligned");

// A tile shape of a family: element type, mc x nc, LDS stages (register-
// staged tile; `run` is its 'N','N' vectorised body).
template <class DT, int MC, int NC, int ST>
struct Shape {
    typedef DT dt;
    static constexpr int mc = MC, nc = NC, st = ST;
    typedef Tile<DT, MC, NC, 2, 2, false, false, true, ST> NN;
    static constexpr int lds = NN::LDS_BYTES;
    static __device__ __forceinline__ void run(const GemmArgs &p, int tm, int tn, char *l)
    {
        NN::run(p, tm, tn, l);
    }
};
// A direct-staged 'N','N' tile shape (NS-deep LDS ring, 16-byte aligned operands).
template <class DT, int MC, int NC, int NS, int KB = 128>
struct DShape {
    typedef DT dt;
    static constexpr int mc = MC, nc = NC;
    typedef DTile<DT, MC, NC, 2, 2, false, false, NS, KB> NN;
    static constexpr int lds = NN::LDS_BYTES;
    static __device__ __forceinline__ void run(const GemmArgs &p, int tm, int tn, char *l)
    {
        NN::run(p, tm, tn, l);
    }
};
// A split-product 'N','N' tile shape on direct-staged FP32 panels.
template <int P, int MC, int NC, int NS>
struct SDShape {
    typedef TSplit<P> dt;
    static constexpr int mc = MC, nc = NC;
    typedef SDTile<P, MC, NC, 2, 2, false, false, NS> NN;
    static constexpr int lds = NN::LDS_BYTES;
    static __device__ __forceinline__ void run(const GemmArgs &p, int tm, int tn, char *l)
    {
        NN::run(p, tm, tn, l);
    }
};
struct NoShape {
    static constexpr int lds = 0;
};

template <class S, bool VEC>
__device__ __forceinline__ void run_shape(int trans, const GemmArgs &p, int tm, int tn, char *lds)
{
    typedef typename S::dt DT;
    switch (trans) {
    case 0: Tile<DT, S::mc, S::nc, 2, 2, false, false, VEC, S::st>::run(p, tm, tn, lds); break;
    case 1: Tile<DT, S::mc, S::nc, 2, 2, false, true, VEC, S::st>::run(p, tm, tn, lds); break;
    case 2: Tile<DT, S::mc, S::nc, 2, 2, true, false, VEC, S::st>::run(p, tm, tn, lds); break;
    default: Tile<DT, S::mc, S::nc, 2, 2, true, true, VEC, S::st>::run(p, tm, tn, lds); break;
    }
}

// Shapes 0 and 2 carry element-wise (unaligned) variants; shape 1 is vectorised only.
template <class S0, class S1, class S2>
__device__ __forceinline__ void run_body(int body, const GemmArgs &p, int tm, int tn, char *lds)
{
    const int shape = body >> 3, trans = (body >> 1) & 3, vec = body & 1;
    if (shape == 0) {
        if (vec) run_shape<S0, true>(trans, p, tm, tn, lds);
        else run_shape<S0, false>(trans, p, tm, tn, lds);
    } else if (shape == 1) {
        run_shape<S1, true>(trans, p, tm, tn, lds);
    } else {
        if constexpr (S2::lds > 0) {
            if (vec) run_shape<S2, true>(trans, p, tm, tn, lds);
            else run_shape<S2, false>(trans, p, tm, tn, lds);
        }
    }
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// All bodies: shapes 0..2 x four transpositions x staging variants.
template <class S0, class S1, class S2, int MINB_>
struct FullBodies {
    static constexpr int LDS = cmax(cmax(S0::lds, S1::lds), S2::lds);
    static constexpr int MINB = MINB_;
    static __device__ __forceinline__ void run(int body, const GemmArgs &p, int tm, int tn, char *lds)
    {
        run_body<S0, S1, S2>(body, p, tm, tn, lds);
    }
};

// Lean bodies: 'N','N' operands with vectorised staging only, a few tile
// shapes of one family (direct-staged, or split at read for the split
// family), chosen per problem: a few thousand instructions per body instead
// of tens of thousands, so the persistent loop runs from the instruction
// cache.  Body b -> the b-th shape.
template <int I, class S0, class... R>
__device__ __forceinline__ void lean_dispatch(int body, const GemmArgs &p, int tm, int tn, char *lds)
{
    if constexpr (sizeof...(R) == 0) {
        S0::run(p, tm, tn, lds);
    } else {
        if (body == I) {
            S0::run(p, tm, tn, lds);
            return;
        }
        lean_dispatch<I + 1, R...>(body, p, tm, tn, lds);
    }
}

template <class S>
constexpr int pieces_of()
{
    if constexpr (S::dt::SPLIT) return S::dt::PLANES;
    else return 0;
}

constexpr int cmaxv(int a) { return a; }
template <class... R>
constexpr int cmaxv(int a, int b, R... r) { return cmaxv(a > b ? a : b, r...); }

template <int MINB_, class... S>
struct LeanBodies {
    static constexpr int N = sizeof...(S);
    static constexpr int LDS = cmaxv(S::lds...);
    static constexpr int MINB = MINB_;
    static __device__ __forceinline__ void run(int body, const GemmArgs &p, int tm, int tn, char *lds)
    {
        lean_dispatch<0, S...>(body, p, tm, tn, lds);
    }
};

// Tile ids are dealt to the XCDs in chunks of kChunk consecutive ids (about
// the number of workgroups one XCD runs at a time; smaller chunks in small
// launches), so the tiles an XCD works on together are neighbours in their
// problem's raster and share A and B panels in that XCD's L2.  Workgroups are dispatched round-robin over the
// XCDs (block b -> XCD b % 8), so group g = b % L collects the workgroups of
// one XCD; with fewer than 8 workgroups, L = grid size and every group still
// has a workgroup.  counters[g] hands out group g's chunk positions;
// counters[8] counts finished workgroups.
constexpr int kChunk = 64;
constexpr int kGroups = 8;
// The prefix array of tables of up to kLdsPrefix problems is copied to LDS at
// the start, so each tile's problem search reads LDS instead of memory.
constexpr int kLdsPrefix = 1024;

template <class BODIES>
__global__ void __launch_bounds__(256, BODIES::MINB) grouped_kernel(const char *__restrict__ table, int *counters)
{
    __shared__ __attribute__((aligned(16))) char lds[BODIES::LDS];
    __shared__ int s_next;
    __shared__ int s_ts[kLdsPrefix];
    const GHeader *h = (const GHeader *)table;
    const GDesc *descs = (const GDesc *)(table + sizeof(GHeader));
    const int total = h->total_tiles, count = h->count;
    const int *ts = (const int *)(table + h->ts_offset);
    const int lane = threadIdx.x & 63;
    const int L = min((int)gridDim.x, kGroups);
    const int g = blockIdx.x % L;
    // Tiles are dealt in chunks of kChunk, or, in launches of fewer than two
    // tiles per workgroup, in chunks of total / (8 L) (at least 1) so that
    // every group gets eight chunks or more: with chunks of kChunk, a launch
    // of up to kChunk tiles would run on one XCD (a 1024^3 INT8 problem, 64
    // tiles: 32.4 against 34.9 us; 640 tiles: 39.5 against 48.0 us).
    const int chunk = total >= 2 * (int)gridDim.x ? kChunk : max(1, min(kChunk, total / (8 * L)));
    // position v of group h -> global tile id; positions 0 .. members(h)-1
    // are the first tiles of group h's workgroups, later ones are claimed
    auto tile_in = [&](int h, int v) { return ((v / chunk) * L + h) * chunk + v % chunk; };
    auto members = [&](int h) { return ((int)gridDim.x - h + L - 1) / L; };
    // Work stealing (thread 0's state): a workgroup draws from its own
    // group's queue, and once that has drained, from the following groups'
    // in turn; a drained queue costs one more claim, so every workgroup ends
    // after at most L - 1 of them.  Only launches of at least four tiles per
    // workgroup steal: in a small launch nearly every workgroup would make
    // its L - 1 claims at once, and those contended atomics cost more than
    // the launch's work (a one-tile launch took 66 us instead of 25 us).
    int src = g, drained = total >= 4 * (int)gridDim.x ? 0 : L;
    auto advance = [&](int nt) {
        while (nt >= total && ++drained < L) {
            src = src + 1 == L ? 0 : src + 1;
            nt = tile_in(src, members(src) + atomicAdd(&counters[src], 1));
        }
        return nt;
    };
    const bool in_lds = count <= kLdsPrefix;
    if (in_lds) {
        for (int i = threadIdx.x; i < count; i += blockDim.x) s_ts[i] = ts[i];
        __syncthreads();
    }
    const int *pre = in_lds ? (const int *)s_ts : ts;
    int t = tile_in(g, (int)blockIdx.x / L);
    if (t >= total) {   // fewer tiles in this group than workgroups: steal at once
        if (threadIdx.x == 0) s_next = advance(t);
        __syncthreads();
        t = __builtin_amdgcn_readfirstlane(s_next);
        __syncthreads();
    }
    while (t < total) {
        // claim the next tile now and use the claim after this tile: the
        // atomic's round trip overlaps the tile instead of delaying its start
        int claim = 0;
        if (threadIdx.x == 0) claim = atomicAdd(&counters[src], 1);
        // last problem whose first tile is <= t: 64-way search per wave over
        // the compact prefix array (in LDS, or two dependent loads for up to
        // 4096 problems)
        int lo = 0, hi = count;
        while (hi - lo > 1) {
            const int step = (hi - lo + 63) >> 6;
            const int i = lo + lane * step;
            const bool le = i < hi && pre[i] <= t;
            const unsigned long long mask = __ballot(le);
            const int last = 63 - __builtin_clzll(mask);   // lane 0 always qualifies
            lo = lo + last * step;
            hi = min(hi, lo + step);
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        const GemmArgs p = descs[lo].a;
        const int body = descs[lo].body;
        int tm, tn;
        raster(t - pre[lo], p.tiles_m, p.tiles_n, p.order, p.group, tm, tn);
        BODIES::run(body, p, tm, tn, lds);
        if (threadIdx.x == 0) s_next = advance(tile_in(src, members(src) + claim));
        __syncthreads();
        t = __builtin_amdgcn_readfirstlane(s_next);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&counters[kGroups], 1) == (int)gridDim.x - 1) {
            for (int i = 0; i < kGroups; ++i) atomicExch(&counters[i], 0);
            atomicExch(&counters[kGroups], 0);
        }
    }
}

// What the host needs to know about one family's kernels.
constexpr int kMaxLean = 8;
struct GroupedFamily {
    const void *func = nullptr;       // all bodies
    int nshapes = 0;
    int mc[3] = {0, 0, 0}, nc[3] = {0, 0, 0};
    const void *lean = nullptr;       // 'N','N', aligned operands only
    int lean_n = 0;                   // lean bodies
    int lean_mc[kMaxLean] = {}, lean_nc[kMaxLean] = {};
    int lean_pieces[kMaxLean] = {};   // split family: bf16 pieces (2: x3, 3: x6); else 0
};

template <class... S>
void lean_shapes(GroupedFamily &f)
{
    const int mc[] = {S::mc...}, nc[] = {S::nc...}, pc[] = {pieces_of<S>()...};
    static_assert(sizeof...(S) <= kMaxLean, "lean body count");
    f.lean_n = (int)sizeof...(S);
    for (int i = 0; i < f.lean_n; ++i) {
        f.lean_mc[i] = mc[i];
        f.lean_nc[i] = nc[i];
        f.lean_pieces[i] = pc[i];
    }
}

template <class LEAN>
struct LeanOf;
template <int MINB, class... S>
struct LeanOf<LeanBodies<MINB, S...>> {
    static void fill(GroupedFamily &f) { lean_shapes<S...>(f); }
};

template <class S0, class S1, class S2, int MINB, class LEAN>
GroupedFamily make_family()
{
    GroupedFamily f;
    f.func = (const void *)&grouped_kernel<FullBodies<S0, S1, S2, MINB>>;
    f.mc[0] = S0::mc;
    f.nc[0] = S0::nc;
    f.mc[1] = S1::mc;
    f.nc[1] = S1::nc;
    f.nshapes = 2;
    if constexpr (S2::lds > 0) {
        f.mc[2] = S2::mc;
        f.nc[2] = S2::nc;
        f.nshapes = 3;
    }
    f.lean = (const void *)&grouped_kernel<LEAN>;
    LeanOf<LEAN>::fill(f);
    return f;
}

enum GFam { G_F32 = 0, G_SPLIT, G_BF16, G_F16, G_F8, G_I8, G_NUM };
GroupedFamily grouped_family(int fam);

}  // namespace mg
