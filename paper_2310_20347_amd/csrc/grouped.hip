// Host side of the grouped persistent launch: validation, per-problem plan
// (tile shape from the tuning table's size bucket, transposition, raster
// order), ordering of problems by descending per-tile cost so the longest
// tiles start first, descriptor tables in pinned host memory copied to the
// device on the launch stream, and the capturable slot API.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "abi_internal.hpp"
#include "grouped.hpp"
#include "mgemm.h"

namespace mg {

GroupedFamily grouped_family_f32();
GroupedFamily grouped_family_split();
GroupedFamily grouped_family_bf16();
GroupedFamily grouped_family_f16();
GroupedFamily grouped_family_f8();
GroupedFamily grouped_family_i8();

GroupedFamily grouped_family(int fam)
{
    switch (fam) {
    case G_F32: return grouped_family_f32();
    case G_SPLIT: return grouped_family_split();
    case G_BF16: return grouped_family_bf16();
    case G_F16: return grouped_family_f16();
    case G_F8: return grouped_family_f8();
    case G_I8: return grouped_family_i8();
    default: return GroupedFamily();
    }
}

constexpr int64_t kCapacity = 8192;   // problems per descriptor table
constexpr int kRotating = 4;          // rotating slots of gemm_grouped per device
constexpr int kCounterInts = 16;      // kGroups tile counters + finished count, padded
// header, descriptors, then the compact tile_start array (one int per problem)
constexpr size_t table_bytes(int64_t cap) { return sizeof(GHeader) + size_t(cap) * (sizeof(GDesc) + 4); }
constexpr size_t kTableBytes = table_bytes(kCapacity);

struct Slot {
    char *host = nullptr;     // pinned staging
    char *dev = nullptr;      // device table
    int *counters = nullptr;  // device {next position per XCD group [8], finished workgroups}
    hipEvent_t done = nullptr;
    bool used = false;
    int family = -1;
    int variant = -1;   // kernel variant fixed by the first write (0 full, 1 lean)
    int device = 0;
    int64_t capacity = kCapacity;
};

struct GroupedDev {
    GroupedFamily fam[G_NUM];
    int grid[G_NUM][2] = {};   // [family][0 full, 1 lean]
    Slot rot[kRotating];
    int next = 0;
    std::mutex mu;
};

static int family_of(int dtype)
{
    switch (dtype) {
    case GEMM_F32: return G_F32;
    case GEMM_F32_BF16X3: case GEMM_F32_BF16X3_ONLY: case GEMM_F32_BF16X6: return G_SPLIT;
    case GEMM_BF16: return G_BF16;
    case GEMM_F16: return G_F16;
    case GEMM_F8E4M3: return G_F8;
    case GEMM_I8: return G_I8;
    default: return -1;
    }
}

static int slot_alloc(Slot &s, int device)
{
    hipError_t e;
    s.device = device;
    if ((e = hipHostMalloc((void **)&s.host, kTableBytes, hipHostMallocDefault)) != hipSuccess) goto fail;
    if ((e = hipMalloc((void **)&s.dev, kTableBytes)) != hipSuccess) goto fail;
    if ((e = hipMalloc((void **)&s.counters, kCounterInts * sizeof(int))) != hipSuccess) goto fail;
    if ((e = hipMemset(s.counters, 0, kCounterInts * sizeof(int))) != hipSuccess) goto fail;
    if ((e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess) goto fail;
    if ((e = hipDeviceSynchronize()) != hipSuccess) goto fail;
    return GEMM_OK;
fail:
    t_tls.hip_err = (int)e;
    return GEMM_E_HIP;
}

static void slot_free(Slot &s)
{
    if (s.done) (void)hipEventSynchronize(s.done);
    if (s.host) (void)hipHostFree(s.host);
    if (s.dev) (void)hipFree(s.dev);
    if (s.counters) (void)hipFree(s.counters);
    if (s.done) (void)hipEventDestroy(s.done);
    s = Slot();
}

int grouped_device_init(DevState *d)
{
    if (d->grouped_ready) return GEMM_OK;
    std::lock_guard<std::mutex> g(g_mu);
    if (d->grouped_ready) return GEMM_OK;
    GroupedDev *gd = new GroupedDev();
    for (int f = 0; f < G_NUM; ++f) {
        gd->fam[f] = grouped_family(f);
        for (int v = 0; v < 2; ++v) {
            int per_cu = 0;
            const void *fn = v ? gd->fam[f].lean : gd->fam[f].func;
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0);
            if (e != hipSuccess || per_cu < 1) per_cu = 1;
            gd->grid[f][v] = d->cus * per_cu;
        }
    }
    for (int i = 0; i < kRotating; ++i) {
        int rc = slot_alloc(gd->rot[i], d->device);
        if (rc != GEMM_OK) {
            for (int j = 0; j <= i; ++j) slot_free(gd->rot[j]);
            delete gd;
            return rc;
        }
    }
    d->grouped = gd;
    d->grouped_ready = true;
    return GEMM_OK;
}

void grouped_device_free(DevState *d)
{
    if (!d->grouped_ready) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(d->device);
    GroupedDev *gd = (GroupedDev *)d->grouped;
    for (int i = 0; i < kRotating; ++i) slot_free(gd->rot[i]);
    delete gd;
    d->grouped = nullptr;
    d->grouped_ready = false;
    (void)hipSetDevice(cur);
}

static int ensure_grouped(DevState **out)
{
    ensure_registered();
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    rc = grouped_device_init(d);
    if (rc != GEMM_OK) return rc;
    *out = d;
    return GEMM_OK;
}

// Lean body of one problem: the body pinned on this thread
// (gemm_grouped_force_body), else the tuning table's grouped entry for the
// size bucket (gemm_tune_grouped), else the body whose tile fits the problem
// best: 32 or 64 rows (columns) for m (n) up to that, 128, and 256 from 1024
// on where such a body exists.  Split family: only bodies of the problem's
// term count (three terms for k >= 64, six below) qualify.
static int lean_body(const GroupedFamily &F, int kclass, int64_t m, int64_t n, int64_t k)
{
    const int want_pieces = kclass == K_SPLIT2 ? 2 : kclass == K_SPLIT3 ? 3 : 0;
    auto ok = [&](int b) { return b >= 0 && b < F.lean_n && F.lean_pieces[b] == want_pieces; };
    if (ok(t_tls.force_body)) return t_tls.force_body;
    const int tuned = grouped_body_lookup(kclass, m, n, k);
    if (ok(tuned)) return tuned;
    auto want = [](int64_t x) { return x <= 32 ? 32.0 : x <= 64 ? 64.0 : x < 1024 ? 128.0 : 256.0; };
    const double wm = want(m), wn = want(n);
    int best = -1;
    double bd = 1e300;
    for (int b = 0; b < F.lean_n; ++b) {
        if (!ok(b)) continue;
        const double d = std::fabs(std::log2(F.lean_mc[b] / wm)) + std::fabs(std::log2(F.lean_nc[b] / wn));
        if (d < bd - 1e-9) {
            bd = d;
            best = b;
        }
    }
    return best;
}

// Builds the descriptor table of `count` problems into `table` (host memory).
// `want`: -1 choose, 0 full kernel, 1 lean kernel.  The lean kernel serves
// batches whose problems are all 'N','N' with vectorisable operands; *variant
// receives the kernel the table was built for.  Returns 0 / -(1000*p + i) /
// GEMM_E_*; sets total tiles in the header.
static int build_table(const GroupedFamily *fams, int cus, int64_t count, const gemm_problem *pr,
                       int dtype, char *table, int want, int *variant, int64_t cap,
                       int *bodies = nullptr)
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -3;
    if (count < 0) return -1;
    if (count > 0 && !pr) return -2;
    if (count > kCapacity) return GEMM_E_WORKSPACE;
    const int fam = family_of(dtype);
    if (fam < 0) return GEMM_E_UNSUPPORTED;
    const GroupedFamily &F = fams[fam];
    for (int64_t p = 0; p < count; ++p) {
        const gemm_problem &q = pr[p];
        const int v = validate(q.transA, q.transB, q.m, q.n, q.k, q.alpha, q.A, q.lda, q.B, q.ldb,
                               q.beta, q.C, q.ldc, dtype);
        if (v != 0) return (int)(-1000 * p + v);
        if (q.m > 0x7FFFFFFF || q.n > 0x7FFFFFFF || q.k > 0x7FFFFFFF) return GEMM_E_UNSUPPORTED;
    }
    bool lean = want != 0;
    for (int64_t p = 0; p < count && lean; ++p) {
        const gemm_problem &q = pr[p];
        const bool nn = (q.transA == 'N' || q.transA == 'n') && (q.transB == 'N' || q.transB == 'n');
        const int es = elem_bytes(kclass_of(dtype, q.k));
        lean = nn && vec_ok(q.A, q.lda, es) && vec_ok(q.B, q.ldb, es);
    }
    if (want == 1 && !lean) return GEMM_E_UNSUPPORTED;
    *variant = lean ? 1 : 0;
    GHeader *h = (GHeader *)table;
    GDesc *descs = (GDesc *)(table + sizeof(GHeader));
    std::vector<GDesc> tmp;
    std::vector<double> cost;
    tmp.reserve((size_t)count);
    for (int64_t p = 0; p < count; ++p) {
        const gemm_problem &q = pr[p];
        if (bodies) bodies[p] = -1;
        if (q.m == 0 || q.n == 0) continue;
        if ((q.alpha == 0.0 || q.k == 0) && q.beta == 1.0) continue;
        const bool ta = q.transA == 'T' || q.transA == 't' || q.transA == 'C' || q.transA == 'c';
        const bool tb = q.transB == 'T' || q.transB == 't' || q.transB == 'C' || q.transB == 'c';
        const int trans = 2 * ta + tb;
        const int kclass = kclass_of(dtype, q.k);
        int cfg = 0, order = 0, group = 8;
        select_config(kclass, trans, q.m, q.n, q.k, cus, cfg, order, group);
        int shape, mc, nc;
        const int es = elem_bytes(kclass);
        const bool vec = vec_ok(q.A, q.lda, es) && vec_ok(q.B, q.ldb, es);
        if (lean) {
            shape = lean_body(F, kclass, q.m, q.n, q.k);
            if (shape < 0) return GEMM_E_UNSUPPORTED;
            mc = F.lean_mc[shape];
            nc = F.lean_nc[shape];
            if (bodies) bodies[p] = shape;
        } else {
            if (kclass == K_SPLIT3)
                shape = 2;
            else
                shape = (cfg == 0 || q.m < F.mc[1] || q.n < F.nc[1]) ? 0 : 1;
            if (!vec && shape == 1) shape = 0;
            mc = F.mc[shape];
            nc = F.nc[shape];
        }
        GDesc d;
        std::memset(&d, 0, sizeof d);
        GemmArgs &a = d.a;
        a.A = q.A;
        a.B = q.B;
        a.C = q.C;
        a.lda = q.lda;
        a.ldb = q.ldb;
        a.ldc = q.ldc;
        a.m = (int)q.m;
        a.n = (int)q.n;
        a.k = (int)q.k;
        a.alpha = (float)q.alpha;
        a.beta = (float)q.beta;
        a.ialpha = dtype == GEMM_I8 ? (int)q.alpha : 0;
        a.ibeta = dtype == GEMM_I8 ? (int)q.beta : 0;
        a.tiles_m = (int)((q.m + mc - 1) / mc);
        a.tiles_n = (int)((q.n + nc - 1) / nc);
        a.order = order;
        a.group = std::max(1, group);
        a.terms = split_terms(kclass);
        d.body = lean ? shape : shape * 8 + trans * 2 + (vec ? 1 : 0);
        tmp.push_back(d);
        // per-tile work: the k loop length times the tile area
        const double kk = (q.alpha == 0.0) ? 0.0 : double(q.k);
        cost.push_back((kk + 64.0) * mc * nc);
    }
    std::vector<size_t> idx(tmp.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    if (cap <= 0) cap = (int64_t)idx.size();
    int *ts = (int *)(table + sizeof(GHeader) + size_t(cap) * sizeof(GDesc));
    int64_t tiles = 0;
    for (size_t i = 0; i < idx.size(); ++i) {
        GDesc d = tmp[idx[i]];
        d.tile_start = (int)tiles;
        ts[i] = (int)tiles;
        tiles += int64_t(d.a.tiles_m) * d.a.tiles_n;
        if (tiles > 0x7FFFFFFF) return GEMM_E_UNSUPPORTED;
        descs[i] = d;
    }
    std::memset(h, 0, sizeof *h);
    h->count = (int)idx.size();
    h->total_tiles = (int)tiles;
    h->family = fam;
    h->ts_offset = (int)(sizeof(GHeader) + size_t(cap) * sizeof(GDesc));
    return GEMM_OK;
}

static int launch_table(const GroupedDev *gd, const Slot &s, int fam, int variant, int grid,
                        size_t bytes, hipStream_t st)
{
    hipError_t e = hipMemcpyAsync(s.dev, s.host, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    const char *table = s.dev;
    int *counters = s.counters;
    void *args[] = {&table, &counters};
    e = hipLaunchKernel(variant ? gd->fam[fam].lean : gd->fam[fam].func, dim3(grid), dim3(256),
                        args, 0, st);
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    return GEMM_OK;
}

}  // namespace mg

using namespace mg;

extern "C" {

int gemm_grouped(int64_t count, const gemm_problem *problems, int dtype)
{
    if (count < 0) return -1;
    if (count > 0 && !problems) return -2;
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -3;
    if (family_of(dtype) < 0) return GEMM_E_UNSUPPORTED;
    if (count > kCapacity) return GEMM_E_WORKSPACE;
    // validate before touching the device (same rules as gemm)
    for (int64_t p = 0; p < count; ++p) {
        const gemm_problem &q = problems[p];
        const int v = validate(q.transA, q.transB, q.m, q.n, q.k, q.alpha, q.A, q.lda, q.B, q.ldb,
                               q.beta, q.C, q.ldc, dtype);
        if (v != 0) return (int)(-1000 * p + v);
    }
    if (count == 0) return GEMM_OK;
    DevState *d = nullptr;
    int rc = ensure_grouped(&d);
    if (rc != GEMM_OK) return rc;
    GroupedDev *gd = (GroupedDev *)d->grouped;
    std::lock_guard<std::mutex> g(gd->mu);
    Slot &s = gd->rot[gd->next];
    gd->next = (gd->next + 1) % kRotating;
    if (s.used) {
        hipError_t e = hipEventSynchronize(s.done);   // previous copy from this slot consumed
        if (e != hipSuccess) {
            t_tls.hip_err = (int)e;
            return GEMM_E_HIP;
        }
    }
    int variant = 0;
    rc = build_table(gd->fam, d->cus, count, problems, dtype, s.host, -1, &variant, 0);
    if (rc != GEMM_OK) return rc;
    const GHeader *h = (const GHeader *)s.host;
    if (h->total_tiles == 0) {
        // only quick-return problems (C untouched)
        return GEMM_OK;
    }
    const int fam = family_of(dtype);
    // the full persistent grid, as for slots, however few the tiles: tiles are
    // dealt to the XCD groups in chunks of kChunk, so a grid cut to the tile
    // count would leave a batch of up to kChunk tiles to the few workgroups of
    // group 0 (one 1024^3 INT8 problem: 140 us instead of 37 us); the
    // workgroups without a tile leave at once
    const int grid = gd->grid[fam][variant];
    const size_t bytes = table_bytes(h->count);
    hipStream_t st = t_tls.stream;
    rc = launch_table(gd, s, fam, variant, grid, bytes, st);
    if (rc != GEMM_OK) return rc;
    hipError_t e = hipEventRecord(s.done, st);
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    s.used = true;
    return GEMM_OK;
}

int64_t gemm_grouped_capacity(void) { return kCapacity; }

int gemm_grouped_slot_create(void **slot, int64_t capacity)
{
    if (!slot) return -1;
    if (capacity < 1 || capacity > kCapacity) return -2;
    DevState *d = nullptr;
    int rc = ensure_grouped(&d);
    if (rc != GEMM_OK) return rc;
    Slot *s = new Slot();
    rc = slot_alloc(*s, d->device);
    if (rc != GEMM_OK) {
        slot_free(*s);
        delete s;
        return rc;
    }
    std::memset(s->host, 0, sizeof(GHeader));
    s->capacity = capacity;
    *slot = s;
    return GEMM_OK;
}

int gemm_grouped_slot_write(void *slot, int64_t count, const gemm_problem *problems, int dtype)
{
    if (!slot) return -1;
    if (count < 0) return -2;
    if (count > 0 && !problems) return -3;
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -4;
    Slot *s = (Slot *)slot;
    if (count > s->capacity) return GEMM_E_WORKSPACE;
    const int fam = family_of(dtype);
    if (fam < 0) return GEMM_E_UNSUPPORTED;
    if (s->family >= 0 && s->family != fam) return GEMM_E_UNSUPPORTED;
    DevState *d = nullptr;
    int rc = ensure_grouped(&d);
    if (rc != GEMM_OK) return rc;
    // build into a private buffer first so a failed validation leaves the slot intact
    std::vector<char> buf(table_bytes(s->capacity));
    int variant = 0;
    rc = build_table(((GroupedDev *)d->grouped)->fam, d->cus, count, problems, dtype, buf.data(),
                     s->variant, &variant, s->capacity);
    if (rc != GEMM_OK) {
        // a problem error is reported as in gemm_grouped: -(1000*p + i)
        return rc;
    }
    std::memcpy(s->host, buf.data(), table_bytes(s->capacity));
    s->family = fam;
    s->variant = variant;
    return GEMM_OK;
}

int gemm_grouped_slot_launch(void *slot)
{
    if (!slot) return -1;
    Slot *s = (Slot *)slot;
    if (s->family < 0) return GEMM_E_UNSUPPORTED;   // never written
    DevState *d = nullptr;
    int rc = ensure_grouped(&d);
    if (rc != GEMM_OK) return rc;
    GroupedDev *gd = (GroupedDev *)d->grouped;
    // the grid does not depend on the table, so a captured launch stays valid
    // when the slot is rewritten; header + capacity descriptors are copied
    const size_t bytes = table_bytes(s->capacity);
    return launch_table(gd, *s, s->family, s->variant, gd->grid[s->family][s->variant], bytes,
                        t_tls.stream);
}

int gemm_grouped_num_bodies(int dtype)
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -1;
    const int fam = family_of(dtype);
    if (fam < 0) return -1;
    return grouped_family(fam).lean_n;
}

int gemm_grouped_body_info(int dtype, int body, int64_t out[3])
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -1;
    const int fam = family_of(dtype);
    if (fam < 0) return GEMM_E_UNSUPPORTED;
    const GroupedFamily F = grouped_family(fam);
    if (body < 0 || body >= F.lean_n) return -2;
    if (!out) return -3;
    out[0] = F.lean_mc[body];
    out[1] = F.lean_nc[body];
    out[2] = F.lean_pieces[body];
    return GEMM_OK;
}

int gemm_grouped_force_body(int body)
{
    if (body < -1 || body >= kMaxGroupedBodies) return -1;
    t_tls.force_body = body;
    return GEMM_OK;
}

int gemm_grouped_bodies(int64_t count, const gemm_problem *problems, int dtype, int *bodies)
{
    if (count < 0) return -1;
    if (count > 0 && !problems) return -2;
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -3;
    if (count > 0 && !bodies) return -4;
    const int fam = family_of(dtype);
    if (fam < 0) return GEMM_E_UNSUPPORTED;
    if (count > kCapacity) return GEMM_E_WORKSPACE;
    ensure_registered();
    GroupedFamily fams[G_NUM];
    for (int f = 0; f < G_NUM; ++f) fams[f] = grouped_family(f);
    int cus = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices && g_dev[dev].init)
        cus = g_dev[dev].cus;
    std::vector<char> buf(table_bytes(std::max<int64_t>(count, 1)));
    int variant = 0;
    return build_table(fams, cus, count, problems, dtype, buf.data(), -1, &variant, 0, bodies);
}

int gemm_tune_grouped(int dtype, int64_t count, const int64_t *shapes, int reps,
                      const char *out_path)
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -1;
    if (count < 1) return -2;
    if (!shapes) return -3;
    if (reps < 1) return -4;
    const int fam = family_of(dtype);
    if (fam < 0) return GEMM_E_UNSUPPORTED;
    for (int64_t i = 0; i < 3 * count; ++i)
        if (shapes[i] < 1 || shapes[i] > 65536) return -3;
    DevState *d = nullptr;
    int rc = ensure_grouped(&d);
    if (rc != GEMM_OK) return rc;
    GroupedDev *gd = (GroupedDev *)d->grouped;
    const GroupedFamily &F = gd->fam[fam];
    // one private slot, operands shared by every problem of a batch, and a C
    // region per problem
    constexpr size_t kCBytes = size_t(1) << 30;
    size_t maxA = 16, maxB = 16;
    for (int64_t i = 0; i < count; ++i) {
        const int64_t m = shapes[3 * i], n = shapes[3 * i + 1], k = shapes[3 * i + 2];
        const int es = elem_bytes(kclass_of(dtype, k));
        const int64_t al = 16 / es;
        maxA = std::max(maxA, size_t(m * ((k + al - 1) / al * al) * es));
        maxB = std::max(maxB, size_t(k * ((n + al - 1) / al * al) * es));
    }
    Slot s;
    void *A = nullptr, *B = nullptr, *C = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const int saved_body = t_tls.force_body;
    auto cleanup = [&]() {
        if (st) (void)hipStreamSynchronize(st);
        slot_free(s);
        if (A) (void)hipFree(A);
        if (B) (void)hipFree(B);
        if (C) (void)hipFree(C);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
        t_tls.force_body = saved_body;
    };
    hipError_t e = hipSuccess;
    if ((rc = slot_alloc(s, d->device)) != GEMM_OK) {
        cleanup();
        return rc;
    }
    if ((e = hipMalloc(&A, maxA)) != hipSuccess || (e = hipMalloc(&B, maxB)) != hipSuccess ||
        (e = hipMalloc(&C, kCBytes)) != hipSuccess || (e = hipStreamCreate(&st)) != hipSuccess ||
        (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        t_tls.hip_err = (int)e;
        cleanup();
        return GEMM_E_HIP;
    }
    const int ckind = fam == G_I8 ? 4 : fam == G_BF16 ? 1 : fam == G_F16 ? 2 : fam == G_F8 ? 3 : 0;
    launch_fill(A, (int64_t)(maxA / (ckind == 0 ? 4 : ckind <= 2 ? 2 : 1)), ckind, 5u, st);
    launch_fill(B, (int64_t)(maxB / (ckind == 0 ? 4 : ckind <= 2 ? 2 : 1)), ckind, 6u, st);
    std::vector<gemm_problem> probs;
    for (int64_t i = 0; i < count; ++i) {
        const int64_t m = shapes[3 * i], n = shapes[3 * i + 1], k = shapes[3 * i + 2];
        const int kclass = kclass_of(dtype, k);
        const int es = elem_bytes(kclass);
        const int64_t al = 16 / es;
        const int64_t lda = (k + al - 1) / al * al, ldb = (n + al - 1) / al * al;
        // enough problems for about four tiles per workgroup slot of the
        // 128x128 body, within the C region and the table
        const int64_t tiles128 = ((m + 127) / 128) * ((n + 127) / 128);
        int64_t N = std::max<int64_t>(1, (4 * int64_t(gd->grid[fam][1]) + tiles128 - 1) / tiles128);
        N = std::min<int64_t>({N, 512, std::max<int64_t>(1, int64_t(kCBytes / (size_t(m) * n * 4)))});
        probs.assign((size_t)N, gemm_problem());
        for (int64_t p = 0; p < N; ++p) {
            gemm_problem &q = probs[(size_t)p];
            q.transA = 'N';
            q.transB = 'N';
            q.m = m;
            q.n = n;
            q.k = k;
            q.alpha = 1.0;
            q.A = A;
            q.lda = lda;
            q.B = B;
            q.ldb = ldb;
            q.beta = 0.0;
            q.C = (char *)C + size_t(p) * m * n * 4;
            q.ldc = n;
        }
        double best_us = 1e300;
        int best = -1;
        for (int b = 0; b < F.lean_n; ++b) {
            const int want = kclass == K_SPLIT2 ? 2 : kclass == K_SPLIT3 ? 3 : 0;
            if (F.lean_pieces[b] != want) continue;
            t_tls.force_body = b;
            int variant = 0;
            rc = build_table(gd->fam, d->cus, N, probs.data(), dtype, s.host, 1, &variant, 0);
            if (rc != GEMM_OK) {
                cleanup();
                return rc;
            }
            const size_t bytes = table_bytes(((const GHeader *)s.host)->count);
            std::vector<float> ms;
            for (int r = 0; r < reps + 1; ++r) {
                (void)hipEventRecord(e0, st);
                rc = launch_table(gd, s, fam, 1, gd->grid[fam][1], bytes, st);
                (void)hipEventRecord(e1, st);
                if (rc != GEMM_OK || (e = hipEventSynchronize(e1)) != hipSuccess) {
                    if (rc == GEMM_OK) {
                        t_tls.hip_err = (int)e;
                        rc = GEMM_E_HIP;
                    }
                    cleanup();
                    return rc;
                }
                float t = 0;
                (void)hipEventElapsedTime(&t, e0, e1);
                if (r > 0) ms.push_back(t);
            }
            std::sort(ms.begin(), ms.end());
            const double us = 1e3 * ms[ms.size() / 2] / double(N);   // per problem
            if (us < best_us) {
                best_us = us;
                best = b;
            }
        }
        if (best >= 0)
            set_table_entry(TuneKey{kclass, kGroupedTrans, bucket(m), bucket(n), bucket(k)},
                            TuneVal{best, 0, 8, best_us});
    }
    cleanup();
    rebuild_lut();
    if (out_path && *out_path) return save_table(out_path);
    return GEMM_OK;
}

void gemm_grouped_slot_destroy(void *slot)
{
    if (!slot) return;
    Slot *s = (Slot *)slot;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    slot_free(*s);
    (void)hipSetDevice(cur);
    delete s;
}

}  // extern "C"
