// C ABI of the GEMM family: argument validation (BLAS conventions), quick
// returns, configuration selection per size bucket, kernel launch on the
// calling thread's stream, tuning table load/save, and introspection.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "abi_internal.hpp"
#include "mgemm.h"

namespace mg {

std::mutex g_mu;
std::vector<KernelCfg> g_cfgs;
std::vector<int> g_by_class[K_NUM];
static bool g_registered = false;
static bool g_table_loaded = false;
DevState g_dev[kMaxDevices];
std::map<TuneKey, TuneVal> g_table;
thread_local Tls t_tls;

// Process-wide defaults read from the environment by gemm_init:
// MGEMM_FORCE_CFG pins a configuration per kernel class (a thread's own pin,
// gemm_force_config, takes precedence); MGEMM_DEBUG turns on the sentinel
// fill and count around every beta = 0 product.
// (The environment's pin is held as id + 1, so that the zero-initialised
// state, before any gemm_init, pins nothing.)
static std::atomic<int> g_env_pin[K_NUM];
static std::atomic<int> g_env_pin_order[K_NUM];
static std::atomic<bool> g_debug{false};

// The configuration pinned for a class: the thread's, else the environment's
// (id < 0: none).
static void pinned(int kclass, int &id, int &order)
{
    id = t_tls.force_id[kclass];
    order = t_tls.force_order[kclass];
    if (id < 0) {
        id = g_env_pin[kclass].load(std::memory_order_relaxed) - 1;
        order = g_env_pin_order[kclass].load(std::memory_order_relaxed);
    }
}

Tls::Tls()
{
    for (int c = 0; c < K_NUM; ++c) {
        force_id[c] = -1;
        force_order[c] = 0;
    }
    for (int i = 0; i < 4; ++i) last[i] = -1;
}

int kclass_of(int dtype, int64_t k)
{
    switch (dtype) {
    case GEMM_F32: return K_F32;
    case GEMM_F32_BF16X3: return k >= 64 ? K_SPLIT2 : K_SPLIT3;
    case GEMM_F32_BF16X3_ONLY: return K_SPLIT2;
    case GEMM_F32_BF16X6: return K_SPLIT3;
    case GEMM_BF16: return K_BF16;
    case GEMM_F16: return K_F16;
    case GEMM_F8E4M3: return K_F8;
    case GEMM_I8: return K_I8;
    case GEMM_F64: return K_F64;
    case GEMM_I16: return K_I16;
    case GEMM_I32: return K_I32;
    default: return -1;
    }
}

int elem_bytes(int kclass)
{
    switch (kclass) {
    case K_F32: case K_SPLIT2: case K_SPLIT3: return 4;
    case K_BF16: case K_F16: case K_I16: return 2;
    case K_F64: return 8;
    case K_I32: return 4;
    default: return 1;
    }
}

int split_terms(int kclass)
{
    return kclass == K_SPLIT2 ? 3 : kclass == K_SPLIT3 ? 6 : 0;
}

int bucket(int64_t x)
{
    int b = 0;
    while (b < 62 && (int64_t(1) << (b + 1)) <= x) ++b;
    return std::min(std::max(b, 4), 12);
}

static bool is_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }
static bool trans_ok(char t) { return t == 'N' || t == 'n' || is_trans(t); }

static bool int32_exact(double v)
{
    return std::isfinite(v) && v == std::floor(v) && v >= -2147483648.0 && v <= 2147483647.0;
}

// Arguments are checked in their order, so the code names the first invalid
// one; checks that need the element size (operand alignment) are skipped
// while the dtype (argument 14) is unknown, which is then reported last.
int validate(char ta, char tb, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
             int64_t lda, const void *B, int64_t ldb, double beta, const void *C, int64_t ldc,
             int dtype)
{
    if (!trans_ok(ta)) return -1;
    if (!trans_ok(tb)) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    const bool dtype_ok = dtype >= 0 && dtype < GEMM_NUM_DTYPES;
    const bool is_int = dtype == GEMM_I8 || dtype == GEMM_I16 || dtype == GEMM_I32;
    if (is_int && !int32_exact(alpha)) return -6;
    const int es = dtype_ok ? elem_bytes(kclass_of(dtype, k)) : 1;
    const bool form = m > 0 && n > 0 && k > 0 && alpha != 0.0;
    if (form && A == nullptr) return -7;
    if (A != nullptr && (reinterpret_cast<uintptr_t>(A) % es) != 0) return -7;
    if (lda < std::max<int64_t>(1, is_trans(ta) ? m : k)) return -8;
    if (form && B == nullptr) return -9;
    if (B != nullptr && (reinterpret_cast<uintptr_t>(B) % es) != 0) return -9;
    if (ldb < std::max<int64_t>(1, is_trans(tb) ? k : n)) return -10;
    if (is_int && !int32_exact(beta)) return -11;
    const bool write = m > 0 && n > 0 && !((alpha == 0.0 || k == 0) && beta == 1.0);
    if (write && C == nullptr) return -12;
    const int ces = !dtype_ok ? 1 : (dtype == GEMM_F64 ? 8 : 4);
    if (C != nullptr && (reinterpret_cast<uintptr_t>(C) % ces) != 0) return -12;
    if (ldc < std::max<int64_t>(1, n)) return -13;
    if (!dtype_ok) return -14;
    return 0;
}

void ensure_registered()
{
    std::lock_guard<std::mutex> g(g_mu);
    if (g_registered) return;
    register_f32(g_cfgs);
    register_split(g_cfgs);
    register_half(g_cfgs);
    register_byte(g_cfgs);
    register_resident_f32(g_cfgs);
    register_resident_split(g_cfgs);
    register_resident_half(g_cfgs);
    register_resident_byte(g_cfgs);
    register_direct_f32(g_cfgs);
    register_direct_half(g_cfgs);
    register_direct_byte(g_cfgs);
    // packed split: every direct bf16 tile, run on operands that a packing
    // pass has split into bf16 pieces (three- and six-term classes)
    auto add_packed = [](size_t from, size_t to) {
        for (int cls : {K_SPLIT2, K_SPLIT3}) {
            for (size_t i = from; i < to; ++i) {
                if (g_cfgs[i].kclass != K_BF16 || !g_cfgs[i].direct) continue;
                KernelCfg p = g_cfgs[i];
                p.kclass = cls;
                p.kind = 5;
                p.direct = false;
                p.packed = (int)i;
                for (int t = 0; t < 4; ++t)
                    for (int v = 0; v < 2; ++v) {
                        p.func[t][v] = split_pack_entry();
                        p.splitk[t][v] = nullptr;
                    }
                g_cfgs.push_back(p);
            }
        }
    };
    const size_t nbase = g_cfgs.size();
    add_packed(0, nbase);
    // split-K: every tile compiled with a sliced form
    const size_t nall = g_cfgs.size();
    for (size_t i = 0; i < nall; ++i) {
        const KernelCfg &b = g_cfgs[i];
        bool any = false;
        for (int t = 0; t < 4; ++t) any = any || b.splitk[t][0] || b.splitk[t][1];
        if (!any) continue;
        KernelCfg p = b;
        p.kind = 6;
        p.base = (int)i;
        for (int t = 0; t < 4; ++t)
            for (int v = 0; v < 2; ++v) {
                p.func[t][v] = b.splitk[t][v];
                p.splitk[t][v] = nullptr;
            }
        g_cfgs.push_back(p);
    }
    // packing configurations (A, B or neither through LDS)
    register_nopack(g_cfgs);
    // split product on direct-staged FP32 panels
    register_splitdirect(g_cfgs);
    register_f64(g_cfgs);
    // appended last, so every configuration number above stays as it was
    register_direct_f32_late(g_cfgs);
    const size_t nlate = g_cfgs.size();
    register_direct_half_late(g_cfgs);
    register_direct_byte_late(g_cfgs);
    add_packed(nlate, g_cfgs.size());
    register_f64_late(g_cfgs);
    register_int_late(g_cfgs);
    const size_t nw32 = g_cfgs.size();
    register_direct_w32_late(g_cfgs);
    register_direct_deep_late(g_cfgs);
    add_packed(nw32, g_cfgs.size());
    for (size_t i = 0; i < g_cfgs.size(); ++i) g_by_class[g_cfgs[i].kclass].push_back((int)i);
    g_registered = true;
}

// Directory of this shared library (for the tuning table shipped beside it).
static std::string lib_dir()
{
    Dl_info info;
    if (dladdr((void *)&lib_dir, &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        size_t s = p.find_last_of('/');
        if (s != std::string::npos) return p.substr(0, s);
    }
    return ".";
}

int device_state(DevState **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        t_tls.hip_err = (int)e;
        return GEMM_E_NOINIT;
    }
    DevState &d = g_dev[dev];
    if (!d.init) {
        std::lock_guard<std::mutex> g(g_mu);
        if (!d.init) {
            int cus = 0;
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) {
                t_tls.hip_err = (int)e;
                return GEMM_E_HIP;
            }
            d.cus = cus;
            d.device = dev;
            d.init = true;
        }
    }
    *out = &d;
    return GEMM_OK;
}

// ---------------------------------------------------------------------------
// Tuning table (JSON, one entry object per line).
// ---------------------------------------------------------------------------
static bool parse_entry(const std::string &obj, TuneKey &key, TuneVal &val)
{
    auto num = [&](const char *name, double &out) -> bool {
        std::string pat = std::string("\"") + name + "\"";
        size_t p = obj.find(pat);
        if (p == std::string::npos) return false;
        p = obj.find(':', p + pat.size());
        if (p == std::string::npos) return false;
        out = std::strtod(obj.c_str() + p + 1, nullptr);
        return true;
    };
    double kc, tr, bm, bn, bk, cfg, order, group, us = 0;
    if (!num("kclass", kc) || !num("trans", tr) || !num("bm", bm) || !num("bn", bn) ||
        !num("bk", bk) || !num("cfg", cfg) || !num("order", order) || !num("group", group))
        return false;
    num("us", us);
    key = TuneKey{(int)kc, (int)tr, (int)bm, (int)bn, (int)bk};
    val = TuneVal{(int)cfg, (int)order, (int)group, us};
    return key.kclass >= 0 && key.kclass < K_NUM && key.trans >= 0 && key.trans <= kGroupedTrans;
}

static void rebuild_lut_locked();
static void ensure_table();

int load_table(const char *path)
{
    std::ifstream f(path);
    if (!f) return GEMM_E_TUNE_TABLE;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t p = s.find("\"entries\"");
    if (p == std::string::npos) return GEMM_E_TUNE_TABLE;
    std::map<TuneKey, TuneVal> table;
    while (true) {
        size_t a = s.find('{', p);
        if (a == std::string::npos) break;
        size_t b = s.find('}', a);
        if (b == std::string::npos) return GEMM_E_TUNE_TABLE;
        TuneKey key;
        TuneVal val;
        if (!parse_entry(s.substr(a, b - a + 1), key, val)) return GEMM_E_TUNE_TABLE;
        // a grouped entry names a body of the class's grouped kernel
        const int ncfg = key.trans == kGroupedTrans ? kMaxGroupedBodies
                                                    : (int)g_by_class[key.kclass].size();
        if (val.cfg < 0 || val.cfg >= ncfg || val.group < 1 || val.order < 0 || val.order > 1)
            return GEMM_E_TUNE_TABLE;
        table[key] = val;
        p = b + 1;
    }
    std::lock_guard<std::mutex> g(g_mu);
    g_table = table;
    rebuild_lut_locked();
    return GEMM_OK;
}

int save_table(const char *path)
{
    std::lock_guard<std::mutex> g(g_mu);
    std::ofstream f(path);
    if (!f) return GEMM_E_TUNE_TABLE;
    f << "{\"version\": 1, \"arch\": \"gfx950\", \"entries\": [\n";
    size_t i = 0;
    for (auto &kv : g_table) {
        const TuneKey &k = kv.first;
        const TuneVal &v = kv.second;
        char line[256];
        std::snprintf(line, sizeof line,
                      " {\"kclass\": %d, \"trans\": %d, \"bm\": %d, \"bn\": %d, \"bk\": %d, "
                      "\"cfg\": %d, \"order\": %d, \"group\": %d, \"us\": %.3f}%s\n",
                      k.kclass, k.trans, k.bm, k.bn, k.bk, v.cfg, v.order, v.group, v.us,
                      ++i < g_table.size() ? "," : "");
        f << line;
    }
    f << "]}\n";
    return f.good() ? GEMM_OK : GEMM_E_TUNE_TABLE;
}

// Lookup table resolved from the tuning table for every (class, trans, size
// bucket): the nearest tuned bucket (L1 distance in log2 buckets, at most 3,
// an entry of another transposition counting half a step more), or cfg -1
// when none is near (the heuristic decides).
static std::vector<TuneVal> g_lut;
static std::vector<int> g_glut;   // grouped bodies: [class][bm][bn][bk], -1 = none near
constexpr int kNB = 9;   // buckets 4..12
static size_t lut_index(int kclass, int trans, int bm, int bn, int bk)
{
    return ((((size_t)kclass * 4 + trans) * kNB + (bm - 4)) * kNB + (bn - 4)) * kNB + (bk - 4);
}

static void rebuild_lut_locked()
{
    g_lut.assign((size_t)K_NUM * 4 * kNB * kNB * kNB, TuneVal{-1, 0, 8, 0.0});
    for (int kc = 0; kc < K_NUM; ++kc)
        for (int tr = 0; tr < 4; ++tr)
            for (int bm = 4; bm <= 12; ++bm)
                for (int bn = 4; bn <= 12; ++bn)
                    for (int bk = 4; bk <= 12; ++bk) {
                        double best = 1e9;
                        TuneVal v{-1, 0, 8, 0.0};
                        for (auto &kv : g_table) {
                            const TuneKey &t = kv.first;
                            if (t.kclass != kc || t.trans == kGroupedTrans) continue;
                            // an entry tuned for another layout only counts
                            // when its configuration has a kernel for this one
                            if (t.trans != tr && kv.second.cfg >= 0 &&
                                kv.second.cfg < (int)g_by_class[kc].size() &&
                                !g_cfgs[g_by_class[kc][kv.second.cfg]].func[tr][1])
                                continue;
                            const double d = std::abs(t.bm - bm) + std::abs(t.bn - bn) +
                                             std::abs(t.bk - bk) + (t.trans == tr ? 0.0 : 0.5);
                            if (d < best) {
                                best = d;
                                v = kv.second;
                            }
                        }
                        if (best <= 3.5) g_lut[lut_index(kc, tr, bm, bn, bk)] = v;
                    }
    // grouped bodies: the nearest grouped entry of the class
    g_glut.assign((size_t)K_NUM * kNB * kNB * kNB, -1);
    for (int kc = 0; kc < K_NUM; ++kc)
        for (int bm = 4; bm <= 12; ++bm)
            for (int bn = 4; bn <= 12; ++bn)
                for (int bk = 4; bk <= 12; ++bk) {
                    double best = 1e9;
                    int body = -1;
                    for (auto &kv : g_table) {
                        const TuneKey &t = kv.first;
                        if (t.kclass != kc || t.trans != kGroupedTrans) continue;
                        const double d = std::abs(t.bm - bm) + std::abs(t.bn - bn) + std::abs(t.bk - bk);
                        if (d < best) {
                            best = d;
                            body = kv.second.cfg;
                        }
                    }
                    if (best <= 3.5)
                        g_glut[(((size_t)kc * kNB + (bm - 4)) * kNB + (bn - 4)) * kNB + (bk - 4)] = body;
                }
}

int grouped_body_lookup(int kclass, int64_t m, int64_t n, int64_t k)
{
    ensure_table();
    std::lock_guard<std::mutex> g(g_mu);
    if (g_glut.empty() || kclass < 0 || kclass >= K_NUM) return -1;
    return g_glut[(((size_t)kclass * kNB + (bucket(m) - 4)) * kNB + (bucket(n) - 4)) * kNB +
                  (bucket(k) - 4)];
}

void set_table_entry(const TuneKey &key, const TuneVal &val)
{
    std::lock_guard<std::mutex> g(g_mu);
    g_table[key] = val;
}

void rebuild_lut()
{
    std::lock_guard<std::mutex> g(g_mu);
    rebuild_lut_locked();
}

static void ensure_table()
{
    if (g_table_loaded) return;
    g_table_loaded = true;
    const char *env = std::getenv("MGEMM_TUNE_TABLE");
    if (env && *env) {
        load_table(env);
        return;
    }
    const std::string def = lib_dir() + "/mgemm_tune.json";
    std::ifstream probe(def);
    if (probe) load_table(def.c_str());
}

// No tuned entry near the size bucket: the configuration the analytical
// model ranks first among those built for the layout.
static void heuristic(int kclass, int trans, int64_t m, int64_t n, int64_t k, int cus, int &id,
                      int &order, int &group)
{
    id = model_best(kclass, trans, true, m, n, k, cus);
    order = 0;
    group = 8;
}

void select_config(int kclass, int trans, int64_t m, int64_t n, int64_t k, int cus, int &id,
                   int &order, int &group)
{
    int pin, pin_order;
    pinned(kclass, pin, pin_order);
    if (pin >= 0 && pin < (int)g_by_class[kclass].size()) {
        id = pin;
        order = pin_order;
        group = t_tls.force_group > 0 ? t_tls.force_group : 8;
        return;
    }
    ensure_table();
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (!g_lut.empty()) {
            const TuneVal &v = g_lut[lut_index(kclass, trans, bucket(m), bucket(n), bucket(k))];
            if (v.cfg >= 0 && v.cfg < (int)g_by_class[kclass].size()) {
                id = v.cfg;
                order = v.order;
                group = v.group;
                return;
            }
        }
    }
    heuristic(kclass, trans, m, n, k, cus, id, order, group);
}

// Reserved workspace of stream s on device d, or NULL when the reservation
// is smaller than `bytes`.  Never allocates, frees or synchronises.
void *stream_workspace(DevState *d, hipStream_t s, size_t bytes, int slot)
{
    std::lock_guard<std::mutex> g(d->ws_mu);
    auto it = d->ws.find({s, slot});
    if (it == d->ws.end() || it->second.second < bytes) return nullptr;
    return it->second.first;
}

Workspace stream_reservation(DevState *d, hipStream_t s, int slot)
{
    std::lock_guard<std::mutex> g(d->ws_mu);
    auto it = d->ws.find({s, slot});
    Workspace w;
    if (it != d->ws.end()) {
        w.ptr = it->second.first;
        w.bytes = it->second.second;
    }
    return w;
}

int reserve_workspace(DevState *d, hipStream_t s, size_t bytes, int slot)
{
    std::lock_guard<std::mutex> g(d->ws_mu);
    std::pair<void *, size_t> &w = d->ws[{s, slot}];
    if (w.second >= bytes) return GEMM_OK;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return GEMM_E_WORKSPACE;
    }
    const size_t gran = size_t(2) << 20;
    const size_t want = (bytes + gran - 1) / gran * gran;
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        (void)hipGetLastError();
        return GEMM_E_HIP;
    }
    // work already enqueued (or being enqueued by another thread) may still
    // read the old buffer: keep it until shutdown / release
    if (w.first) d->retired.push_back({{s, slot}, w.first});
    w = {p, want};
    return GEMM_OK;
}

void release_workspaces(DevState *d, hipStream_t s)
{
    std::lock_guard<std::mutex> g(d->ws_mu);
    (void)hipStreamSynchronize(s);
    for (auto it = d->ws.begin(); it != d->ws.end();) {
        if (it->first.first == s) {
            if (it->second.first) (void)hipFree(it->second.first);
            it = d->ws.erase(it);
        } else {
            ++it;
        }
    }
    for (auto it = d->retired.begin(); it != d->retired.end();) {
        if (it->first.first == s) {
            (void)hipFree(it->second);
            it = d->retired.erase(it);
        } else {
            ++it;
        }
    }
}

void free_workspaces(DevState *d)
{
    std::lock_guard<std::mutex> g(d->ws_mu);
    for (auto &kv : d->ws)
        if (kv.second.first) (void)hipFree(kv.second.first);
    d->ws.clear();
    for (auto &r : d->retired) (void)hipFree(r.second);
    d->retired.clear();
}

// Split-K plan: S slices of k (each a whole number of stages, at least two)
// chosen to give about two workgroups per CU; S <= 1 runs the plain tile.
static void splitk_plan(const KernelCfg &c, const GemmArgs &a, int cus, int64_t &S, int64_t &kslice)
{
    const int64_t tiles = int64_t(a.tiles_m) * a.tiles_n;
    const int64_t nk = (int64_t(a.k) + c.kc - 1) / c.kc;
    S = (2 * int64_t(cus) + tiles - 1) / tiles;
    S = std::min<int64_t>(S, std::min<int64_t>(16, nk / 2));
    kslice = 0;
    if (S <= 1) return;
    kslice = (nk + S - 1) / S * c.kc;
    S = (a.k + kslice - 1) / kslice;
}

static void packed_sizes(const GemmArgs &a, int64_t &kp, size_t &abytes, size_t &bbytes)
{
    kp = packed_k(a.k, a.terms);
    abytes = (size_t(a.m) * kp * 2 + 255) / 256 * 256;
    bbytes = size_t(a.n) * kp * 2;
}

size_t workspace_need(const KernelCfg &c, const GemmArgs &a, int cus)
{
    if (c.kind == 7) return (size_t)digit_layout(c.kclass, a.m, a.n, a.k).total;
    if (c.packed >= 0) {
        int64_t kp;
        size_t ab, bb;
        packed_sizes(a, kp, ab, bb);
        return ab + bb;
    }
    if (c.base >= 0) {
        int64_t S, kslice;
        splitk_plan(c, a, cus, S, kslice);
        return S > 1 ? size_t(S) * a.m * a.n * 4 : 0;
    }
    return 0;
}

int no_workspace_id(int kclass, int reg, bool vec)
{
    const KernelCfg &c = g_cfgs[reg];
    if (c.kind == 7) return 0;               // the vector-ALU tile
    if (c.packed >= 0) return vec ? 1 : 0;   // the fused split tile
    if (c.base >= 0) {
        const std::vector<int> &ids = g_by_class[kclass];
        for (size_t i = 0; i < ids.size(); ++i)
            if (ids[i] == c.base) return (int)i;   // the unsliced tile
    }
    return 0;
}

// Packed split product: pack op(A) and op(B) into k-contiguous bf16 pieces
// in the workspace w, then run the bf16 tile c.packed ('N','T') over the
// packed k.
static int launch_packed(const KernelCfg &c, int trans, const GemmArgs &a, hipStream_t s,
                         Workspace w)
{
    const int terms = a.terms;
    int64_t kp;
    size_t abytes, bbytes;
    packed_sizes(a, kp, abytes, bbytes);
    if (kp > 0x7FFFFFFF || terms <= 0) return kPackUnavailable;
    if (!w.ptr || w.bytes < abytes + bbytes) return kPackUnavailable;
    char *ws = (char *)w.ptr;
    unsigned short *pa = (unsigned short *)ws, *pb = (unsigned short *)(ws + abytes);
    const bool ta = (trans >> 1) != 0, tb = (trans & 1) != 0;
    int rc = launch_split_pack((const float *)a.A, a.lda, !ta, a.m, a.k, terms, true, pa, s);
    if (rc == GEMM_E_UNSUPPORTED) return kPackUnavailable;
    if (rc != GEMM_OK) return rc;
    rc = launch_split_pack((const float *)a.B, a.ldb, tb, a.n, a.k, terms, false, pb, s);
    if (rc != GEMM_OK) return rc;
    GemmArgs b = a;
    b.A = pa;
    b.lda = kp;
    b.B = pb;
    b.ldb = kp;
    b.k = (int)kp;
    return launch_gemm(g_cfgs[c.packed], 1, true, b, s);
}

// Split-K: partial tiles in the workspace w, then the ordered reduction.
// Without enough workspace (or with one slice) the plain tile runs.
static int launch_splitk(const KernelCfg &c, int trans, bool vec, const GemmArgs &a, hipStream_t s,
                         Workspace w)
{
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    int64_t S, kslice;
    splitk_plan(c, a, d->cus, S, kslice);
    const KernelCfg &b = g_cfgs[c.base];
    if (S <= 1) return launch_gemm(b, trans, vec, a, s);
    const int64_t tiles = int64_t(a.tiles_m) * a.tiles_n;
    if (!w.ptr || w.bytes < size_t(S) * a.m * a.n * 4) return launch_gemm(b, trans, vec, a, s);
    void *ws = w.ptr;
    const void *f = c.func[trans][vec ? 1 : 0];
    if (!f) return GEMM_E_UNSUPPORTED;
    GemmArgs copy = a;
    int ks = (int)kslice;
    void *args[] = {&copy, &ks, &ws};
    hipError_t e = hipLaunchKernel(f, dim3((unsigned)(tiles * S)), dim3(c.threads), args, 0, s);
    if (e == hipSuccess) {
        launch_splitk_reduce(ws, (int)S, a.C, a.ldc, a.m, a.n, a, c.kclass == K_I8, s);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    return GEMM_OK;
}

int launch_gemm(const KernelCfg &c, int trans, bool vec, const GemmArgs &a, hipStream_t s,
                Workspace w)
{
    if (c.packed >= 0) return launch_packed(c, trans, a, s, w);
    if (c.base >= 0) return launch_splitk(c, trans, vec, a, s, w);
    if (c.kind == 7) return launch_digits(c, a, trans, s, w);
    const void *f = c.func[trans][vec ? 1 : 0];
    if (!f) return GEMM_E_UNSUPPORTED;
    const int64_t blocks = int64_t(a.tiles_m) * a.tiles_n;
    if (blocks <= 0 || blocks > 0x7FFFFFFF) return GEMM_E_UNSUPPORTED;
    GemmArgs copy = a;
    void *args[] = {&copy};
    hipError_t e = hipLaunchKernel(f, dim3((unsigned)blocks), dim3(c.threads), args, 0, s);
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    return GEMM_OK;
}

bool vec_ok(const void *X, int64_t ld, int es)
{
    return (reinterpret_cast<uintptr_t>(X) % 16) == 0 && ((ld * es) % 16) == 0;
}

// Fills kernel arguments and picks configuration + staging variant.
// Returns the registry index, or -1 when nothing fits.
int plan_gemm(int dtype, char ta, char tb, int64_t m, int64_t n, int64_t k, double alpha,
              const void *A, int64_t lda, const void *B, int64_t ldb, double beta, void *C,
              int64_t ldc, int cus, GemmArgs &a, int &trans, bool &vec, int &cfg_id, int &kclass)
{
    kclass = kclass_of(dtype, k);
    trans = 2 * (is_trans(ta) ? 1 : 0) + (is_trans(tb) ? 1 : 0);
    int order = 0, group = 8;
    select_config(kclass, trans, m, n, k, cus, cfg_id, order, group);
    const int es = elem_bytes(kclass);
    vec = vec_ok(A, lda, es) && vec_ok(B, ldb, es);
    int reg = g_by_class[kclass][cfg_id];
    if (!g_cfgs[reg].func[trans][vec ? 1 : 0]) {
        // no kernel of this configuration for the layout / staging: a tuned
        // choice gives way to the model's best among the configurations that
        // have one; a forced one to the class's first configuration, which
        // carries every element-wise staging variant
        int pin, pin_order;
        pinned(kclass, pin, pin_order);
        const bool forced = pin >= 0;
        cfg_id = forced ? 0 : model_best(kclass, trans, vec, m, n, k, cus);
        reg = g_by_class[kclass][cfg_id];
        if (!g_cfgs[reg].func[trans][vec ? 1 : 0]) {
            cfg_id = 0;
            reg = g_by_class[kclass][0];
            if (!g_cfgs[reg].func[trans][vec ? 1 : 0]) return -1;
        }
    }
    const KernelCfg &c = g_cfgs[reg];
    a.A = A;
    a.B = B;
    a.C = C;
    a.lda = lda;
    a.ldb = ldb;
    a.ldc = ldc;
    a.m = (int)m;
    a.n = (int)n;
    a.k = (int)k;
    a.alpha = (float)alpha;
    a.beta = (float)beta;
    const bool int_out = dtype == GEMM_I8 || dtype == GEMM_I16 || dtype == GEMM_I32;
    a.ialpha = int_out ? (int)alpha : 0;
    a.ibeta = int_out ? (int)beta : 0;
    a.tiles_m = (int)((m + c.mc - 1) / c.mc);
    a.tiles_n = (int)((n + c.nc - 1) / c.nc);
    a.order = order;
    a.group = std::max(1, group);
    a.terms = split_terms(kclass);
    a.dalpha = alpha;
    a.dbeta = beta;
    return reg;
}

int gemm_ws(char transA, char transB, int64_t m, int64_t n, int64_t k, double alpha,
            const void *A, int64_t lda, const void *B, int64_t ldb, double beta, void *C,
            int64_t ldc, int dtype, Workspace w, bool reject_short)
{
    const int v = validate(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (v != 0) return v;
    if (m == 0 || n == 0) return GEMM_OK;
    if ((alpha == 0.0 || k == 0) && beta == 1.0) return GEMM_OK;
    if (m > 0x7FFFFFFF || n > 0x7FFFFFFF || k > 0x7FFFFFFF) return GEMM_E_UNSUPPORTED;
    ensure_registered();
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    hipStream_t s = t_tls.stream;
    if (alpha == 0.0 || k == 0) {
        const int elem = (dtype == GEMM_I8 || dtype == GEMM_I16 || dtype == GEMM_I32) ? 1
                         : (dtype == GEMM_F64 ? 2 : 0);
        launch_scale(C, ldc, (int)m, (int)n, beta, elem, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            t_tls.hip_err = (int)e;
            return GEMM_E_HIP;
        }
        t_tls.last[0] = dtype;
        t_tls.last[1] = -1;
        t_tls.last[2] = -1;
        t_tls.last[3] = 0;
        return GEMM_OK;
    }
    GemmArgs a;
    int trans = 0, cfg = 0, kclass = 0;
    bool vec = true;
    const int reg = plan_gemm(dtype, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                              d->cus, a, trans, vec, cfg, kclass);
    if (reg < 0) return GEMM_E_UNSUPPORTED;
    int run = reg;
    const size_t need = workspace_need(g_cfgs[reg], a, d->cus);
    if (need > 0 && (!w.ptr || w.bytes < need)) {
        if (reject_short) return GEMM_E_WORKSPACE;
        // the workspace is too small (nothing is allocated here): the
        // class's configuration that needs none
        const int saved = t_tls.force_id[kclass];
        t_tls.force_id[kclass] = no_workspace_id(kclass, reg, vec);
        run = plan_gemm(dtype, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                        d->cus, a, trans, vec, cfg, kclass);
        t_tls.force_id[kclass] = saved;
        if (run < 0) return GEMM_E_UNSUPPORTED;
    }
    const bool debug = g_debug.load(std::memory_order_relaxed) && d->debug_count && beta == 0.0;
    const int es = dtype == GEMM_F64 ? 8 : 4;
    if (debug) launch_debug_fill(C, ldc, m, n, es, s);
    rc = launch_gemm(g_cfgs[run], trans, vec, a, s, w);
    if (rc == kPackUnavailable) rc = GEMM_E_UNSUPPORTED;   // packing pass not built for this case
    if (rc == GEMM_OK && debug) launch_debug_count(C, ldc, m, n, es, d->debug_count, s);
    if (rc == GEMM_OK) {
        t_tls.last[0] = dtype;
        t_tls.last[1] = cfg;
        t_tls.last[2] = a.order;
        t_tls.last[3] = a.terms;
    }
    return rc;
}

// The debug counter of a device (allocated once, zeroed; outside any capture).
static int debug_device_init(DevState *d)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (d->debug_count) return GEMM_OK;
    unsigned long long *p = nullptr;
    hipError_t e = hipMalloc((void **)&p, sizeof *p);
    if (e == hipSuccess) e = hipMemset(p, 0, sizeof *p);
    if (e != hipSuccess) {
        if (p) (void)hipFree(p);
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    d->debug_count = p;
    return GEMM_OK;
}

// The kernel class whose configurations a query about dtype lists (the x3
// split: its three-term class).
static int class_for_query(int dtype)
{
    if (dtype == GEMM_F32_BF16X3) return K_SPLIT2;
    return kclass_of(dtype, 0);
}

// MGEMM_DEBUG (non-empty and not "0") and MGEMM_FORCE_CFG, a comma-separated
// list of dtype:id[:order] (dtype codes as in mgemm.h; entries that do not
// parse or name no configuration are ignored).
static void apply_env_settings()
{
    const char *dbg = std::getenv("MGEMM_DEBUG");
    g_debug.store(dbg && *dbg && std::strcmp(dbg, "0") != 0);
    int pin[K_NUM], pin_order[K_NUM];
    for (int c = 0; c < K_NUM; ++c) {
        pin[c] = -1;
        pin_order[c] = 0;
    }
    const char *v = std::getenv("MGEMM_FORCE_CFG");
    while (v && *v) {
        char *end = nullptr;
        const long dt = std::strtol(v, &end, 10);
        long id = -1, order = 0;
        bool ok = end != v && *end == ':';
        if (ok) {
            v = end + 1;
            id = std::strtol(v, &end, 10);
            ok = end != v;
            if (ok && *end == ':') {
                v = end + 1;
                order = std::strtol(v, &end, 10);
                ok = end != v && (order == 0 || order == 1);
            }
        }
        if (ok && dt >= 0 && dt < GEMM_NUM_DTYPES && id >= 0) {
            int classes[2] = {class_for_query((int)dt), dt == GEMM_F32_BF16X3 ? K_SPLIT3 : -1};
            for (int c : classes)
                if (c >= 0 && id < (long)g_by_class[c].size()) {
                    pin[c] = (int)id;
                    pin_order[c] = (int)order;
                }
        }
        const char *comma = std::strchr(end ? end : v, ',');
        v = comma ? comma + 1 : nullptr;
    }
    for (int c = 0; c < K_NUM; ++c) {
        g_env_pin_order[c].store(pin_order[c], std::memory_order_relaxed);
        g_env_pin[c].store(pin[c] + 1, std::memory_order_relaxed);
    }
}

}  // namespace mg

using namespace mg;

extern "C" {

int gemm(char transA, char transB, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
         int64_t lda, const void *B, int64_t ldb, double beta, void *C, int64_t ldc, int dtype)
{
    // argument errors before any runtime call
    const int v = validate(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (v != 0) return v;
    // the workspace reserved for the calling thread's stream (none when the
    // device has no state yet: gemm_ws reports that device's error itself)
    Workspace w;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices && g_dev[dev].init)
        w = stream_reservation(&g_dev[dev], t_tls.stream, 0);
    return gemm_ws(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, w, false);
}

int gemm_set_stream(void *hip_stream)
{
    t_tls.stream = (hipStream_t)hip_stream;
    return GEMM_OK;
}

// Default reservations of gemm_init on the calling thread's stream (bytes;
// MGEMM_WORKSPACE_BYTES / MGEMM_SCALED_WORKSPACE_BYTES override, 0 = none):
// enough for the packed split product at 8192^3 (2 (m + n) 3k bf16 values,
// 805 MB) and for the scaled path's quantised operands and partial product
// at 8192^3 in binary16 with beta != 0 (about 537 MB).
constexpr int64_t kDefaultWorkspace = int64_t(1) << 30;
constexpr int64_t kDefaultScaledWorkspace = int64_t(768) << 20;

static int64_t env_bytes(const char *name, int64_t dflt)
{
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    char *end = nullptr;
    const long long x = std::strtoll(v, &end, 10);
    return (end && *end == '\0' && x >= 0) ? (int64_t)x : dflt;
}

int gemm_init(const char *tune_table_path)
{
    ensure_registered();
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    if (tune_table_path && *tune_table_path) {
        g_table_loaded = true;
        rc = load_table(tune_table_path);
        if (rc != GEMM_OK) return rc;
    } else {
        ensure_table();
    }
    rc = grouped_device_init(d);
    if (rc != GEMM_OK) return rc;
    rc = scratch_device_init(d->device);
    if (rc != GEMM_OK) return rc;
    rc = debug_device_init(d);
    if (rc != GEMM_OK) return rc;
    apply_env_settings();
    const hipStream_t s = t_tls.stream;
    rc = reserve_workspace(d, s, (size_t)env_bytes("MGEMM_WORKSPACE_BYTES", kDefaultWorkspace), 0);
    if (rc != GEMM_OK) return rc;
    return reserve_workspace(d, s,
                             (size_t)env_bytes("MGEMM_SCALED_WORKSPACE_BYTES", kDefaultScaledWorkspace), 1);
}

void gemm_shutdown(void)
{
    for (int i = 0; i < kMaxDevices; ++i) {
        grouped_device_free(&g_dev[i]);
        free_workspaces(&g_dev[i]);
        if (g_dev[i].debug_count) {
            (void)hipFree(g_dev[i].debug_count);
            g_dev[i].debug_count = nullptr;
        }
    }
}

int gemm_reserve_workspace(int64_t bytes, int64_t scaled_bytes)
{
    if (bytes < 0) return -1;
    if (scaled_bytes < 0) return -2;
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    const hipStream_t s = t_tls.stream;
    if (bytes > 0 && (rc = reserve_workspace(d, s, (size_t)bytes, 0)) != GEMM_OK) return rc;
    if (scaled_bytes > 0 && (rc = reserve_workspace(d, s, (size_t)scaled_bytes, 1)) != GEMM_OK)
        return rc;
    return GEMM_OK;
}

int gemm_release_workspace(void)
{
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    release_workspaces(d, t_tls.stream);
    return GEMM_OK;
}

int64_t gemm_workspace_bytes(char transA, char transB, int64_t m, int64_t n, int64_t k, int dtype)
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES || !trans_ok(transA) || !trans_ok(transB) || m < 0 ||
        n < 0 || k < 0)
        return -1;
    if (m == 0 || n == 0 || k == 0) return 0;
    if (m > 0x7FFFFFFF || n > 0x7FFFFFFF || k > 0x7FFFFFFF) return -1;
    ensure_registered();
    DevState *d = nullptr;
    if (device_state(&d) != GEMM_OK) return -1;
    // 16-byte aligned stand-in operands with the smallest leading dimensions
    const int es = elem_bytes(kclass_of(dtype, k));
    const int64_t lda = is_trans(transA) ? m : k, ldb = is_trans(transB) ? k : n;
    const int64_t al = 16 / es;
    const void *fake = (const void *)uintptr_t(4096);
    GemmArgs a;
    int trans = 0, cfg = 0, kclass = 0;
    bool vec = true;
    const int reg = plan_gemm(dtype, transA, transB, m, n, k, 1.0, fake, (lda + al - 1) / al * al,
                              fake, (ldb + al - 1) / al * al, 0.0, (void *)fake, n, d->cus, a, trans,
                              vec, cfg, kclass);
    if (reg < 0) return 0;
    return (int64_t)workspace_need(g_cfgs[reg], a, d->cus);
}

const char *gemm_strerror(int code)
{
    if (code < 0) return "invalid argument (the code's magnitude is the argument number)";
    switch (code) {
    case GEMM_OK: return "success";
    case GEMM_E_HIP: return "HIP runtime error";
    case GEMM_E_UNSUPPORTED: return "unsupported dtype, size or configuration";
    case GEMM_E_NOINIT: return "no usable GPU device";
    case GEMM_E_WORKSPACE: return "workspace too small (grouped problem count, or the workspace a configuration needs)";
    case GEMM_E_TUNE_TABLE: return "tuning table unreadable or malformed";
    case GEMM_E_SERVE: return "serving loop configuration or backend failure";
    default: return "unknown error";
    }
}

int gemm_last_hip_error(void) { return t_tls.hip_err; }

int gemm_num_configs(int dtype)
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -1;
    ensure_registered();
    return (int)g_by_class[class_for_query(dtype)].size();
}

int gemm_config_info(int dtype, int id, int64_t out[8])
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -1;
    ensure_registered();
    const std::vector<int> &ids = g_by_class[class_for_query(dtype)];
    if (id < 0 || id >= (int)ids.size()) return -2;
    if (!out) return -3;
    const KernelCfg &c = g_cfgs[ids[id]];
    out[0] = c.mc;
    out[1] = c.nc;
    out[2] = c.kc;
    out[3] = c.mc / c.wm;
    out[4] = c.nc / c.wn;
    out[5] = c.threads;
    out[6] = c.lds;
    out[7] = c.kind;
    return GEMM_OK;
}

int gemm_config_staging(int dtype, int id)
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -1;
    ensure_registered();
    const std::vector<int> &ids = g_by_class[class_for_query(dtype)];
    if (id < 0 || id >= (int)ids.size()) return -2;
    const KernelCfg &c = g_cfgs[ids[id]];
    if (c.kind == 7) return 6;
    if (c.unpacked) return 2 + c.unpacked;
    return c.packed >= 0 ? 2 : (c.direct ? 1 : 0);
}

int gemm_config_mfma(int dtype, int id)
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -1;
    ensure_registered();
    const std::vector<int> &ids = g_by_class[class_for_query(dtype)];
    if (id < 0 || id >= (int)ids.size()) return -2;
    return g_cfgs[ids[id]].mfma;
}

int gemm_config_layouts(int dtype, int id)
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -1;
    ensure_registered();
    const std::vector<int> &ids = g_by_class[class_for_query(dtype)];
    if (id < 0 || id >= (int)ids.size()) return -2;
    const KernelCfg &c = g_cfgs[ids[id]];
    int mask = 0;
    for (int t = 0; t < 4; ++t)
        for (int v = 0; v < 2; ++v)
            if (c.func[t][v]) mask |= 1 << (2 * t + v);
    return mask;
}

int gemm_force_config(int dtype, int id, int order)
{
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -1;
    if (order < 0 || order > 1) return -3;
    ensure_registered();
    int classes[2] = {class_for_query(dtype), -1};
    if (dtype == GEMM_F32_BF16X3) classes[1] = K_SPLIT3;
    for (int c : classes) {
        if (c < 0) continue;
        if (id >= (int)g_by_class[c].size()) {
            if (dtype != GEMM_F32_BF16X3) return -2;
            continue;
        }
        t_tls.force_id[c] = id < 0 ? -1 : id;
        t_tls.force_order[c] = order;
    }
    return GEMM_OK;
}

int gemm_debug_count(const void *C, int64_t m, int64_t n, int64_t ldc, int dtype)
{
    if (!C && m > 0 && n > 0) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (ldc < std::max<int64_t>(1, n)) return -4;
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -5;
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    if (!d->debug_count) return GEMM_E_NOINIT;
    if (m == 0 || n == 0) return GEMM_OK;
    launch_debug_count(C, ldc, m, n, dtype == GEMM_F64 ? 8 : 4, d->debug_count, t_tls.stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    return GEMM_OK;
}

int64_t gemm_debug_unwritten(void)
{
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return -rc;
    if (!d->debug_count) return -GEMM_E_NOINIT;
    unsigned long long v = 0;
    hipError_t e = hipStreamSynchronize(t_tls.stream);
    if (e == hipSuccess) e = hipMemcpy(&v, d->debug_count, sizeof v, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemset(d->debug_count, 0, sizeof v);
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        return -GEMM_E_HIP;
    }
    return (int64_t)v;
}

int gemm_last_config(int64_t out[4])
{
    if (!out) return -1;
    for (int i = 0; i < 4; ++i) out[i] = t_tls.last[i];
    return GEMM_OK;
}

}  // extern "C"
