// Shared host-side state and helpers of the C ABI (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "registry.hpp"

namespace mg {

constexpr int kMaxDevices = 64;

// Per-device state: created on first use (or gemm_init) of a device.
struct DevState {
    bool init = false;
    int device = 0;
    int cus = 0;
    // grouped launches: device descriptor tables and pinned host staging
    bool grouped_ready = false;
    void *grouped = nullptr;
    // workspaces reserved per stream (work on one stream is ordered, so its
    // GEMMs can share one); only gemm_init, gemm_reserve_workspace and the
    // tuner allocate them, GEMM calls only look them up
    std::mutex ws_mu;
    std::map<std::pair<hipStream_t, int>, std::pair<void *, size_t>> ws;   // (stream, slot)
    // buffers replaced by a larger reservation: a call on another thread may
    // still be enqueuing work that reads them, so they are freed only at
    // gemm_shutdown (or gemm_release_workspace of their stream)
    std::vector<std::pair<std::pair<hipStream_t, int>, void *>> retired;
    // debug mode: count of sentinel elements found (allocated by gemm_init)
    unsigned long long *debug_count = nullptr;
};

// Internal status of launch_gemm: a packed configuration could not get its
// workspace (the caller falls back to a fused configuration).
constexpr int kPackUnavailable = 100;

// Tuning table key: kernel class, trans index (2*tA + tB), log2 size buckets.
// Entries with trans == kGroupedTrans choose the grouped kernel's tile body
// for the bucket (cfg = body index, below kMaxGroupedBodies).
constexpr int kGroupedTrans = 4;
constexpr int kMaxGroupedBodies = 8;
struct TuneKey {
    int kclass, trans, bm, bn, bk;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(kclass, trans, bm, bn, bk) < std::tie(o.kclass, o.trans, o.bm, o.bn, o.bk);
    }
};
struct TuneVal {
    int cfg, order, group;
    double us;
};

// Per-thread state.
struct Tls {
    hipStream_t stream = nullptr;
    int force_id[K_NUM];
    int force_order[K_NUM];
    int force_group = 0;
    int force_body = -1;      // grouped kernel: body for every problem (-1: per bucket)
    int64_t last[4];
    int hip_err = 0;
    Tls();
};

extern std::mutex g_mu;
extern std::vector<KernelCfg> g_cfgs;
extern std::vector<int> g_by_class[K_NUM];
extern DevState g_dev[kMaxDevices];
extern std::map<TuneKey, TuneVal> g_table;
extern thread_local Tls t_tls;

int kclass_of(int dtype, int64_t k);
int elem_bytes(int kclass);
int split_terms(int kclass);
int bucket(int64_t x);
int validate(char ta, char tb, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
             int64_t lda, const void *B, int64_t ldb, double beta, const void *C, int64_t ldc,
             int dtype);
void ensure_registered();
int device_state(DevState **out);
int load_table(const char *path);
// Tuned grouped body of (class, size bucket), or -1 when no entry is near.
int grouped_body_lookup(int kclass, int64_t m, int64_t n, int64_t k);
// Adds or replaces one tuning-table entry (call rebuild_lut afterwards).
void set_table_entry(const TuneKey &key, const TuneVal &val);
int save_table(const char *path);
void rebuild_lut();
void select_config(int kclass, int trans, int64_t m, int64_t n, int64_t k, int cus, int &id,
                   int &order, int &group);
bool vec_ok(const void *X, int64_t ld, int es);
int plan_gemm(int dtype, char ta, char tb, int64_t m, int64_t n, int64_t k, double alpha,
              const void *A, int64_t lda, const void *B, int64_t ldb, double beta, void *C,
              int64_t ldc, int cus, GemmArgs &a, int &trans, bool &vec, int &cfg_id, int &kclass);
// Device workspace handed to a launch: the packed split's operand pieces or
// split-K's partial tiles live in [ptr, ptr + bytes).
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};
int launch_gemm(const KernelCfg &c, int trans, bool vec, const GemmArgs &a, hipStream_t s,
                Workspace w = Workspace());
// gemm() with an explicit workspace.  When the planned configuration needs
// more than w.bytes: reject_short ? GEMM_E_WORKSPACE (nothing launched) : the
// class's configuration that needs none.  Validation and quick returns as gemm().
int gemm_ws(char transA, char transB, int64_t m, int64_t n, int64_t k, double alpha,
            const void *A, int64_t lda, const void *B, int64_t ldb, double beta, void *C,
            int64_t ldc, int dtype, Workspace w, bool reject_short);

// kernels_int.hip: INT16 / INT32 digit products.  Workspace layout of one
// call: A's planes (m rows of P*kp int8), B's (n rows), then (INT16) the
// row sums of op(A) and column sums of op(B) (int32).
struct DigitLayout {
    int P = 0;           // digit planes per operand (2 or 4)
    int64_t kp = 0;      // k rounded up to 64
    int64_t a_off = 0, b_off = 0, sums_off = 0, total = 0;   // bytes
};
DigitLayout digit_layout(int kclass, int64_t m, int64_t n, int64_t k);
int launch_digits(const KernelCfg &c, const GemmArgs &a, int trans, hipStream_t s, Workspace w);

// noalloc.hip: the fixed device scratch array of gemm_noalloc (bytes), and
// the per-device lookup of its address (gemm_init, or the first call).
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
int scratch_device_init(int device);

// misc.hip: fills `count` elements of the tuner's operands (kind: 0 f32,
// 1 bf16, 2 f16, 3 e4m3, 4 int8, 5 f64, 6 int16, 7 int32).
void launch_fill(void *p, int64_t count, int kind, uint32_t seed, hipStream_t s);

// grouped.hip
int grouped_device_init(DevState *d);
void grouped_device_free(DevState *d);

// pack.hip: split-product packing
int64_t packed_k(int64_t k, int terms);
int launch_split_pack(const float *X, int64_t ld, bool kmode, int64_t rows, int64_t k, int terms,
                      bool a_side, unsigned short *out, hipStream_t s);
const void *split_pack_entry();
// slot 0: the kernels' own workspace (packed split, split-K); slot 1: the
// scaled path's quantised operands, which outlive the GEMM it calls.
// stream_workspace returns the stream's reserved buffer when it holds at
// least `bytes`, else NULL; it never allocates, frees or synchronises.
void *stream_workspace(DevState *d, hipStream_t s, size_t bytes, int slot = 0);
// The whole reservation of (s, slot); {NULL, 0} when there is none.
Workspace stream_reservation(DevState *d, hipStream_t s, int slot = 0);
// Grows the reservation of (s, slot) to at least `bytes` (allocates; refused
// during a graph capture).  The replaced buffer is retired, not freed.
int reserve_workspace(DevState *d, hipStream_t s, size_t bytes, int slot);
// Frees every reservation of stream s (and its retired buffers) after
// synchronising the stream.
void release_workspaces(DevState *d, hipStream_t s);
// Workspace bytes configuration c needs for the planned call a (0: none).
size_t workspace_need(const KernelCfg &c, const GemmArgs &a, int cus);
// Configuration of the same class that needs no workspace, for c (id within
// the class), when c's workspace is not available.
int no_workspace_id(int kclass, int reg, bool vec);

// Analytical model (model.cpp): cycles / microseconds of configuration c on
// an m x n x k problem, and the class's configuration it ranks first.
double model_cycles(const KernelCfg &c, int kclass, int64_t m, int64_t n, int64_t k, int cus);
double model_us(const KernelCfg &c, int kclass, int64_t m, int64_t n, int64_t k, int cus);
int model_best(int kclass, int trans, bool vec, int64_t m, int64_t n, int64_t k, int cus);
void free_workspaces(DevState *d);

}  // namespace mg
