/*
 * mgemm: blocked GEMM family for AMD Instinct MI355X (gfx950) - C ABI.
 *
 * The operation is the paper's matrix multiplication C = C + A B
 * (section 3.1, "The baseline algorithm"; A is m x k, B is k x n, C is
 * m x n), generalised to the BLAS form
 *
 *     C = alpha * op(A) * op(B) + beta * C
 *
 * and computed with the five loops around a micro-kernel of section 3
 * (Figures "Baseline (B3A2C0) and A3B2C0 algorithms" and "B3C2A0 and
 * A3C2B0 algorithms"), panel packing (section 5.3) and a register-resident
 * micro-tile (section 4.1), re-derived for CDNA4: packing is global->LDS
 * staging, the micro-kernel is a tile of MFMA instructions.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout: ROW-MAJOR.  lda, ldb, ldc are row strides in elements.
 *   transA 'N': A is stored m x k, lda >= max(1,k);  'T': stored k x m, lda >= max(1,m)
 *   transB 'N': B is stored k x n, ldb >= max(1,n);  'T': stored n x k, ldb >= max(1,k)
 *   ldc >= max(1,n).  Accepted trans characters: N n T t C c ('C' = 'T', real data).
 * Types (by dtype):
 *   GEMM_F32, GEMM_F32_BF16X3, GEMM_F32_BF16X3_ONLY, GEMM_F32_BF16X6:
 *                       A, B float32;  C float32
 *   GEMM_BF16:          A, B bfloat16 (raw 16-bit patterns); C float32
 *   GEMM_F16:           A, B IEEE binary16;                   C float32
 *   GEMM_F8E4M3:        A, B OCP FP8 E4M3FN bytes;            C float32
 *   GEMM_I8:            A, B int8;                            C int32
 *   GEMM_F64:           A, B float64;                         C float64
 *   GEMM_I16:           A, B int16;                           C int32
 *   GEMM_I32:           A, B int32;                           C int32
 *   Accumulation is FP32 for the float types up to FP32, FP64 for GEMM_F64
 *   and INT32 for GEMM_I8.  alpha and beta are passed as double, used as
 *   float32 by the FP32-output paths and as double by GEMM_F64; for the
 *   integer types they must be integers representable in int32 and the
 *   result is the exact integer alpha*op(A)*op(B) + beta*C modulo 2^32
 *   (two's complement).
 * Pointers: A, B, C are DEVICE pointers owned by the caller, aligned at least
 *   to their element size.  The library never frees or retains them.
 * Semantics (BLAS):
 *   m == 0 or n == 0                    -> returns 0, nothing is read or written
 *   (alpha == 0 or k == 0), beta == 1   -> returns 0, nothing is read or written
 *   alpha == 0 or k == 0                -> C = beta*C; A and B are not read
 *   beta == 0                           -> C is not read (NaN/Inf in C are overwritten)
 * Execution: asynchronous on the calling thread's current stream (see
 *   gemm_set_stream); no host synchronisation.  Device faults surface at the
 *   caller's next synchronisation.  Results are deterministic run to run: each
 *   kernel configuration fixes its k-summation order.
 * Errors: 0 on success; -i when the i-th argument (1-based, BLAS xerbla
 *   convention) is invalid; a positive GEMM_E_* code otherwise.  No C++
 *   exception crosses this interface.
 * Threads: entry points may be called from several host threads; stream and
 *   last-error state are per thread.
 */
#ifndef MGEMM_H
#define MGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GEMM_F32 = 0,             /* plain FP32: FP32 MFMA (v_mfma_f32_16x16x4_f32)            */
    GEMM_F32_BF16X3 = 1,      /* FP32-accurate: A, B split into bf16 pieces on the fly;    */
                              /* 3 piece products when k >= 64, 6 when k < 64              */
    GEMM_BF16 = 2,            /* bfloat16 inputs                                           */
    GEMM_F16 = 3,             /* binary16 inputs                                           */
    GEMM_F8E4M3 = 4,          /* OCP e4m3fn inputs, unit block scales                      */
    GEMM_I8 = 5,              /* int8 inputs, int32 accumulate, bit-exact                  */
    GEMM_F32_BF16X3_ONLY = 6, /* split product, always 3 terms (hi*hi, hi*mid, mid*hi)     */
    GEMM_F32_BF16X6 = 7,      /* split product, always 6 terms (adds mid*mid, hi*lo, lo*hi)*/
    GEMM_F64 = 8,             /* FP64 inputs, FP64 accumulate (v_mfma_f64_16x16x4f64) and  */
                              /* FP64 C; alpha and beta used in full double precision;     */
                              /* gemm() only (the grouped and serving paths return         */
                              /* GEMM_E_UNSUPPORTED / reject it)                           */
    GEMM_I16 = 9,             /* int16 inputs, int32 C: four INT8 MFMA digit products      */
                              /* and a rank-two correction (or the vector ALUs); exact     */
                              /* value modulo 2^32; gemm() only                            */
    GEMM_I32 = 10,            /* int32 inputs and C: ten INT8 MFMA digit products modulo   */
                              /* 2^32 (or the vector ALUs); gemm() only                    */
    GEMM_NUM_DTYPES = 11
} gemm_dtype;

enum {
    GEMM_OK = 0,
    GEMM_E_HIP = 1,          /* a HIP runtime call failed; see gemm_last_hip_error()      */
    GEMM_E_UNSUPPORTED = 2,  /* no kernel built for this dtype / configuration             */
    GEMM_E_NOINIT = 3,       /* no usable GPU device                                       */
    GEMM_E_WORKSPACE = 4,    /* workspace too small: grouped count above capacity, or a    */
                             /* configuration's workspace above what the call may use      */
    GEMM_E_TUNE_TABLE = 5,   /* tuning table file unreadable or malformed                  */
    GEMM_E_SERVE = 6         /* serving loop: invalid configuration or backend failure     */
};

/*
 * gemm: C = alpha * op(A) * op(B) + beta * C on the current stream.
 *   Arguments (1-based numbers used by the -i error convention):
 *    1 transA, 2 transB, 3 m, 4 n, 5 k, 6 alpha, 7 A, 8 lda, 9 B, 10 ldb,
 *   11 beta, 12 C, 13 ldc, 14 dtype.
 *   Invalid: trans not in NnTtCc; m, n or k < 0; ld below the minimum above;
 *   A or B NULL when they must be read; C NULL when it must be written;
 *   dtype unknown; for GEMM_I8, alpha (-6) or beta (-11) not an int32 integer.
 *   The loop order, the block sizes (mc, nc, kc) and the MFMA wave tile are
 *   chosen per (dtype, trans, size bucket) from the tuning table (gemm_init).
 *   Packed split and split-K configurations use the workspace reserved for
 *   the calling thread's stream (gemm_init, gemm_reserve_workspace); gemm()
 *   itself never allocates, frees or synchronises.  When the reservation is
 *   smaller than the chosen configuration needs (gemm_workspace_bytes), the
 *   call runs the class's configuration that needs none (the unsliced tile
 *   for split-K, the fused split tile for the packed split); the result is
 *   equal to the oracle's at the same tolerance either way.
 */
int gemm(char transA, char transB, int64_t m, int64_t n, int64_t k,
         double alpha, const void *A, int64_t lda, const void *B, int64_t ldb,
         double beta, void *C, int64_t ldc, int dtype);

/*
 * gemm_noalloc: gemm() for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, layouts, semantics and results as gemm() (the
 * same configuration is chosen, so results are bitwise equal to gemm()'s
 * whenever gemm() has the workspace that configuration needs).  Packed split
 * and split-K configurations take their workspace from a fixed device array
 * of gemm_noalloc_scratch_bytes() = 64 MiB that the library holds on each
 * GPU it runs on until the process ends; no reservation or gemm_init is
 * needed (gemm_init looks the array up ahead of time; otherwise the first
 * call on a device does).  The call never allocates, frees or synchronises.
 * When the chosen configuration needs more than 64 MiB of workspace
 * (gemm_workspace_bytes), the call returns GEMM_E_WORKSPACE and launches
 * nothing: run gemm() instead.  All calls on one GPU share the array, and
 * each call overwrites what the last left there: calls that may execute at
 * the same time on one GPU (different streams without ordering between
 * them) race; calls on one stream, or otherwise ordered, are safe.  Nothing
 * in the array needs to start at zero (every byte a launch reads was written
 * earlier in the same call).  Argument errors as gemm().
 */
int gemm_noalloc(char transA, char transB, int64_t m, int64_t n, int64_t k,
                 double alpha, const void *A, int64_t lda, const void *B, int64_t ldb,
                 double beta, void *C, int64_t ldc, int dtype);

/* Size in bytes of gemm_noalloc's fixed device scratch array. */
int64_t gemm_noalloc_scratch_bytes(void);

/*
 * Power-of-two scaled low-precision GEMM on FP32 operands (A, B, C float32,
 * the layouts and BLAS semantics of gemm()).  Each row i of op(A) and each
 * column j of op(B) is scaled by 2^-e_i, 2^-f_j so that its largest
 * magnitude M lands in [2^T, 2^(T+1)) (e = floor(log2 M) - T; rows that are
 * zero or hold Inf/NaN: e = 0), rounded to the format of `dtype` (nearest,
 * ties to even; E4M3 saturates at 448) and multiplied by that format's GEMM
 * (FP32 accumulation); then C = alpha * 2^(e_i + f_j) * product + beta * C.
 * dtype: GEMM_BF16 (T = 0), GEMM_F16 (T = 14) or GEMM_F8E4M3 (T = 7); other
 * values return -14.  For data whose rows and columns span more magnitudes
 * than the format holds (A = Dr A0 Dc with diagonal scalings over 2^+-20,
 * say), where the plain FP16 and FP8 paths overflow or flush to zero.  The
 * quantised operands live in the stream's second reserved workspace, of
 * gemm_scaled_workspace_bytes() bytes: about (m*k + k*n)*bytes + 16*(m + n)
 * (exponents and the partial maxima of the strided exponent reductions;
 * + 4*m*n when beta != 0).  When the reservation is smaller the call returns
 * GEMM_E_WORKSPACE and launches nothing; it never allocates.  Asynchronous on
 * the current stream like gemm().  Argument errors follow gemm(), with
 * argument 14 (dtype) checked after the others.
 */
int gemm_scaled(char transA, char transB, int64_t m, int64_t n, int64_t k, double alpha,
                const void *A, int64_t lda, const void *B, int64_t ldb, double beta, void *C,
                int64_t ldc, int dtype);

/* Bytes of the scaled path's workspace one gemm_scaled call of these sizes
 * needs; -1 for invalid sizes or a dtype gemm_scaled does not take. */
int64_t gemm_scaled_workspace_bytes(char transA, char transB, int64_t m, int64_t n, int64_t k,
                                    double beta, int dtype);

/* One problem of a grouped call; the fields mean what gemm()'s arguments do. */
typedef struct {
    char transA, transB;
    int64_t m, n, k;
    double alpha;
    const void *A;
    int64_t lda;
    const void *B;
    int64_t ldb;
    double beta;
    void *C;
    int64_t ldc;
} gemm_problem;

/*
 * gemm_grouped: `count` independent problems of one dtype in ONE persistent
 * kernel launch (plus one host-to-device copy of the descriptor table) on the
 * current stream.  `problems` is a HOST array, copied into library-owned
 * pinned staging before return, so the caller may reuse it immediately.
 * Each problem is validated as gemm() would: an invalid argument i of problem
 * p returns -(1000*p + i) and nothing is launched.  Problems that gemm()
 * would quick-return are skipped.  Output regions of different problems
 * must not overlap.  Returns GEMM_E_WORKSPACE when count exceeds
 * gemm_grouped_capacity().  Calls rotate over a few library staging slots;
 * a slot is reused only after the stream has consumed its previous table (an
 * event guards reuse), so back-to-back calls are safe, and a call whose slot
 * still has a copy in flight waits on the host for that copy.  Loops that
 * must never wait, and graph capture, use the slots below.
 */
int gemm_grouped(int64_t count, const gemm_problem *problems, int dtype);

/* Maximum `count` accepted by gemm_grouped (fixed at initialisation). */
int64_t gemm_grouped_capacity(void);

/*
 * Graph-capturable grouped launch.
 *   gemm_grouped_slot_create(&slot, capacity): a library-owned descriptor slot
 *     (pinned host table, device table, device counters) for up to `capacity`
 *     problems (1 <= capacity <= gemm_grouped_capacity()).  Allocates; call it
 *     outside any capture.
 *   gemm_grouped_slot_write(slot, count, problems, dtype): validates like
 *     gemm_grouped (errors -(1000*p + i)) and writes the table into the slot's
 *     pinned memory.  The dtype family (FP32 / split / BF16 / FP16 / FP8 /
 *     INT8) of a slot is fixed by its first write, and so is its kernel: a
 *     first batch whose problems are all 'N','N' with 16-byte aligned A, B
 *     and leading dimensions selects the compact kernel for that case, and
 *     later batches that do not qualify return GEMM_E_UNSUPPORTED (any
 *     other first batch selects the general kernel, which takes anything).
 *     count <= capacity.
 *   gemm_grouped_slot_launch(slot): enqueues, on the current stream, one copy
 *     of the pinned table (header + capacity descriptors) to the device and
 *     one persistent kernel launch whose grid does not depend on the table.
 *     Capture this call into a HIP graph; each replay re-reads the pinned
 *     table, so the problem list can be rewritten between replays.  Rewrite
 *     a slot only while no launch or replay that uses it is in flight.
 *   gemm_grouped_slot_destroy(slot): synchronises the slot's device and frees it.
 */
/*
 * Tile bodies of the grouped kernel for batches of 'N','N' problems with
 * 16-byte aligned operands and leading dimensions (the compact kernel).
 * The paper's finding that the best micro-kernel depends on the operand
 * shape (section 8.4, "In search of the best micro-kernel") applies per
 * problem: each problem of such a batch runs the body chosen for its size
 * bucket by gemm_tune_grouped (tuning-table entries with "trans": 4), or,
 * without an entry near the bucket, the body whose tile fits m and n best
 * (32 or 64 rows / columns up to that size, then 128, then 256).  The
 * split dtype uses three-term bodies for k >= 64 and six-term ones below.
 *   gemm_grouped_num_bodies(dtype): number of bodies of the dtype's family
 *     (-1 for a dtype the grouped kernel does not take).
 *   gemm_grouped_body_info(dtype, body, out[3]): {mc, nc, split pieces
 *     (2: three terms, 3: six terms, 0: not a split dtype)}.
 *   gemm_grouped_force_body(body): this thread's later grouped tables use
 *     `body` for every problem it qualifies for (-1 clears; other values
 *     below -1 or from 8 on return -1).
 *   gemm_grouped_bodies(count, problems, dtype, bodies): validates like
 *     gemm_grouped and writes the body each problem would run (-1: skipped
 *     as a quick return, or the batch takes the general kernel); launches
 *     nothing.
 *   gemm_tune_grouped(dtype, count, shapes, reps, out_path): for every
 *     (m, n, k) of `shapes` (3*count values, each 1..65536) times a batch of
 *     identical problems of that size in one launch with each qualifying
 *     body (median of `reps` launches), stores the fastest per size bucket
 *     and writes the table to `out_path` (NULL: memory only).  Synchronous;
 *     allocates its operands, a 1 GiB output region and a private stream,
 *     all freed before it returns.
 */
int gemm_grouped_num_bodies(int dtype);
int gemm_grouped_body_info(int dtype, int body, int64_t out[3]);
int gemm_grouped_force_body(int body);
int gemm_grouped_bodies(int64_t count, const gemm_problem *problems, int dtype, int *bodies);
int gemm_tune_grouped(int dtype, int64_t count, const int64_t *shapes, int reps,
                      const char *out_path);

int gemm_grouped_slot_create(void **slot, int64_t capacity);
int gemm_grouped_slot_write(void *slot, int64_t count, const gemm_problem *problems,
                            int dtype);
int gemm_grouped_slot_launch(void *slot);
void gemm_grouped_slot_destroy(void *slot);

/*
 * Stream for this host thread's subsequent calls: a hipStream_t, or NULL for
 * the null stream.  The library does not take ownership.
 */
int gemm_set_stream(void *hip_stream);

/*
 * Initialise the library on the current device: query the device, register
 * the compiled kernel family, load the tuning table from `tune_table_path`
 * (JSON written by gemm_tune; NULL or "" = built-in defaults, or the path in
 * the MGEMM_TUNE_TABLE environment variable), allocate the grouped launch's
 * descriptor tables and reserve workspace on the calling thread's current
 * stream: 1 GiB for gemm() and 768 MiB for gemm_scaled() (environment
 * MGEMM_WORKSPACE_BYTES / MGEMM_SCALED_WORKSPACE_BYTES override the sizes;
 * 0 reserves none).  Call it before any graph capture.  gemm() also works
 * without it (no workspace: the configurations that need none run).
 */
int gemm_init(const char *tune_table_path);
/* Frees everything the library allocated on every device.  Call it only
 * when no work that uses library memory is in flight. */
void gemm_shutdown(void);

/*
 * Reserve workspace for the calling thread's current stream on the current
 * device: at least `bytes` for gemm()'s packed split and split-K
 * configurations and `scaled_bytes` for gemm_scaled() (0 leaves a
 * reservation as it is; reservations only grow).  This call allocates
 * (outside any graph capture: during one it returns GEMM_E_WORKSPACE); a
 * replaced, smaller buffer is kept until gemm_shutdown or
 * gemm_release_workspace, since work enqueued on the stream may still read
 * it.  Errors: -1 / -2 for a negative size, GEMM_E_HIP when the allocation
 * fails.  A reservation belongs to the stream handle: release it (or finish
 * the stream's work) before destroying the stream.
 */
int gemm_reserve_workspace(int64_t bytes, int64_t scaled_bytes);

/* Synchronises the calling thread's current stream and frees its
 * reservations (and the buffers they replaced). */
int gemm_release_workspace(void);

/* Workspace bytes the configuration gemm() picks for these sizes (16-byte
 * aligned operands) needs on the current device; 0 when it needs none, -1 for
 * invalid arguments. */
int64_t gemm_workspace_bytes(char transA, char transB, int64_t m, int64_t n, int64_t k, int dtype);

/* Text of an error code (static storage). */
const char *gemm_strerror(int code);

/* The hipError_t behind the last GEMM_E_HIP on this thread. */
int gemm_last_hip_error(void);

/*
 * Kernel family introspection (used by the tuner and the tests).
 *   gemm_num_configs(dtype): number of compiled tile configurations.
 *   gemm_config_info(dtype, id, out[8]): out = {mc, nc, kc, wave tile m,
 *     wave tile n, threads, lds bytes, kind}; kind 0 = C resident in
 *     registers (B3A2C0 / A3B2C0), 1..4 = operand resident (B3C2A0, A3C2B0,
 *     C3A2B0, C3B2A0; paper section 4), 5 = packed split product (split
 *     dtypes: a packing pass writes the operands' bf16 pieces, then a bf16
 *     tile multiplies them), 6 = split-K (the k loop is cut into slices of
 *     whole stages run by separate workgroups, about two per CU, whose
 *     partial tiles go to a per-stream workspace and are then summed in
 *     slice order; deterministic, but float results differ in the last bits
 *     from the unsliced order), 7 = digit products (GEMM_I16 / GEMM_I32: a
 *     packing pass writes each operand's int8 digit planes to the workspace,
 *     then INT8 tiles multiply windows of them, one per weight class).
 *   gemm_config_staging(dtype, id): how the configuration fills its LDS
 *     panels: 0 = global loads through registers (converted, transposed and
 *     stored by the workgroup), 1 = direct global -> LDS loads into a ring of
 *     stages, 2 = packed split (packing pass, then a direct bf16 tile);
 *     packing configurations (paper section 5.3 / 8.6): 3 = A not packed
 *     (its fragments go straight from global memory to registers; B through
 *     LDS), 4 = B not packed, 5 = neither packed (no LDS), 6 = digit planes
 *     (INT16 / INT32: a packing pass writes int8 digit planes, then INT8
 *     tiles); negative as gemm_config_info's errors.
 *   gemm_config_mfma(dtype, id): the edge of the MFMA blocks its wave
 *     tiles are made of: 16 (16x16 MFMAs) or 32 (32x32 MFMAs: BF16, FP16,
 *     FP8 and INT8 direct-staged tiles, and the packed split tiles built on
 *     the BF16 ones); negative as gemm_config_info's errors.
 *   gemm_config_layouts(dtype, id): bit (2*t + v) is set when the
 *     configuration has a kernel for trans index t = 2*(transA is T) +
 *     (transB is T) with vectorised (v = 1: 16-byte aligned operands and
 *     leading dimensions) or element-wise (v = 0) staging; for other
 *     layouts a call forced to it runs the class's configuration 0.
 *   gemm_force_config(dtype, id, order): pin the next calls on this thread
 *     to configuration `id` with raster order `order` (0 = B3A2C0, column
 *     panels outer; 1 = A3B2C0, row panels outer); id < 0 clears the pin.
 *   gemm_last_config(out[3]): {dtype, id, order} used by this thread's last
 *     gemm() launch, and the split-term count in out[3] (0 if not split).
 */
int gemm_num_configs(int dtype);
int gemm_config_info(int dtype, int id, int64_t out[8]);
int gemm_config_staging(int dtype, int id);
int gemm_config_mfma(int dtype, int id);
int gemm_config_layouts(int dtype, int id);
int gemm_force_config(int dtype, int id, int order);
int gemm_last_config(int64_t out[4]);

/*
 * Debug aids (no part of the paper's method: checks that every tile writes
 * its part of C).
 *   Environment, read by gemm_init:
 *     MGEMM_FORCE_CFG=dtype:id[:order][,dtype:id[:order]...] pins
 *       configuration `id` (raster order `order`, default 0) for the dtype
 *       (codes as in gemm_dtype) on every thread that has no pin of its own
 *       (gemm_force_config); entries that do not parse, and ids the dtype
 *       does not have, are ignored.
 *     MGEMM_DEBUG (set, and not "0"): every gemm() / gemm_noalloc() call with
 *       beta = 0 that runs a product kernel first fills the m x n block of C
 *       with a sentinel (the NaN 0x7FC0DEAD; FP64 0x7FF8DEADDEADDEAD; int32 C
 *       the same 32 bits), then counts the block's sentinel elements after
 *       the product, so an element the product left unwritten is counted (as
 *       is a computed value with exactly those bits).  Two extra kernels per
 *       call, on the call's stream; nothing is counted for grouped launches.
 *   gemm_debug_count(C, m, n, ldc, dtype): enqueue the same count, on the
 *     calling thread's stream, for any m x n block of C (row-major, leading
 *     dimension ldc, element type of dtype's C).  Returns -i for an invalid
 *     i-th argument.
 *   gemm_debug_unwritten(): synchronise the calling thread's stream and
 *     return the count accumulated on the current device since the last
 *     call (which resets it to 0); on failure minus a GEMM_E_* code.
 * Both need gemm_init on the current device (GEMM_E_NOINIT otherwise, as
 * -GEMM_E_NOINIT from gemm_debug_unwritten).
 */
int gemm_debug_count(const void *C, int64_t m, int64_t n, int64_t ldc, int dtype);
int64_t gemm_debug_unwritten(void);

/*
 * Autotuner (paper section 8.4, "In search of the best micro-kernel": a
 * search over micro-kernel shapes of a few dozen experiments).  For every
 * (m, n, k) in `shapes` (3*count int64) it times each compiled configuration
 * of `dtype` that has a kernel for the layout (both raster orders) on
 * library-allocated scratch operands, in each of the four layouts
 * ('N','N', 'N','T', 'T','N', 'T','T'), keeps the fastest by median of `reps`
 * launches, stores it under (layout, size bucket) and writes the table as
 * JSON to `out_path` (NULL: keep in memory only).  Synchronous; allocates
 * (its scratch operands and the workspace of its candidates, on a private
 * stream, all freed before it returns).
 */
int gemm_tune(int dtype, int64_t count, const int64_t *shapes, int reps,
              const char *out_path);

/* gemm_tune_pruned restricted to the layouts whose bit is set in trans_mask
 * (bit t = 2*(transA is 'T') + (transB is 'T'), 1..15; else -7). */
int gemm_tune_layouts(int dtype, int64_t count, const int64_t *shapes, int reps,
                      const char *out_path, int model_keep, int trans_mask);

/*
 * gemm_tune restricted to the model_keep configurations the analytical model
 * ranks first for each shape (0: all of them, which is gemm_tune); -6 when
 * model_keep < 0.  The model (gemm_model_us) predicts occupancy from LDS and
 * register use, the rounds of tiles over the compute units, and a tile's
 * time as the largest of its MFMA, L2->LDS and LDS-read times plus the load
 * latency its stage ring leaves exposed.  It also picks the configuration
 * for sizes the tuning table does not cover.
 */
int gemm_tune_pruned(int dtype, int64_t count, const int64_t *shapes, int reps,
                     const char *out_path, int model_keep);

/* Modelled time in microseconds of configuration `id` of `dtype` on an
 * m x n x k problem over `cus` compute units; -1 on invalid arguments. */
double gemm_model_us(int dtype, int id, int64_t m, int64_t n, int64_t k, int cus);

/*
 * Fraction of a memory of `capacity_bytes` occupied by a rows x cols panel of
 * `elem_bytes`-byte values: the occupancy measure of the paper's analytical
 * cache model (section 8.4, Table 2: the L1 share of the micro-panel Br =
 * kc x nr FP32 values in a 64 KiB L1).  The tuner uses it to prune
 * configurations whose staged panels exceed a CU's LDS.  Returns -1 for
 * negative sizes or non-positive element size / capacity.
 */
double gemm_panel_occupancy(int64_t rows, int64_t cols, int64_t elem_bytes,
                            int64_t capacity_bytes);

#ifdef __cplusplus
}
#endif

#endif /* MGEMM_H */
