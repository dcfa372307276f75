/*
 * mgemm serving loop: continuous batching of independent GEMM requests on one
 * GPU, built on the grouped persistent launch of mgemm.h.
 *
 * Requests arrive over time (arrival times are inputs).  A request is
 * admitted when a slot is free and the device arena (the HBM budget) can hold
 * its operands; at admission its A and B are copied device-to-device from
 * caller-owned source memory into the arena and stay resident until the
 * request completes.  Work is issued in steps: each step takes whole row
 * panels of C from every active request (oldest first, a per-request cap and
 * a per-step cap, in 128x128-tile units) and launches one grouped kernel per
 * dtype on that dtype's stream; requests that arrive while steps run join the
 * next step.  A request completes when the step holding its last row panel
 * has finished; latency = completion time - arrival time (release time in
 * closed-loop mode, see serve_config).
 *
 * Layout of a request (row-major, transA = transB = 'N', alpha = 1, beta = 0):
 * A is m x k with lda = k rounded up to a 16-byte multiple, B is k x n with
 * ldb = n rounded up likewise, C is m x n float32 (int32 for GEMM_I8) with
 * ldc = n.  serve_layout() returns these strides and the arena bytes.
 *
 * Errors: 0 on success; -i when argument i is invalid; GEMM_E_SERVE when a
 * step fails at launch (its requests are marked failed and the loop goes on)
 * is reported per request, while a step that does not complete within the
 * watchdog time ends the run with GEMM_E_SERVE.
 */
#ifndef MGEMM_SERVE_H
#define MGEMM_SERVE_H

#include <stdint.h>

#include "mgemm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double arrival_s;     /* arrival time in seconds from the start of the run     */
    int64_t m, n, k;      /* problem size, all > 0                                   */
    int dtype;            /* a gemm_dtype                                            */
    const void *a_src;    /* DEVICE memory holding m*lda elements of A (serve_layout) */
    const void *b_src;    /* DEVICE memory holding k*ldb elements of B                */
    void *result;         /* optional HOST buffer of m*n*4 bytes that receives C,    */
                          /* or NULL                                                 */
} serve_request;

typedef struct {
    int64_t budget_bytes;      /* device arena size: the HBM budget for operands         */
    int max_active;            /* requests admitted at once (slots)                       */
    int64_t step_tile_budget;  /* max 128x128 output tiles issued per step                */
    int64_t request_tile_cap;  /* max tiles of one request per step                       */
    int inflight_steps;        /* steps in flight per dtype stream, 1..4 (1 keeps the     */
                               /* latency lowest: arrivals join the next step instead of  */
                               /* queueing behind a second launch on the stream)          */
    double watchdog_s;         /* a step unfinished after this long ends the run          */
    int64_t warmup_requests;   /* first requests (by arrival) left out of the statistics  */
    int closed_loop;           /* 0: requests arrive at their arrival times (open loop).  */
                               /* 1: one request in the system at a time: each is        */
                               /* released, in arrival order, at the later of its arrival */
                               /* and the completion of the one before, and its latency   */
                               /* counts from its release.  Serving a set of requests     */
                               /* this way gives each one's alone-latency (on an          */
                               /* otherwise idle GPU, same path and overheads).           */
    int graph_replay;          /* step loop: 1 = each step's grouped launch of a dtype is  */
                               /* the replay of a HIP graph captured once per launch slot  */
                               /* (the slot's table copy and persistent kernel), 0 =       */
                               /* direct launches.  The queue mode ignores it.            */
} serve_config;

typedef struct {
    int64_t completed, failed, rejected;   /* over all requests                          */
    int64_t measured;                      /* completed requests in the statistics       */
    double window_s;                       /* first measured arrival -> last completion  */
    double req_per_s, tflops;              /* over the window                            */
    double p50_ms, p99_ms, mean_ms, max_ms;
    int64_t count_by_dtype[GEMM_NUM_DTYPES];
    double p50_ms_by_dtype[GEMM_NUM_DTYPES], p99_ms_by_dtype[GEMM_NUM_DTYPES];
    int64_t steps, launches;
    int64_t peak_arena_bytes, peak_active;
    double mean_requests_per_launch;
} serve_stats;

typedef struct {
    double admit_s, done_s;   /* seconds from the start of the run (-1 if never)        */
    double latency_ms;        /* done - arrival (release, closed loop), -1 if the      */
                              /* request did not complete                               */
    int status;               /* 0 completed, GEMM_E_SERVE failed, GEMM_E_WORKSPACE      */
                              /* rejected (does not fit the budget)                     */
} serve_outcome;

/* Strides and arena bytes of a request (see the layout above). */
int serve_layout(int64_t m, int64_t n, int64_t k, int dtype, int64_t *lda, int64_t *ldb,
                 int64_t *ldc, int64_t *arena_bytes);

/*
 * Runs the loop in real time on the current device until every request has
 * completed, failed or been rejected.  Allocates the arena (budget_bytes) and
 * its streams at the start and frees them at the end.  `outcomes` (count
 * entries) and `stats` may be NULL.
 *   Arguments: 1 cfg, 2 count, 3 reqs, 4 stats, 5 outcomes.
 */
int serve_run(const serve_config *cfg, int64_t count, const serve_request *reqs,
              serve_stats *stats, serve_outcome *outcomes);

/*
 * Queue mode: the same admission (FIFO, slots, arena budget) without steps.
 * One persistent kernel stays resident (one workgroup per compute unit,
 * at most half of each unit's registers) and takes work from a ring of tile
 * records in pinned host memory, in publication order.  A request is
 * published at admission as copy tiles (its A and B into the arena, 256 KiB
 * each, done by the kernel) followed by the first chunk of its output tiles,
 * which wait for those copies; its further chunks are published (oldest
 * request first) only while fewer than backlog_tiles published tiles are
 * unclaimed, so a request admitted later waits behind at most that backlog,
 * not behind all of an earlier large request.  A request completes
 * when its last output tile is done; the kernel reports that through pinned
 * host memory and the host polls it.  Output tiles: 128x128 (64x64 for the
 * six-term split), the bodies of the grouped kernel's compact variant, so
 * every result equals the standalone gemm() call bit for bit.
 *
 * Every wait in the kernel is bounded: after idle_polls empty polls of the
 * ring (about 4 us each) the kernel leaves, and the host relaunches it when
 * work is waiting (stats.launches counts the instances).  At the end the
 * host sets a stop word and waits for the kernel to leave.  A request whose
 * tiles do not fit the ring is rejected (GEMM_E_WORKSPACE); a request is
 * admitted only when the ring can take all of its tiles, so its later chunks
 * always find room.  stats.steps is 0; mean_requests_per_launch is completed
 * requests per kernel instance.
 */
typedef struct {
    int64_t ring_tiles;   /* tile records in the ring: a power of two in          */
                          /* [1024, 2^24], or 0 for 65536 (144 bytes each)        */
    int workgroups;       /* persistent workgroups, 0 = one per compute unit;      */
                          /* larger values are reduced to that                     */
    int64_t idle_polls;   /* empty polls before the kernel leaves, 0 = 20000       */
    int64_t chunk_tiles;  /* output tiles per published chunk, 0 = the number of    */
                          /* workgroups                                            */
    int64_t backlog_tiles;/* later chunks wait while this many published tiles are  */
                          /* unclaimed, 0 = workgroups + 17 (the least it may be:   */
                          /* smaller values are raised to it)                       */
} serve_queue_config;

/* Arguments: 1 cfg, 2 qcfg (NULL = defaults), 3 count, 4 reqs, 5 stats,
 * 6 outcomes.  Returns as serve_run. */
int serve_run_queue(const serve_config *cfg, const serve_queue_config *qcfg, int64_t count,
                    const serve_request *reqs, serve_stats *stats, serve_outcome *outcomes);

/* Simulated device for testing the scheduler without a GPU: a virtual clock,
 * a cost model per launch and forced failures. */
typedef struct {
    double launch_overhead_s;   /* fixed cost of one grouped launch                  */
    double flops_per_s;         /* compute rate of the simulated device              */
    double bytes_per_s;         /* memory rate (operand traffic of a launch)         */
    int64_t fail_launch;        /* index of a launch that fails to start (-1: none)  */
    int64_t hang_launch;        /* index of a launch that never completes (-1: none) */
} serve_sim;

/* The same scheduler on the simulated device (no GPU, operands not touched;
 * `result` buffers are ignored).  Arguments: 1 cfg, 2 count, 3 reqs, 4 sim,
 * 5 stats, 6 outcomes. */
int serve_run_sim(const serve_config *cfg, int64_t count, const serve_request *reqs,
                  const serve_sim *sim, serve_stats *stats, serve_outcome *outcomes);

#ifdef __cplusplus
}
#endif

#endif /* MGEMM_SERVE_H */
