// Serving loop: continuous batching of GEMM requests under an HBM budget.
//
// One host thread runs the scheduler.  Arrivals go to a FIFO queue; the head
// is admitted when a slot is free and the arena (first-fit, coalescing free
// list over one device allocation) can hold its operands.  Each step takes a
// row panel chunk of C from every active request (oldest first), groups the
// chunks by dtype and issues one grouped persistent launch per dtype on that
// dtype's stream; up to `inflight_steps` launches per stream are in flight.
// Completions are observed by polling events; a request's memory is released
// when its last launch has retired.  The scheduler talks to a Backend: the
// real one (HIP) or a simulated one (virtual clock, cost model, forced
// failures) used by the CPU tests.
//
// The queue mode (run_queue) has no steps: admitted requests are published
// tile by tile to a persistent kernel that polls a host-written ring
// (queue.hpp, queue.hip), and completions are read from host memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <list>
#include <limits>
#include <map>
#include <thread>
#include <vector>

#include "abi_internal.hpp"
#include "mgemm.h"
#include "mgemm_serve.h"
#include "queue.hpp"

namespace mg {
namespace {

constexpr int64_t kPanel = 128;     // rows of C per chunk unit (one tile row)
constexpr int64_t kAlign = 256;     // arena alignment
constexpr double kInf = std::numeric_limits<double>::infinity();

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

int in_bytes(int dtype)
{
    switch (dtype) {
    case GEMM_BF16: case GEMM_F16: return 2;
    case GEMM_F8E4M3: case GEMM_I8: return 1;
    default: return 4;
    }
}

struct Req {
    int64_t idx = 0;
    const serve_request *in = nullptr;
    int64_t lda = 0, ldb = 0, ldc = 0, a_bytes = 0, b_bytes = 0, bytes = 0;
    int64_t off = -1;
    int64_t rows_issued = 0;
    int outstanding = 0;
    bool finished = false, failed = false, released = false, counted = false;
    double arr_t = 0;   // latency counts from here: the arrival, or the release (closed loop)
    double admit_t = -1, done_t = -1;
    int status = 0;
    // queue mode
    int qslot = -1, qgen = 0;
    int64_t qtiles = 0, qcopies = 0;
    int64_t qpub = 0;      // output tiles published so far
    int64_t qfirst = -1;   // ring position of the request's first tile
    GemmArgs qargs;        // its output tiles' arguments
    double publish_t = -1;
};

struct Launch {
    int dtype = 0, slot = 0;
    int64_t index = 0;
    std::vector<int64_t> reqs, finishing;
    double t_launch = 0, done_at = kInf;   // done_at: simulated completion
    bool failed = false;
};

class Arena {
public:
    void init(int64_t size)
    {
        free_.clear();
        if (size > 0) free_[0] = size;
        used_ = peak_ = 0;
    }
    int64_t alloc(int64_t bytes)
    {
        bytes = round_up(bytes, kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, rem = it->second - bytes;
                free_.erase(it);
                if (rem > 0) free_[off + bytes] = rem;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes)
    {
        bytes = round_up(bytes, kAlign);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t peak() const { return peak_; }

private:
    std::map<int64_t, int64_t> free_;
    int64_t used_ = 0, peak_ = 0;
};

// The host loops poll (events, completion words), so they yield rather than
// sleep: a sleep of a few microseconds lasts tens (the kernel's timer
// slack).  They sleep only when nothing is outstanding and the next arrival
// is far off.
void idle_wait(double dt, bool outstanding)
{
    if (!outstanding && dt > 300e-6) std::this_thread::sleep_for(std::chrono::duration<double>(dt - 200e-6));
    else std::this_thread::yield();
}

class Backend {
public:
    virtual ~Backend() {}
    virtual int begin(const serve_config &cfg) = 0;
    virtual void end() = 0;
    virtual double now() = 0;
    virtual void idle_until(double t) = 0;
    virtual char *base() = 0;
    virtual int admit(const Req &r) = 0;
    virtual int launch(Launch &l, const std::vector<gemm_problem> &probs) = 0;
    virtual int query(Launch &l) = 0;   // 1 done, 0 pending, < 0 error
    virtual double completion_hint() = 0;
    virtual void fetch(const Req &r) = 0;
};

// ---------------------------------------------------------------------------
// Real device.
// ---------------------------------------------------------------------------
class HipBackend : public Backend {
public:
    int begin(const serve_config &cfg) override
    {
        hipError_t e = hipMalloc((void **)&base_, (size_t)std::max<int64_t>(cfg.budget_bytes, kAlign));
        if (e != hipSuccess) return fail(e);
        slots_per_dtype_ = cfg.inflight_steps;
        for (int d = 0; d < GEMM_NUM_DTYPES; ++d) {
            if ((e = hipStreamCreate(&stream_[d])) != hipSuccess) return fail(e);
            for (int s = 0; s < slots_per_dtype_; ++s) {
                int rc = gemm_grouped_slot_create(&slot_[d][s], cfg.max_active);
                if (rc != GEMM_OK) return rc;
                if ((e = hipEventCreateWithFlags(&ev_[d][s], hipEventDisableTiming)) != hipSuccess)
                    return fail(e);
                if (cfg.graph_replay && gemm_grouped_num_bodies(d) > 0) {
                    rc = capture(d, s);
                    if (rc != GEMM_OK) return rc;
                }
            }
        }
        // arrivals count from here: the arena and slot set-up (hundreds of
        // milliseconds for a large arena once earlier ones were freed) is not
        // part of any request's latency
        t0_ = std::chrono::steady_clock::now();
        return GEMM_OK;
    }
    void end() override
    {
        (void)hipDeviceSynchronize();
        for (int d = 0; d < GEMM_NUM_DTYPES; ++d) {
            for (int s = 0; s < slots_per_dtype_; ++s) {
                if (exec_[d][s]) (void)hipGraphExecDestroy(exec_[d][s]);
                exec_[d][s] = nullptr;
                if (slot_[d][s]) gemm_grouped_slot_destroy(slot_[d][s]);
                if (ev_[d][s]) (void)hipEventDestroy(ev_[d][s]);
                slot_[d][s] = nullptr;
                ev_[d][s] = nullptr;
            }
            if (stream_[d]) (void)hipStreamDestroy(stream_[d]);
            stream_[d] = nullptr;
        }
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
    }
    double now() override
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
    }
    void idle_until(double t) override { idle_wait(t - now(), false); }
    char *base() override { return base_; }
    int admit(const Req &r) override
    {
        hipStream_t s = stream_[r.in->dtype];
        hipError_t e = hipMemcpyAsync(base_ + r.off, r.in->a_src, (size_t)(r.in->m * r.lda * in_bytes(r.in->dtype)),
                                      hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(base_ + r.off + r.a_bytes, r.in->b_src,
                               (size_t)(r.in->k * r.ldb * in_bytes(r.in->dtype)), hipMemcpyDeviceToDevice, s);
        return e == hipSuccess ? GEMM_OK : fail(e);
    }
    int launch(Launch &l, const std::vector<gemm_problem> &probs) override
    {
        void *slot = slot_[l.dtype][l.slot];
        int rc = gemm_grouped_slot_write(slot, (int64_t)probs.size(), probs.data(), l.dtype);
        if (rc != GEMM_OK) return rc;
        if (hipGraphExec_t g = exec_[l.dtype][l.slot]) {
            // the captured copy re-reads the slot's pinned table just written
            hipError_t e = hipGraphLaunch(g, stream_[l.dtype]);
            if (e != hipSuccess) return fail(e);
        } else {
            hipStream_t saved = t_tls.stream;
            t_tls.stream = stream_[l.dtype];
            rc = gemm_grouped_slot_launch(slot);
            t_tls.stream = saved;
            if (rc != GEMM_OK) return rc;
        }
        hipError_t e = hipEventRecord(ev_[l.dtype][l.slot], stream_[l.dtype]);
        return e == hipSuccess ? GEMM_OK : fail(e);
    }
    int query(Launch &l) override
    {
        hipError_t e = hipEventQuery(ev_[l.dtype][l.slot]);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        t_tls.hip_err = (int)e;
        return -1;
    }
    double completion_hint() override { return kInf; }
    void fetch(const Req &r) override
    {
        if (!r.in->result) return;
        (void)hipMemcpy(r.in->result, base_ + r.off + r.a_bytes + r.b_bytes,
                        (size_t)(r.in->m * r.ldc * 4), hipMemcpyDeviceToHost);
    }

private:
    int fail(hipError_t e)
    {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    // Captures slot s of dtype d's launch (table copy + persistent kernel) on
    // the dtype's stream into a graph.  The slot is first written with a
    // one-problem 'N','N' table of the dtype, which fixes its kernel (the
    // compact one: arena operands are aligned, as every request's are).
    int capture(int d, int s)
    {
        gemm_problem q;
        std::memset(&q, 0, sizeof q);
        q.transA = q.transB = 'N';
        q.m = q.n = q.k = 16;
        q.alpha = 1.0;
        q.A = q.B = q.C = base_;
        q.lda = q.ldb = q.ldc = 16;
        int rc = gemm_grouped_slot_write(slot_[d][s], 1, &q, d);
        if (rc != GEMM_OK) return rc;
        hipStream_t st = stream_[d];
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail(e);
        hipStream_t saved = t_tls.stream;
        t_tls.stream = st;
        rc = gemm_grouped_slot_launch(slot_[d][s]);
        t_tls.stream = saved;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(st, &g);
        if (rc == GEMM_OK && e == hipSuccess)
            e = hipGraphInstantiate(&exec_[d][s], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (rc != GEMM_OK) return rc;
        return e == hipSuccess ? GEMM_OK : fail(e);
    }
    std::chrono::steady_clock::time_point t0_;
    char *base_ = nullptr;
    hipStream_t stream_[GEMM_NUM_DTYPES] = {};
    void *slot_[GEMM_NUM_DTYPES][4] = {};
    hipEvent_t ev_[GEMM_NUM_DTYPES][4] = {};
    hipGraphExec_t exec_[GEMM_NUM_DTYPES][4] = {};
    int slots_per_dtype_ = 0;
};

// ---------------------------------------------------------------------------
// Simulated device: virtual time, one in-order queue per dtype.
// ---------------------------------------------------------------------------
class SimBackend : public Backend {
public:
    explicit SimBackend(const serve_sim &s) : sim_(s) {}
    int begin(const serve_config &) override
    {
        t_ = 0;
        for (double &f : stream_free_) f = 0;
        return GEMM_OK;
    }
    void end() override {}
    double now() override { return t_; }
    void idle_until(double t) override { t_ = std::max(t_, t); }
    char *base() override { return nullptr; }
    int admit(const Req &) override { return GEMM_OK; }
    int launch(Launch &l, const std::vector<gemm_problem> &probs) override
    {
        const int64_t idx = count_++;
        if (idx == sim_.fail_launch) return GEMM_E_HIP;
        double cost = sim_.launch_overhead_s;
        for (const gemm_problem &p : probs) {
            const double flops = 2.0 * p.m * p.n * p.k;
            const double bytes = double(in_bytes(l.dtype)) * (p.m * p.k + p.k * p.n) + 4.0 * p.m * p.n;
            cost += std::max(flops / sim_.flops_per_s, bytes / sim_.bytes_per_s);
        }
        const double start = std::max(t_, stream_free_[l.dtype]);
        l.done_at = (idx == sim_.hang_launch) ? kInf : start + cost;
        stream_free_[l.dtype] = l.done_at;
        pending_.push_back(&l);
        return GEMM_OK;
    }
    int query(Launch &l) override
    {
        if (t_ >= l.done_at) {
            pending_.erase(std::remove(pending_.begin(), pending_.end(), &l), pending_.end());
            return 1;
        }
        return 0;
    }
    double completion_hint() override
    {
        double h = kInf;
        for (Launch *l : pending_) h = std::min(h, l->done_at);
        return h;
    }
    void fetch(const Req &) override {}

private:
    serve_sim sim_;
    double t_ = 0;
    double stream_free_[GEMM_NUM_DTYPES] = {};
    int64_t count_ = 0;
    std::vector<Launch *> pending_;
};

// ---------------------------------------------------------------------------
// Scheduler.
// ---------------------------------------------------------------------------
double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return -1.0;
    std::sort(v.begin(), v.end());
    const double pos = q * double(v.size() - 1);
    const size_t lo = (size_t)std::floor(pos), hi = (size_t)std::ceil(pos);
    return v[lo] + (v[hi] - v[lo]) * (pos - double(lo));
}

int check_config(const serve_config *cfg)
{
    if (!cfg) return -1;
    if (cfg->budget_bytes <= 0 || cfg->max_active < 1 || cfg->max_active > 8192 ||
        cfg->step_tile_budget < 1 || cfg->request_tile_cap < 1 || cfg->inflight_steps < 1 ||
        cfg->inflight_steps > 4 || !(cfg->watchdog_s > 0) || cfg->warmup_requests < 0 ||
        (cfg->closed_loop != 0 && cfg->closed_loop != 1) ||
        (cfg->graph_replay != 0 && cfg->graph_replay != 1))
        return -1;
    return 0;
}

int check_requests(int64_t count, const serve_request *reqs, bool need_src)
{
    if (count < 0) return -2;
    if (count > 0 && !reqs) return -3;
    for (int64_t i = 0; i < count; ++i) {
        const serve_request &r = reqs[i];
        if (r.m <= 0 || r.n <= 0 || r.k <= 0 || r.m > 0x7FFFFFFF || r.n > 0x7FFFFFFF ||
            r.k > 0x7FFFFFFF || r.dtype < 0 || r.dtype >= GEMM_F64 ||
            !std::isfinite(r.arrival_s) || r.arrival_s < 0 ||
            (need_src && (!r.a_src || !r.b_src)))
            return -3;
    }
    return 0;
}

// Moves the requests whose arrival time has passed into the admission queue
// (both loops).  Closed loop: at most one, and only when the system is empty
// (nothing queued or admitted); its latency then counts from now.
void release_arrivals(const serve_config &cfg, const std::vector<int64_t> &order, std::vector<Req> &R,
                      double now, bool system_empty, size_t &next_arrival, std::deque<int64_t> &queue)
{
    while (next_arrival < order.size()) {
        Req &r = R[(size_t)order[next_arrival]];
        if (r.in->arrival_s > now) break;
        if (cfg.closed_loop) {
            if (!system_empty) break;
            r.arr_t = now;
            queue.push_back(order[next_arrival++]);
            break;
        }
        r.arr_t = r.in->arrival_s;
        queue.push_back(order[next_arrival++]);
    }
}

// Outcomes and statistics of a finished run (both loops).
void fill_stats(const serve_config &cfg, const std::vector<int64_t> &order, const std::vector<Req> &R,
                int64_t peak_arena, int64_t peak_active, int64_t steps, int64_t launches,
                int64_t reqs_in_launches, serve_stats *stats, serve_outcome *outcomes)
{
    std::vector<double> lat, lat_by[GEMM_NUM_DTYPES];
    double t_first = kInf, t_last = 0, flops = 0;
    int64_t completed = 0, failed = 0, rejected = 0;
    for (size_t pos = 0; pos < order.size(); ++pos) {
        const Req &r = R[(size_t)order[pos]];
        if (r.finished) ++completed;
        else if (r.status == GEMM_E_WORKSPACE) ++rejected;
        else ++failed;
        if (outcomes) {
            serve_outcome &o = outcomes[r.idx];
            o.admit_s = r.admit_t;
            o.done_s = r.finished ? r.done_t : -1.0;
            o.latency_ms = r.finished ? 1e3 * (r.done_t - r.arr_t) : -1.0;
            o.status = r.finished ? 0 : (r.status ? r.status : GEMM_E_SERVE);
        }
        if ((int64_t)pos < cfg.warmup_requests || !r.finished) continue;
        const double ms = 1e3 * (r.done_t - r.arr_t);
        lat.push_back(ms);
        lat_by[r.in->dtype].push_back(ms);
        t_first = std::min(t_first, r.arr_t);
        t_last = std::max(t_last, r.done_t);
        flops += 2.0 * r.in->m * r.in->n * r.in->k;
    }
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->completed = completed;
        stats->failed = failed;
        stats->rejected = rejected;
        stats->measured = (int64_t)lat.size();
        stats->window_s = lat.empty() ? 0.0 : t_last - t_first;
        stats->req_per_s = stats->window_s > 0 ? lat.size() / stats->window_s : 0.0;
        stats->tflops = stats->window_s > 0 ? flops / stats->window_s / 1e12 : 0.0;
        stats->p50_ms = percentile(lat, 0.50);
        stats->p99_ms = percentile(lat, 0.99);
        double sum = 0, mx = 0;
        for (double v : lat) {
            sum += v;
            mx = std::max(mx, v);
        }
        stats->mean_ms = lat.empty() ? -1.0 : sum / lat.size();
        stats->max_ms = lat.empty() ? -1.0 : mx;
        for (int d = 0; d < GEMM_NUM_DTYPES; ++d) {
            stats->count_by_dtype[d] = (int64_t)lat_by[d].size();
            stats->p50_ms_by_dtype[d] = percentile(lat_by[d], 0.50);
            stats->p99_ms_by_dtype[d] = percentile(lat_by[d], 0.99);
        }
        stats->steps = steps;
        stats->launches = launches;
        stats->peak_arena_bytes = peak_arena;
        stats->peak_active = peak_active;
        stats->mean_requests_per_launch = launches ? double(reqs_in_launches) / launches : 0.0;
    }
}

int run(Backend &be, const serve_config &cfg, int64_t count, const serve_request *reqs,
        serve_stats *stats, serve_outcome *outcomes)
{
    std::vector<Req> R((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        Req &r = R[(size_t)i];
        r.idx = i;
        r.in = &reqs[i];
        serve_layout(r.in->m, r.in->n, r.in->k, r.in->dtype, &r.lda, &r.ldb, &r.ldc, &r.bytes);
        r.a_bytes = round_up(r.in->m * r.lda * in_bytes(r.in->dtype), kAlign);
        r.b_bytes = round_up(r.in->k * r.ldb * in_bytes(r.in->dtype), kAlign);
    }
    std::vector<int64_t> order((size_t)count);
    for (int64_t i = 0; i < count; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return reqs[a].arrival_s < reqs[b].arrival_s; });

    int rc = be.begin(cfg);
    if (rc != GEMM_OK) {
        be.end();
        return rc;
    }
    Arena arena;
    arena.init(cfg.budget_bytes);
    std::deque<int64_t> queue;
    std::vector<int64_t> active;             // admission order
    std::list<Launch> inflight;              // launch records (stable addresses)
    int inflight_per[GEMM_NUM_DTYPES] = {};
    int next_slot[GEMM_NUM_DTYPES] = {};
    size_t next_arrival = 0;
    int64_t done = 0, launches = 0, steps = 0, peak_active = 0, reqs_in_launches = 0;
    int result = GEMM_OK;

    auto finish_req = [&](Req &r) {
        if (!r.counted) {
            r.counted = true;
            ++done;
        }
        if (r.outstanding == 0 && !r.released && r.off >= 0) {
            arena.release(r.off, r.bytes);
            r.released = true;
            active.erase(std::remove(active.begin(), active.end(), r.idx), active.end());
        }
    };

    while (done < count) {
        const double now = be.now();
        release_arrivals(cfg, order, R, now, queue.empty() && active.empty(), next_arrival, queue);
        // admission: FIFO, head of line waits for a slot and arena space
        while (!queue.empty() && (int64_t)active.size() < cfg.max_active) {
            Req &r = R[(size_t)queue.front()];
            if (round_up(r.bytes, kAlign) > cfg.budget_bytes) {
                r.status = GEMM_E_WORKSPACE;
                queue.pop_front();
                finish_req(r);
                continue;
            }
            const int64_t off = arena.alloc(r.bytes);
            if (off < 0) break;
            r.off = off;
            r.admit_t = now;
            queue.pop_front();
            active.push_back(r.idx);
            peak_active = std::max<int64_t>(peak_active, (int64_t)active.size());
            if (be.admit(r) != GEMM_OK) {
                r.failed = true;
                r.status = GEMM_E_SERVE;
                finish_req(r);
            }
        }
        bool progressed = false;
        // retire finished launches: in launch order within a dtype stream (a
        // later launch of a stream is not retired before an earlier one), any
        // order across streams
        bool blocked[GEMM_NUM_DTYPES] = {};
        for (auto it = inflight.begin(); it != inflight.end();) {
            Launch &l = *it;
            const int q = blocked[l.dtype] ? 0 : be.query(l);
            if (q == 0) {
                blocked[l.dtype] = true;
                if (now - l.t_launch > cfg.watchdog_s) {
                    result = GEMM_E_SERVE;
                    break;
                }
                ++it;
                continue;
            }
            for (int64_t ri : l.reqs) {
                Req &r = R[(size_t)ri];
                --r.outstanding;
                if (q < 0) {
                    r.failed = true;
                    r.status = GEMM_E_SERVE;
                }
            }
            for (int64_t ri : l.finishing) {
                Req &r = R[(size_t)ri];
                if (!r.failed) {
                    r.finished = true;
                    r.done_t = be.now();
                    be.fetch(r);
                }
            }
            for (int64_t ri : l.reqs) {
                Req &r = R[(size_t)ri];
                if (r.finished || r.failed) finish_req(r);
            }
            --inflight_per[l.dtype];
            it = inflight.erase(it);
            progressed = true;
        }
        if (result != GEMM_OK) break;
        // one step: a chunk from every active request with work left
        std::vector<gemm_problem> probs[GEMM_NUM_DTYPES];
        std::vector<int64_t> who[GEMM_NUM_DTYPES], last[GEMM_NUM_DTYPES];
        int64_t step_tiles = 0;
        for (int64_t ri : active) {
            Req &r = R[(size_t)ri];
            const int dt = r.in->dtype;
            if (r.failed || r.rows_issued >= r.in->m || inflight_per[dt] >= cfg.inflight_steps) continue;
            const int64_t tpp = (r.in->n + kPanel - 1) / kPanel;   // tiles per row panel
            const int64_t cap_rows = std::max<int64_t>(1, cfg.request_tile_cap / tpp) * kPanel;
            const int64_t rows = std::min(r.in->m - r.rows_issued, cap_rows);
            const int64_t tiles = (rows + kPanel - 1) / kPanel * tpp;
            if (step_tiles > 0 && step_tiles + tiles > cfg.step_tile_budget) break;
            step_tiles += tiles;
            char *b = be.base();
            const int es = in_bytes(dt);
            gemm_problem p;
            std::memset(&p, 0, sizeof p);
            p.transA = 'N';
            p.transB = 'N';
            p.m = rows;
            p.n = r.in->n;
            p.k = r.in->k;
            p.alpha = 1.0;
            p.beta = 0.0;
            p.lda = r.lda;
            p.ldb = r.ldb;
            p.ldc = r.ldc;
            if (b) {
                p.A = b + r.off + r.rows_issued * r.lda * es;
                p.B = b + r.off + r.a_bytes;
                p.C = b + r.off + r.a_bytes + r.b_bytes + r.rows_issued * r.ldc * 4;
            }
            r.rows_issued += rows;
            probs[dt].push_back(p);
            who[dt].push_back(ri);
            if (r.rows_issued >= r.in->m) last[dt].push_back(ri);
        }
        bool stepped = false;
        for (int dt = 0; dt < GEMM_NUM_DTYPES; ++dt) {
            if (probs[dt].empty()) continue;
            inflight.emplace_back();
            Launch &l = inflight.back();
            l.dtype = dt;
            l.slot = next_slot[dt];
            next_slot[dt] = (next_slot[dt] + 1) % cfg.inflight_steps;
            l.index = launches++;
            l.reqs = who[dt];
            l.finishing = last[dt];
            l.t_launch = be.now();
            for (int64_t ri : l.reqs) ++R[(size_t)ri].outstanding;
            reqs_in_launches += (int64_t)l.reqs.size();
            ++inflight_per[dt];
            stepped = true;
            if (be.launch(l, probs[dt]) != GEMM_OK) {
                // the launch did not start: its requests fail, the loop goes on
                for (int64_t ri : l.reqs) {
                    Req &r = R[(size_t)ri];
                    --r.outstanding;
                    r.failed = true;
                    r.status = GEMM_E_SERVE;
                    finish_req(r);
                }
                --inflight_per[dt];
                inflight.pop_back();
            }
        }
        if (stepped) {
            ++steps;
            progressed = true;
        }
        if (!progressed && done < count) {
            double t_next = be.now() + 1e-4;
            // (closed loop: an arrival held back until the system empties is no wake-up time)
            if (next_arrival < order.size() && (!cfg.closed_loop || (queue.empty() && active.empty())))
                t_next = std::min(t_next, reqs[order[next_arrival]].arrival_s);
            t_next = std::min(t_next, be.completion_hint());
            be.idle_until(std::max(t_next, be.now()));
        }
    }
    be.end();
    fill_stats(cfg, order, R, arena.peak(), peak_active, steps, launches, reqs_in_launches, stats,
               outcomes);
    return result;
}


// ---------------------------------------------------------------------------
// Queue mode: one persistent kernel fed through a host-written ring.
// ---------------------------------------------------------------------------
constexpr int64_t kRingDefault = 1 << 16;
constexpr int64_t kIdleDefault = 20000;

// Tile shape of a request's dtype class in the queue kernel.
int64_t queue_tiles(const serve_request &q, int64_t *mc_out = nullptr, int64_t *nc_out = nullptr)
{
    const int64_t t = kclass_of(q.dtype, q.k) == K_SPLIT3 ? 64 : 128;
    if (mc_out) *mc_out = t;
    if (nc_out) *nc_out = t;
    return ((q.m + t - 1) / t) * ((q.n + t - 1) / t);
}

// Device and pinned resources of one queue run.
struct QueueRes {
    char *base = nullptr;             // the arena
    QTile *ring_h = nullptr, *ring_d = nullptr;
    QCtl *ctl_h = nullptr, *ctl_d = nullptr;
    int *done_h = nullptr, *done_d = nullptr;
    QDev *dev = nullptr;
    size_t dev_bytes = 0;
    hipStream_t ks = nullptr, cs = nullptr;   // kernel, result copies
    hipEvent_t kev = nullptr;                 // kernel instance finished

    int init(const serve_config &cfg, int64_t ring)
    {
        hipError_t e;
        const int slots = cfg.max_active;
        if ((e = hipMalloc((void **)&base, (size_t)std::max<int64_t>(cfg.budget_bytes, kAlign))) != hipSuccess)
            return fail(e);
        const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
        if ((e = hipHostMalloc((void **)&ring_h, (size_t)ring * sizeof(QTile), fl)) != hipSuccess) return fail(e);
        if ((e = hipHostMalloc((void **)&ctl_h, sizeof(QCtl), fl)) != hipSuccess) return fail(e);
        if ((e = hipHostMalloc((void **)&done_h, (size_t)slots * sizeof(int), fl)) != hipSuccess) return fail(e);
        std::memset(ring_h, 0, (size_t)ring * sizeof(QTile));
        std::memset(ctl_h, 0, sizeof(QCtl));
        std::memset(done_h, 0, (size_t)slots * sizeof(int));
        if ((e = hipHostGetDevicePointer((void **)&ring_d, ring_h, 0)) != hipSuccess) return fail(e);
        if ((e = hipHostGetDevicePointer((void **)&ctl_d, ctl_h, 0)) != hipSuccess) return fail(e);
        if ((e = hipHostGetDevicePointer((void **)&done_d, done_h, 0)) != hipSuccess) return fail(e);
        dev_bytes = offsetof(QDev, counters) + 2 * (size_t)slots * sizeof(int32_t);
        if ((e = hipMalloc((void **)&dev, dev_bytes)) != hipSuccess) return fail(e);
        if ((e = hipStreamCreateWithFlags(&ks, hipStreamNonBlocking)) != hipSuccess) return fail(e);
        if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return fail(e);
        if ((e = hipEventCreateWithFlags(&kev, hipEventDisableTiming)) != hipSuccess) return fail(e);
        if ((e = hipMemsetAsync(dev, 0, dev_bytes, ks)) != hipSuccess) return fail(e);
        if ((e = hipStreamSynchronize(ks)) != hipSuccess) return fail(e);
        return GEMM_OK;
    }
    // Frees everything; the kernel must have left (the caller synchronises).
    void free_all()
    {
        if (kev) (void)hipEventDestroy(kev);
        if (cs) (void)hipStreamDestroy(cs);
        if (ks) (void)hipStreamDestroy(ks);
        if (dev) (void)hipFree(dev);
        if (done_h) (void)hipHostFree(done_h);
        if (ctl_h) (void)hipHostFree(ctl_h);
        if (ring_h) (void)hipHostFree(ring_h);
        if (base) (void)hipFree(base);
        *this = QueueRes();
    }
    static int fail(hipError_t e)
    {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
};

int run_queue(const serve_config &cfg, const serve_queue_config &qc, int64_t count,
              const serve_request *reqs, int cus, serve_stats *stats, serve_outcome *outcomes)
{
    std::vector<Req> R((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        Req &r = R[(size_t)i];
        r.idx = i;
        r.in = &reqs[i];
        serve_layout(r.in->m, r.in->n, r.in->k, r.in->dtype, &r.lda, &r.ldb, &r.ldc, &r.bytes);
        r.a_bytes = round_up(r.in->m * r.lda * in_bytes(r.in->dtype), kAlign);
        r.b_bytes = round_up(r.in->k * r.ldb * in_bytes(r.in->dtype), kAlign);
        r.qtiles = queue_tiles(*r.in);
        r.qcopies = (r.in->m * r.lda * in_bytes(r.in->dtype) + kCopyChunk - 1) / kCopyChunk +
                    (r.in->k * r.ldb * in_bytes(r.in->dtype) + kCopyChunk - 1) / kCopyChunk;
    }
    std::vector<int64_t> order((size_t)count);
    for (int64_t i = 0; i < count; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return reqs[a].arrival_s < reqs[b].arrival_s; });

    const int64_t ring = qc.ring_tiles > 0 ? qc.ring_tiles : kRingDefault;
    const int64_t idle = qc.idle_polls > 0 ? qc.idle_polls : kIdleDefault;
    // at most one workgroup per compute unit: the result copies (and any
    // other work on the device) need the rest of each unit's registers
    const int grid = qc.workgroups > 0 ? std::min(qc.workgroups, cus) : cus;
    const int64_t chunk = qc.chunk_tiles > 0 ? qc.chunk_tiles : grid;
    // the claimed word trails the claims by fewer than 16 + grid (it is
    // stored for every 16th tile, and the claiming workgroups' stores land in
    // any order), so a smaller backlog could read as full with every tile taken
    const int64_t backlog = std::max<int64_t>(qc.backlog_tiles > 0 ? qc.backlog_tiles : (int64_t)grid + 17,
                                              (int64_t)grid + 17);
    QueueRes q;
    int rc = q.init(cfg, ring);
    if (rc != GEMM_OK) {
        (void)hipDeviceSynchronize();
        q.free_all();
        return rc;
    }
    const auto t0 = std::chrono::steady_clock::now();
    auto now_s = [&]() {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    };
    int64_t launches = 0;
    bool running = false;
    auto launch = [&]() {
        int r2 = launch_queue_kernel(q.ring_d, ring - 1, q.ctl_d, q.done_d, q.dev, cfg.max_active, idle,
                                     grid, q.ks);
        if (r2 == GEMM_OK && hipEventRecord(q.kev, q.ks) != hipSuccess) r2 = GEMM_E_HIP;
        if (r2 == GEMM_OK) {
            ++launches;
            running = true;
        }
        return r2;
    };
    int result = launch();

    Arena arena;
    arena.init(cfg.budget_bytes);
    std::deque<int64_t> queue;
    std::vector<int64_t> published;   // admitted, not finished
    std::deque<int64_t> partial;      // admitted with output tiles still to publish, oldest first
    std::vector<int> free_slots, slot_gen((size_t)cfg.max_active, 0);
    for (int i = cfg.max_active - 1; i >= 0; --i) free_slots.push_back(i);
    size_t next_arrival = 0;
    int64_t done = 0, peak_active = 0, active = 0, tail = 0;
    int64_t unpublished = 0;   // output tiles of admitted requests not yet published
    int64_t claimed_seen = -1;
    double claimed_t = 0;      // when the claimed word last changed

    // Ring positions below the watermark hold records of finished requests
    // only (each of which was read before its tile ran), so the host may
    // overwrite them.  Admission keeps tail + unpublished <= watermark + ring,
    // so every later chunk of an admitted request has room.
    auto watermark = [&]() {
        int64_t w = tail;
        for (int64_t i : published) w = std::min(w, R[(size_t)i].qfirst);
        return w;
    };
    auto put_outputs = [&](Req &r, int64_t count) {
        int64_t pos = tail;
        for (int64_t t = r.qpub; t < r.qpub + count; ++t) {
            QTile &rec = q.ring_h[pos++ & (ring - 1)];
            rec.a = r.qargs;
            rec.t = (int)t;
            rec.slot = r.qslot;
            rec.ntiles = (int)r.qtiles;
            rec.body = kclass_of(r.in->dtype, r.in->k);
            rec.gen = r.qgen;
            rec.kind = 0;
            rec.ncopy = (int)r.qcopies;
            rec.pad = 0;
        }
        r.qpub += count;
        unpublished -= count;
        tail = pos;
    };

    auto finish = [&](Req &r) {
        ++done;
        if (r.off >= 0) {
            arena.release(r.off, r.bytes);
            r.off = -1;
        }
        if (r.qslot >= 0) {
            free_slots.push_back(r.qslot);
            r.qslot = -1;
            --active;
        }
    };

    while (result == GEMM_OK && done < count) {
        const double now = now_s();
        bool progressed = false;
        release_arrivals(cfg, order, R, now, queue.empty() && active == 0, next_arrival, queue);
        // admission: FIFO; a request is published at once, its operand copies
        // as the first tiles
        while (!queue.empty() && !free_slots.empty()) {
            Req &r = R[(size_t)queue.front()];
            if (round_up(r.bytes, kAlign) > cfg.budget_bytes || r.qtiles + r.qcopies > ring) {
                r.status = GEMM_E_WORKSPACE;
                queue.pop_front();
                finish(r);
                continue;
            }
            if (tail + unpublished + r.qcopies + r.qtiles > watermark() + ring) break;   // ring full
            const int64_t off = arena.alloc(r.bytes);
            if (off < 0) break;
            queue.pop_front();
            r.off = off;
            r.admit_t = now;
            r.qslot = free_slots.back();
            free_slots.pop_back();
            peak_active = std::max(peak_active, ++active);
            r.qgen = ++slot_gen[(size_t)r.qslot];
            const int es = in_bytes(r.in->dtype);
            int64_t pos = tail;
            r.qfirst = tail;
            auto put_copies = [&](const void *src, char *dst, int64_t bytes) {
                for (int64_t o = 0; o < bytes; o += kCopyChunk) {
                    QTile &rec = q.ring_h[pos++ & (ring - 1)];
                    std::memset(&rec, 0, sizeof rec);
                    rec.a.A = (const char *)src + o;
                    rec.a.C = dst + o;
                    rec.a.lda = std::min(kCopyChunk, bytes - o);
                    rec.slot = r.qslot;
                    rec.kind = 1;
                }
            };
            put_copies(r.in->a_src, q.base + r.off, r.in->m * r.lda * es);
            put_copies(r.in->b_src, q.base + r.off + r.a_bytes, r.in->k * r.ldb * es);
            int64_t mc = 128, nc = 128;
            queue_tiles(*r.in, &mc, &nc);
            const int kclass = kclass_of(r.in->dtype, r.in->k);
            GemmArgs a;
            std::memset(&a, 0, sizeof a);
            a.A = q.base + r.off;
            a.B = q.base + r.off + r.a_bytes;
            a.C = q.base + r.off + r.a_bytes + r.b_bytes;
            a.lda = r.lda;
            a.ldb = r.ldb;
            a.ldc = r.ldc;
            a.m = (int)r.in->m;
            a.n = (int)r.in->n;
            a.k = (int)r.in->k;
            a.alpha = 1.0f;
            a.beta = 0.0f;
            a.ialpha = 1;
            a.ibeta = 0;
            a.tiles_m = (int)((r.in->m + mc - 1) / mc);
            a.tiles_n = (int)((r.in->n + nc - 1) / nc);
            a.order = 0;
            a.group = 8;
            a.terms = split_terms(kclass);
            r.qargs = a;
            tail = pos;
            // the first chunk now; the rest as the kernel takes the ring
            r.qpub = 0;
            unpublished += r.qtiles;
            put_outputs(r, std::min(chunk, r.qtiles));
            if (r.qpub < r.qtiles) partial.push_back(r.idx);
            __atomic_store_n(&q.ctl_h->tail, tail, __ATOMIC_RELEASE);
            r.publish_t = now_s();
            published.push_back(r.idx);
            progressed = true;
        }
        // later chunks, oldest request first, while the unclaimed backlog is
        // short; should the claimed word stand still for 100 us (its stores
        // are not ordered, so it could rest below the claims) one chunk goes
        // out regardless, so progress never depends on it
        if (!partial.empty()) {
            const int64_t claimed = __atomic_load_n(&q.ctl_h->claimed, __ATOMIC_ACQUIRE);
            if (claimed != claimed_seen) {
                claimed_seen = claimed;
                claimed_t = now;
            }
            bool put = false, force = now - claimed_t > 100e-6;
            while (!partial.empty() && (tail - claimed < backlog || force)) {
                Req &r = R[(size_t)partial.front()];
                put_outputs(r, std::min(chunk, r.qtiles - r.qpub));
                if (r.qpub >= r.qtiles) partial.pop_front();
                put = true;
                if (force) {
                    force = false;
                    claimed_t = now;
                }
            }
            if (put) {
                __atomic_store_n(&q.ctl_h->tail, tail, __ATOMIC_RELEASE);
                progressed = true;
            }
        }
        if (__atomic_load_n(&q.ctl_h->fault, __ATOMIC_ACQUIRE)) {
            result = GEMM_E_SERVE;
            break;
        }
        // completions, in any order
        for (size_t i = 0; i < published.size();) {
            Req &r = R[(size_t)published[i]];
            if (__atomic_load_n(&q.done_h[r.qslot], __ATOMIC_ACQUIRE) == r.qgen) {
                r.finished = true;
                r.done_t = now_s();
                if (r.in->result) {
                    const char *c = q.base + r.off + r.a_bytes + r.b_bytes;
                    if (hipMemcpyAsync(r.in->result, c, (size_t)(r.in->m * r.ldc * 4), hipMemcpyDeviceToHost,
                                       q.cs) != hipSuccess ||
                        hipStreamSynchronize(q.cs) != hipSuccess) {
                        r.finished = false;
                        r.failed = true;
                        r.status = GEMM_E_SERVE;
                    }
                }
                finish(r);
                published[i] = published.back();
                published.pop_back();
                progressed = true;
                continue;
            }
            if (now - r.publish_t > cfg.watchdog_s) {
                result = GEMM_E_SERVE;
                break;
            }
            ++i;
        }
        if (result != GEMM_OK) break;
        // a kernel instance that left while idle is relaunched when work is waiting
        if (running && hipEventQuery(q.kev) == hipSuccess) running = false;
        if (!running && !published.empty()) {
            QDev h;
            std::memset(&h, 0, sizeof h);
            hipError_t e = hipMemcpyAsync(&h.tail, &q.dev->tail, sizeof h.tail, hipMemcpyDeviceToHost, q.ks);
            if (e == hipSuccess) e = hipStreamSynchronize(q.ks);
            h.claim = h.tail;
            h.stop = 0;
            if (e == hipSuccess)
                e = hipMemcpyAsync(q.dev, &h, offsetof(QDev, counters), hipMemcpyHostToDevice, q.ks);
            if (e == hipSuccess) e = hipStreamSynchronize(q.ks);
            if (e != hipSuccess) {
                t_tls.hip_err = (int)e;
                result = GEMM_E_SERVE;
                break;
            }
            result = launch();
            progressed = true;
        }
        if (!progressed) {
            const double dt = next_arrival < order.size() ? reqs[order[next_arrival]].arrival_s - now : 1.0;
            idle_wait(dt, !published.empty() || !queue.empty());
        }
    }
    // the kernel leaves on the stop word (or, at the latest, after its idle bound)
    __atomic_store_n(&q.ctl_h->stop, 1, __ATOMIC_RELEASE);
    (void)hipStreamSynchronize(q.ks);
    (void)hipStreamSynchronize(q.cs);
    q.free_all();
    for (int64_t i = 0; i < count; ++i) {
        Req &r = R[(size_t)i];
        if (!r.finished && !r.failed && r.status == 0) r.status = GEMM_E_SERVE;
    }
    fill_stats(cfg, order, R, arena.peak(), peak_active, 0, launches, done, stats, outcomes);
    return result;
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

int serve_layout(int64_t m, int64_t n, int64_t k, int dtype, int64_t *lda, int64_t *ldb,
                 int64_t *ldc, int64_t *arena_bytes)
{
    if (m <= 0) return -1;
    if (n <= 0) return -2;
    if (k <= 0) return -3;
    if (dtype < 0 || dtype >= GEMM_NUM_DTYPES) return -4;
    const int es = in_bytes(dtype);
    const int64_t q = 16 / es;
    const int64_t a = round_up(k, q), b = round_up(n, q);
    if (lda) *lda = a;
    if (ldb) *ldb = b;
    if (ldc) *ldc = n;
    if (arena_bytes)
        *arena_bytes = round_up(m * a * es, kAlign) + round_up(k * b * es, kAlign) +
                       round_up(m * n * 4, kAlign);
    return GEMM_OK;
}

int serve_run(const serve_config *cfg, int64_t count, const serve_request *reqs,
              serve_stats *stats, serve_outcome *outcomes)
{
    if (check_config(cfg)) return -1;
    int v = check_requests(count, reqs, true);
    if (v) return v;
    ensure_registered();
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    rc = grouped_device_init(d);
    if (rc != GEMM_OK) return rc;
    HipBackend be;
    return run(be, *cfg, count, reqs, stats, outcomes);
}

int serve_run_queue(const serve_config *cfg, const serve_queue_config *qcfg, int64_t count,
                    const serve_request *reqs, serve_stats *stats, serve_outcome *outcomes)
{
    if (check_config(cfg)) return -1;
    serve_queue_config qc;
    std::memset(&qc, 0, sizeof qc);
    if (qcfg) qc = *qcfg;
    if (qc.ring_tiles < 0 || (qc.ring_tiles > 0 && (qc.ring_tiles < 1024 || qc.ring_tiles > (1 << 24) ||
                                                    (qc.ring_tiles & (qc.ring_tiles - 1)))) ||
        qc.workgroups < 0 || qc.workgroups > 8192 || qc.idle_polls < 0 || qc.chunk_tiles < 0 ||
        qc.backlog_tiles < 0)
        return -2;
    int v = check_requests(count, reqs, true);
    if (v) return v - 1;
    ensure_registered();
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    return run_queue(*cfg, qc, count, reqs, d->cus, stats, outcomes);
}

int serve_run_sim(const serve_config *cfg, int64_t count, const serve_request *reqs,
                  const serve_sim *sim, serve_stats *stats, serve_outcome *outcomes)
{
    if (check_config(cfg)) return -1;
    int v = check_requests(count, reqs, false);
    if (v) return v;
    if (!sim || !(sim->flops_per_s > 0) || !(sim->bytes_per_s > 0) || sim->launch_overhead_s < 0)
        return -4;
    SimBackend be(*sim);
    return run(be, *cfg, count, reqs, stats, outcomes);
}

}  // extern "C"
