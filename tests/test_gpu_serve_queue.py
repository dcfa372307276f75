"""GPU queue-mode serving (a persistent kernel fed through a host-written
ring): every sampled request's result equals the same GEMM run alone through
gemm() bit for bit and matches the oracle; the kernel's bounded idle exit
and the host's relaunch lose no work."""
import numpy as np
import pytest

import paper_2310_20347_amd as mg
from paper_2310_20347_amd import serve as sv

from serve_cases import Pools, check_results, workload

pytestmark = pytest.mark.gpu


def test_queue_results_same_alone_and_in_the_mix():
    mg.gemm_init(None)
    pools = Pools(64 << 20, seed=9101)
    reqs, meta = workload(600, 5000.0, 9102, pools, lo=16, hi=1024, result_every=15)
    # a burst: 60 requests arrive together, among them three with a dimension
    # of 4096 (the batching workload's upper end), so their tiles share the
    # ring and the workgroups
    t0 = reqs[100].arrival_s
    for i in range(100, 160):
        reqs[i].arrival_s = t0
    for j, (m, n, k) in enumerate([(4096, 256, 512), (384, 4096, 256), (256, 640, 4096)]):
        r, md = workload(1, 1.0, 9150 + j, pools, lo=16, hi=16, result_every=1)
        md = md[0]
        dt = md["dtype"]
        lda, ldb, ldc, _ = sv.serve_layout(m, n, k, dt)
        md.update(m=m, n=n, k=k, lda=lda, ldb=ldb, ldc=ldc, a_off=0, b_off=0,
                  result=np.zeros((m, n), dtype=np.int32 if dt == mg.GEMM_I8 else np.float32))
        reqs[110 + j] = sv.Request(t0, m, n, k, dt, pools.ptr(dt, 0), pools.ptr(dt, 0),
                                   md["result"].ctypes.data)
        meta[110 + j] = md
    for i in range(100, 160, 3):   # results of several burst members
        md = meta[i]
        if md["result"] is None:
            md["result"] = np.zeros((md["m"], md["n"]),
                                    dtype=np.int32 if md["dtype"] == mg.GEMM_I8 else np.float32)
            reqs[i].result = md["result"].ctypes.data
    cfg = sv.config(budget_bytes=2 << 30, max_active=256, warmup_requests=50, watchdog_s=20.0)
    print("queue mode: 600 requests at 5k req/s", flush=True)
    rc, st, oc = sv.serve_run_queue(cfg, reqs)
    print(f"completed {st.completed} p50 {st.p50_ms:.3f} ms p99 {st.p99_ms:.3f} ms "
          f"kernel launches {st.launches}", flush=True)
    assert rc == 0 and st.completed == 600 and st.failed == 0 and st.rejected == 0
    assert st.steps == 0 and st.launches >= 1
    assert st.peak_arena_bytes <= cfg.budget_bytes
    assert st.p50_ms > 0 and st.p99_ms >= st.p50_ms
    assert all(o.status == 0 for o in oc)
    # every checked burst member was in flight together with another request
    for i in range(100, 160):
        if meta[i]["result"] is None:
            continue
        assert any(j != i and oc[j].admit_s < oc[i].done_s and oc[i].admit_s < oc[j].done_s
                   for j in range(100, 160)), f"request {i} ran alone"
    assert check_results(pools, meta) >= 50


def test_queue_idle_exit_and_relaunch_lose_no_work():
    # a tiny idle bound: the kernel leaves in every gap between arrivals (mean
    # gap 2 ms) and the host relaunches it from the device's tail
    mg.gemm_init(None)
    pools = Pools(32 << 20, seed=9201)
    reqs, meta = workload(120, 500.0, 9202, pools, lo=16, hi=512, result_every=4)
    cfg = sv.config(budget_bytes=1 << 30, max_active=64, watchdog_s=20.0)
    print("queue mode, idle bound 32 polls: 120 requests at 500 req/s", flush=True)
    rc, st, oc = sv.serve_run_queue(cfg, reqs, sv.queue_config(ring_tiles=1024, idle_polls=32))
    print(f"completed {st.completed} kernel launches {st.launches} p99 {st.p99_ms:.3f} ms",
          flush=True)
    assert rc == 0 and st.completed == 120 and st.failed == 0
    assert st.launches > 1
    assert check_results(pools, meta) >= 25


def test_queue_chunked_publication_and_ring_wrap():
    # chunks of 8 output tiles and a 1024-record ring: large requests are
    # published over many chunks while later requests interleave, and the
    # ring wraps many times (records are rewritten only below the watermark
    # of unfinished requests); a closed-loop pass over the same requests
    # checks the one-at-a-time release as well
    mg.gemm_init(None)
    pools = Pools(64 << 20, seed=9301)
    # up to 1024^3: at most 256 output tiles + 32 copy tiles per request, so
    # every request fits the ring and the ring wraps many times over the run
    reqs, meta = workload(300, 8000.0, 9302, pools, lo=16, hi=1024, result_every=6)
    cfg = sv.config(budget_bytes=2 << 30, max_active=128, watchdog_s=20.0)
    q = sv.queue_config(ring_tiles=1024, chunk_tiles=8)
    print("queue mode, chunks of 8 tiles, ring 1024: 300 requests at 8k req/s", flush=True)
    rc, st, oc = sv.serve_run_queue(cfg, reqs, q)
    print(f"completed {st.completed} p99 {st.p99_ms:.3f} ms", flush=True)
    assert rc == 0 and st.completed == 300 and st.failed == 0 and st.rejected == 0
    assert all(o.status == 0 for o in oc)
    assert check_results(pools, meta) >= 45
    for md in meta:
        if md["result"] is not None:
            md["result"][:] = 0
    cfg1 = sv.config(budget_bytes=2 << 30, max_active=128, watchdog_s=20.0, closed_loop=1)
    print("the same requests in closed loop", flush=True)
    rc, st1, oc1 = sv.serve_run_queue(cfg1, reqs, q)
    assert rc == 0 and st1.completed == 300 and st1.failed == 0
    for a, b in zip(oc1[1:], oc1[:-1]):   # arrivals are increasing: index order
        assert a.admit_s >= b.done_s
    assert check_results(pools, meta) >= 45
