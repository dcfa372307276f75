"""GPU serving loop: every sampled request's result from the mix equals the same
GEMM run alone through gemm() (bitwise: same tile bodies, same k order) and
matches the oracle; the budget holds; statistics are populated."""
import numpy as np
import pytest

import paper_2310_20347_amd as mg
from paper_2310_20347_amd import serve as sv

from serve_cases import Pools, check_results, workload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graph_replay", [1, 0], ids=["graph", "direct"])
def test_serving_results_same_alone_and_in_the_mix(graph_replay):
    mg.gemm_init(None)
    pools = Pools(64 << 20, seed=9001)
    reqs, meta = workload(600, 5000.0, 9002, pools, lo=16, hi=1024, result_every=15)
    # a burst: 60 requests arrive together (they share launches), among them
    # some with a dimension of 4096 (the batching workload's upper end)
    t0 = reqs[100].arrival_s
    for i in range(100, 160):
        reqs[i].arrival_s = t0
    big = [(4096, 256, 512), (384, 4096, 256), (256, 640, 4096)]
    for j, (m, n, k) in enumerate(big):
        r, md = workload(1, 1.0, 9100 + j, pools, lo=16, hi=16, result_every=1)
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
    cfg = sv.config(budget_bytes=2 << 30, max_active=256, warmup_requests=50,
                    graph_replay=graph_replay)
    print(f"serving 600 requests at 5k req/s, graph_replay={graph_replay}", flush=True)
    rc, st, oc = sv.serve_run(cfg, reqs)
    print(f"completed {st.completed} p50 {st.p50_ms:.3f} ms p99 {st.p99_ms:.3f} ms "
          f"launches {st.launches} req/launch {st.mean_requests_per_launch:.2f}", flush=True)
    assert rc == 0 and st.completed == 600 and st.failed == 0 and st.rejected == 0
    assert st.peak_arena_bytes <= cfg.budget_bytes
    assert st.p50_ms > 0 and st.p99_ms >= st.p50_ms
    assert st.mean_requests_per_launch > 1.0
    # every checked burst member was on the GPU together with another request
    for i in range(100, 160):
        if meta[i]["result"] is None:
            continue
        assert any(j != i and oc[j].admit_s < oc[i].done_s and oc[i].admit_s < oc[j].done_s
                   for j in range(100, 160)), f"request {i} ran alone"
    assert check_results(pools, meta) >= 50


def test_closed_loop_serves_one_request_at_a_time():
    # closed loop: each request is released when the one before it has
    # completed, so admissions and completions alternate in arrival order, one
    # grouped launch per request, and the results are those of the open loop
    mg.gemm_init(None)
    pools = Pools(32 << 20, seed=9011)
    reqs, meta = workload(120, 5000.0, 9012, pools, lo=16, hi=512, result_every=6)
    cfg = sv.config(budget_bytes=1 << 30, max_active=64, closed_loop=1)
    print("step loop, closed loop: 120 requests", flush=True)
    rc, st, oc = sv.serve_run(cfg, reqs)
    print(f"completed {st.completed} launches {st.launches} p50 {st.p50_ms:.3f} ms", flush=True)
    assert rc == 0 and st.completed == 120 and st.failed == 0
    assert st.peak_active == 1
    for a, b in zip(oc[1:], oc[:-1]):   # arrivals are increasing: index order
        assert a.admit_s >= b.done_s
    assert all(o.latency_ms > 0 for o in oc)
    assert check_results(pools, meta) >= 18
