"""GPU serving loop: every sampled request's result from the mix equals the same
GEMM run alone through gemm() (bitwise: same tile bodies, same k order) and
matches the oracle; the budget holds; statistics are populated."""
import pytest

import paper_2310_20347_amd as mg
from paper_2310_20347_amd import serve as sv

from serve_cases import Pools, check_results, workload

pytestmark = pytest.mark.gpu


def test_serving_results_same_alone_and_in_the_mix():
    mg.gemm_init(None)
    pools = Pools(64 << 20, seed=9001)
    reqs, meta = workload(600, 5000.0, 9002, pools, lo=16, hi=1024, result_every=15)
    cfg = sv.config(budget_bytes=2 << 30, max_active=256, warmup_requests=50)
    print("serving 600 requests at 5k req/s", flush=True)
    rc, st, oc = sv.serve_run(cfg, reqs)
    print(f"completed {st.completed} p50 {st.p50_ms:.3f} ms p99 {st.p99_ms:.3f} ms "
          f"launches {st.launches} req/launch {st.mean_requests_per_launch:.1f}", flush=True)
    assert rc == 0 and st.completed == 600 and st.failed == 0 and st.rejected == 0
    assert st.peak_arena_bytes <= cfg.budget_bytes
    assert st.p50_ms > 0 and st.p99_ms >= st.p50_ms
    assert check_results(pools, meta) >= 30


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
