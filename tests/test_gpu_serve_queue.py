"""GPU queue-mode serving (a persistent kernel fed through a host-written
ring): every sampled request's result equals the same GEMM run alone through
gemm() bit for bit and matches the oracle; the kernel's bounded idle exit
and the host's relaunch lose no work."""
import pytest

import paper_2310_20347_amd as mg
from paper_2310_20347_amd import serve as sv

from serve_cases import Pools, check_results, workload

pytestmark = pytest.mark.gpu


def test_queue_results_same_alone_and_in_the_mix():
    mg.gemm_init(None)
    pools = Pools(64 << 20, seed=9101)
    reqs, meta = workload(600, 5000.0, 9102, pools, lo=16, hi=1024, result_every=15)
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
    assert check_results(pools, meta) >= 30


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
