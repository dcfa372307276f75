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
