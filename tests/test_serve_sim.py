"""The serving scheduler on the simulated device (virtual clock): admission
under the HBM budget, slot limits, FIFO order, continuous batching, latency
accounting, and forced failures.  No GPU."""
import numpy as np
import pytest

import paper_2310_20347_amd as mg
from paper_2310_20347_amd import inputs
from paper_2310_20347_amd import serve as sv


def sim(overhead=10e-6, flops=100e12, bw=5e12, fail=-1, hang=-1):
    return sv.Sim(overhead, flops, bw, fail, hang)


def reqs_of(shapes, arrivals, dtypes):
    return [sv.Request(float(t), m, n, k, int(d), 1, 1, None)
            for (m, n, k), t, d in zip(shapes, arrivals, dtypes)]


def test_layout_strides_are_16_byte_multiples():
    lda, ldb, ldc, nbytes = sv.serve_layout(100, 30, 17, mg.GEMM_I8)
    assert (lda, ldb, ldc) == (32, 32, 30)
    lda, ldb, ldc, nbytes = sv.serve_layout(100, 30, 17, mg.GEMM_BF16)
    assert (lda, ldb) == (24, 32)
    lda, ldb, ldc, nbytes = sv.serve_layout(100, 30, 17, mg.GEMM_F32_BF16X3)
    assert (lda, ldb) == (20, 32) and nbytes == 8192 + 2304 + 12032
    assert mg.lib().serve_layout(0, 1, 1, 0, None, None, None, None) == -1


def test_single_request_latency_is_its_cost():
    r = reqs_of([(256, 256, 256)], [0.5], [mg.GEMM_BF16])
    rc, st, oc = sv.serve_run_sim(sv.config(), r, sim(overhead=1e-5, flops=1e12, bw=1e15))
    assert rc == 0 and st.completed == 1
    cost = 1e-5 + 2 * 256 ** 3 / 1e12
    assert oc[0].latency_ms == pytest.approx(1e3 * cost, rel=1e-9)
    assert oc[0].admit_s == pytest.approx(0.5)


def test_closed_loop_latency_is_each_requests_alone_latency():
    # closed loop: one request in the system at a time, latency from its
    # release; each equals the latency of a run holding that request alone,
    # whatever the arrival times (here a burst, all due at once)
    shapes = inputs.log_uniform_shapes(40, seed=3)
    dts = [mg.GEMM_F32_BF16X3, mg.GEMM_BF16, mg.GEMM_I8, mg.GEMM_F32] * 10
    r = reqs_of(shapes, [0.0] * 40, dts)
    rc, st, oc = sv.serve_run_sim(sv.config(closed_loop=1), r, sim())
    assert rc == 0 and st.completed == 40
    for i, (shape, d) in enumerate(zip(shapes, dts)):
        _, _, solo = sv.serve_run_sim(sv.config(), reqs_of([shape], [0.0], [d]), sim())
        assert oc[i].latency_ms == pytest.approx(solo[0].latency_ms, rel=1e-9), i
    # released one after another, in arrival order (index order here)
    for i in range(1, 40):
        assert oc[i].admit_s >= oc[i - 1].done_s
    # an open-loop run whose arrivals are far apart gives the same latencies
    rc, _, spaced = sv.serve_run_sim(sv.config(), reqs_of(shapes, np.arange(40) * 1.0, dts), sim())
    assert rc == 0
    assert [o.latency_ms for o in spaced] == pytest.approx([o.latency_ms for o in oc], rel=1e-9)


def test_budget_is_never_exceeded_and_oversize_is_rejected():
    shapes = inputs.log_uniform_shapes(300, seed=1)
    arrivals = np.sort(np.random.default_rng(2).uniform(0, 0.01, 300))
    dt = [mg.GEMM_F32_BF16X3, mg.GEMM_BF16, mg.GEMM_I8] * 100
    budget = 256 << 20
    r = reqs_of(shapes, arrivals, dt)
    big = sv.Request(0.0, 20000, 20000, 20000, mg.GEMM_F32_BF16X3, 1, 1, None)
    rc, st, oc = sv.serve_run_sim(sv.config(budget_bytes=budget, max_active=64), r + [big],
                                  sim())
    assert rc == 0
    assert st.peak_arena_bytes <= budget
    assert st.rejected == 1 and oc[-1].status == 4        # GEMM_E_WORKSPACE
    assert st.completed == 300 and st.peak_active <= 64


def test_fifo_admission_and_continuous_batching():
    # a large request arrives first, small ones while it runs: they are admitted
    # and finish before it (continuous batching), and admission is FIFO
    shapes = [(4096, 4096, 4096)] + [(64, 64, 64)] * 20
    arrivals = [0.0] + list(np.linspace(1e-4, 2e-3, 20))
    r = reqs_of(shapes, arrivals, [mg.GEMM_F32_BF16X3] * 21)
    rc, st, oc = sv.serve_run_sim(sv.config(request_tile_cap=64, step_tile_budget=256), r,
                                  sim(flops=20e12))
    assert rc == 0 and st.completed == 21
    admits = [o.admit_s for o in oc]
    assert admits == sorted(admits)                       # FIFO
    assert all(oc[i].done_s < oc[0].done_s for i in range(1, 21))
    assert st.mean_requests_per_launch > 1.5              # several requests per launch


def test_slot_limit_serialises_admission():
    shapes = [(512, 512, 512)] * 10
    r = reqs_of(shapes, [0.0] * 10, [mg.GEMM_BF16] * 10)
    rc, st, oc = sv.serve_run_sim(sv.config(max_active=2), r, sim(flops=1e12))
    assert rc == 0 and st.peak_active == 2 and st.completed == 10


def test_percentiles_and_per_dtype_accounting():
    rng = np.random.default_rng(3)
    n = 400
    shapes = inputs.log_uniform_shapes(n, seed=4, hi=512)
    arrivals = inputs.poisson_arrivals(n, 5000.0, 5)
    dts = [[mg.GEMM_F32_BF16X3, mg.GEMM_BF16, mg.GEMM_I8][i] for i in
           inputs.categorical(n, [0.5, 0.3, 0.2], 6)]
    r = reqs_of(shapes, arrivals, dts)
    rc, st, oc = sv.serve_run_sim(sv.config(warmup_requests=50), r, sim())
    assert rc == 0 and st.completed == n and st.measured == n - 50
    order = np.argsort(arrivals, kind="stable")
    lat = np.array([oc[i].latency_ms for i in order[50:]])
    assert st.p50_ms == pytest.approx(np.percentile(lat, 50))
    assert st.p99_ms == pytest.approx(np.percentile(lat, 99))
    assert st.max_ms == pytest.approx(lat.max())
    for d in (mg.GEMM_F32_BF16X3, mg.GEMM_BF16, mg.GEMM_I8):
        sel = [oc[i].latency_ms for i in order[50:] if dts[i] == d]
        assert st.count_by_dtype[d] == len(sel)
        assert st.p99_ms_by_dtype[d] == pytest.approx(np.percentile(sel, 99))
    assert st.window_s > 0 and st.req_per_s == pytest.approx(st.measured / st.window_s)


def test_failed_launch_fails_its_requests_and_the_loop_goes_on():
    shapes = [(300, 300, 300)] * 12
    r = reqs_of(shapes, np.linspace(0, 1e-3, 12), [mg.GEMM_BF16] * 12)
    rc, st, oc = sv.serve_run_sim(sv.config(max_active=3), r, sim(fail=1))
    assert rc == 0
    assert st.failed >= 1 and st.completed == 12 - st.failed
    assert any(o.status == 6 for o in oc) and all(o.status in (0, 6) for o in oc)


def test_hung_launch_trips_the_watchdog():
    shapes = [(128, 128, 128)] * 5
    r = reqs_of(shapes, [0.0] * 5, [mg.GEMM_I8] * 5)
    rc, st, oc = sv.serve_run_sim(sv.config(watchdog_s=0.05), r, sim(hang=0))
    assert rc == 6          # GEMM_E_SERVE


def test_invalid_configuration_and_requests():
    r = reqs_of([(8, 8, 8)], [0.0], [mg.GEMM_BF16])
    bad = sv.config(max_active=0)
    assert sv.serve_run_sim(bad, r, sim())[0] == -1
    assert sv.serve_run_sim(sv.config(closed_loop=2), r, sim())[0] == -1
    r[0].m = 0
    assert sv.serve_run_sim(sv.config(), r, sim())[0] == -3
    assert sv.serve_run_sim(sv.config(), reqs_of([(8, 8, 8)], [0.0], [1]),
                            sv.Sim(0, 0, 1, -1, -1))[0] == -4


def test_queue_mode_rejects_invalid_arguments_before_touching_the_device():
    r = reqs_of([(8, 8, 8)], [0.0], [mg.GEMM_BF16])
    assert sv.serve_run_queue(sv.config(max_active=0), r, check=False)[0] == -1
    assert sv.serve_run_queue(sv.config(), r, sv.queue_config(ring_tiles=1000), check=False)[0] == -2
    assert sv.serve_run_queue(sv.config(), r, sv.queue_config(ring_tiles=512), check=False)[0] == -2
    assert sv.serve_run_queue(sv.config(), r, sv.queue_config(idle_polls=-1), check=False)[0] == -2
    assert sv.serve_run_queue(sv.config(), r, sv.queue_config(workgroups=-3), check=False)[0] == -2
    assert sv.serve_run_queue(sv.config(), r, sv.queue_config(chunk_tiles=-1), check=False)[0] == -2
    assert sv.serve_run_queue(sv.config(), r, sv.queue_config(backlog_tiles=-1), check=False)[0] == -2
    r[0].m = 0
    assert sv.serve_run_queue(sv.config(), r, check=False)[0] == -4
