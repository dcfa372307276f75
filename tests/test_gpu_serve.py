"""GPU serving loop: every sampled request's result from the mix equals the same
GEMM run alone through gemm() (bitwise: same tile bodies, same k order) and
matches the oracle; the budget holds; statistics are populated."""
import numpy as np
import pytest

import oracle
import paper_2310_20347_amd as mg
from paper_2310_20347_amd import serve as sv

from gemm_cases import QUANT_TOL, decode, terms_for
from serve_cases import Pools, workload

pytestmark = pytest.mark.gpu


def alone(pools, md):
    import torch
    m, n, k, dt = md["m"], md["n"], md["k"], md["dtype"]
    out_t = torch.int32 if dt == mg.GEMM_I8 else torch.float32
    C = torch.zeros((m, n), dtype=out_t, device="cuda")
    # an unsliced configuration (not split-K): the serving launches run
    # unsliced tiles, and every unsliced configuration sums k in one order
    mg.force_config(dt, 1, 0)
    try:
        mg.gemm("N", "N", m, n, k, 1, pools.ptr(dt, md["a_off"]), md["lda"],
                pools.ptr(dt, md["b_off"]), md["ldb"], 0, C, n, dt)
    finally:
        mg.force_config(dt, -1, 0)
    torch.cuda.synchronize()
    return C.cpu().numpy()


def host_operand(pools, dt, off, rows, ld):
    t = pools.t[dt]
    es = t.element_size()
    flat = t.cpu().numpy().reshape(-1)
    x = flat[off // es: off // es + rows * ld].reshape(rows, ld)
    if dt == mg.GEMM_BF16:
        x = x.view(np.uint16)
    return x


def test_serving_results_same_alone_and_in_the_mix():
    import torch
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
    checked = 0
    for md in meta:
        if md["result"] is None:
            continue
        mix = md["result"]
        solo = alone(pools, md)
        assert np.array_equal(mix, solo), f"mix != alone for {md['m']}x{md['n']}x{md['k']}"
        dt, m, n, k = md["dtype"], md["m"], md["n"], md["k"]
        A = host_operand(pools, dt, md["a_off"], m, md["lda"])
        B = host_operand(pools, dt, md["b_off"], k, md["ldb"])
        if dt == mg.GEMM_I8:
            ref = oracle.gemm_i8("N", "N", m, n, k, 1, A, md["lda"], B, md["ldb"])
            assert np.array_equal(mix, ref)
        else:
            terms = terms_for(dt, k)
            if terms is not None:
                npc = 3 if len(terms) > 3 else 2
                PA = [oracle.decode_bf16(x) for x in oracle.split_bf16(A, npc)]
                PB = [oracle.decode_bf16(x) for x in oracle.split_bf16(B, npc)]
                ref = oracle.gemm_pieces("N", "N", m, n, k, 1.0, PA, md["lda"], PB, md["ldb"], terms)
                ma, mb = np.abs(A).max(), np.abs(B).max()
            else:
                Aq, Bq = decode(A, dt), decode(B, dt)
                ref = oracle.gemm_f64("N", "N", m, n, k, 1.0, Aq, md["lda"], Bq, md["ldb"])
                ma, mb = np.abs(Aq).max(), np.abs(Bq).max()
            assert oracle.normalized_error(mix, ref, k, ma, mb) <= QUANT_TOL
        checked += 1
    assert checked >= 30
