"""The boundary's workspace rules on the GPU: gemm() and gemm_scaled() take
their workspace from the stream's reservation (gemm_init /
gemm_reserve_workspace) and never allocate, free or synchronise; without a
large enough reservation gemm() runs the configuration that needs none and
gemm_scaled() returns GEMM_E_WORKSPACE."""
import numpy as np
import pytest

import oracle
import paper_2310_20347_amd as mg
from gemm_cases import Case, gpu_init, make_operands, to_device

pytestmark = pytest.mark.gpu

GEMM_E_WORKSPACE = 4


def _kind_cfg(dtype, kind):
    return [i for i in range(mg.num_configs(dtype)) if mg.config_info(dtype, i)["kind"] == kind][0]


def test_no_allocation_across_a_growing_sequence():
    """Free device memory (hipMemGetInfo) is unchanged across split-K and
    packed-split calls of growing size once the stream's workspace is
    reserved, and each call ran the configuration that uses the workspace."""
    import torch
    gpu_init()
    shapes = [(96, 256, 1024), (196, 1024, 2304), (196, 1024, 4608), (512, 768, 4096)]
    cases = []
    for dtype, kind in [(mg.GEMM_F32, 6), (mg.GEMM_F32_BF16X3, 5), (mg.GEMM_I8, 6)]:
        cfg = _kind_cfg(dtype, kind)
        for (m, n, k) in shapes:
            c = Case(dtype, "N", "N", m, n, k, 1.0, 0.0, seed=21)
            a, b, _ = make_operands(c)
            enc = (lambda x: x.astype(np.int8)) if dtype == mg.GEMM_I8 else (lambda x: x)
            dA, dB = to_device(enc(a)), to_device(enc(b))
            dC = torch.zeros((m, n), dtype=torch.int32 if dtype == mg.GEMM_I8 else torch.float32,
                             device="cuda")
            cases.append((dtype, cfg, c, dA, dB, dC, a, b))
    need = 0
    try:
        for dtype, cfg, c, *_ in cases:
            mg.force_config(dtype, cfg, 0)
            need = max(need, mg.workspace_bytes("N", "N", c.m, c.n, c.k, dtype))
            mg.force_config(dtype, -1, 0)
        assert need > 0
        mg.reserve_workspace(need, 0)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for dtype, cfg, c, dA, dB, dC, a, b in cases:
            mg.force_config(dtype, cfg, 0)
            print(f"dtype {mg.DTYPE_NAMES[dtype]} cfg {cfg} {c.m}x{c.n}x{c.k}", flush=True)
            mg.gemm("N", "N", c.m, c.n, c.k, 1.0, dA, c.k, dB, c.n, 0.0, dC, c.n, dtype)
            assert mg.last_config()["cfg"] == cfg
            mg.force_config(dtype, -1, 0)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        # and the results are right: a sampled row band against the oracle
        for dtype, cfg, c, dA, dB, dC, a, b in cases:
            rows = slice(0, 8)
            got = dC.cpu().numpy()[rows]
            if dtype == mg.GEMM_I8:
                ref = oracle.gemm_i8("N", "N", 8, c.n, c.k, 1, a[rows].astype(np.int8), c.k,
                                     b.astype(np.int8), c.n, 0, None, c.n)
                assert np.array_equal(got, ref)
            else:
                ref = oracle.gemm_f64("N", "N", 8, c.n, c.k, 1.0, a[rows].astype(np.float64),
                                      c.k, b.astype(np.float64), c.n)
                err = oracle.normalized_error(got, ref, c.k, float(np.abs(a).max()),
                                              float(np.abs(b).max()))
                assert err <= 2e-6, f"{mg.DTYPE_NAMES[dtype]} {c} error {err:.3g}"
    finally:
        for dtype, *_ in cases:
            mg.force_config(dtype, -1, 0)


def test_gemm_returns_before_its_kernel_finishes():
    """No host synchronisation: right after an 8192^3 FP32 call returns, the
    stream still has work (hipStreamQuery not ready)."""
    import torch
    gpu_init()
    n = 8192
    dA = torch.empty((n, n), dtype=torch.float32, device="cuda").uniform_(-1, 1)
    dB = torch.empty((n, n), dtype=torch.float32, device="cuda").uniform_(-1, 1)
    dC = torch.empty((n, n), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    mg.gemm("N", "N", n, n, n, 1.0, dA, n, dB, n, 0.0, dC, n, mg.GEMM_F32)
    busy = not s.query()
    torch.cuda.synchronize()
    assert busy, "gemm() returned after its work had finished (a host synchronisation?)"
    assert s.query()


def test_scaled_without_reservation_returns_workspace_error():
    """gemm_scaled() on a stream with no reservation launches nothing and
    returns GEMM_E_WORKSPACE; after a reservation the same call succeeds."""
    import torch
    gpu_init()
    m, n, k = 128, 96, 64
    dA = torch.ones((m, k), dtype=torch.float32, device="cuda")
    dB = torch.ones((k, n), dtype=torch.float32, device="cuda")
    dC = torch.full((m, n), 3.0, dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rc = mg.gemm_scaled("N", "N", m, n, k, 1.0, dA, k, dB, n, 0.0, dC, n, mg.GEMM_F16,
                            stream=s, check=False)
        assert rc == GEMM_E_WORKSPACE
        torch.cuda.synchronize()
        assert bool((dC == 3.0).all())
        mg.reserve_workspace(0, mg.scaled_workspace_bytes("N", "N", m, n, k, 0.0, mg.GEMM_F16),
                             stream=s)
        mg.gemm_scaled("N", "N", m, n, k, 1.0, dA, k, dB, n, 0.0, dC, n, mg.GEMM_F16, stream=s)
        torch.cuda.synchronize()
        assert bool((dC == float(k)).all())
        mg.release_workspace(stream=s)
