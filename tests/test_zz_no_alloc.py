"""gemm_noalloc, the entry point for callers that cannot allocate: through the
C ABI its results equal gemm()'s bit for bit (same configuration, workspace
from the library's fixed device array instead of the stream's reservation)
and the oracle's at the parity bar, on two calls in a row with the second
smaller; it allocates nothing; a configuration needing more than the array
holds is refused with GEMM_E_WORKSPACE and nothing is written."""
import numpy as np
import pytest

import oracle
import paper_2310_20347_amd as mg
from gemm_cases import Case, gpu_init, make_operands, to_device

pytestmark = pytest.mark.gpu

GEMM_E_WORKSPACE = 4


def _kind_cfg(dtype, kind):
    return [i for i in range(mg.num_configs(dtype)) if mg.config_info(dtype, i)["kind"] == kind][0]


def _operands(dtype, m, n, k, seed):
    import torch
    c = Case(dtype, "N", "N", m, n, k, 1.0, 0.0, seed=seed)
    a, b, _ = make_operands(c)
    enc = (lambda x: x.astype(np.int8)) if dtype == mg.GEMM_I8 else (lambda x: x)
    ct = torch.int32 if dtype == mg.GEMM_I8 else torch.float32
    return c, a, b, to_device(enc(a)), to_device(enc(b)), ct


def _oracle_rows(dtype, c, a, b, rows):
    if dtype == mg.GEMM_I8:
        return oracle.gemm_i8("N", "N", rows, c.n, c.k, 1, a[:rows].astype(np.int8), c.k,
                              b.astype(np.int8), c.n, 0, None, c.n)
    return oracle.gemm_f64("N", "N", rows, c.n, c.k, 1.0, a[:rows].astype(np.float64), c.k,
                           b.astype(np.float64), c.n)


@pytest.mark.parametrize("dtype,kind", [(mg.GEMM_F32, 6), (mg.GEMM_F32_BF16X3, 5),
                                        (mg.GEMM_I8, 6)])
def test_noalloc_equals_gemm_on_two_calls(dtype, kind):
    import torch
    gpu_init()
    cfg = _kind_cfg(dtype, kind)
    limit = mg.noalloc_scratch_bytes()
    assert limit == 64 << 20
    try:
        for (m, n, k), seed in (((196, 1024, 4608), 31), ((96, 256, 1024), 32)):
            print(f"noalloc {mg.DTYPE_NAMES[dtype]} cfg {cfg} {m}x{n}x{k}", flush=True)
            c, a, b, dA, dB, ct = _operands(dtype, m, n, k, seed)
            mg.force_config(dtype, cfg, 0)
            need = mg.workspace_bytes("N", "N", m, n, k, dtype)
            assert 0 < need <= limit
            ref = torch.full((m, n), 7, dtype=ct, device="cuda")
            got = torch.full((m, n), -7, dtype=ct, device="cuda")
            mg.gemm("N", "N", m, n, k, 1.0, dA, k, dB, n, 0.0, ref, n, dtype)
            assert mg.last_config()["cfg"] == cfg
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            mg.gemm_noalloc("N", "N", m, n, k, 1.0, dA, k, dB, n, 0.0, got, n, dtype)
            assert mg.last_config()["cfg"] == cfg
            torch.cuda.synchronize()
            assert torch.cuda.mem_get_info()[0] == free0, "gemm_noalloc allocated device memory"
            g, r = got.cpu().numpy(), ref.cpu().numpy()
            assert np.array_equal(g.view(np.uint32), r.view(np.uint32)), "differs from gemm()"
            rows = 8
            want = _oracle_rows(dtype, c, a, b, rows)
            if dtype == mg.GEMM_I8:
                assert np.array_equal(g[:rows], want)
            else:
                err = oracle.normalized_error(g[:rows], want, k, float(np.abs(a).max()),
                                              float(np.abs(b).max()))
                assert err <= 2e-6, f"error {err:.3g}"
            mg.force_config(dtype, -1, 0)
    finally:
        mg.force_config(dtype, -1, 0)


def test_noalloc_refuses_workspace_above_its_array():
    """A packed split product whose pieces need more than the array holds:
    GEMM_E_WORKSPACE, C untouched; gemm() runs the same call."""
    import torch
    gpu_init()
    dtype = mg.GEMM_F32_BF16X3
    cfg = _kind_cfg(dtype, 5)
    m, n, k = 2048, 2048, 4096
    try:
        mg.force_config(dtype, cfg, 0)
        assert mg.workspace_bytes("N", "N", m, n, k, dtype) > mg.noalloc_scratch_bytes()
        dA = torch.zeros((m, k), dtype=torch.float32, device="cuda")
        dB = torch.zeros((k, n), dtype=torch.float32, device="cuda")
        dC = torch.full((m, n), 5.0, dtype=torch.float32, device="cuda")
        rc = mg.gemm_noalloc("N", "N", m, n, k, 1.0, dA, k, dB, n, 0.0, dC, n, dtype, check=False)
        assert rc == GEMM_E_WORKSPACE
        torch.cuda.synchronize()
        assert bool((dC == 5.0).all())
        mg.gemm("N", "N", m, n, k, 1.0, dA, k, dB, n, 0.0, dC, n, dtype)
        torch.cuda.synchronize()
        assert bool((dC == 0.0).all())
    finally:
        mg.force_config(dtype, -1, 0)
