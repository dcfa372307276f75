"""Debug aids on the GPU: with MGEMM_DEBUG the sentinel fill and count
around every beta = 0 product find no unwritten element of C in any
configuration of a ragged problem, while the count itself finds planted
sentinels; MGEMM_FORCE_CFG pins a configuration for threads without a pin
of their own.  (gemm_init reads both variables.)"""
import os

import numpy as np
import pytest

import paper_2310_20347_amd as mg

pytestmark = pytest.mark.gpu

SENTINEL32 = np.uint32(0x7FC0DEAD)


@pytest.fixture
def env():
    saved = {k: os.environ.get(k) for k in ("MGEMM_DEBUG", "MGEMM_FORCE_CFG")}
    yield os.environ
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    mg.gemm_init(None)   # back to the defaults


def _operands(torch, m, n, k, dtype):
    g = torch.Generator(device="cpu").manual_seed(11)
    if dtype == mg.GEMM_I8:
        A = torch.randint(-128, 128, (m, k), generator=g, dtype=torch.int8)
        B = torch.randint(-128, 128, (k, n), generator=g, dtype=torch.int8)
        C = torch.zeros((m, n + 3), dtype=torch.int32)
        return A.cuda(), B.cuda(), C.cuda(), A.long() @ B.long()
    A = torch.rand((m, k), generator=g) * 2 - 1
    B = torch.rand((k, n), generator=g) * 2 - 1
    C = torch.zeros((m, n + 3))
    return A.cuda(), B.cuda(), C.cuda(), A.double() @ B.double()


@pytest.mark.parametrize("dtype", [mg.GEMM_F32, mg.GEMM_BF16, mg.GEMM_I8],
                         ids=lambda d: mg.DTYPE_NAMES[d])
def test_every_configuration_writes_its_block(env, dtype):
    import torch
    env["MGEMM_DEBUG"] = "1"
    env.pop("MGEMM_FORCE_CFG", None)
    mg.gemm_init(None)
    assert mg.debug_unwritten() == 0
    m, n, k = 263, 197, 160
    A, B, C, ref = _operands(torch, m, n, k, dtype)
    if dtype == mg.GEMM_BF16:
        A, B = A.bfloat16(), B.bfloat16()
        ref = A.double().cpu() @ B.double().cpu()
    one = 1 if dtype == mg.GEMM_I8 else 1.0
    zero = 0 if dtype == mg.GEMM_I8 else 0.0
    pad = C[:, n:].clone()
    for cfg in range(mg.num_configs(dtype)):
        info = mg.config_info(dtype, cfg)
        print(f"{mg.DTYPE_NAMES[dtype]} cfg {cfg} {info['mc']}x{info['nc']} {info['staging']}", flush=True)
        mg.force_config(dtype, cfg, 0)
        try:
            mg.gemm("N", "N", m, n, k, one, A, k, B, n, zero, C, n + 3, dtype)
        finally:
            mg.force_config(dtype, -1, 0)
        assert mg.debug_unwritten() == 0, f"configuration {cfg} left elements of C unwritten"
        got = C[:, :n].cpu().double()
        tol = 0 if dtype == mg.GEMM_I8 else (1e-4 if dtype == mg.GEMM_F32 else 1e-2) * k
        assert float((got - ref.double()).abs().max()) <= tol
        assert torch.equal(C[:, n:], pad), "columns past n were written"


def test_count_finds_planted_sentinels(env):
    import torch
    env["MGEMM_DEBUG"] = "1"
    mg.gemm_init(None)
    mg.debug_unwritten()
    C = torch.zeros((40, 37), dtype=torch.int32, device="cuda")
    C.view(-1)[[0, 5, 41, 1479]] = int(SENTINEL32.view(np.int32))
    mg.debug_count(C, 40, 37, 37, mg.GEMM_F32)
    assert mg.debug_unwritten() == 4
    mg.debug_count(C, 1, 37, 37, mg.GEMM_F32)   # first row only: elements 0 and 5
    assert mg.debug_unwritten() == 2
    D = torch.full((8, 8), 0x7FF8DEADDEADDEAD, dtype=torch.int64, device="cuda")
    mg.debug_count(D, 8, 6, 8, mg.GEMM_F64)
    assert mg.debug_unwritten() == 48


def test_environment_pin(env):
    import torch
    env["MGEMM_FORCE_CFG"] = f"{mg.GEMM_F32}:0:1,{mg.GEMM_I8}:1, junk"
    env.pop("MGEMM_DEBUG", None)
    mg.gemm_init(None)
    A = torch.rand((512, 512), device="cuda")
    C = torch.zeros((512, 512), device="cuda")
    mg.gemm("N", "N", 512, 512, 512, 1.0, A, 512, A, 512, 0.0, C, 512, mg.GEMM_F32)
    assert mg.last_config()["cfg"] == 0 and mg.last_config()["order"] == 1
    mg.force_config(mg.GEMM_F32, 2, 0)   # the thread's own pin wins
    try:
        mg.gemm("N", "N", 512, 512, 512, 1.0, A, 512, A, 512, 0.0, C, 512, mg.GEMM_F32)
        assert mg.last_config()["cfg"] == 2
    finally:
        mg.force_config(mg.GEMM_F32, -1, 0)
    Ai = torch.ones((256, 256), dtype=torch.int8, device="cuda")
    Ci = torch.zeros((256, 256), dtype=torch.int32, device="cuda")
    mg.gemm("N", "N", 256, 256, 256, 1, Ai, 256, Ai, 256, 0, Ci, 256, mg.GEMM_I8)
    assert mg.last_config()["cfg"] == 1
    assert int(Ci[0, 0]) == 256
