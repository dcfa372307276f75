"""Offsets beyond 32 bits: a 50000 x 50000 C (2.5e9 elements, 10 GB) with
k = 32, so that row * ldc passes 2^31 for the rows from 42950 on, through
the tuned dispatch (FP32, the x3 split, INT8) and the grouped launch (INT8);
sampled rows and columns match the float64 / int64 product of the operands."""
import numpy as np
import pytest

import paper_2310_20347_amd as mg

pytestmark = pytest.mark.gpu

M = N = 50000
K = 32
ROWS = [0, 1, 32767, 32768, 42949, 42950, 49999]
COLS = [0, 1, 127, 128, 12345, 49871, 49999]


def _operands(torch, dt):
    g = torch.Generator().manual_seed(3)
    if dt == mg.GEMM_I8:
        A = torch.randint(-128, 128, (M, K), generator=g, dtype=torch.int8)
        B = torch.randint(-128, 128, (K, N), generator=g, dtype=torch.int8)
        return A, B, torch.int32, 1, 0
    A = torch.rand((M, K), generator=g) * 2 - 1
    B = torch.rand((K, N), generator=g) * 2 - 1
    return A, B, torch.float32, 1.0, 0.0


def _check(torch, C, A, B, dt):
    r = torch.tensor(ROWS)
    c = torch.tensor(COLS)
    got = C[r][:, c].cpu().double()
    ref = A[r].double() @ B[:, c].double()
    if dt == mg.GEMM_I8:
        assert torch.equal(got, ref)
    else:
        assert float((got - ref).abs().max()) <= 2e-6 * K
    assert not torch.isnan(got).any()


@pytest.mark.parametrize("dt", [mg.GEMM_F32, mg.GEMM_F32_BF16X3, mg.GEMM_I8],
                         ids=lambda d: mg.DTYPE_NAMES[d])
def test_gemm_beyond_32_bit_offsets(dt):
    import torch
    mg.gemm_init(None)
    A, B, ct, one, zero = _operands(torch, dt)
    dA, dB = A.cuda(), B.cuda()
    C = torch.full((M, N), -7, dtype=ct, device="cuda")
    print(f"{mg.DTYPE_NAMES[dt]} {M}x{N}x{K}", flush=True)
    mg.gemm("N", "N", M, N, K, one, dA, K, dB, N, zero, C, N, dt)
    torch.cuda.synchronize()
    print("config", mg.last_config(), flush=True)
    _check(torch, C, A, B, dt)
    del C
    torch.cuda.empty_cache()


def test_grouped_beyond_32_bit_offsets():
    import torch
    mg.gemm_init(None)
    dt = mg.GEMM_I8
    A, B, ct, one, zero = _operands(torch, dt)
    dA, dB = A.cuda(), B.cuda()
    C = torch.full((M, N), -7, dtype=ct, device="cuda")
    small = torch.zeros((16, 16), dtype=ct, device="cuda")
    probs = [mg.Problem("N", "N", 16, 16, K, one, dA, K, dB, N, zero, small, 16),
             mg.Problem("N", "N", M, N, K, one, dA, K, dB, N, zero, C, N)]
    mg.gemm_grouped(probs, dt)
    torch.cuda.synchronize()
    _check(torch, C, A, B, dt)
    ref = A[:16].long() @ B[:, :16].long()
    assert torch.equal(small.cpu().long(), ref)
    del C
    torch.cuda.empty_cache()
