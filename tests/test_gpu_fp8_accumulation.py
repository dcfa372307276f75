"""The FP8 MFMA's accumulation precision, measured through the library: every
product of two E4M3 values is exact in FP32, yet one instruction sums its
products (128 for the 16x16 form, 64 for the 32x32 one) with about 12 bits
relative to the largest of them.  With k equal to one instruction's k (one
instruction per output) the error of each C entry against the exact sum of
its decoded products, divided by that entry's largest |product|, stays
within 2^-11 (the allowance the FP8 parity tolerance adds per instruction's
chunk of k) and is far above FP32 accumulation's rounding (the sums are not
exact).  Small-integer data, whose products and sums are exact in fewer
bits, come out exact."""
import numpy as np
import pytest

import oracle
import paper_2310_20347_amd as mg
from gemm_cases import gpu_init
from paper_2310_20347_amd import inputs

pytestmark = pytest.mark.gpu


def _config(form):
    """The first configuration whose wave tiles are made of form x form MFMAs."""
    ids = [i for i in range(mg.num_configs(mg.GEMM_F8E4M3))
           if mg.config_info(mg.GEMM_F8E4M3, i)["mfma"] == form
           and mg.config_supports(mg.GEMM_F8E4M3, i, "N", "N")]
    assert ids, f"no {form}x{form} FP8 configuration"
    return ids[0]


def _run(a32, b32, cfg):
    import torch
    gpu_init()
    m, k = a32.shape
    n = b32.shape[1]
    A = inputs.to_e4m3_bits(a32)
    B = inputs.to_e4m3_bits(b32)
    C = torch.empty((m, n), dtype=torch.float32, device="cuda")
    mg.force_config(mg.GEMM_F8E4M3, cfg, 0)
    try:
        mg.gemm("N", "N", m, n, k, 1.0, torch.from_numpy(A).cuda(), k, torch.from_numpy(B).cuda(),
                n, 0.0, C, n, mg.GEMM_F8E4M3)
        torch.cuda.synchronize()
        assert mg.last_config()["cfg"] == cfg
    finally:
        mg.force_config(mg.GEMM_F8E4M3, -1, 0)
    return C.cpu().numpy().astype(np.float64), oracle.decode_e4m3(A).reshape(m, k), \
        oracle.decode_e4m3(B).reshape(k, n)


@pytest.mark.parametrize("form", [16, 32], ids=["16x16x128", "32x32x64"])
def test_fp8_mfma_sums_with_about_12_bits(form):
    m = n = 128
    k = 128 if form == 16 else 64
    a32 = inputs.normal((m, k), 501)
    b32 = inputs.normal((k, n), 502)
    C, Ad, Bd = _run(a32, b32, _config(form))
    exact = Ad @ Bd                                        # products exact, summed in FP64
    pmax = np.abs(Ad)[:, :, None] * np.abs(Bd)[None, :, :]
    pmax = pmax.max(axis=1)                                # largest |a_ip b_pj| per entry
    ratio = np.abs(C - exact) / np.maximum(pmax, np.finfo(np.float64).tiny)
    worst = float(ratio.max())
    print(f"max |C - exact| / max|product| = 2^{np.log2(worst):.2f}", flush=True)
    assert worst <= 2.0 ** -11
    # FP32 accumulation of 128 such products would stay near 2^-24 k; the
    # measured error is orders of magnitude above it
    assert worst >= 2.0 ** -16


@pytest.mark.parametrize("form", [16, 32], ids=["16x16x128", "32x32x64"])
def test_fp8_small_integers_exact(form):
    k = 128
    a32 = inputs.small_ints((64, k), 503, -4, 4)
    b32 = inputs.small_ints((k, 64), 504, -4, 4)
    C, Ad, Bd = _run(a32, b32, _config(form))
    assert np.array_equal(C, Ad @ Bd)
