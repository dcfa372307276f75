"""INT16 and INT32 GEMM on the GPU against the oracle, bit for bit: both
configurations (vector ALUs; INT8 MFMA digit products) in all four layouts on
ragged shapes that span several tiles, padded and unaligned operands,
alpha / beta, extreme values, and sampled entries at full size."""
import numpy as np
import pytest

import oracle
import paper_2310_20347_amd as mg
from gemm_cases import gpu_init

pytestmark = pytest.mark.gpu

TRANS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]
NP = {16: np.int16, 32: np.int32}
DT = {16: mg.GEMM_I16, 32: mg.GEMM_I32}


def _operand(rng, shape, bits, kind="uniform"):
    lo, hi = -2 ** (bits - 1), 2 ** (bits - 1)
    if kind == "min":
        return np.full(shape, lo, NP[bits])
    if kind == "max":
        return np.full(shape, hi - 1, NP[bits])
    return rng.integers(lo, hi, size=shape, dtype=np.int64).astype(NP[bits])


def _stored(op, t, pad):
    s = np.ascontiguousarray(op.T if t == "T" else op)
    return np.pad(s, ((0, 0), (0, pad))) if pad else s


def _device(x, offset=0):
    """A device copy of x; `offset` elements of slack in front make the
    pointer unaligned for 16-byte loads."""
    import torch
    flat = np.concatenate([np.zeros(offset, x.dtype), x.reshape(-1)])
    t = torch.from_numpy(flat).cuda()
    return t, t[offset:]


def run(bits, ta, tb, m, n, k, alpha, beta, cfg, seed=0, kind="uniform", pad=0, offset=0):
    import torch
    gpu_init()
    rng = np.random.default_rng(seed)
    A = _operand(rng, (m, k), bits, kind)
    B = _operand(rng, (k, n), bits, kind)
    C0 = rng.integers(-2 ** 31, 2 ** 31, size=(m, n), dtype=np.int64).astype(np.int32)
    As, Bs = _stored(A, ta, pad), _stored(B, tb, pad)
    lda, ldb = As.shape[1], Bs.shape[1]
    keepA, dA = _device(As, offset)
    keepB, dB = _device(Bs, offset)
    dC = torch.from_numpy(C0.copy()).cuda()
    dt = DT[bits]
    try:
        mg.force_config(dt, cfg, 0)
        mg.gemm(ta, tb, m, n, k, alpha, dA, lda, dB, ldb, beta, dC, n, dt)
        used = mg.last_config()
    finally:
        mg.force_config(dt, -1, 0)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    want = oracle.gemm_int(bits, ta, tb, m, n, k, alpha, As, lda, Bs, ldb, beta, C0, n)
    return got, want, used


@pytest.mark.parametrize("bits", [16, 32])
@pytest.mark.parametrize("cfg", [0, 1])
@pytest.mark.parametrize("ta,tb", TRANS)
def test_every_layout_ragged(bits, cfg, ta, tb):
    print(f"i{bits} cfg {cfg} {ta}{tb}", flush=True)
    got, want, used = run(bits, ta, tb, 200, 136, 300, 3, -2, cfg, seed=1, pad=5)
    assert used["cfg"] == cfg
    assert np.array_equal(got, want)


@pytest.mark.parametrize("bits", [16, 32])
@pytest.mark.parametrize("shape", [(257, 129, 1001), (1, 300, 77), (65, 1, 64), (130, 70, 1),
                                   (64, 64, 64), (333, 517, 129)])
def test_digit_products_ragged_shapes(bits, shape):
    m, n, k = shape
    print(f"i{bits} digits {shape}", flush=True)
    got, want, _ = run(bits, "N", "N", m, n, k, 1, 0, 1, seed=2)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("bits", [16, 32])
@pytest.mark.parametrize("kind", ["min", "max"])
@pytest.mark.parametrize("cfg", [0, 1])
def test_extreme_values(bits, kind, cfg):
    # all -2^(w-1) (or all 2^(w-1)-1): every sum wraps modulo 2^32
    got, want, _ = run(bits, "N", "T", 96, 80, 515, 7, 1, cfg, kind=kind)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("bits", [16, 32])
def test_unaligned_operands(bits):
    # pointers one element past a 16-byte boundary, odd leading dimensions
    for cfg in (0, 1):
        got, want, _ = run(bits, "T", "N", 150, 90, 211, -1, 3, cfg, seed=3, pad=1, offset=1)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("bits", [16, 32])
def test_alpha_beta_extremes(bits):
    for alpha, beta in ((2 ** 31 - 1, -2 ** 31), (-2 ** 31, 0), (0, 5), (65536, 1)):
        got, want, _ = run(bits, "N", "N", 70, 50, 130, alpha, beta, 1, seed=4)
        assert np.array_equal(got, want), (alpha, beta)


@pytest.mark.parametrize("bits", [16, 32])
def test_full_size_sampled(bits):
    """4096 x 4096 x 4096 through the tuned dispatch: 2000 sampled entries
    against the oracle's entries, and the same call on the other
    configuration agrees everywhere."""
    import torch
    gpu_init()
    n = 4096
    rng = np.random.default_rng(5)
    A = _operand(rng, (n, n), bits)
    B = _operand(rng, (n, n), bits)
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    dC = torch.empty((n, n), dtype=torch.int32, device="cuda")
    dt = DT[bits]
    mg.gemm("N", "N", n, n, n, 1, dA, n, dB, n, 0, dC, n, dt)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    rows = rng.integers(0, n, 2000)
    cols = rng.integers(0, n, 2000)
    want = oracle.entries_int(bits, "N", "N", n, 1, A, n, B, n, 0, None, n, rows, cols)
    assert np.array_equal(got[rows, cols], want)
    other = 0 if mg.last_config()["cfg"] == 1 else 1
    dC2 = torch.empty_like(dC)
    try:
        mg.force_config(dt, other, 0)
        mg.gemm("N", "N", n, n, n, 1, dA, n, dB, n, 0, dC2, n, dt)
    finally:
        mg.force_config(dt, -1, 0)
    torch.cuda.synchronize()
    assert torch.equal(dC, dC2)


def test_digit_products_without_workspace_run_the_vector_tile():
    """On a stream without a reservation the digit configuration cannot get
    its planes: the call runs configuration 0 with the same result."""
    import torch
    gpu_init()
    s = torch.cuda.Stream()
    m, n, k = 96, 64, 200
    rng = np.random.default_rng(6)
    A = _operand(rng, (m, k), 32)
    B = _operand(rng, (k, n), 32)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.zeros((m, n), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    try:
        mg.force_config(mg.GEMM_I32, 1, 0)
        with torch.cuda.stream(s):
            mg.gemm("N", "N", m, n, k, 1, dA, k, dB, n, 0, dC, n, mg.GEMM_I32, stream=s)
            assert mg.last_config()["cfg"] == 0
        torch.cuda.synchronize()
    finally:
        mg.force_config(mg.GEMM_I32, -1, 0)
        mg.set_stream(None)
    assert np.array_equal(dC.cpu().numpy(), oracle.gemm_int(32, "N", "N", m, n, k, 1, A, k, B, n))
