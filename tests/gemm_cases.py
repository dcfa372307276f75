"""Shared helpers of the GPU parity tests: seeded operands in every storage
format, a GPU call through the C ABI, and the oracle's result on the same
inputs (both on the quantised inputs the kernel sees and on the FP32 source).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle
import paper_2310_20347_amd as mg
from paper_2310_20347_amd import inputs

FLOAT_SPLIT = (mg.GEMM_F32_BF16X3, mg.GEMM_F32_BF16X3_ONLY, mg.GEMM_F32_BF16X6)
ALL_DTYPES = (mg.GEMM_F32, mg.GEMM_F32_BF16X3, mg.GEMM_BF16, mg.GEMM_F16, mg.GEMM_F8E4M3,
              mg.GEMM_I8, mg.GEMM_F32_BF16X3_ONLY, mg.GEMM_F32_BF16X6, mg.GEMM_F64)

# Graded tolerance of the normalised error max|C-Cref| / (k max|A| max|B|)
# against the FP64 oracle on the FP32 source inputs (FP64: its own inputs).
SOURCE_TOL = {mg.GEMM_F32: 2e-6, mg.GEMM_F32_BF16X3: 2e-6, mg.GEMM_F32_BF16X6: 2e-6,
              mg.GEMM_BF16: 8e-3, mg.GEMM_F16: 8e-3, mg.GEMM_F8E4M3: 6.25e-2,
              mg.GEMM_F32_BF16X3_ONLY: None, mg.GEMM_F64: None}
# Kernel-correctness gate: against the oracle on the inputs the kernel actually
# multiplies, the only error left is FP32 accumulation.
QUANT_TOL = 2e-6


def quant_tol(c, fp8_chunk=128):
    """Tolerance of the quantised-input gate.  FP8 MFMA instructions sum the
    products of one instruction (128 of them for the 16x16 form, 64 for the
    32x32 one) with about 12 bits relative to the largest product (measured
    on gfx950), so the FP8 bound adds 2^-11 * max|product| per fp8_chunk-long
    chunk of k; quantised magnitudes exceed the source's by at most 2^-4
    (1.07 covers it)."""
    if c.dtype == mg.GEMM_F8E4M3 and c.k > 0:
        return QUANT_TOL + 1.07 * 2.0 ** -11 * ((c.k + fp8_chunk - 1) // fp8_chunk) / c.k
    if c.dtype == mg.GEMM_F64:
        # FP64 accumulation of k products, plus the alpha/beta roundings:
        # |error| <= (k + 2) u sum|a||b| + ..., so (k + 4) u covers the
        # normalised error with u = 2^-53
        return (c.k + 4) * 2.0 ** -53
    return QUANT_TOL


def terms_for(dtype, k):
    if dtype == mg.GEMM_F32_BF16X3:
        return oracle.TERMS_X3 if k >= 64 else oracle.TERMS_X6
    if dtype == mg.GEMM_F32_BF16X3_ONLY:
        return oracle.TERMS_X3
    if dtype == mg.GEMM_F32_BF16X6:
        return oracle.TERMS_X6
    return None


def stored(op_mat, t, ld):
    """Row-major storage of an operand with op() = op_mat, padded to ld columns."""
    s = op_mat.T if t in "Tt" else op_mat
    out = np.zeros((s.shape[0], ld), dtype=s.dtype)
    out[:, :s.shape[1]] = s
    return out


def encode(x32, dtype):
    """FP32 source values -> the storage the GEMM of `dtype` reads."""
    if dtype == mg.GEMM_BF16:
        return inputs.to_bf16_bits(x32)
    if dtype == mg.GEMM_F16:
        return inputs.to_f16_bits(x32)
    if dtype == mg.GEMM_F8E4M3:
        return inputs.to_e4m3_bits(x32)
    if dtype == mg.GEMM_I8:
        return x32.astype(np.int8)
    if dtype == mg.GEMM_F64:
        return np.ascontiguousarray(x32, dtype=np.float64)
    return np.ascontiguousarray(x32, dtype=np.float32)


def decode(stored_arr, dtype):
    """Exact values the kernel multiplies (oracle decoders)."""
    if dtype == mg.GEMM_BF16:
        return oracle.decode_bf16(stored_arr)
    if dtype == mg.GEMM_F16:
        return oracle.decode_f16(stored_arr)
    if dtype == mg.GEMM_F8E4M3:
        return oracle.decode_e4m3(stored_arr)
    return stored_arr.astype(np.float64)


_INITIALISED = False


def gpu_init():
    """gemm_init once per process: the tuning table, the grouped tables and
    the default workspace reservations of the current stream."""
    global _INITIALISED
    if not _INITIALISED:
        mg.gemm_init(None)
        _INITIALISED = True


def to_device(arr):
    import torch
    gpu_init()
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(a).cuda()


@dataclass
class Case:
    dtype: int
    ta: str
    tb: str
    m: int
    n: int
    k: int
    alpha: float = 1.0
    beta: float = 0.0
    pad: int = 0          # extra leading-dimension elements on A, B, C
    misalign: int = 0     # element offset of A and B in their buffers
    dist: str = "uniform"
    seed: int = 0


def make_operands(c: Case):
    """FP32 sources of op(A) (m x k), op(B) (k x n) and C0 (m x n)."""
    s = 1000 * c.seed
    if c.dtype == mg.GEMM_I8:
        a = inputs.int8_uniform((c.m, c.k), s + 1).astype(np.float32)
        b = inputs.int8_uniform((c.k, c.n), s + 2).astype(np.float32)
        c0 = np.random.default_rng(s + 3).integers(-1000, 1000, size=(c.m, c.n)).astype(np.int32)
        return a, b, c0
    ft = np.float64 if c.dtype == mg.GEMM_F64 else np.float32
    if c.dist == "uniform":
        a = inputs.uniform((c.m, c.k), s + 1, dtype=ft)
        b = inputs.uniform((c.k, c.n), s + 2, dtype=ft)
    elif c.dist == "normal":
        a = inputs.normal((c.m, c.k), s + 1, dtype=ft)
        b = inputs.normal((c.k, c.n), s + 2, dtype=ft)
    elif c.dist == "ints":
        a = inputs.small_ints((c.m, c.k), s + 1, dtype=ft)
        b = inputs.small_ints((c.k, c.n), s + 2, dtype=ft)
    elif c.dist == "badly_scaled":
        a = inputs.badly_scaled(c.m, c.k, s + 1, dtype=ft)
        b = inputs.badly_scaled(c.k, c.n, s + 2, dtype=ft)
    else:
        raise ValueError(c.dist)
    c0 = inputs.uniform((c.m, c.n), s + 3, dtype=ft)
    return a, b, c0


def run_case(c: Case, sample=None):
    """Runs the GPU GEMM; returns dict with C (GPU), Cq (oracle on quantised
    inputs), Cs (oracle on FP32 source; float paths) and the error metrics.
    With `sample` (rows, cols) only those entries are compared."""
    import torch
    a32, b32, c0 = make_operands(c)
    lda = (c.m if c.ta in "Tt" else c.k) + c.pad
    ldb = (c.k if c.tb in "Tt" else c.n) + c.pad
    ldc = c.n + c.pad
    As = stored(encode(a32, c.dtype), c.ta, lda)
    Bs = stored(encode(b32, c.dtype), c.tb, ldb)
    Cs0 = stored(c0, "N", ldc)

    dA = to_device(np.concatenate([np.zeros(c.misalign, As.dtype), As.reshape(-1)]))
    dB = to_device(np.concatenate([np.zeros(c.misalign, Bs.dtype), Bs.reshape(-1)]))
    dC = to_device(Cs0.reshape(-1).copy())
    esz = dA.element_size()
    mg.gemm(c.ta, c.tb, c.m, c.n, c.k, c.alpha, dA.data_ptr() + c.misalign * esz, lda,
            dB.data_ptr() + c.misalign * esz, ldb, c.beta, dC, ldc, c.dtype)
    torch.cuda.synchronize()
    cfg = mg.last_config()
    C = dC.cpu().numpy().reshape(c.m, ldc)[:, :c.n] if c.m else np.zeros((0, c.n))

    out = {"C": C, "cfg": cfg}
    if c.dtype == mg.GEMM_I8:
        if sample is None:
            out["Cq"] = oracle.gemm_i8(c.ta, c.tb, c.m, c.n, c.k, int(c.alpha), As, lda, Bs, ldb,
                                       int(c.beta), Cs0, ldc)
        else:
            r, q = sample
            out["Cq"] = oracle.entries_i8(c.ta, c.tb, c.k, int(c.alpha), As, lda, Bs, ldb,
                                          int(c.beta), Cs0, ldc, r, q)
            out["C"] = C[r, q]
        return out

    terms = terms_for(c.dtype, c.k)
    if terms is not None:
        # quantised oracle: the FP32 operands' bf16 pieces, listed products only
        npieces = 3 if len(terms) > 3 else 2
        PA = [oracle.decode_bf16(p) for p in oracle.split_bf16(As, npieces)]
        PB = [oracle.decode_bf16(p) for p in oracle.split_bf16(Bs, npieces)]
        if sample is None:
            out["Cq"] = oracle.gemm_pieces(c.ta, c.tb, c.m, c.n, c.k, c.alpha, PA, lda, PB, ldb,
                                           terms, c.beta, Cs0, ldc)
        else:
            out["Cq"] = None   # sampled checks use the source oracle only
    else:
        Aq, Bq = decode(As, c.dtype), decode(Bs, c.dtype)
        if sample is None:
            out["Cq"] = oracle.gemm_f64(c.ta, c.tb, c.m, c.n, c.k, c.alpha, Aq, lda, Bq, ldb,
                                        c.beta, Cs0, ldc)
        else:
            r, q = sample
            out["Cq"] = oracle.entries_f64(c.ta, c.tb, c.k, c.alpha, Aq, lda, Bq, ldb, c.beta,
                                           Cs0, ldc, r, q)
    As32, Bs32 = stored(a32, c.ta, lda), stored(b32, c.tb, ldb)
    if sample is None:
        out["Cs"] = oracle.gemm_f64(c.ta, c.tb, c.m, c.n, c.k, c.alpha, As32, lda, Bs32, ldb,
                                    c.beta, Cs0, ldc)
    else:
        r, q = sample
        out["Cs"] = oracle.entries_f64(c.ta, c.tb, c.k, c.alpha, As32, lda, Bs32, ldb, c.beta,
                                       Cs0, ldc, r, q)
        out["C"] = C[r, q]
    # graded error: max|C - Cref| / (k max|A| max|B|) on the source operands
    ma = float(np.max(np.abs(a32))) if a32.size else 0.0
    mb = float(np.max(np.abs(b32))) if b32.size else 0.0
    kk = max(c.k, 1) * max(abs(c.alpha), 1e-300)
    out["err_source"] = oracle.normalized_error(out["C"], out["Cs"], kk, ma, mb)
    if out["Cq"] is not None:
        out["err_quant"] = oracle.normalized_error(out["C"], out["Cq"], kk, ma, mb)
    return out


def check(c: Case, res, qtol=None):
    """Asserts the parity bar for case c."""
    if qtol is None:
        chunk = 128
        if c.dtype == mg.GEMM_F8E4M3 and res.get("cfg") is not None:
            chunk = 64 if mg.config_info(c.dtype, res["cfg"]["cfg"])["mfma"] == 32 else 128
        qtol = quant_tol(c, chunk)
    if c.dtype == mg.GEMM_I8:
        assert np.array_equal(res["C"], res["Cq"]), f"INT8 not bit-exact: {c}"
        return
    assert np.all(np.isfinite(res["C"])) or c.dist == "badly_scaled", f"non-finite output: {c}"
    if res.get("err_quant") is not None:
        assert res["err_quant"] <= qtol, f"quantised-input error {res['err_quant']:.3g}: {c}"
    tol = SOURCE_TOL.get(c.dtype)
    if tol is not None and c.dist != "badly_scaled":
        assert res["err_source"] <= tol, f"source error {res['err_source']:.3g} > {tol}: {c}"
