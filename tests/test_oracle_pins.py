"""Pins of the oracle against facts it does not compute itself.

Each pin is a function of a GEMM callable with the oracle's ``gemm_f64``
signature, so the same pins run on the oracle (must pass) and on planted
mistakes of it (each must fail at least one pin):

* identity / permutation matrices (closed forms: C = op(B) or a row/column
  permutation of it, exactly);
* rank-one closed form C(i,j) = alpha*k*u_i*v_j + beta*C0(i,j), exactly;
* small-integer matrices against numpy's exact int64 matmul (library);
* random real matrices against numpy's float64 matmul (library) to 1e-12;
* BLAS special cases (alpha = 0 / beta = 0 do not read A,B / C0; k = 0).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2310_20347_amd import inputs

TRANS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]


def stored(op_mat, t):
    """Stored (row-major) form of an operand whose op() is op_mat."""
    return np.ascontiguousarray(op_mat.T if t in "Tt" else op_mat)


def run(g, ta, tb, alpha, opA, opB, beta=0.0, C0=None, pad=0):
    """Call a gemm_f64-like callable on op() matrices, with padded leading dims."""
    m, k = opA.shape
    n = opB.shape[1]
    As, Bs = stored(opA, ta), stored(opB, tb)
    if pad:
        As = np.pad(As, ((0, 0), (0, pad)), constant_values=np.nan)
        Bs = np.pad(Bs, ((0, 0), (0, pad)), constant_values=np.nan)
    C0s = None
    ldc0 = n
    if C0 is not None:
        C0s = np.pad(C0, ((0, 0), (0, pad)), constant_values=np.nan) if pad else C0
        ldc0 = C0s.shape[1]
    return g(ta, tb, m, n, k, alpha, As, As.shape[1], Bs, Bs.shape[1], beta, C0s, ldc0)


# -- pins -----------------------------------------------------------------------

def pin_identity(g):
    rng = np.random.default_rng(11)
    for ta, tb in TRANS:
        m, k, n = 7, 7, 5
        B = rng.integers(-9, 10, size=(k, n)).astype(np.float64)
        C0 = rng.integers(-9, 10, size=(m, n)).astype(np.float64)
        C = run(g, ta, tb, 2.0, np.eye(m), B, 0.5, C0, pad=3)
        if not np.array_equal(C, 2.0 * B + 0.5 * C0):
            return False
        A = rng.integers(-9, 10, size=(m, k)).astype(np.float64)
        C = run(g, ta, tb, 1.0, A, np.eye(k), 0.0, None, pad=1)
        if not np.array_equal(C, A):
            return False
    return True


def pin_permutation(g):
    rng = np.random.default_rng(12)
    for ta, tb in TRANS:
        m, k, n = 9, 9, 6
        perm = rng.permutation(m)
        P = np.eye(m)[perm]                    # (P B)[i] = B[perm[i]]
        B = rng.integers(-50, 51, size=(k, n)).astype(np.float64)
        if not np.array_equal(run(g, ta, tb, 1.0, P, B), B[perm]):
            return False
        Q = np.eye(n)[:, rng.permutation(n)]   # right permutation of columns
        A = rng.integers(-50, 51, size=(5, n)).astype(np.float64)
        if not np.array_equal(run(g, ta, tb, 1.0, A, Q), A @ Q):
            return False
    return True


def pin_rank_one(g):
    rng = np.random.default_rng(13)
    for ta, tb in TRANS:
        m, n, k = 6, 8, 37
        u = rng.integers(-7, 8, size=m).astype(np.float64)
        v = rng.integers(-7, 8, size=n).astype(np.float64)
        A = np.repeat(u[:, None], k, axis=1)
        B = np.repeat(v[None, :], k, axis=0)
        C0 = rng.integers(-3, 4, size=(m, n)).astype(np.float64)
        C = run(g, ta, tb, -3.0, A, B, 2.0, C0, pad=2)
        if not np.array_equal(C, -3.0 * k * np.outer(u, v) + 2.0 * C0):
            return False
    return True


def pin_small_int_exact(g):
    rng = np.random.default_rng(14)
    for ta, tb in TRANS:
        m, n, k = 13, 11, 29
        A = rng.integers(-8, 9, size=(m, k))
        B = rng.integers(-8, 9, size=(k, n))
        C0 = rng.integers(-8, 9, size=(m, n))
        ref = 3 * (A @ B) - 2 * C0             # numpy exact int64 matmul
        C = run(g, ta, tb, 3.0, A.astype(np.float64), B.astype(np.float64), -2.0,
                C0.astype(np.float64), pad=4)
        if not np.array_equal(C, ref.astype(np.float64)):
            return False
    return True


def pin_numpy_f64(g):
    rng = np.random.default_rng(15)
    for ta, tb in TRANS:
        m, n, k = 17, 23, 31
        A = rng.uniform(-1, 1, size=(m, k))
        B = rng.uniform(-1, 1, size=(k, n))
        C0 = rng.uniform(-1, 1, size=(m, n))
        ref = 0.75 * (A @ B) + 1.25 * C0
        C = run(g, ta, tb, 0.75, A, B, 1.25, C0, pad=5)
        if np.max(np.abs(C - ref)) > 1e-12 * max(1.0, np.max(np.abs(ref))):
            return False
    return True


def pin_blas_special(g):
    nan = np.full((4, 3), np.nan)
    C0 = np.arange(20, dtype=np.float64).reshape(4, 5)
    # alpha == 0: A and B are not read
    C = g("N", "N", 4, 5, 3, 0.0, nan, 3, np.full((3, 5), np.nan), 5, 2.0, C0, 5)
    if not np.array_equal(C, 2.0 * C0):
        return False
    # beta == 0: C0 is not read
    A = np.ones((4, 3))
    B = np.ones((3, 5))
    C = g("N", "N", 4, 5, 3, 1.0, A, 3, B, 5, 0.0, np.full((4, 5), np.nan), 5)
    if not np.array_equal(C, np.full((4, 5), 3.0)):
        return False
    # k == 0: C = beta * C0
    C = g("N", "N", 4, 5, 0, 1.0, np.zeros(1), 1, np.zeros(1), 5, -1.0, C0, 5)
    return np.array_equal(C, -C0)


PINS = [pin_identity, pin_permutation, pin_rank_one, pin_small_int_exact, pin_numpy_f64,
        pin_blas_special]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_oracle_passes_pin(pin):
    assert pin(oracle.gemm_f64)


# -- planted mistakes: each must be caught by at least one pin -----------------------

def _mut_drop_last_term(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0):
    return oracle.gemm_f64(ta, tb, m, n, max(k - 1, 0), alpha, A, lda, B, ldb, beta, C0, ldc0)


def _mut_transposed_operand(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0):
    # reads B's storage with the other trans flag when that fits (square-ish cases)
    tb2 = "N" if tb in "Tt" else "T"
    try:
        return oracle.gemm_f64(ta, tb2, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0)
    except ValueError:
        return np.full((m, n), np.nan)


def _mut_beta_sign(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0):
    return oracle.gemm_f64(ta, tb, m, n, k, alpha, A, lda, B, ldb, -beta, C0, ldc0)


def _mut_alpha_dropped(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0):
    return oracle.gemm_f64(ta, tb, m, n, k, 1.0 if alpha != 0 else 0.0, A, lda, B, ldb,
                           beta, C0, ldc0)


def _mut_ld_off_by_one(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0):
    # wrong row stride for A (a classic index bug), kept in bounds
    A = np.asarray(A).reshape(-1)
    rows = k if ta in "Tt" else m
    cols = m if ta in "Tt" else k
    if rows > 1 and lda > cols:
        return oracle.gemm_f64(ta, tb, m, n, k, alpha, A, lda - 1, B, ldb, beta, C0, ldc0)
    return oracle.gemm_f64(ta, tb, m, n, k, alpha, A[1:] if A.size > 1 else A, lda, B, ldb,
                           beta, C0, ldc0) if A.size > (rows - 1) * lda + cols else \
        np.full((m, n), np.nan)


MUTANTS = [_mut_drop_last_term, _mut_transposed_operand, _mut_beta_sign, _mut_alpha_dropped,
           _mut_ld_off_by_one]


@pytest.mark.parametrize("mutant", MUTANTS, ids=lambda f: f.__name__)
def test_pins_catch_planted_mistake(mutant):
    def safe(pin):
        try:
            return pin(mutant)
        except ValueError:
            return False
    assert not all(safe(p) for p in PINS), "no pin caught this planted mistake"


# -- entries / int8 / pieces ------------------------------------------------------

def test_entries_equal_full_product():
    rng = np.random.default_rng(21)
    m, n, k = 19, 27, 33
    for ta, tb in TRANS:
        A = stored(rng.uniform(-1, 1, size=(m, k)), ta)
        B = stored(rng.uniform(-1, 1, size=(k, n)), tb)
        C0 = rng.uniform(-1, 1, size=(m, n))
        full = oracle.gemm_f64(ta, tb, m, n, k, 1.5, A, A.shape[1], B, B.shape[1], -0.5, C0, n)
        rows = rng.integers(0, m, 40)
        cols = rng.integers(0, n, 40)
        e = oracle.entries_f64(ta, tb, k, 1.5, A, A.shape[1], B, B.shape[1], -0.5, C0, n,
                               rows, cols)
        assert np.array_equal(e, full[rows, cols])


@pytest.mark.parametrize("ta,tb", TRANS)
def test_i8_matches_numpy_int64(ta, tb):
    m, n, k = 23, 19, 301
    A = inputs.int8_uniform((m, k), 31)
    B = inputs.int8_uniform((k, n), 32)
    C0 = np.random.default_rng(33).integers(-1000, 1000, size=(m, n)).astype(np.int32)
    As, Bs = stored(A, ta), stored(B, tb)
    C = oracle.gemm_i8(ta, tb, m, n, k, 3, As, As.shape[1], Bs, Bs.shape[1], -2, C0, n)
    ref = 3 * (A.astype(np.int64) @ B.astype(np.int64)) - 2 * C0.astype(np.int64)
    assert np.array_equal(C, ref.astype(np.int32))
    rows = np.arange(m)
    cols = (rows * 7) % n
    e = oracle.entries_i8(ta, tb, k, 3, As, As.shape[1], Bs, Bs.shape[1], -2, C0, n, rows, cols)
    assert np.array_equal(e, C[rows, cols])


def test_i8_extremes_closed_form():
    k = 4096
    A = np.full((3, k), -128, np.int8)
    B = np.full((k, 2), -128, np.int8)
    C = oracle.gemm_i8("N", "N", 3, 2, k, 1, A, k, B, 2, 0)
    assert np.all(C == 16384 * k)
    A2 = np.tile(np.array([127, -127], np.int8), (2, k // 2))
    B2 = np.full((k, 2), 127, np.int8)
    C2 = oracle.gemm_i8("N", "N", 2, 2, k, 1, A2, k, B2, 2, 0)
    assert np.all(C2 == 0)


def test_i8_wraps_to_int32():
    k = 64
    A = np.full((2, k), 127, np.int8)
    B = np.full((k, 2), 127, np.int8)
    alpha = 200000                          # 127*127*64*200000 overflows int32
    C = oracle.gemm_i8("N", "N", 2, 2, k, alpha, A, k, B, 2, 0)
    exact = np.int64(127 * 127 * k) * alpha
    assert np.all(C == np.array(exact).astype(np.int32))   # numpy wraps modulo 2^32
    assert exact > 2**31


def test_pieces_single_term_equals_plain():
    rng = np.random.default_rng(41)
    m, n, k = 9, 14, 40
    for ta, tb in TRANS:
        A = stored(rng.uniform(-1, 1, size=(m, k)), ta)
        B = stored(rng.uniform(-1, 1, size=(k, n)), tb)
        C0 = rng.uniform(-1, 1, size=(m, n))
        p = oracle.gemm_pieces(ta, tb, m, n, k, 0.5, [A], A.shape[1], [B], B.shape[1],
                               [(0, 0)], 2.0, C0)
        f = oracle.gemm_f64(ta, tb, m, n, k, 0.5, A, A.shape[1], B, B.shape[1], 2.0, C0, n)
        assert np.array_equal(p, f)


def test_pieces_all_terms_distribute():
    """With every piece pair formed, sum_u sum_v PA_u PB_v = (sum PA)(sum PB)."""
    rng = np.random.default_rng(42)
    m, n, k = 8, 10, 24
    x = rng.integers(-4, 5, size=(3, m, k)).astype(np.float64)
    y = rng.integers(-4, 5, size=(3, k, n)).astype(np.float64)
    terms = [(u, v) for u in range(3) for v in range(3)]
    p = oracle.gemm_pieces("N", "N", m, n, k, 1.0, list(x), k, list(y), n, terms)
    assert np.array_equal(p, x.sum(0) @ y.sum(0))


# -- number formats -----------------------------------------------------------------

def test_decode_e4m3_all_codes():
    import torch
    codes = np.arange(256, dtype=np.uint8)
    mine = oracle.decode_e4m3(codes)
    lib = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float32).numpy()
    nan = np.isnan(lib)
    assert np.array_equal(np.isnan(mine), nan)
    assert set(np.flatnonzero(nan)) == {0x7F, 0xFF}
    assert np.array_equal(mine[~nan], lib[~nan].astype(np.float64))
    assert mine[0x7E] == 448.0 and mine[0x01] == 2.0 ** -9 and mine[0x38] == 1.0
    assert mine[0x08] == 2.0 ** -6 and mine[0xFE] == -448.0


def test_decode_bf16_and_f16_match_library():
    import torch
    bits = np.arange(0, 65536, 7, dtype=np.uint16)
    lib_bf = torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    mine = oracle.decode_bf16(bits)
    ok = ~np.isnan(lib_bf)
    assert np.array_equal(np.isnan(mine), ~ok)
    assert np.array_equal(mine[ok], lib_bf[ok])
    lib_h = bits.view(np.float16).astype(np.float64)
    mine_h = oracle.decode_f16(bits)
    okh = ~np.isnan(lib_h)
    assert np.array_equal(np.isnan(mine_h), ~okh)
    assert np.array_equal(mine_h[okh], lib_h[okh])


def test_split_bf16_exact_and_rne():
    rng = np.random.default_rng(51)
    x = (rng.standard_normal(200000) * np.exp2(rng.uniform(-60, 60, 200000))).astype(np.float32)
    x[:4] = [0.0, -0.0, 1.0, np.float32(1.0) + np.float32(2.0 ** -23)]
    hi, mid, lo = oracle.split_bf16(x, 3)
    # hi is the library's round-to-nearest-even bf16 cast
    assert np.array_equal(hi, inputs.to_bf16_bits(x))
    h, md, l_ = (oracle.decode_bf16(v) for v in (hi, mid, lo))
    # the three pieces reproduce every normal FP32 value exactly
    assert np.array_equal(h + md + l_, x.astype(np.float64))
    # each residual is at most half an ulp of bf16 of the previous piece
    nz = h != 0
    assert np.all(np.abs(md[nz]) <= np.abs(h[nz]) * 2.0 ** -8)
    # two pieces keep 16 significant bits: relative error <= 2^-16
    assert np.all(np.abs((h + md) - x) <= np.abs(x.astype(np.float64)) * 2.0 ** -16)


def test_split_x6_not_worse_than_x3():
    rng = np.random.default_rng(52)
    m, n, k = 32, 32, 16
    A = rng.uniform(-1, 1, size=(m, k)).astype(np.float32)
    B = rng.uniform(-1, 1, size=(k, n)).astype(np.float32)
    pa = [oracle.decode_bf16(p) for p in oracle.split_bf16(A, 3)]
    pb = [oracle.decode_bf16(p) for p in oracle.split_bf16(B, 3)]
    ref = oracle.gemm("N", "N", 1.0, A, B)
    e3 = np.abs(oracle.gemm_pieces("N", "N", m, n, k, 1.0, pa, k, pb, n, oracle.TERMS_X3) - ref).max()
    e6 = np.abs(oracle.gemm_pieces("N", "N", m, n, k, 1.0, pa, k, pb, n, oracle.TERMS_X6) - ref).max()
    e1 = np.abs(oracle.gemm_pieces("N", "N", m, n, k, 1.0, pa, k, pb, n, [(0, 0)]) - ref).max()
    assert e6 <= e3 <= e1
    assert e3 < 2.0 ** -14 * k and e1 > 2.0 ** -10


def test_normalized_error_closed_form():
    C = np.array([[1.0, 2.0], [3.0, 4.5]])
    R = np.array([[1.0, 2.0], [3.0, 4.0]])
    assert math.isclose(oracle.normalized_error(C, R, 8, 2.0, 0.25), 0.5 / (8 * 2.0 * 0.25))
    assert oracle.normalized_error(R, R, 8, 0.0, 0.0) == 0.0


def test_empty_shapes():
    assert oracle.gemm_f64("N", "N", 0, 5, 3, 1.0, np.zeros(1), 3, np.zeros(15), 5).shape == (0, 5)
    assert oracle.gemm_i8("N", "N", 4, 0, 3, 1, np.zeros(12), 3, np.zeros(1), 1).shape == (4, 0)


# --- scaled low-precision path: exponents and format encoders --------------

def _sweep_values():
    """Magnitudes over the binary16 / E4M3 ranges incl. subnormals, exact
    ties between neighbouring codes, and signs."""
    rng = np.random.default_rng(17)
    v = np.concatenate([rng.uniform(-1, 1, 4000) * np.exp2(rng.integers(-26, 16, 4000)),
                        np.exp2(np.arange(-26, 16, dtype=np.float64)),
                        (np.arange(1, 2048) + 0.5) * 2.0 ** -24,       # f16 subnormal ties
                        (np.arange(1024, 2047) + 0.5) * 2.0 ** -10])   # f16 normal ties
    return np.concatenate([v, -v]).astype(np.float32)


def test_f16_encoder_matches_library_rounding():
    # numpy's float32 -> float16 conversion rounds to nearest even
    x = _sweep_values()
    x = x[np.abs(x) < 65504]
    codes = oracle.scaled_codes(x[None, :], np.zeros(1, np.int32), "f16")[0]
    assert np.array_equal(codes, x.astype(np.float16).view(np.uint16))


def test_e4m3_encoder_matches_library_rounding():
    # torch's float32 -> float8_e4m3fn conversion rounds to nearest even in range
    import torch
    rng = np.random.default_rng(18)
    x = np.concatenate([rng.uniform(-1, 1, 5000) * np.exp2(rng.integers(-11, 9, 5000)),
                        (np.arange(1, 16) + 0.5) * 2.0 ** -9,          # subnormal ties
                        (np.arange(8, 16) + 0.5) * 2.0 ** 4]).astype(np.float32)
    x = x[np.abs(x) <= 448]
    codes = oracle.scaled_codes(x[None, :], np.zeros(1, np.int32), "e4m3")[0]
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(codes, ref)
    # saturation, not infinity or NaN, past 448
    big = np.array([[500.0, -1e6, 449.0]], np.float32)
    assert list(oracle.scaled_codes(big, np.zeros(1, np.int32), "e4m3")[0]) == [0x7E, 0xFE, 0x7E]


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
def test_scale_exponents_place_each_row_max(fmt):
    _, T = oracle.SCALED_FORMATS[fmt]
    x = inputs.badly_scaled(40, 70, 19)
    e = oracle.scale_exponents(x, T)
    mx = np.max(np.abs(x), axis=1).astype(np.float64)
    scaled = mx * np.exp2(-e.astype(np.float64))
    assert np.all(scaled >= 2.0 ** T) and np.all(scaled < 2.0 ** (T + 1))
    # shifting a row by 2^s shifts its exponent by s and leaves its codes alone
    s = np.arange(-5, 35, dtype=np.int32)
    x2 = np.ldexp(x.astype(np.float64), s[:, None]).astype(np.float32)
    e2 = oracle.scale_exponents(x2, T)
    assert np.array_equal(e2, e + s)
    assert np.array_equal(oracle.scaled_codes(x2, e2, fmt), oracle.scaled_codes(x, e, fmt))
    # zero and non-finite rows are not scaled
    z = np.zeros((2, 5), np.float32)
    z[1, 2] = np.inf
    assert list(oracle.scale_exponents(z, T)) == [0, 0]


@pytest.mark.parametrize("fmt,rel", [("bf16", 2.0 ** -8), ("f16", 2.0 ** -11), ("e4m3", 2.0 ** -4)])
def test_scaled_codes_round_trip_within_unit_roundoff(fmt, rel):
    _, T = oracle.SCALED_FORMATS[fmt]
    x = inputs.normal((30, 200), 20)
    e = oracle.scale_exponents(x, T)
    back = np.ldexp(oracle.decode_codes(oracle.scaled_codes(x, e, fmt), fmt),
                    e[:, None].astype(np.int64))
    # values within the format's normal range relative to their row maximum
    rowmax = np.max(np.abs(x), axis=1, keepdims=True)
    normal = np.abs(x) >= rowmax * 2.0 ** -(T + 5 if fmt != "bf16" else 100)
    err = np.abs(back - x)[normal] / np.abs(x)[normal]
    assert err.max() <= rel


def test_gemm_scaled_reference_equals_definition():
    # C = alpha * diag(2^e) (Qa Qb) diag(2^f) + beta C0, with Qa, Qb the codes
    m, n, k = 7, 5, 9
    a = inputs.badly_scaled(m, k, 21)
    b = inputs.badly_scaled(k, n, 22)
    c0 = inputs.uniform((m, n), 23, dtype=np.float64)
    C, qa, e, qbt, f = oracle.gemm_scaled("N", "N", m, n, k, 1.5, a, k, b, n, "f16", -0.5, c0, n)
    da = oracle.decode_f16(qa) * np.exp2(e[:, None].astype(np.float64))
    db = oracle.decode_f16(qbt) * np.exp2(f[:, None].astype(np.float64))
    ref = np.empty((m, n))
    for i in range(m):
        for j in range(n):
            ref[i, j] = 1.5 * sum(da[i, p] * db[j, p] for p in range(k)) - 0.5 * c0[i, j]
    assert np.allclose(C, ref, rtol=1e-12, atol=0)
    # transposed storage gives the same result
    Ct = oracle.gemm_scaled("T", "T", m, n, k, 1.5, a.T.copy(), m, b.T.copy(), k, "f16",
                            -0.5, c0, n)[0]
    assert np.array_equal(C, Ct)


# -- INT16 / INT32: exact integer value modulo 2^32 ------------------------------------

INT_DT = {16: np.int16, 32: np.int32}


def _int_operand(rng, shape, bits, extremes=True):
    lo, hi = -2 ** (bits - 1), 2 ** (bits - 1)
    x = rng.integers(lo, hi, size=shape, dtype=np.int64)
    if extremes and x.size >= 4:
        flat = x.reshape(-1)
        flat[0], flat[1], flat[-1] = lo, hi - 1, lo   # the most negative, most positive values
    return x.astype(INT_DT[bits])


def _run_int(g, bits, ta, tb, alpha, opA, opB, beta=0, C0=None, pad=0):
    m, k = opA.shape
    n = opB.shape[1]
    As, Bs = stored(opA, ta), stored(opB, tb)
    if pad:
        As = np.pad(As, ((0, 0), (0, pad)), constant_values=-1)
        Bs = np.pad(Bs, ((0, 0), (0, pad)), constant_values=-1)
    return g(bits, ta, tb, m, n, k, alpha, As, As.shape[1], Bs, Bs.shape[1], beta, C0, n)


def _wrap32_py(v):
    v &= 0xFFFFFFFF
    return v - (1 << 32) if v >= 1 << 31 else v


def pin_int_python_bigints(g):
    """Brute force in Python's exact integers on small inputs with extreme values."""
    rng = np.random.default_rng(61)
    for bits in (16, 32):
        for ta, tb in TRANS:
            m, n, k = 3, 4, 5
            A = _int_operand(rng, (m, k), bits)
            B = _int_operand(rng, (k, n), bits)
            C0 = rng.integers(-2**31, 2**31, size=(m, n), dtype=np.int64).astype(np.int32)
            alpha, beta = int(rng.integers(-2**31, 2**31)), int(rng.integers(-2**31, 2**31))
            C = _run_int(g, bits, ta, tb, alpha, A, B, beta, C0, pad=2)
            for i in range(m):
                for j in range(n):
                    s = sum(int(A[i, p]) * int(B[p, j]) for p in range(k))
                    if C[i, j] != _wrap32_py(alpha * s + beta * int(C0[i, j])):
                        return False
    return True


def pin_int_numpy(g):
    """int16: numpy's int64 matmul is exact; int32: numpy's uint64 matmul wraps
    modulo 2^64, which keeps the low 32 bits exact."""
    rng = np.random.default_rng(62)
    m, n, k = 13, 11, 67
    for ta, tb in TRANS:
        A = _int_operand(rng, (m, k), 16)
        B = _int_operand(rng, (k, n), 16)
        ref = (A.astype(np.int64) @ B.astype(np.int64)) * 3
        if not np.array_equal(_run_int(g, 16, ta, tb, 3, A, B, pad=1), ref.astype(np.int32)):
            return False
        A = _int_operand(rng, (m, k), 32)
        B = _int_operand(rng, (k, n), 32)
        ref = (A.astype(np.int64).astype(np.uint64) @ B.astype(np.int64).astype(np.uint64))
        ref = (ref * np.uint64(2**32 - 7)) & np.uint64(0xFFFFFFFF)   # alpha = -7 modulo 2^32
        if not np.array_equal(_run_int(g, 32, ta, tb, -7, A, B, pad=1),
                              ref.astype(np.uint32).view(np.int32)):
            return False
    return True


def pin_int_closed_forms(g):
    """All -32768 (int16): C = k 2^30 modulo 2^32; identity: C = op(B) exactly;
    rank one with u_i = 2^16 + i, v_j = 2^16 - j: C = k u_i v_j modulo 2^32."""
    for k, want in ((1, 2**30), (2, -2**31), (3, -2**30), (4, 0), (5, 2**30)):
        A = np.full((2, k), -32768, np.int16)
        B = np.full((k, 3), -32768, np.int16)
        if not np.all(_run_int(g, 16, "N", "N", 1, A, B) == want):
            return False
    rng = np.random.default_rng(63)
    for ta, tb in TRANS:
        Bm = _int_operand(rng, (6, 4), 32)
        C = _run_int(g, 32, ta, tb, 1, np.eye(6, dtype=np.int32), Bm, pad=3)
        if not np.array_equal(C, Bm):
            return False
    m, n, k = 4, 3, 9
    u = np.array([2**16 + i for i in range(m)], np.int64)
    v = np.array([2**16 - j for j in range(n)], np.int64)
    A = np.repeat(u[:, None], k, axis=1).astype(np.int32)
    B = np.repeat(v[None, :], k, axis=0).astype(np.int32)
    C = _run_int(g, 32, "N", "N", 1, A, B)
    want = [[_wrap32_py(k * int(u[i]) * int(v[j])) for j in range(n)] for i in range(m)]
    return np.array_equal(C, np.array(want, np.int32))


def pin_int_blas_special(g):
    """alpha == 0 reads neither A nor B (C = beta C0); beta == 0 does not read C0;
    k == 0 gives beta C0."""
    rng = np.random.default_rng(64)
    C0 = rng.integers(-2**31, 2**31, size=(3, 4), dtype=np.int64).astype(np.int32)
    A = _int_operand(rng, (3, 5), 32)
    B = _int_operand(rng, (5, 4), 32)
    C = _run_int(g, 32, "N", "N", 0, A, B, 3, C0)
    if not np.array_equal(C, (C0.astype(np.int64) * 3).astype(np.int32)):
        return False
    C = _run_int(g, 32, "N", "N", 1, A, B, 0, np.full((3, 4), 123456, np.int32))
    ref = (A.astype(np.int64).astype(np.uint64) @ B.astype(np.int64).astype(np.uint64))
    return np.array_equal(C, (ref & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.int32))


INT_PINS = [pin_int_python_bigints, pin_int_numpy, pin_int_closed_forms, pin_int_blas_special]


@pytest.mark.parametrize("pin", INT_PINS, ids=lambda p: p.__name__)
def test_int_oracle_passes_pin(pin):
    assert pin(oracle.gemm_int)


def _mut_int_drop_last_term(bits, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0):
    return oracle.gemm_int(bits, ta, tb, m, n, max(k - 1, 0), alpha, A, lda, B, ldb, beta, C0,
                           ldc0)


def _mut_int_int32_accumulator(bits, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0):
    # products kept in int32 before the sum: wrong whenever a product exceeds 2^31
    A = np.asarray(A).reshape(-1).astype(np.int64)
    B = np.asarray(B).reshape(-1).astype(np.int64)
    opA = (A[:k * lda].reshape(k, lda)[:, :m].T if ta in "Tt" else A[:m * lda].reshape(m, lda)[:, :k])
    opB = (B[:n * ldb].reshape(n, ldb)[:, :k].T if tb in "Tt" else B[:k * ldb].reshape(k, ldb)[:, :n])
    prod = np.clip(opA[:, :, None] * opB[None, :, :], -2**31, 2**31 - 1).sum(axis=1)
    v = alpha * prod
    if beta != 0:
        v = v + beta * np.asarray(C0, np.int64).reshape(m, -1)[:, :n]
    return (v & 0xFFFFFFFF).astype(np.uint32).view(np.int32)


def _mut_int_narrow_operand(bits, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0):
    # 32-bit operands read through 16 bits
    A = np.asarray(A).astype(np.int16) if bits == 32 else A
    return oracle.gemm_int(bits, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0)


def _mut_int_transposed(bits, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0):
    ta2 = "N" if ta in "Tt" else "T"
    try:
        return oracle.gemm_int(bits, ta2, tb, m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc0)
    except ValueError:
        return np.full((m, n), 0, np.int32)


INT_MUTANTS = [_mut_int_drop_last_term, _mut_int_int32_accumulator, _mut_int_narrow_operand,
               _mut_int_transposed]


@pytest.mark.parametrize("mutant", INT_MUTANTS, ids=lambda f: f.__name__)
def test_int_pins_catch_planted_mistake(mutant):
    def safe(pin):
        try:
            return pin(mutant)
        except (ValueError, IndexError):
            return False
    assert not all(safe(p) for p in INT_PINS), "no pin caught this planted mistake"


def test_int_entries_equal_full_product():
    rng = np.random.default_rng(65)
    m, n, k = 17, 21, 45
    for bits in (16, 32):
        for ta, tb in TRANS:
            A = stored(_int_operand(rng, (m, k), bits), ta)
            B = stored(_int_operand(rng, (k, n), bits), tb)
            C0 = rng.integers(-2**31, 2**31, size=(m, n), dtype=np.int64).astype(np.int32)
            full = oracle.gemm_int(bits, ta, tb, m, n, k, -5, A, A.shape[1], B, B.shape[1], 7,
                                   C0, n)
            rows = rng.integers(0, m, 40)
            cols = rng.integers(0, n, 40)
            e = oracle.entries_int(bits, ta, tb, k, -5, A, A.shape[1], B, B.shape[1], 7, C0, n,
                                   rows, cols)
            assert np.array_equal(e, full[rows, cols])
