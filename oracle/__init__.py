"""Oracle: a plain CPU reference for the GEMM family, in FP64 / exact int64.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product library (the HIP path)
never imports, links or calls it, and this package imports nothing from the
product package: the two share no code.

Every routine is a thin ctypes wrapper over ``oracle_gemm.c``:

* ``gemm_f64``      C = alpha*op(A)*op(B) + beta*C0 in FP64, the definition
                    of paper section 3.1 (C += AB) with BLAS alpha/beta/trans,
                    summed as the plain i -> p -> j triple loop of section 5.1.
* ``gemm_i8``       the same over int8 inputs with exact int64 sums, wrapped to
                    int32 at the end.
* ``gemm_int``      int16 or int32 inputs: the exact integer value of
                    alpha*op(A)*op(B) + beta*C0 modulo 2^32 (int32 C).
* ``gemm_pieces``   the split-product form used by the FP32-accurate path:
                    op(A) = sum of bf16 pieces, only listed piece pairs formed.
* ``entries_*``     individual entries C(i, j) of the same definitions, for
                    sampled checks at sizes where the full product is too slow.
* ``decode_*``      exact decoders for bfloat16, binary16 and OCP E4M3FN codes.
* ``split_bf16``    round-to-nearest-even split of FP32 into bf16 pieces.
* ``gemm_scaled``   the power-of-two scaled low-precision GEMM (per-row
                    exponents of op(A), per-column of op(B), format codes).
* ``normalized_error`` the graded error max|C - Cref| / (k max|A| max|B|).

Storage is row-major; ``lda``/``ldb``/``ldc`` are row strides in elements.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# Piece products of the split-product path, as (piece of A, piece of B),
# piece 0 = hi, 1 = mid, 2 = lo.  Three terms keep hi*hi, hi*mid, mid*hi;
# six terms add mid*mid, hi*lo, lo*hi.
TERMS_X3 = ((0, 0), (0, 1), (1, 0))
TERMS_X6 = TERMS_X3 + ((1, 1), (0, 2), (2, 0))

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double
_C = ctypes.c_char
_INT = ctypes.c_int


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_threads.restype = _INT
    lib.oracle_set_threads.argtypes = [_INT]
    lib.oracle_set_threads.restype = None
    lib.oracle_gemm_f64.argtypes = [_C, _C, _I64, _I64, _I64, _D, _P, _I64, _P, _I64,
                                    _D, _P, _I64, _P, _I64]
    lib.oracle_gemm_entries_f64.argtypes = [_C, _C, _I64, _D, _P, _I64, _P, _I64, _D,
                                            _P, _I64, _I64, _P, _P, _P]
    lib.oracle_gemm_pieces_f64.argtypes = [_C, _C, _I64, _I64, _I64, _D, _INT, _P, _I64,
                                           _INT, _P, _I64, _INT, _P, _P, _D, _P, _I64,
                                           _P, _I64]
    lib.oracle_gemm_i8.argtypes = [_C, _C, _I64, _I64, _I64, _I64, _P, _I64, _P, _I64,
                                   _I64, _P, _I64, _P, _I64]
    lib.oracle_gemm_entries_i8.argtypes = [_C, _C, _I64, _I64, _P, _I64, _P, _I64, _I64,
                                           _P, _I64, _I64, _P, _P, _P]
    lib.oracle_gemm_int.argtypes = [_INT, _C, _C, _I64, _I64, _I64, _I64, _P, _I64, _P, _I64,
                                    _I64, _P, _I64, _P, _I64]
    lib.oracle_gemm_entries_int.argtypes = [_INT, _C, _C, _I64, _I64, _P, _I64, _P, _I64, _I64,
                                            _P, _I64, _I64, _P, _P, _P]
    lib.oracle_decode_bf16.argtypes = [_P, _I64, _P]
    lib.oracle_decode_f16.argtypes = [_P, _I64, _P]
    lib.oracle_decode_e4m3.argtypes = [_P, _I64, _P]
    lib.oracle_split_bf16.argtypes = [_P, _I64, _INT, _P, _P, _P]
    lib.oracle_scale_exponents.argtypes = [_P, _I64, _I64, _INT, _P]
    lib.oracle_scaled_codes.argtypes = [_P, _I64, _I64, _P, _INT, _P]
    for f in ("oracle_gemm_f64", "oracle_gemm_entries_f64", "oracle_gemm_pieces_f64",
              "oracle_gemm_i8", "oracle_gemm_entries_i8", "oracle_gemm_int",
              "oracle_gemm_entries_int", "oracle_decode_bf16",
              "oracle_decode_f16", "oracle_decode_e4m3", "oracle_split_bf16",
              "oracle_scale_exponents", "oracle_scaled_codes"):
        getattr(lib, f).restype = None
    _lib = lib
    return lib


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's following calls (n >= 1)."""
    _load().oracle_set_threads(int(n))


def threads() -> int:
    """OpenMP threads the oracle runs on (OMP_NUM_THREADS or all cores)."""
    return int(_load().oracle_threads())


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else None


def _flat(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype).reshape(-1)


def _tc(t):
    t = t.decode() if isinstance(t, bytes) else t
    if t not in "NnTtCc" or len(t) != 1:
        raise ValueError(f"trans must be one of N,T,C: {t!r}")
    return t.encode()


def _is_t(t):
    return _tc(t) in (b"T", b"t", b"C", b"c")


def _check_ld(ta, tb, m, n, k, lda, ldb, ldc0, A, B, C0, beta):
    """Storage extents implied by the row-major layout; raise on undersize."""
    ra, ca = (k, m) if _is_t(ta) else (m, k)
    rb, cb = (n, k) if _is_t(tb) else (k, n)
    if ra and ca and (lda < ca or A.size < (ra - 1) * lda + ca):
        raise ValueError("A too small for its lda/shape")
    if rb and cb and (ldb < cb or B.size < (rb - 1) * ldb + cb):
        raise ValueError("B too small for its ldb/shape")
    if beta != 0 and m and n and (ldc0 < n or C0.size < (m - 1) * ldc0 + n):
        raise ValueError("C0 too small for its ldc/shape")


def gemm_f64(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta=0.0, C0=None, ldc0=None):
    """C = alpha*op(A)*op(B) + beta*C0 in FP64; returns an (m, n) float64 array.

    A, B, C0 are buffers of the stored matrices (any real dtype, read as FP64),
    row-major with row strides lda, ldb, ldc0.  C0 is not read when beta == 0.
    """
    lib = _load()
    A = _flat(A, np.float64)
    B = _flat(B, np.float64)
    ldc0 = n if ldc0 is None else ldc0
    C0f = _flat(C0, np.float64) if (C0 is not None and beta != 0) else np.zeros(0)
    _check_ld(ta, tb, m, n, k, lda, ldb, ldc0, A, B, C0f, beta)
    C = np.empty((m, n), dtype=np.float64)
    if m and n:
        lib.oracle_gemm_f64(_tc(ta), _tc(tb), m, n, k, float(alpha), _ptr(A), lda,
                            _ptr(B), ldb, float(beta), _ptr(C0f), ldc0, _ptr(C), n)
    return C


def gemm(ta, tb, alpha, A, B, beta=0.0, C0=None):
    """Convenience form over 2-D arrays of the stored matrices (ld = columns)."""
    A = np.asarray(A)
    B = np.asarray(B)
    m, k = (A.shape[1], A.shape[0]) if _is_t(ta) else A.shape
    n = B.shape[0] if _is_t(tb) else B.shape[1]
    return gemm_f64(ta, tb, m, n, k, alpha, A, A.shape[1], B, B.shape[1], beta, C0, n)


def entries_f64(ta, tb, k, alpha, A, lda, B, ldb, beta, C0, ldc0, rows, cols):
    """C(rows[t], cols[t]) of the FP64 definition, for sampled checks."""
    lib = _load()
    A = _flat(A, np.float64)
    B = _flat(B, np.float64)
    rows = _flat(rows, np.int64)
    cols = _flat(cols, np.int64)
    C0f = _flat(C0, np.float64) if (C0 is not None and beta != 0) else np.zeros(0)
    out = np.empty(rows.size, dtype=np.float64)
    if rows.size:
        lib.oracle_gemm_entries_f64(_tc(ta), _tc(tb), k, float(alpha), _ptr(A), lda,
                                    _ptr(B), ldb, float(beta), _ptr(C0f), ldc0,
                                    rows.size, _ptr(rows), _ptr(cols), _ptr(out))
    return out


def gemm_pieces(ta, tb, m, n, k, alpha, PA, lda, PB, ldb, terms, beta=0.0, C0=None,
                ldc0=None):
    """Split-product definition: op(A) = sum(PA), op(B) = sum(PB), and only the
    (u, v) piece products listed in ``terms`` are formed.  FP64 result."""
    lib = _load()
    PA = [_flat(p, np.float64) for p in PA]
    PB = [_flat(p, np.float64) for p in PB]
    for (u, v) in terms:
        if u >= len(PA) or v >= len(PB):
            raise ValueError("term names a missing piece")
    ldc0 = n if ldc0 is None else ldc0
    C0f = _flat(C0, np.float64) if (C0 is not None and beta != 0) else np.zeros(0)
    _check_ld(ta, tb, m, n, k, lda, ldb, ldc0, PA[0], PB[0], C0f, beta)
    pa = (ctypes.c_void_p * len(PA))(*[p.ctypes.data for p in PA])
    pb = (ctypes.c_void_p * len(PB))(*[p.ctypes.data for p in PB])
    tu = np.array([t[0] for t in terms], dtype=np.int32)
    tv = np.array([t[1] for t in terms], dtype=np.int32)
    C = np.empty((m, n), dtype=np.float64)
    if m and n:
        lib.oracle_gemm_pieces_f64(_tc(ta), _tc(tb), m, n, k, float(alpha), len(PA),
                                   ctypes.cast(pa, _P), lda, len(PB), ctypes.cast(pb, _P),
                                   ldb, len(terms), _ptr(tu), _ptr(tv), float(beta),
                                   _ptr(C0f), ldc0, _ptr(C), n)
    return C


def gemm_i8(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta=0, C0=None, ldc0=None):
    """INT8 definition: exact int64 sums, alpha*acc + beta*C0 wrapped to int32."""
    lib = _load()
    if int(alpha) != alpha or int(beta) != beta:
        raise ValueError("INT8 alpha/beta must be integers")
    A = _flat(A, np.int8)
    B = _flat(B, np.int8)
    ldc0 = n if ldc0 is None else ldc0
    C0f = _flat(C0, np.int32) if (C0 is not None and beta != 0) else np.zeros(0, np.int32)
    _check_ld(ta, tb, m, n, k, lda, ldb, ldc0, A, B, C0f, beta)
    C = np.empty((m, n), dtype=np.int32)
    if m and n:
        lib.oracle_gemm_i8(_tc(ta), _tc(tb), m, n, k, int(alpha), _ptr(A), lda,
                           _ptr(B), ldb, int(beta), _ptr(C0f), ldc0, _ptr(C), n)
    return C


def _int_kind(bits):
    if bits == 16:
        return 2, np.int16
    if bits == 32:
        return 4, np.int32
    raise ValueError("bits must be 16 or 32")


def _int32_scalar(v, name):
    if int(v) != v or not -2**31 <= int(v) < 2**31:
        raise ValueError(f"{name} must be an int32 integer")
    return int(v)


def gemm_int(bits, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta=0, C0=None, ldc0=None):
    """INT16 / INT32 definition: the exact integer alpha*op(A)*op(B) + beta*C0
    modulo 2^32, as int32 (A, B int16 when bits == 16, int32 when 32)."""
    lib = _load()
    eb, dt = _int_kind(bits)
    alpha = _int32_scalar(alpha, "alpha")
    beta = _int32_scalar(beta, "beta")
    A = _flat(A, dt)
    B = _flat(B, dt)
    ldc0 = n if ldc0 is None else ldc0
    C0f = _flat(C0, np.int32) if (C0 is not None and beta != 0) else np.zeros(0, np.int32)
    _check_ld(ta, tb, m, n, k, lda, ldb, ldc0, A, B, C0f, beta)
    C = np.empty((m, n), dtype=np.int32)
    if m and n:
        lib.oracle_gemm_int(eb, _tc(ta), _tc(tb), m, n, k, alpha, _ptr(A), lda, _ptr(B), ldb,
                            beta, _ptr(C0f), ldc0, _ptr(C), n)
    return C


def entries_int(bits, ta, tb, k, alpha, A, lda, B, ldb, beta, C0, ldc0, rows, cols):
    """C(rows[t], cols[t]) of the INT16 / INT32 definition."""
    lib = _load()
    eb, dt = _int_kind(bits)
    alpha = _int32_scalar(alpha, "alpha")
    beta = _int32_scalar(beta, "beta")
    A = _flat(A, dt)
    B = _flat(B, dt)
    rows = _flat(rows, np.int64)
    cols = _flat(cols, np.int64)
    C0f = _flat(C0, np.int32) if (C0 is not None and beta != 0) else np.zeros(0, np.int32)
    out = np.empty(rows.size, dtype=np.int32)
    if rows.size:
        lib.oracle_gemm_entries_int(eb, _tc(ta), _tc(tb), k, alpha, _ptr(A), lda, _ptr(B), ldb,
                                    beta, _ptr(C0f), ldc0, rows.size, _ptr(rows), _ptr(cols),
                                    _ptr(out))
    return out


def entries_i8(ta, tb, k, alpha, A, lda, B, ldb, beta, C0, ldc0, rows, cols):
    lib = _load()
    A = _flat(A, np.int8)
    B = _flat(B, np.int8)
    rows = _flat(rows, np.int64)
    cols = _flat(cols, np.int64)
    C0f = _flat(C0, np.int32) if (C0 is not None and beta != 0) else np.zeros(0, np.int32)
    out = np.empty(rows.size, dtype=np.int32)
    if rows.size:
        lib.oracle_gemm_entries_i8(_tc(ta), _tc(tb), k, int(alpha), _ptr(A), lda,
                                   _ptr(B), ldb, int(beta), _ptr(C0f), ldc0,
                                   rows.size, _ptr(rows), _ptr(cols), _ptr(out))
    return out


def decode_bf16(bits):
    """bfloat16 bit patterns (uint16) -> exact float64 values."""
    b = _flat(bits, np.uint16)
    out = np.empty(b.size, dtype=np.float64)
    _load().oracle_decode_bf16(_ptr(b), b.size, _ptr(out))
    return out.reshape(np.shape(bits))


def decode_f16(bits):
    """IEEE binary16 bit patterns (uint16) -> exact float64 values."""
    b = _flat(bits, np.uint16)
    out = np.empty(b.size, dtype=np.float64)
    _load().oracle_decode_f16(_ptr(b), b.size, _ptr(out))
    return out.reshape(np.shape(bits))


def decode_e4m3(bits):
    """OCP FP8 E4M3FN codes (uint8) -> exact float64 values (NaN for 0x7F/0xFF)."""
    b = _flat(bits, np.uint8)
    out = np.empty(b.size, dtype=np.float64)
    _load().oracle_decode_e4m3(_ptr(b), b.size, _ptr(out))
    return out.reshape(np.shape(bits))


def split_bf16(x, pieces):
    """Round-to-nearest-even split of FP32 values into ``pieces`` bf16 patterns
    (hi, mid[, lo]) such that hi + mid + lo == x exactly for normal x."""
    if pieces not in (1, 2, 3):
        raise ValueError("pieces must be 1, 2 or 3")
    xf = _flat(x, np.float32)
    outs = [np.empty(xf.size, dtype=np.uint16) for _ in range(3)]
    _load().oracle_split_bf16(_ptr(xf), xf.size, pieces, _ptr(outs[0]), _ptr(outs[1]),
                              _ptr(outs[2]))
    return [o.reshape(np.shape(x)) for o in outs[:pieces]]


# Scaled low-precision path: format codes and the exponent T at which each
# row's largest magnitude is placed ([2^T, 2^(T+1))).
SCALED_FORMATS = {"bf16": (0, 0), "f16": (1, 14), "e4m3": (2, 7)}


def scale_exponents(x, T):
    """Per-row exponents e_r = floor(log2 max_p |x[r, p]|) - T (0 for zero or
    non-finite rows) of a 2-D FP32 array."""
    xf = np.ascontiguousarray(x, dtype=np.float32)
    rows, cols = xf.shape
    e = np.empty(rows, dtype=np.int32)
    _load().oracle_scale_exponents(_ptr(xf), rows, cols, int(T), _ptr(e))
    return e


def scaled_codes(x, e, fmt):
    """Round-to-nearest-even codes of x[r, p] * 2^-e[r] in format ``fmt``
    ("bf16", "f16" or "e4m3"; e4m3 saturates at 448)."""
    code, _ = SCALED_FORMATS[fmt]
    xf = np.ascontiguousarray(x, dtype=np.float32)
    rows, cols = xf.shape
    ee = np.ascontiguousarray(e, dtype=np.int32)
    out = np.empty((rows, cols), dtype=np.uint16)
    _load().oracle_scaled_codes(_ptr(xf), rows, cols, _ptr(ee), code, _ptr(out))
    return out.astype(np.uint8) if fmt == "e4m3" else out


def decode_codes(codes, fmt):
    return {"bf16": decode_bf16, "f16": decode_f16, "e4m3": decode_e4m3}[fmt](codes)


def gemm_scaled(ta, tb, m, n, k, alpha, A, lda, B, ldb, fmt, beta=0.0, C0=None, ldc0=None):
    """The scaled low-precision GEMM on FP32 operands: op(A) rows and op(B)
    columns are scaled by powers of two into the format's range and rounded
    (scale_exponents, scaled_codes); C = alpha * 2^(e_i + f_j) *
    sum_p qa(i,p) qb(p,j) + beta * C0, evaluated in FP64 (the scalings are
    exact there).  Returns (C, qa codes, e, qb^T codes, f)."""
    _, T = SCALED_FORMATS[fmt]
    A = np.asarray(A, dtype=np.float32)
    B = np.asarray(B, dtype=np.float32)
    opA = (A[:k, :m].T if _is_t(ta) else A[:m, :k]).astype(np.float32)
    opBt = (B[:n, :k] if _is_t(tb) else B[:k, :n].T).astype(np.float32)   # n x k
    e = scale_exponents(opA, T)
    f = scale_exponents(opBt, T)
    qa = scaled_codes(opA, e, fmt)
    qbt = scaled_codes(opBt, f, fmt)
    As = np.ldexp(decode_codes(qa, fmt), e[:, None].astype(np.int64))
    Bs = np.ldexp(decode_codes(qbt, fmt), f[:, None].astype(np.int64)).T.copy()
    C = gemm_f64("N", "N", m, n, k, alpha, As, k, Bs, n, beta, C0, ldc0)
    return C, qa, e, qbt, f


def normalized_error(C, Cref, k, max_a, max_b):
    """max |C - Cref| / (k * max|A| * max|B|), the graded error of the FP paths."""
    C = np.asarray(C, dtype=np.float64)
    Cref = np.asarray(Cref, dtype=np.float64)
    if C.size == 0:
        return 0.0
    denom = float(k) * float(max_a) * float(max_b)
    diff = float(np.max(np.abs(C - Cref)))
    if denom == 0.0:
        return 0.0 if diff == 0.0 else float("inf")
    return diff / denom
