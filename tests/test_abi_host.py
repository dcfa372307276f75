"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the public headers declare, validates arguments with the BLAS
-i convention before touching a device, and quick-returns where BLAS does."""
import ctypes
import glob
import os
import re

import pytest

import paper_2310_20347_amd as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, re.M):
            if m.group(1) not in ("if", "while", "for", "return", "sizeof"):
                names.add(m.group(1))
    return names


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert {"gemm", "gemm_grouped", "gemm_init", "gemm_tune"} <= names
    lib = ctypes.CDLL(mg.lib_path())
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def call(ta="N", tb="N", m=4, n=5, k=3, alpha=1.0, A=0x1000, lda=3, B=0x2000, ldb=5, beta=0.0,
         C=0x3000, ldc=5, dtype=mg.GEMM_F32):
    return mg.lib().gemm(ta.encode(), tb.encode(), m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                         dtype)


@pytest.mark.parametrize("kw,code", [
    (dict(ta="X"), -1), (dict(tb="q"), -2), (dict(m=-1), -3), (dict(n=-1), -4), (dict(k=-1), -5),
    (dict(A=None), -7), (dict(A=0x1001), -7), (dict(lda=2), -8), (dict(ta="T", lda=3), -8),
    (dict(B=None), -9), (dict(ldb=4), -10), (dict(tb="T", ldb=2), -10), (dict(C=None), -12),
    (dict(ldc=4), -13), (dict(dtype=99), -14), (dict(dtype=-1), -14),
    (dict(dtype=mg.GEMM_I8, alpha=0.5), -6), (dict(dtype=mg.GEMM_I8, beta=2.5), -11),
    (dict(dtype=mg.GEMM_I8, alpha=2.0 ** 31), -6),
])
def test_invalid_arguments_report_their_position(kw, code):
    assert call(**kw) == code


def test_first_invalid_argument_wins():
    assert call(ta="X", m=-1, ldc=0) == -1
    assert call(m=-1, ldc=0) == -3
    # the dtype is argument 14: a bad lda (8) or C (12) together with a bad dtype reports 8 / 12
    assert call(lda=2, dtype=99) == -8
    assert call(C=None, dtype=-1) == -12
    assert call(ldc=4, dtype=99) == -13
    # an operand misaligned for some element size is not judged while the dtype is unknown
    assert call(A=0x1001, dtype=99) == -14


def test_workspace_entry_points_validate_on_the_host():
    L = mg.lib()
    assert L.gemm_reserve_workspace(-1, 0) == -1
    assert L.gemm_reserve_workspace(0, -5) == -2
    assert L.gemm_workspace_bytes(b"X", b"N", 4, 4, 4, mg.GEMM_F32) == -1
    assert L.gemm_workspace_bytes(b"N", b"N", 4, 4, 4, 99) == -1
    assert L.gemm_workspace_bytes(b"N", b"N", -1, 4, 4, mg.GEMM_F32) == -1
    assert L.gemm_workspace_bytes(b"N", b"N", 0, 4, 4, mg.GEMM_F32) == 0
    assert mg.scaled_workspace_bytes("N", "N", 4, 4, 4, 0.0, mg.GEMM_F32) == -1
    # exponents (256-byte rounded) x 2, partial maxima x 2, quantised A and B, no P at beta 0
    m, n, k = 100, 60, 36
    qa = -(-(m * 40 * 2) // 256) * 256   # rows of k rounded up to 8 binary16 values
    qb = -(-(k * 64 * 2) // 256) * 256   # rows of n rounded up to 8 values
    e, f = 512, 256
    assert mg.scaled_workspace_bytes("N", "N", m, n, k, 0.0, mg.GEMM_F16) == 2 * (e + f) + qa + qb
    assert (mg.scaled_workspace_bytes("N", "N", m, n, k, 1.0, mg.GEMM_F16)
            == 2 * (e + f) + qa + qb + 4 * m * n)


def test_transposed_leading_dimensions():
    # 'T' A is stored k x m: lda >= m; 'T' B stored n x k: ldb >= k
    assert call(ta="T", lda=4, ldc=0) == -13       # lda ok, fails later at ldc
    assert call(tb="T", ldb=3, ldc=0) == -13
    assert call(ta="t", tb="c", lda=4, ldb=3, ldc=0) == -13   # lower case and 'C' accepted


def test_quick_returns_touch_nothing():
    # no device is needed: nothing is launched
    assert call(m=0, A=None, B=None, C=None) == 0
    assert call(n=0, A=None, B=None, C=None) == 0
    assert call(k=0, beta=1.0, A=None, B=None, C=None, lda=1) == 0
    assert call(alpha=0.0, beta=1.0, A=None, B=None, C=None) == 0


def test_null_operands_allowed_when_not_read():
    # alpha == 0: A, B not read; the call proceeds to the device (which may be absent)
    rc = call(alpha=0.0, beta=2.0, A=None, B=None)
    assert rc in (0, 3)


def test_strerror_and_config_introspection():
    assert "invalid" in mg.strerror(-3)
    assert mg.strerror(0) == "success"
    for dt in range(mg.GEMM_NUM_DTYPES):
        n = mg.num_configs(dt)
        assert n >= 2
        for c in range(n):
            info = mg.config_info(dt, c)
            assert info["mc"] % info["mr"] == 0 and info["nc"] % info["nr"] == 0
            assert info["lds_bytes"] <= 160 * 1024
            if dt in (mg.GEMM_I16, mg.GEMM_I32):
                continue   # vector-ALU tile (16 values of k per stage) and digit products
            # a stage holds 128 bytes of k per panel row (64 for the deep-ring
            # direct configurations)
            kb = info["kc"] * {0: 4, 1: 2, 2: 2, 3: 2, 4: 1, 5: 1, 6: 2, 7: 2, 8: 8}[dt]
            assert kb == 128 or (kb == 64 and info["staging"] in ("direct", "packed"))


def test_panel_occupancy_reproduces_paper_table2():
    rows = [list(map(float, ln.split())) for ln in open(os.path.join(GOLDEN, "table2_l1_occupancy.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 14
    for layer, kc, nr, pct in rows:
        got = 100.0 * mg.panel_occupancy(int(kc), int(nr), 4, 64 * 1024)
        # the table prints 3 significant figures (e.g. 18.75 -> 18.80)
        assert float(f"{got:.3g}") == pct, (layer, kc, nr, got, pct)
    assert mg.panel_occupancy(-1, 1, 4, 10) == -1.0


def test_integer_dtypes_validate_on_the_host():
    # INT16 / INT32: integer alpha and beta (-6, -11), element alignment of A (-7)
    assert call(dtype=mg.GEMM_I16, alpha=0.5) == -6
    assert call(dtype=mg.GEMM_I32, beta=1.5) == -11
    assert call(dtype=mg.GEMM_I32, alpha=2.0 ** 31) == -6
    assert call(dtype=mg.GEMM_I16, A=0x1001) == -7
    assert call(dtype=mg.GEMM_I32, A=0x1002) == -7
    assert call(dtype=mg.GEMM_I16, m=0) == 0
    # two configurations each: the vector-ALU tile (every layout, any
    # alignment) and the digit products (kind 7)
    for dt in (mg.GEMM_I16, mg.GEMM_I32):
        assert mg.num_configs(dt) == 2
        assert mg.config_info(dt, 0)["kind"] == 0
        assert mg.config_info(dt, 1)["kind"] == 7
        assert mg.lib().gemm_config_layouts(dt, 0) == 255
        assert mg.lib().gemm_config_layouts(dt, 1) == 255
    # the grouped launch does not take them
    P = mg._binding._Problem
    arr = (P * 1)()
    arr[0] = P(b"N", b"N", 4, 5, 3, 1.0, 0x1000, 3, 0x2000, 5, 0.0, 0x3000, 5)
    assert mg.lib().gemm_grouped(1, arr, mg.GEMM_I16) == 2   # GEMM_E_UNSUPPORTED


def test_noalloc_validates_like_gemm():
    L = mg.lib()

    def na(ta=b"N", m=4, lda=3, dtype=mg.GEMM_F32, beta=0.0, C=0x3000):
        return L.gemm_noalloc(ta, b"N", m, 5, 3, 1.0, 0x1000, lda, 0x2000, 5, beta, C, 5, dtype)

    assert na(ta=b"X") == -1
    assert na(lda=2) == -8
    assert na(lda=2, dtype=99) == -8
    assert na(dtype=99) == -14
    assert na(C=None) == -12
    assert na(m=0) == 0                              # quick return before any device call
    assert L.gemm_noalloc_scratch_bytes() == 64 << 20


def test_no_device_reports_noinit():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert call() == 3


def test_grouped_validation_before_device():
    P = mg._binding._Problem
    arr = (P * 3)()
    for i in range(3):
        arr[i] = P(b"N", b"N", 4, 5, 3, 1.0, 0x1000, 3, 0x2000, 5, 0.0, 0x3000, 5)
    arr[2].ldb = 4                                   # problem 2, argument 10
    assert mg.lib().gemm_grouped(3, arr, mg.GEMM_F32) == -(1000 * 2 + 10)
    arr[2].ldb = 5
    arr[0].transA = b"x"                             # problem 0, argument 1
    assert mg.lib().gemm_grouped(3, arr, mg.GEMM_F32) == -1
    assert mg.lib().gemm_grouped(-1, arr, mg.GEMM_F32) == -1
    assert mg.lib().gemm_grouped(3, None, mg.GEMM_F32) == -2
    assert mg.lib().gemm_grouped(3, arr, 42) == -3
    assert mg.lib().gemm_grouped(0, None, mg.GEMM_F32) == 0
    assert mg.gemm_grouped_capacity() >= 512


def test_gemm_scaled_validates_before_touching_the_device():
    # only the narrow formats; FP32 argument rules; quick return for m == 0
    L = mg.lib()
    n_, p_ = b"N", 0x1000
    assert L.gemm_scaled(n_, n_, 4, 4, 4, 1.0, p_, 4, p_, 4, 0.0, p_, 4, mg.GEMM_F32) == -14
    # arguments are checked in order: a missing A (7) is reported before the format (14)
    assert L.gemm_scaled(n_, n_, 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, mg.GEMM_F32) == -7
    assert L.gemm_scaled(n_, n_, 4, 4, 4, 1.0, p_, 2, p_, 4, 0.0, p_, 4, 99) == -8
    assert L.gemm_scaled(n_, n_, 4, 4, 4, 1.0, p_, 2, p_, 4, 0.0, p_, 4, mg.GEMM_F16) == -8
    assert L.gemm_scaled(b"X", n_, 4, 4, 4, 1.0, p_, 4, p_, 4, 0.0, p_, 4, mg.GEMM_F8E4M3) == -1
    assert L.gemm_scaled(n_, n_, 0, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, mg.GEMM_BF16) == 0


def test_analytical_model_structure():
    """The analytical model's rules, on the CPU (no device: register counts
    estimated): invalid arguments; time grows with k; one round of tiles
    costs the same whatever the tile count; split-K first for a tall-k
    problem whose output fills a quarter of the compute units."""
    assert mg.model_us(mg.GEMM_F32, 0, 0, 64, 64) == -1.0
    assert mg.model_us(mg.GEMM_F32, 999, 64, 64, 64) == -1.0
    t = [mg.model_us(mg.GEMM_F32, 0, 512, 512, k) for k in (256, 1024, 4096)]
    assert 0 < t[0] < t[1] < t[2]
    one = mg.model_us(mg.GEMM_BF16, 0, 64, 64, 1024)
    assert mg.model_us(mg.GEMM_BF16, 0, 640, 640, 1024) == pytest.approx(one, rel=1e-9)
    assert mg.model_us(mg.GEMM_BF16, 0, 64 * 64, 64 * 64, 1024) > 1.5 * one
    ranked = sorted(range(mg.num_configs(mg.GEMM_F32)),
                    key=lambda c: mg.model_us(mg.GEMM_F32, c, 196, 1024, 4608))
    assert mg.config_info(mg.GEMM_F32, ranked[0])["kind"] == 6


def test_shipped_tuning_table_names_existing_configurations():
    """Configurations are only ever appended to a class, so the shipped table
    keeps naming the tiles it was tuned on: every entry's configuration exists
    in its class and has a kernel for the entry's layout (trans = 2 tA + tB);
    grouped entries (trans 4) name one of the family's grouped bodies."""
    import json
    path = os.path.join(os.path.dirname(os.path.abspath(mg.__file__)), "mgemm_tune.json")
    table = json.load(open(path))
    assert table["arch"].startswith("gfx950")
    family = {0: mg.GEMM_F32, 1: mg.GEMM_F32_BF16X3_ONLY, 2: mg.GEMM_F32_BF16X6, 3: mg.GEMM_BF16,
              4: mg.GEMM_F16, 5: mg.GEMM_F8E4M3, 6: mg.GEMM_I8, 7: mg.GEMM_F64,
              8: mg.GEMM_I16, 9: mg.GEMM_I32}
    layouts = {0: ("N", "N"), 1: ("N", "T"), 2: ("T", "N"), 3: ("T", "T")}
    seen, grouped = set(), set()
    for e in table["entries"]:
        dt = family[e["kclass"]]
        if e["trans"] == 4:
            assert 0 <= e["cfg"] < len(mg.grouped_bodies_info(dt)), e
            grouped.add(e["kclass"])
        else:
            assert 0 <= e["cfg"] < mg.num_configs(dt), e
            assert mg.config_supports(dt, e["cfg"], *layouts[e["trans"]]), e
            seen.add((e["kclass"], e["trans"]))
        assert e["order"] in (0, 1) and e["group"] > 0 and e["us"] > 0, e
        assert all(4 <= e[b] <= 12 for b in ("bm", "bn", "bk")), e
    assert seen == {(kc, tr) for kc in family for tr in range(4)}
    assert grouped >= {6}


def test_config_mfma_form():
    """gemm_config_mfma: 32 for the 32x32-block tiles (BF16, FP16, FP8, INT8
    direct tiles and the x3/x6 packed split built on the BF16 ones), 16 for
    every other configuration; negative for a bad dtype or id."""
    L = mg.lib()
    w32 = {}
    for dt in range(mg.GEMM_NUM_DTYPES):
        n = mg.num_configs(dt)
        forms = [L.gemm_config_mfma(dt, i) for i in range(n)]
        assert set(forms) <= {16, 32}, (dt, forms)
        w32[dt] = [i for i, f in enumerate(forms) if f == 32]
        for i in w32[dt]:
            info = mg.config_info(dt, i)
            assert info["mr"] % 32 == 0 and info["nr"] % 32 == 0, (dt, i, info)
            assert info["staging"] in ("direct", "packed"), (dt, i, info)
    for dt in (mg.GEMM_BF16, mg.GEMM_F16, mg.GEMM_F8E4M3, mg.GEMM_I8):
        assert len(w32[dt]) >= 4, mg.DTYPE_NAMES[dt]
    for dt in (mg.GEMM_F32, mg.GEMM_F64, mg.GEMM_I16, mg.GEMM_I32):
        assert not w32[dt], mg.DTYPE_NAMES[dt]
    assert L.gemm_config_mfma(99, 0) == -1
    assert L.gemm_config_mfma(mg.GEMM_BF16, -1) == -2
    assert L.gemm_config_mfma(mg.GEMM_BF16, mg.num_configs(mg.GEMM_BF16)) == -2


def test_debug_count_validates_before_the_device():
    L = mg.lib()
    L.gemm_debug_count.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_int]
    L.gemm_debug_count.restype = ctypes.c_int
    assert L.gemm_debug_count(None, 4, 5, 5, mg.GEMM_F32) == -1
    assert L.gemm_debug_count(0x1000, -1, 5, 5, mg.GEMM_F32) == -2
    assert L.gemm_debug_count(0x1000, 4, -1, 5, mg.GEMM_F32) == -3
    assert L.gemm_debug_count(0x1000, 4, 5, 4, mg.GEMM_F32) == -4
    assert L.gemm_debug_count(0x1000, 4, 5, 5, 99) == -5
    assert L.gemm_debug_count(None, 0, 5, 5, 99) == -5   # C unused when the block is empty
    import torch
    if not torch.cuda.is_available():
        assert L.gemm_debug_count(0x1000, 4, 5, 5, mg.GEMM_F32) == 3   # no device
        L.gemm_debug_unwritten.restype = ctypes.c_int64
        assert L.gemm_debug_unwritten() == -3
