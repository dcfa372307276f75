"""GPU parity of the single-GEMM path (through the C ABI) against the oracle.

Bars: INT8 bit-exact; every float path within 2e-6 (normalised) of the oracle
run on the inputs the kernel multiplies; FP32 and the split path within 2e-6
and BF16/FP16 within 8e-3 of the oracle on the FP32 source; small-integer
data bit-exact on every path.
"""
import numpy as np
import pytest

import oracle
import paper_2310_20347_amd as mg
from paper_2310_20347_amd import inputs

from gemm_cases import ALL_DTYPES, Case, check, run_case, to_device

pytestmark = pytest.mark.gpu

TRANS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]
SHAPES = [(257, 191, 203), (1, 1, 1), (17, 15, 255), (130, 300, 517), (64, 128, 16)]


def _ab(dtype):
    return (3.0, -2.0) if dtype == mg.GEMM_I8 else (1.5, -0.5)


@pytest.mark.parametrize("dtype", ALL_DTYPES, ids=lambda d: mg.DTYPE_NAMES[d])
@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_parity_ragged_shapes(dtype, ta, tb, shape):
    m, n, k = shape
    alpha, beta = _ab(dtype)
    c = Case(dtype, ta, tb, m, n, k, alpha, beta, pad=3, seed=7)
    print(f"case {c}", flush=True)
    check(c, run_case(c))


@pytest.mark.parametrize("dtype", ALL_DTYPES, ids=lambda d: mg.DTYPE_NAMES[d])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "T")])
def test_parity_unaligned_operands(dtype, ta, tb):
    # odd leading dimensions and a one-element offset: element-wise staging
    c = Case(dtype, ta, tb, 99, 77, 131, *_ab(dtype), pad=1, misalign=1, seed=8)
    print(f"case {c}", flush=True)
    check(c, run_case(c))


@pytest.mark.parametrize("dtype", ALL_DTYPES, ids=lambda d: mg.DTYPE_NAMES[d])
def test_every_configuration_and_raster_order(dtype):
    """The whole family computes the same C: exact on small integers."""
    results = []
    try:
        for cfg in range(mg.num_configs(dtype)):
            for order in (0, 1):
                mg.force_config(dtype, cfg, order)
                # leading dimensions are 16-byte multiples for every element size,
                # so each configuration runs its own (vectorised) staging
                c = Case(dtype, "N", "N", 300, 272, 288, 1.0, 1.0, dist="ints", seed=9)
                print(f"cfg {cfg} order {order} case {c}", flush=True)
                r = run_case(c)
                # a configuration without an 'N','N' kernel runs configuration 0
                expect = cfg if mg.config_supports(dtype, cfg, "N", "N") else 0
                assert r["cfg"]["cfg"] == expect and r["cfg"]["order"] == order
                check(c, r)
                ref = r["Cq"] if r.get("Cq") is not None else r["Cs"]
                assert np.array_equal(r["C"], np.asarray(ref).astype(r["C"].dtype)), \
                    f"not exact on integers: cfg {cfg} order {order}"
                results.append(r["C"])
    finally:
        mg.force_config(dtype, -1, 0)
    for r in results[1:]:
        assert np.array_equal(r, results[0])


@pytest.mark.parametrize("dtype", [mg.GEMM_F32, mg.GEMM_F32_BF16X3, mg.GEMM_F32_BF16X6,
                                   mg.GEMM_BF16, mg.GEMM_F16, mg.GEMM_F8E4M3, mg.GEMM_I8,
                                   mg.GEMM_F64],
                         ids=lambda d: mg.DTYPE_NAMES[d])
def test_every_configuration_every_layout_ragged(dtype):
    """Every configuration (register-staged, operand-resident and the LDS-ring
    ones fed by direct global->LDS loads) in all four layouts, with m, n and k
    ragged against the tile, the 16-byte vector and the k stage, and leading
    dimensions that are 16-byte multiples (so every configuration runs its
    own vectorised staging): exact on small integers."""
    import torch
    from gemm_cases import decode, encode, make_operands, stored
    pad = 7   # dimensions = 9 mod 16, leading dimensions = 0 mod 16
    for (m, n, k) in [(297, 265, 1001), (41, 57, 41)]:
        for ta, tb in TRANS:
            c = Case(dtype, ta, tb, m, n, k, 1.0, -1.0, pad=pad, dist="ints", seed=11)
            a32, b32, c0 = make_operands(c)
            lda = (m if ta == "T" else k) + pad
            ldb = (k if tb == "T" else n) + pad
            ldc = n + pad
            As, Bs = stored(encode(a32, dtype), ta, lda), stored(encode(b32, dtype), tb, ldb)
            # padding between rows holds NaN (int8: 127): a vector that runs
            # past m, n or k must not leak it into a valid output
            junk = {mg.GEMM_BF16: 0x7FC0, mg.GEMM_F16: 0x7E00, mg.GEMM_F8E4M3: 0x7F,
                    mg.GEMM_I8: 127}.get(dtype, np.nan)
            As[:, (m if ta == "T" else k):] = junk
            Bs[:, (k if tb == "T" else n):] = junk
            Cs0 = stored(c0, "N", ldc)
            if dtype == mg.GEMM_I8:
                ref = oracle.gemm_i8(ta, tb, m, n, k, 1, As, lda, Bs, ldb, -1, Cs0, ldc)
            else:
                ref = oracle.gemm_f64(ta, tb, m, n, k, 1.0, decode(As, dtype), lda,
                                      decode(Bs, dtype), ldb, -1.0, Cs0, ldc)
            dA, dB = to_device(As), to_device(Bs)
            # the split dtype takes the six-term family (and its configurations) when k < 64
            fam = mg.GEMM_F32_BF16X6 if (dtype == mg.GEMM_F32_BF16X3 and k < 64) else dtype
            try:
                for cfg in range(mg.num_configs(fam)):
                    mg.force_config(dtype, cfg, cfg % 2)
                    dC = to_device(Cs0.copy())
                    print(f"cfg {cfg} {ta}{tb} {m}x{n}x{k}", flush=True)
                    mg.gemm(ta, tb, m, n, k, 1.0, dA, lda, dB, ldb, -1.0, dC, ldc, dtype)
                    torch.cuda.synchronize()
                    expect = cfg if mg.config_supports(fam, cfg, ta, tb) else 0
                    assert mg.last_config()["cfg"] == expect
                    C = dC.cpu().numpy().reshape(m, ldc)[:, :n]
                    assert np.array_equal(C, np.asarray(ref).astype(C.dtype)), \
                        f"cfg {cfg} {ta}{tb} {m}x{n}x{k} not exact"
            finally:
                mg.force_config(dtype, -1, 0)


@pytest.mark.parametrize("dtype", [mg.GEMM_F32_BF16X3, mg.GEMM_F32_BF16X6],
                         ids=lambda d: mg.DTYPE_NAMES[d])
@pytest.mark.parametrize("ta,tb", TRANS)
def test_packed_split_equals_fused_split_bitwise(dtype, ta, tb):
    """The packed split (a packing pass writes the bf16 pieces, then a bf16
    tile multiplies them) issues the same MFMA sequence on every accumulator
    as the fused split tile: equal bits, on normal inputs with ragged k."""
    import torch
    from gemm_cases import encode, make_operands, stored
    m, n, k = 200, 304, 520   # 16-byte rows in every layout; k ragged against 32 and 64
    c = Case(dtype, ta, tb, m, n, k, 1.25, -0.5, dist="normal", seed=12)
    a32, b32, c0 = make_operands(c)
    lda, ldb, ldc = (m if ta == "T" else k), (k if tb == "T" else n), n
    dA = to_device(stored(encode(a32, dtype), ta, lda))
    dB = to_device(stored(encode(b32, dtype), tb, ldb))
    # (the packed split on 32x32 MFMA tiles sums in another order: it is
    # checked against the oracle in the 32x32 tests)
    packed = [i for i in range(mg.num_configs(dtype))
              if mg.config_info(dtype, i)["kind"] == 5 and mg.config_info(dtype, i)["mfma"] == 16]
    assert packed, "no packed split configuration registered"
    # the split on direct-staged FP32 panels forms the same pieces as it reads
    packed += [i for i in range(mg.num_configs(dtype))
               if mg.config_info(dtype, i)["staging"] == "direct"
               and mg.config_supports(dtype, i, ta, tb)]
    outs = {}
    try:
        for cfg in [0] + packed:   # configuration 0 also takes unaligned operands
            mg.force_config(dtype, cfg, 0)
            dC = to_device(stored(c0, "N", ldc))
            print(f"cfg {cfg} {ta}{tb} {m}x{n}x{k}", flush=True)
            mg.gemm(ta, tb, m, n, k, 1.25, dA, lda, dB, ldb, -0.5, dC, ldc, dtype)
            torch.cuda.synchronize()
            assert mg.last_config()["cfg"] == cfg
            outs[cfg] = dC.cpu().numpy()
    finally:
        mg.force_config(dtype, -1, 0)
    for cfg in packed:
        assert np.array_equal(outs[cfg], outs[0]), f"packed cfg {cfg} differs from fused"


@pytest.mark.parametrize("dtype", [mg.GEMM_F32, mg.GEMM_F32_BF16X3, mg.GEMM_BF16, mg.GEMM_F8E4M3,
                                   mg.GEMM_I8], ids=lambda d: mg.DTYPE_NAMES[d])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "T")])
def test_split_k_configurations_vs_oracle(dtype, ta, tb):
    """Split-K (k cut into slices of whole stages, partial tiles summed in
    order): the tall-k shape (196, 1024, 4608) of the sweep and a ragged one,
    to the parity bar (INT8 bit-exact)."""
    sk = [i for i in range(mg.num_configs(dtype)) if mg.config_info(dtype, i)["kind"] == 6]
    assert sk, "no split-K configuration registered"
    try:
        for shape in [(196, 1024, 4608), (144, 80, 1008)]:   # 16-byte leading dimensions
            m, n, k = shape
            es = {mg.GEMM_BF16: 2, mg.GEMM_F8E4M3: 1, mg.GEMM_I8: 1}.get(dtype, 4)
            lds = ((m if ta == "T" else k), (k if tb == "T" else n))
            aligned = all(ld * es % 16 == 0 for ld in lds)
            for cfg in sk:
                mg.force_config(dtype, cfg, 0)
                c = Case(dtype, ta, tb, *shape, *_ab(dtype), seed=13)
                print(f"cfg {cfg} case {c}", flush=True)
                r = run_case(c)
                # direct-staged tiles need 16-byte rows; otherwise configuration 0 runs
                direct = mg.config_info(dtype, cfg)["staging"] == "direct"
                assert r["cfg"]["cfg"] == (cfg if aligned or not direct else 0)
                check(c, r)
    finally:
        mg.force_config(dtype, -1, 0)


@pytest.mark.parametrize("dtype,kind", [(mg.GEMM_F32, 6), (mg.GEMM_F32_BF16X3, 5),
                                        (mg.GEMM_F32_BF16X3, 6)],
                         ids=["f32-splitk", "bf16x3-packed", "bf16x3-splitk"])
def test_workspace_configurations_under_graph_capture(dtype, kind):
    """Configurations that use the per-stream workspace (packed split, split-K)
    inside a captured HIP graph.  With the workspace reserved before capture
    the replays reproduce the eager result bit for bit (each replay checked,
    with eager work in between); on a stream that has none the capture takes
    a configuration that needs no workspace, allocating nothing, and the
    replay still matches the oracle."""
    import torch
    from gemm_cases import stored
    cfg = [i for i in range(mg.num_configs(dtype)) if mg.config_info(dtype, i)["kind"] == kind][0]
    m, n, k = 196, 1024, 2304
    c = Case(dtype, "N", "N", m, n, k, 1.0, 0.0, seed=14)
    from gemm_cases import make_operands
    a32, b32, _ = make_operands(c)
    dA, dB = to_device(a32), to_device(b32)
    dC = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    ref_q = oracle.gemm_f64("N", "N", m, n, k, 1.0, a32.astype(np.float64), k,
                            b32.astype(np.float64), n)
    try:
        mg.force_config(dtype, cfg, 0)
        s1 = torch.cuda.Stream()
        need = mg.workspace_bytes("N", "N", m, n, k, dtype)
        assert need > 0
        mg.reserve_workspace(need, 0, stream=s1)
        mg.gemm("N", "N", m, n, k, 1.0, dA, k, dB, n, 0.0, dC, n, dtype, stream=s1)
        torch.cuda.synchronize()
        assert mg.last_config()["cfg"] == cfg
        eager = dC.cpu().numpy().copy()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s1):
            with torch.cuda.graph(g, stream=s1):
                mg.gemm("N", "N", m, n, k, 1.0, dA, k, dB, n, 0.0, dC, n, dtype, stream=s1)
        for rep in range(3):
            dC.fill_(7.0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(dC.cpu().numpy(), eager), f"replay {rep} differs from eager"
        s2 = torch.cuda.Stream()   # no workspace on this stream yet
        g2 = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s2):
            with torch.cuda.graph(g2, stream=s2):
                mg.gemm("N", "N", m, n, k, 1.0, dA, k, dB, n, 0.0, dC, n, dtype, stream=s2)
        assert mg.last_config()["cfg"] != cfg   # the configuration without workspace
        dC.fill_(7.0)
        torch.cuda.synchronize()
        g2.replay()
        torch.cuda.synchronize()
        err = oracle.normalized_error(dC.cpu().numpy(), ref_q, k, float(np.abs(a32).max()),
                                      float(np.abs(b32).max()))
        assert err <= 2e-6, f"fallback capture error {err:.3g}"
        del g, g2
        mg.release_workspace(stream=s1)
    finally:
        mg.force_config(dtype, -1, 0)


@pytest.mark.parametrize("dtype", [mg.GEMM_F32, mg.GEMM_BF16], ids=lambda d: mg.DTYPE_NAMES[d])
def test_packing_configurations_vs_oracle(dtype):
    """Packing configurations (A, B or neither staged in LDS; the others'
    fragments loaded straight into registers) in every layout they support,
    on shapes ragged against the tile, the fragment vector and the stage."""
    cfgs = [i for i in range(mg.num_configs(dtype))
            if mg.config_info(dtype, i)["staging"] in ("a_unpacked", "b_unpacked", "unpacked")]
    assert len(cfgs) >= 3, "packing configurations missing"
    try:
        for cfg in cfgs:
            for ta, tb in TRANS:
                if not mg.config_supports(dtype, cfg, ta, tb):
                    continue
                for shape in [(64, 64, 64), (100, 200, 296), (257, 136, 1000)]:
                    mg.force_config(dtype, cfg, 0)
                    c = Case(dtype, ta, tb, *shape, *_ab(dtype), dist="normal", seed=15)
                    print(f"cfg {cfg} case {c}", flush=True)
                    r = run_case(c)
                    m, n, k = shape
                    es = 4 if dtype == mg.GEMM_F32 else 2
                    lds = ((m if ta == "T" else k), (k if tb == "T" else n))
                    aligned = all(ld * es % 16 == 0 for ld in lds)
                    assert r["cfg"]["cfg"] == (cfg if aligned else 0)
                    check(c, r)
    finally:
        mg.force_config(dtype, -1, 0)


@pytest.mark.parametrize("dtype", ALL_DTYPES, ids=lambda d: mg.DTYPE_NAMES[d])
@pytest.mark.parametrize("ta,tb", TRANS)
def test_identity_and_permutation_pins(dtype, ta, tb):
    import torch
    from gemm_cases import encode, stored
    n = 96
    rng = np.random.default_rng(5)
    B = rng.integers(-8, 9, size=(n, 70)).astype(np.float32)
    P = np.eye(n, dtype=np.float32)[rng.permutation(n)]
    for A in (np.eye(n, dtype=np.float32), P):
        As = stored(encode(A, dtype), ta, n)
        Bs = stored(encode(B, dtype), tb, n if tb in "Tt" else 70)
        out_t = {mg.GEMM_I8: torch.int32, mg.GEMM_F64: torch.float64}.get(dtype, torch.float32)
        dC = torch.full((n, 70), 7, dtype=out_t, device="cuda")
        mg.gemm(ta, tb, n, 70, n, 1, to_device(As), As.shape[1], to_device(Bs), Bs.shape[1], 0,
                dC, 70, dtype)
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy(), (A @ B).astype(dC.cpu().numpy().dtype))


@pytest.mark.parametrize("dtype", [mg.GEMM_F32, mg.GEMM_F32_BF16X3, mg.GEMM_BF16, mg.GEMM_I8,
                                   mg.GEMM_F64])
def test_blas_special_cases(dtype):
    import torch
    is_int = dtype == mg.GEMM_I8
    ct = torch.int32 if is_int else (torch.float64 if dtype == mg.GEMM_F64 else torch.float32)
    m, n, k = 37, 29, 41
    C0 = torch.arange(m * n, dtype=ct, device="cuda").reshape(m, n)
    esz = {mg.GEMM_F32: 4, mg.GEMM_F32_BF16X3: 4, mg.GEMM_BF16: 2, mg.GEMM_I8: 1,
           mg.GEMM_F64: 8}[dtype]
    nanbuf = torch.full((m * k * 4,), -1, dtype=torch.uint8, device="cuda")  # NaN patterns
    # k == 0: C = beta * C (A, B not read)
    C = C0.clone()
    mg.gemm("N", "N", m, n, 0, 1, None, 1, None, n, 2, C, n, dtype)
    torch.cuda.synchronize()
    assert torch.equal(C, 2 * C0)
    # alpha == 0: C = beta * C, A and B (NaN) not read
    C = C0.clone()
    mg.gemm("N", "N", m, n, k, 0, nanbuf, k, nanbuf, n, 3, C, n, dtype)
    torch.cuda.synchronize()
    assert torch.equal(C, 3 * C0)
    # beta == 0: NaN in C is overwritten, not propagated
    if not is_int:
        C = torch.full((m, n), float("nan"), dtype=ct, device="cuda")
        A = torch.ones(m * k * 4 // esz, dtype=torch.float32, device="cuda")
        if dtype == mg.GEMM_BF16:
            A = torch.ones(m * k, dtype=torch.bfloat16, device="cuda")
        if dtype == mg.GEMM_F64:
            A = torch.ones(m * k, dtype=torch.float64, device="cuda")
        B = torch.ones_like(A)
        mg.gemm("N", "N", m, n, k, 1, A, k, B, n, 0, C, n, dtype)
        torch.cuda.synchronize()
        assert torch.equal(C, torch.full_like(C, float(k)))
    # m == 0: nothing happens
    mg.gemm("N", "N", 0, n, k, 1, None, k, None, n, 0, None, n, dtype)


@pytest.mark.parametrize("dtype", [d for d in ALL_DTYPES if d != mg.GEMM_I8],
                         ids=lambda d: mg.DTYPE_NAMES[d])
def test_small_integers_exact_every_float_path(dtype):
    c = Case(dtype, "N", "N", 200, 180, 1000, 1.0, 0.0, dist="ints", seed=10)
    r = run_case(c)
    ref = r["Cq"] if r.get("Cq") is not None else r["Cs"]
    assert np.array_equal(r["C"].astype(np.float64), ref)


def test_config1_full_fp32_256():
    """C = A*B + C, m = n = k = 256, U[-1,1], plain FP32, compared in full."""
    c = Case(mg.GEMM_F32, "N", "N", 256, 256, 256, 1.0, 1.0, seed=1)
    r = run_case(c)
    check(c, r)
    assert r["err_source"] <= 2e-6


SWEEP = [(1024, 1024, 1024), (2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192),
         (50176, 64, 576), (3136, 256, 2304), (196, 1024, 4608), (12544, 128, 1152)]


def _sample(m, n, count=192, seed=3):
    rng = np.random.default_rng(seed)
    r = np.concatenate([rng.integers(0, m, count), [0, m - 1, m - 1, 0]])
    q = np.concatenate([rng.integers(0, n, count), [0, n - 1, 0, n - 1]])
    return r, q


@pytest.mark.parametrize("shape", SWEEP, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_fp32_sweep_sampled(shape, beta):
    m, n, k = shape
    c = Case(mg.GEMM_F32, "N", "N", m, n, k, 1.0, beta, seed=2)
    r = run_case(c, sample=_sample(m, n))
    print(f"{shape} beta={beta} err={r['err_source']:.3g}", flush=True)
    check(c, r)


@pytest.mark.parametrize("dtype", [mg.GEMM_F32_BF16X3, mg.GEMM_F32_BF16X6, mg.GEMM_BF16,
                                   mg.GEMM_F16, mg.GEMM_F8E4M3],
                         ids=lambda d: mg.DTYPE_NAMES[d])
@pytest.mark.parametrize("dist", ["normal", "badly_scaled"])
# badly scaled FP16 inputs overflow on conversion (the case this test records)
@pytest.mark.filterwarnings("ignore:overflow encountered in cast:RuntimeWarning")
@pytest.mark.filterwarnings("ignore:invalid value encountered in subtract:RuntimeWarning")
def test_precision_8192_sampled(dtype, dist):
    c = Case(dtype, "N", "N", 8192, 8192, 8192, 1.0, 0.0, dist=dist, seed=3)
    r = run_case(c, sample=_sample(8192, 8192, 128))
    print(f"{mg.DTYPE_NAMES[dtype]} {dist} err={r['err_source']:.3g}", flush=True)
    if dist == "normal":
        check(c, r)
    elif dtype in (mg.GEMM_F32_BF16X3, mg.GEMM_F32_BF16X6):
        # the split path keeps FP32 accuracy on badly scaled inputs as well
        assert r["err_source"] <= 2e-6


def test_int8_4096_sampled_exact():
    c = Case(mg.GEMM_I8, "N", "N", 4096, 4096, 4096, 1.0, 1.0, seed=4)
    r = run_case(c, sample=_sample(4096, 4096, 256))
    check(c, r)
