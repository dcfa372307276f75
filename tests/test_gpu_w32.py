"""Tiles of 32x32 MFMA blocks (BF16, FP16, FP8, INT8 direct-staged, and the
packed split built on the BF16 ones) against the oracle: normal data in all
four layouts with m, n and k ragged against the tile, the stage and the
16-byte vector (INT8 bit-exact, floats to the parity bar); every result
equals the 16x16 tile of the same shape on small integers (exact sums); and
an 8192^3-class shape on sampled entries."""
import numpy as np
import pytest

import paper_2310_20347_amd as mg
from gemm_cases import Case, check, run_case

pytestmark = pytest.mark.gpu

TRANS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]

W32_DTYPES = [mg.GEMM_BF16, mg.GEMM_F16, mg.GEMM_F8E4M3, mg.GEMM_I8]


def w32_configs(dtype):
    return [i for i in range(mg.num_configs(dtype)) if mg.config_info(dtype, i)["mfma"] == 32]


def test_32x32_configurations_registered():
    for dt in W32_DTYPES:
        ids = w32_configs(dt)
        assert len(ids) >= 4, mg.DTYPE_NAMES[dt]
        for i in ids:
            info = mg.config_info(dt, i)
            assert info["staging"] == "direct" and info["layouts"] & 0xAA == 0xAA
            assert info["mr"] % 32 == 0 and info["nr"] % 32 == 0
    # the x3 split's packed configurations include ones on the 32x32 BF16 tiles
    packed = [i for i in w32_configs(mg.GEMM_F32_BF16X3_ONLY)
              if mg.config_info(mg.GEMM_F32_BF16X3_ONLY, i)["kind"] == 5]
    assert len(packed) == len(w32_configs(mg.GEMM_BF16))


@pytest.mark.parametrize("dtype", W32_DTYPES, ids=lambda d: mg.DTYPE_NAMES[d])
@pytest.mark.parametrize("ta,tb", TRANS)
def test_32x32_tiles_normal_data_ragged(dtype, ta, tb):
    # leading dimensions m+4, n+4, k+4 are multiples of 16 elements, so the
    # direct-staged kernels run; k = 1004 leaves a partial vector in the
    # last stage (k-contiguous panels zero its tail)
    dist = "uniform" if dtype == mg.GEMM_I8 else "normal"
    try:
        for cfg in w32_configs(dtype):
            ab = (2, -1) if dtype == mg.GEMM_I8 else (1.25, -0.75)
            c = Case(dtype, ta, tb, 300, 268, 1004, *ab, pad=4, dist=dist, seed=31)
            mg.force_config(dtype, cfg, cfg % 2)
            print(f"cfg {cfg} {ta}{tb} {c.m}x{c.n}x{c.k}", flush=True)
            r = run_case(c)
            assert r["cfg"]["cfg"] == cfg
            check(c, r)
    finally:
        mg.force_config(dtype, -1, 0)


@pytest.mark.parametrize("dtype", W32_DTYPES, ids=lambda d: mg.DTYPE_NAMES[d])
def test_32x32_equals_16x16_on_small_integers(dtype):
    """Same tile shape, 16x16 against 32x32 blocks: exact sums, equal bits."""
    ids16 = {}
    for i in range(mg.num_configs(dtype)):
        info = mg.config_info(dtype, i)
        if info["mfma"] == 16 and info["staging"] == "direct" and info["kind"] == 0:
            ids16.setdefault((info["mc"], info["nc"], info["mr"], info["nr"]), i)
    pairs = []
    for i in w32_configs(dtype):
        info = mg.config_info(dtype, i)
        key = (info["mc"], info["nc"], info["mr"], info["nr"])
        if key in ids16:
            pairs.append((ids16[key], i))
    assert pairs
    try:
        for a, b in pairs:
            outs = []
            for cfg in (a, b):
                mg.force_config(dtype, cfg, 0)
                c = Case(dtype, "N", "T", 520, 392, 784, 1.0, 1.0, dist="ints", seed=33)
                print(f"cfg {cfg} {c.m}x{c.n}x{c.k}", flush=True)
                r = run_case(c)
                assert r["cfg"]["cfg"] == cfg
                check(c, r)
                outs.append(r["C"])
            assert np.array_equal(outs[0], outs[1]), f"configurations {a} and {b} differ"
    finally:
        mg.force_config(dtype, -1, 0)


@pytest.mark.parametrize("dtype", W32_DTYPES, ids=lambda d: mg.DTYPE_NAMES[d])
def test_32x32_large_sampled(dtype):
    """The 256x256 8-wave 32x32 tile on a 4096 x 4096 x 8192 product,
    checked on sampled entries (the oracle computes each one alone)."""
    cfg = [i for i in w32_configs(dtype)
           if (mg.config_info(dtype, i)["mc"], mg.config_info(dtype, i)["threads"]) == (256, 512)][0]
    rng = np.random.default_rng(35)
    rows = rng.integers(0, 4096, 256)
    cols = rng.integers(0, 4096, 256)
    dist = "uniform" if dtype == mg.GEMM_I8 else "normal"
    try:
        mg.force_config(dtype, cfg, 1)
        ab = (1, 3) if dtype == mg.GEMM_I8 else (1.0, 0.5)
        c = Case(dtype, "N", "N", 4096, 4096, 8192, *ab, dist=dist, seed=36)
        print(f"cfg {cfg} {c.m}x{c.n}x{c.k} sampled", flush=True)
        r = run_case(c, sample=(rows, cols))
        assert r["cfg"]["cfg"] == cfg
        check(c, r)
    finally:
        mg.force_config(dtype, -1, 0)


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N")])
def test_32x32_packed_split_vs_oracle(ta, tb):
    """The x3 split product on the 32x32 BF16 tiles (packing pass, then the
    tile): the FP32 parity bar against the oracle."""
    dtype = mg.GEMM_F32_BF16X3
    ids = [i for i in w32_configs(dtype) if mg.config_info(dtype, i)["kind"] == 5]
    assert ids
    try:
        for cfg in ids:
            mg.force_config(dtype, cfg, 0)
            c = Case(dtype, ta, tb, 300, 268, 1004, 1.0, 0.5, pad=4, dist="normal", seed=37)
            print(f"cfg {cfg} {ta}{tb} {c.m}x{c.n}x{c.k}", flush=True)
            r = run_case(c)
            assert r["cfg"]["cfg"] == cfg
            check(c, r)
    finally:
        mg.force_config(dtype, -1, 0)
