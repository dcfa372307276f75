"""The autotuner on the GPU: gemm_tune times the configurations of each
shape in all four layouts, the table it writes reloads through
gemm_init(path), the dispatch then runs the stored configuration of each
(layout, size bucket), and the results match the oracle."""
import json
import os

import numpy as np
import pytest

import paper_2310_20347_amd as mg
from gemm_cases import Case, check, run_case

pytestmark = pytest.mark.gpu

LAYOUTS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]
# multiples of 16: every operand and leading dimension is 16-byte aligned,
# as the tuner's own operands are
SHAPES = [(96, 80, 208), (320, 256, 64), (1024, 512, 384)]


def _bucket(x):
    return min(12, max(4, int(np.floor(np.log2(x)))))


@pytest.mark.parametrize("dtype", [mg.GEMM_F32, mg.GEMM_I8], ids=lambda d: mg.DTYPE_NAMES[d])
def test_tune_reload_dispatch(dtype, tmp_path):
    mg.gemm_init(None)
    path = str(tmp_path / "table.json")
    default = os.path.join(os.path.dirname(mg.lib_path()), "mgemm_tune.json")
    try:
        print(f"tuning {mg.DTYPE_NAMES[dtype]} on {SHAPES}", flush=True)
        mg.gemm_tune(dtype, SHAPES, reps=3, out_path=path)
        table = json.load(open(path))["entries"]
        kclass = 0 if dtype == mg.GEMM_F32 else 6
        mine = {(e["trans"], e["bm"], e["bn"], e["bk"]): e for e in table if e["kclass"] == kclass}
        mg.gemm_init(path)
        for (m, n, k) in SHAPES:
            for t, (ta, tb) in enumerate(LAYOUTS):
                key = (t, _bucket(m), _bucket(n), _bucket(k))
                assert key in mine, f"no entry for layout {ta}{tb} bucket {key[1:]}"
                e = mine[key]
                # the stored configuration has a kernel for its layout
                assert mg.config_supports(dtype, e["cfg"], ta, tb)
                ab = (2, -1) if dtype == mg.GEMM_I8 else (1.0, 0.5)
                c = Case(dtype, ta, tb, m, n, k, ab[0], ab[1], seed=7)
                r = run_case(c)
                check(c, r)
                got = mg.last_config()
                assert (got["cfg"], got["order"]) == (e["cfg"], e["order"]), (key, got, e)
    finally:
        mg.gemm_init(default)
