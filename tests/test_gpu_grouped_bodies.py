"""The grouped compact kernel's tile bodies: every body, forced on a batch of
ragged 'N','N' problems, gives each problem the bits of the standalone gemm()
and the oracle's result at the parity bar; the benchmark's mixed batch runs
more than one body; the grouped tuner's choices survive a round trip through
the tuning-table file."""
import os

import numpy as np
import pytest

import paper_2310_20347_amd as mg
from paper_2310_20347_amd import inputs

from grouped_cases import Batch
from test_gpu_grouped import oracle_check, standalone

pytestmark = pytest.mark.gpu

FAMILIES = [mg.GEMM_F32, mg.GEMM_F32_BF16X3, mg.GEMM_BF16, mg.GEMM_F16, mg.GEMM_F8E4M3,
            mg.GEMM_I8]


def _shapes(pieces):
    # several tiles of every body and ragged edges; k below 64 for the six-term bodies
    if pieces == 3:
        return [(130, 200, 40), (64, 64, 16), (257, 129, 63), (33, 300, 1)]
    return [(300, 260, 200), (64, 128, 64), (129, 257, 300), (17, 140, 96), (520, 130, 130)]


@pytest.mark.parametrize("dtype", FAMILIES, ids=lambda d: mg.DTYPE_NAMES[d])
def test_every_body_forced_equals_standalone_and_oracle(dtype):
    import torch
    mg.gemm_init(None)
    bodies = mg.grouped_bodies_info(dtype)
    assert len(bodies) >= 2
    for b, info in enumerate(bodies):
        shapes = _shapes(info["pieces"])
        is_int = dtype == mg.GEMM_I8
        batch = Batch(dtype, shapes, seed=70 + b, alpha=2 if is_int else 1.5,
                      beta=-1 if is_int else 0.5)
        print(f"{mg.DTYPE_NAMES[dtype]} body {b} {info}", flush=True)
        try:
            mg.grouped_force_body(b)
            assert set(mg.grouped_bodies(batch.problems, dtype)) == {b}
            mg.gemm_grouped(batch.problems, dtype)
        finally:
            mg.grouped_force_body(-1)
        torch.cuda.synchronize()
        got = batch.results()
        for p, h, C in zip(batch.problems, batch.host, got):
            oracle_check(dtype, p, h, C)
        batch.reset_c()
        alone = standalone(dtype, batch, lambda p: 0)
        for i, (C, A1) in enumerate(zip(got, alone)):
            assert np.array_equal(C, A1), f"body {b} problem {i} differs from gemm()"


@pytest.mark.parametrize("dtype", [mg.GEMM_F32_BF16X3, mg.GEMM_I8], ids=lambda d: mg.DTYPE_NAMES[d])
def test_mixed_batch_runs_several_bodies(dtype):
    """The batching workload's 512 problems (m, n, k log-uniform on [16, 4096])
    are spread over more than one body, and a sample of them equals gemm()."""
    import torch
    mg.gemm_init(None)
    shapes = inputs.log_uniform_shapes(512, 0)
    small = [s for s in shapes if s[0] * s[1] * s[2] <= 2 ** 24][:40]
    batch = Batch(dtype, small, seed=81)
    used = mg.grouped_bodies(batch.problems, dtype)
    assert min(used) >= 0 and len(set(used)) > 1, used
    mg.gemm_grouped(batch.problems, dtype)
    torch.cuda.synchronize()
    got = batch.results()
    batch.reset_c()
    alone = standalone(dtype, batch, lambda p: 0)
    for i, (C, A1) in enumerate(zip(got, alone)):
        assert np.array_equal(C, A1), f"problem {i} {small[i]} differs from gemm()"
    # all 512 problems: bodies chosen for every one of them
    import torch as _t  # noqa: F401
    full = Batch(dtype, shapes, seed=82, keep_host=False)
    used = mg.grouped_bodies(full.problems, dtype)
    assert min(used) >= 0 and len(set(used)) > 1


def test_grouped_tuner_round_trip(tmp_path):
    """gemm_tune_grouped stores one body per size bucket; gemm_init(path) of
    the written table makes the grouped launch use those bodies."""
    import json
    import torch
    dtype = mg.GEMM_I8
    shapes = [(48, 300, 200), (1500, 1400, 300)]
    path = str(tmp_path / "grouped_table.json")
    default = os.path.join(os.path.dirname(mg.lib_path()), "mgemm_tune.json")
    # start from an empty table, so the written file holds only what the tuner stored
    empty = str(tmp_path / "empty.json")
    with open(empty, "w") as f:
        json.dump({"version": 1, "arch": "gfx950", "entries": []}, f)
    try:
        mg.gemm_init(empty)
        mg.gemm_tune_grouped(dtype, shapes, reps=2, out_path=path)
        entries = [e for e in json.load(open(path))["entries"] if e["trans"] == 4]
        assert len(entries) == len(shapes)
        mg.gemm_init(path)
        batch = Batch(dtype, shapes, seed=91)
        used = mg.grouped_bodies(batch.problems, dtype)
        want = {(e["bm"], e["bn"], e["bk"]): e["cfg"] for e in entries}
        buckets = [tuple(min(12, max(4, int(np.floor(np.log2(x))))) for x in s) for s in shapes]
        assert used == [want[b] for b in buckets]
        mg.gemm_grouped(batch.problems, dtype)
        torch.cuda.synchronize()
        for p, h, C in zip(batch.problems, batch.host, batch.results()):
            oracle_check(dtype, p, h, C)
    finally:
        mg.gemm_init(default)
