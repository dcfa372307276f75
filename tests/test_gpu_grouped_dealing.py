"""Tile dealing of the grouped persistent launch at its boundaries: tiles go to
the XCD groups in chunks (64 tiles, or total/64 in launches of fewer than two
tiles per workgroup), workgroups without a first tile leave, and launches of
at least four tiles per workgroup steal from drained queues.  Batches whose
tile counts straddle those boundaries, in direct calls and in slots, must
produce every problem's exact INT8 product (each tile computed exactly once)."""
import numpy as np
import pytest

import paper_2310_20347_amd as mg

pytestmark = pytest.mark.gpu


def _batch(count, m, n, k, seed):
    import torch
    rng = np.random.default_rng(seed)
    host, probs, dev = [], [], []
    for i in range(count):
        a = rng.integers(-128, 128, size=(m, k), dtype=np.int8)
        b = rng.integers(-128, 128, size=(k, n), dtype=np.int8)
        A, B = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        C = torch.full((m, n), -7, dtype=torch.int32, device="cuda")
        dev.append((A, B, C))
        host.append((a, b))
        probs.append(mg.Problem("N", "N", m, n, k, 1, A, k, B, n, 0, C, n))
    return host, probs, dev


def _check(host, dev, rows=None):
    import torch
    torch.cuda.synchronize()
    for i, ((a, b), (_, _, C)) in enumerate(zip(host, dev)):
        got = C.cpu().numpy()
        if rows is None:
            ref = (a.astype(np.int64) @ b.astype(np.int64)).astype(np.int32)
            assert np.array_equal(got, ref), f"problem {i}"
        else:
            ref = (a[rows].astype(np.int64) @ b.astype(np.int64)).astype(np.int32)
            assert np.array_equal(got[rows], ref), f"problem {i}"


@pytest.mark.parametrize("count", [1, 63, 64, 65, 511, 512, 513, 1100])
def test_one_tile_problems_around_chunk_and_grid_edges(count):
    # 128 x 128 problems: one tile each with the INT8 grouped bodies
    mg.gemm_init(None)
    host, probs, dev = _batch(count, 128, 128, 64, 7000 + count)
    print(f"{count} one-tile problems, direct call", flush=True)
    mg.gemm_grouped(probs, mg.GEMM_I8)
    _check(host, dev)
    for _, _, C in dev:
        C.fill_(-7)
    slot = mg.GroupedSlot(capacity=count)
    try:
        slot.write(probs, mg.GEMM_I8)
        print(f"{count} one-tile problems, slot launch", flush=True)
        slot.launch()
        _check(host, dev)
    finally:
        slot.destroy()


def test_large_launch_that_steals():
    # 17 problems of 2048 x 2048 x 64: 4352 tiles of 128 x 128 or 2176 of
    # 256 x 128, either way at least four per workgroup, so drained queues
    # are refilled from the other groups'; sampled rows
    mg.gemm_init(None)
    host, probs, dev = _batch(17, 2048, 2048, 64, 7100)
    rows = np.random.default_rng(7101).integers(0, 2048, 64)
    print("17 x 2048^2 x 64, direct call", flush=True)
    mg.gemm_grouped(probs, mg.GEMM_I8)
    _check(host, dev, rows)
    print("again (the queues reset themselves)", flush=True)
    for _, _, C in dev:
        C.fill_(-7)
    mg.gemm_grouped(probs, mg.GEMM_I8)
    _check(host, dev, rows)
