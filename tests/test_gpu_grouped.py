"""GPU parity of the grouped persistent launch and of its graph-captured slot.

Each problem of a grouped launch must equal (bitwise) the same problem run
alone through gemm() with the same tile shape, and match the oracle to the
same bar as single GEMMs (INT8 bit-exact).
"""
import numpy as np
import pytest

import oracle
import paper_2310_20347_amd as mg
from paper_2310_20347_amd import inputs

from gemm_cases import QUANT_TOL, SOURCE_TOL, decode, terms_for
from grouped_cases import Batch

pytestmark = pytest.mark.gpu


def oracle_check(dtype, p, h, C, rows=None, cols=None):
    """Asserts problem p's result C against the oracle (full or sampled)."""
    ta, tb, m, n, k = p.transA, p.transB, p.m, p.n, p.k
    if dtype == mg.GEMM_I8:
        if rows is None:
            ref = oracle.gemm_i8(ta, tb, m, n, k, int(p.alpha), h["As"], h["lda"], h["Bs"],
                                 h["ldb"], int(p.beta), h["C0"], h["ldc"])
            assert np.array_equal(C, ref), f"INT8 mismatch {m}x{n}x{k}"
        else:
            ref = oracle.entries_i8(ta, tb, k, int(p.alpha), h["As"], h["lda"], h["Bs"],
                                    h["ldb"], int(p.beta), h["C0"], h["ldc"], rows, cols)
            assert np.array_equal(C[rows, cols], ref), f"INT8 mismatch {m}x{n}x{k}"
        return 0.0
    terms = terms_for(dtype, k)
    ma = float(np.abs(h["a32"]).max()) if h["a32"].size else 0.0
    mb = float(np.abs(h["b32"]).max()) if h["b32"].size else 0.0
    kk = max(k, 1) * max(abs(p.alpha), 1e-300)
    if rows is None:
        if terms is not None:
            npieces = 3 if len(terms) > 3 else 2
            PA = [oracle.decode_bf16(x) for x in oracle.split_bf16(h["As"], npieces)]
            PB = [oracle.decode_bf16(x) for x in oracle.split_bf16(h["Bs"], npieces)]
            q = oracle.gemm_pieces(ta, tb, m, n, k, p.alpha, PA, h["lda"], PB, h["ldb"], terms,
                                   p.beta, h["C0"], h["ldc"])
        else:
            q = oracle.gemm_f64(ta, tb, m, n, k, p.alpha, decode(h["As"], dtype), h["lda"],
                                decode(h["Bs"], dtype), h["ldb"], p.beta, h["C0"], h["ldc"])
        eq = oracle.normalized_error(C, q, kk, ma, mb)
        qt = QUANT_TOL
        if dtype == mg.GEMM_F8E4M3 and k > 0:   # FP8 MFMA accumulation (see gemm_cases)
            qt += 1.07 * 2.0 ** -11 * ((k + 127) // 128) / k
        assert eq <= qt, f"quantised error {eq:.3g} for {m}x{n}x{k}"
        As32 = h["a32"].T if ta == "T" else h["a32"]
        Bs32 = h["b32"].T if tb == "T" else h["b32"]
        s = oracle.gemm_f64(ta, tb, m, n, k, p.alpha, np.ascontiguousarray(As32),
                            As32.shape[1], np.ascontiguousarray(Bs32), Bs32.shape[1], p.beta,
                            h["C0"], h["ldc"])
    else:
        As32 = h["a32"].T if ta == "T" else h["a32"]
        Bs32 = h["b32"].T if tb == "T" else h["b32"]
        s = oracle.entries_f64(ta, tb, k, p.alpha, np.ascontiguousarray(As32), As32.shape[1],
                               np.ascontiguousarray(Bs32), Bs32.shape[1], p.beta, h["C0"],
                               h["ldc"], rows, cols)
        C = C[rows, cols]
    es = oracle.normalized_error(C, s, kk, ma, mb)
    tol = SOURCE_TOL.get(dtype)
    if tol is not None and dtype != mg.GEMM_F8E4M3:
        assert es <= tol, f"source error {es:.3g} for {m}x{n}x{k}"
    return es


def standalone(dtype, batch, shape_of):
    """Runs every problem alone through gemm() with the grouped tile shape."""
    import torch
    outs = []
    for p in batch.problems:
        dC = p._keep[2]
        saved = dC.clone()
        mg.force_config(dtype, shape_of(p), 0)
        try:
            mg.gemm(p.transA, p.transB, p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B, p.ldb, p.beta,
                    dC, p.ldc, dtype)
        finally:
            mg.force_config(dtype, -1, 0)
        torch.cuda.synchronize()
        outs.append(dC.cpu().numpy().reshape(p.m, p.ldc)[:, :p.n].copy())
        dC.copy_(saved)
    return outs


def grouped_shape(dtype, p):
    """Tile shape the grouped launch uses without a tuning table: 64x64 (config
    0) for small or unaligned problems, 128x128 (config 1) otherwise."""
    return 1 if (p.m >= 128 and p.n >= 128) else 0


GROUPED_DTYPES = [mg.GEMM_F32, mg.GEMM_F32_BF16X3, mg.GEMM_BF16, mg.GEMM_F16, mg.GEMM_F8E4M3,
                  mg.GEMM_I8]


@pytest.mark.parametrize("dtype", GROUPED_DTYPES, ids=lambda d: mg.DTYPE_NAMES[d])
def test_grouped_small_batch_vs_oracle_and_standalone(dtype):
    import torch
    shapes = inputs.log_uniform_shapes(48, seed=21, lo=1, hi=300)
    shapes += [(1, 1, 1), (128, 128, 64), (129, 257, 63), (200, 300, 16)]
    trans = [(("N", "N"), ("T", "N"), ("N", "T"), ("T", "T"))[i % 4] for i in range(len(shapes))]
    is_int = dtype == mg.GEMM_I8
    alpha = [(2 if is_int else 1.25) if i % 5 else (0 if i % 10 == 0 else 1) for i in range(len(shapes))]
    beta = [(-1 if is_int else -0.5) if i % 4 else 0 for i in range(len(shapes))]
    b = Batch(dtype, shapes, seed=23, trans=trans, alpha=alpha, beta=beta, misalign_every=7)
    mg.gemm_init(None)
    print(f"grouped {mg.DTYPE_NAMES[dtype]}: {len(shapes)} problems", flush=True)
    mg.gemm_grouped(b.problems, dtype)
    torch.cuda.synchronize()
    got = b.results()
    for p, h, C in zip(b.problems, b.host, got):
        oracle_check(dtype, p, h, C)
    # bitwise equal to the standalone call: every C-resident tile body sums
    # each entry in the same k order, so the tile shape does not change bits
    b.reset_c()
    alone = standalone(dtype, b, lambda p: grouped_shape(dtype, p))
    for i, (p, C, A1) in enumerate(zip(b.problems, got, alone)):
        assert np.array_equal(C, A1), f"problem {i} {p.m}x{p.n}x{p.k} differs from standalone"


@pytest.mark.parametrize("dtype", [mg.GEMM_F32_BF16X3, mg.GEMM_I8], ids=lambda d: mg.DTYPE_NAMES[d])
def test_grouped_batching_config_512_sampled(dtype):
    """The batching workload: 512 GEMMs, m, n, k log-uniform on [16, 4096]."""
    import torch
    shapes = inputs.log_uniform_shapes(512, seed=0)
    b = Batch(dtype, shapes, seed=4, keep_host=True)
    mg.gemm_init(None)
    print(f"batch {mg.DTYPE_NAMES[dtype]} 512 problems, {b.flops() / 1e12:.3f} TFLOP", flush=True)
    mg.gemm_grouped(b.problems, dtype)
    torch.cuda.synchronize()
    got = b.results()
    rng = np.random.default_rng(5)
    worst = 0.0
    for p, h, C in zip(b.problems, b.host, got):
        rows = rng.integers(0, p.m, 12)
        cols = rng.integers(0, p.n, 12)
        worst = max(worst, oracle_check(dtype, p, h, C, rows, cols))
    print(f"worst sampled normalised error {worst:.3g}", flush=True)


def test_grouped_graph_replay_with_rewrites():
    """A captured slot launch replays correctly after the problem list changes."""
    import torch
    dtype = mg.GEMM_F32_BF16X3
    mg.gemm_init(None)
    b1 = Batch(dtype, inputs.log_uniform_shapes(24, seed=31, lo=8, hi=260), seed=32)
    b2 = Batch(dtype, inputs.log_uniform_shapes(30, seed=33, lo=8, hi=260), seed=34)
    slot = mg.GroupedSlot(capacity=64)
    try:
        s = torch.cuda.Stream()
        slot.write(b1.problems, dtype)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                slot.launch(stream=s)
        torch.cuda.synchronize()
        for rep in range(3):
            for batch in (b1, b2):
                batch.reset_c()
                slot.write(batch.problems, dtype)
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                got = batch.results()
                # eager reference between replays
                batch.reset_c()
                mg.gemm_grouped(batch.problems, dtype)
                torch.cuda.synchronize()
                ref = batch.results()
                for i, (x, y) in enumerate(zip(got, ref)):
                    assert np.array_equal(x, y), f"replay {rep} problem {i} differs"
        for p, h, C in zip(b2.problems, b2.host, b2.results()):
            oracle_check(dtype, p, h, C)
    finally:
        slot.destroy()


def test_grouped_rejects_bad_problem_and_capacity():
    import torch
    b = Batch(mg.GEMM_F32, [(8, 8, 8), (9, 9, 9)], seed=41)
    bad = list(b.problems)
    bad[1] = mg.Problem("N", "N", 9, 9, 9, 1.0, bad[1].A, 3, bad[1].B, bad[1].ldb, 0.0,
                        bad[1].C, bad[1].ldc)
    assert mg.gemm_grouped(bad, mg.GEMM_F32, check=False) == -(1000 * 1 + 8)
    assert mg.lib().gemm_grouped(mg.gemm_grouped_capacity() + 1, None, mg.GEMM_F32) == -2
    torch.cuda.synchronize()


def test_slot_keeps_the_kernel_of_its_first_write():
    """A slot first written with an all-'N','N' aligned batch uses the compact
    kernel and rejects a later batch it cannot run; the general kernel accepts
    everything."""
    import torch
    dtype = mg.GEMM_BF16
    mg.gemm_init(None)
    nn = Batch(dtype, [(64, 64, 64), (130, 70, 90)], seed=51)
    mixed = Batch(dtype, [(64, 64, 64), (30, 20, 10)], seed=52, trans=[("N", "N"), ("T", "N")])
    s1, s2 = mg.GroupedSlot(capacity=8), mg.GroupedSlot(capacity=8)
    try:
        s1.write(nn.problems, dtype)
        assert s1.write(mixed.problems, dtype, check=False) == 2      # GEMM_E_UNSUPPORTED
        s2.write(mixed.problems, dtype)
        s2.write(nn.problems, dtype)                                  # general kernel: fine
        s2.launch()
        torch.cuda.synchronize()
        for p, h, C in zip(nn.problems, nn.host, nn.results()):
            oracle_check(dtype, p, h, C)
    finally:
        s1.destroy()
        s2.destroy()
