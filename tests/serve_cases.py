"""Synthetic serving workloads: Poisson arrivals, log-uniform shapes, a dtype
mix, and device pools from which request operands are copied at admission."""
from __future__ import annotations

import numpy as np

import paper_2310_20347_amd as mg
from paper_2310_20347_amd import inputs
from paper_2310_20347_amd import serve as sv

MIX = ((mg.GEMM_F32_BF16X3, 0.5), (mg.GEMM_BF16, 0.3), (mg.GEMM_I8, 0.2))


class Pools:
    """One device pool per dtype holding valid values of that input format."""

    def __init__(self, nbytes, seed):
        import torch
        n32 = nbytes // 4
        self.t = {
            mg.GEMM_F32_BF16X3: torch.from_numpy(inputs.uniform((n32,), seed)).cuda(),
            mg.GEMM_BF16: torch.from_numpy(
                inputs.to_bf16_bits(inputs.uniform((nbytes // 2,), seed + 1)).view(np.int16)).cuda(),
            mg.GEMM_I8: torch.from_numpy(inputs.int8_uniform((nbytes,), seed + 2)).cuda(),
        }
        self.nbytes = nbytes

    def ptr(self, dtype, off):
        return self.t[dtype].data_ptr() + off


def workload(count, rate, seed, pools, lo=16, hi=4096, result_every=0):
    """count requests; returns (requests, meta) where meta holds what a check needs."""
    shapes = inputs.log_uniform_shapes(count, seed, lo, hi)
    arrivals = inputs.poisson_arrivals(count, rate, seed + 1)
    kinds = inputs.categorical(count, [p for _, p in MIX], seed + 2)
    rng = np.random.default_rng(seed + 3)
    reqs, meta = [], []
    for i, ((m, n, k), t, c) in enumerate(zip(shapes, arrivals, kinds)):
        dt = MIX[c][0]
        lda, ldb, ldc, _ = sv.serve_layout(m, n, k, dt)
        es = {mg.GEMM_F32_BF16X3: 4, mg.GEMM_BF16: 2, mg.GEMM_I8: 1}[dt]
        a_bytes, b_bytes = m * lda * es, k * ldb * es
        if max(a_bytes, b_bytes) > pools.nbytes:
            raise ValueError("pool too small")
        a_off = int(rng.integers(0, (pools.nbytes - a_bytes) // 256 + 1)) * 256
        b_off = int(rng.integers(0, (pools.nbytes - b_bytes) // 256 + 1)) * 256
        res = None
        if result_every and i % result_every == 0:
            res = np.zeros((m, n), dtype=np.int32 if dt == mg.GEMM_I8 else np.float32)
        reqs.append(sv.Request(float(t), m, n, k, dt, pools.ptr(dt, a_off), pools.ptr(dt, b_off),
                               res.ctypes.data if res is not None else None))
        meta.append(dict(m=m, n=n, k=k, dtype=dt, lda=lda, ldb=ldb, ldc=ldc, a_off=a_off,
                         b_off=b_off, result=res))
    return reqs, meta


def alone(pools, md):
    """The request run by itself through gemm() with an unsliced configuration
    (not split-K): the serving launches run unsliced tiles, and every unsliced
    configuration sums k in one order."""
    import torch
    m, n, k, dt = md["m"], md["n"], md["k"], md["dtype"]
    out_t = torch.int32 if dt == mg.GEMM_I8 else torch.float32
    C = torch.zeros((m, n), dtype=out_t, device="cuda")
    mg.force_config(dt, 1, 0)
    try:
        mg.gemm("N", "N", m, n, k, 1, pools.ptr(dt, md["a_off"]), md["lda"],
                pools.ptr(dt, md["b_off"]), md["ldb"], 0, C, n, dt)
    finally:
        mg.force_config(dt, -1, 0)
    torch.cuda.synchronize()
    return C.cpu().numpy()


def host_operand(pools, dt, off, rows, ld):
    t = pools.t[dt]
    es = t.element_size()
    flat = t.cpu().numpy().reshape(-1)
    x = flat[off // es: off // es + rows * ld].reshape(rows, ld)
    if dt == mg.GEMM_BF16:
        x = x.view(np.uint16)
    return x


def check_results(pools, meta):
    """Every request that returned its C: equal to the request alone (bit for
    bit) and within the quantised-input tolerance of the oracle.  Returns the
    number checked."""
    import oracle
    from gemm_cases import QUANT_TOL, decode, terms_for
    checked = 0
    for md in meta:
        if md["result"] is None:
            continue
        mix = md["result"]
        solo = alone(pools, md)
        assert np.array_equal(mix, solo), f"mix != alone for {md['m']}x{md['n']}x{md['k']}"
        dt, m, n, k = md["dtype"], md["m"], md["n"], md["k"]
        A = host_operand(pools, dt, md["a_off"], m, md["lda"])
        B = host_operand(pools, dt, md["b_off"], k, md["ldb"])
        if dt == mg.GEMM_I8:
            ref = oracle.gemm_i8("N", "N", m, n, k, 1, A, md["lda"], B, md["ldb"])
            assert np.array_equal(mix, ref)
        else:
            terms = terms_for(dt, k)
            if terms is not None:
                npc = 3 if len(terms) > 3 else 2
                PA = [oracle.decode_bf16(x) for x in oracle.split_bf16(A, npc)]
                PB = [oracle.decode_bf16(x) for x in oracle.split_bf16(B, npc)]
                ref = oracle.gemm_pieces("N", "N", m, n, k, 1.0, PA, md["lda"], PB, md["ldb"], terms)
                ma, mb = np.abs(A).max(), np.abs(B).max()
            else:
                Aq, Bq = decode(A, dt), decode(B, dt)
                ref = oracle.gemm_f64("N", "N", m, n, k, 1.0, Aq, md["lda"], Bq, md["ldb"])
                ma, mb = np.abs(Aq).max(), np.abs(Bq).max()
            assert oracle.normalized_error(mix, ref, k, ma, mb) <= QUANT_TOL
        checked += 1
    return checked
