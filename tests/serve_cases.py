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
