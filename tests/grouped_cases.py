"""Batches of independent GEMMs for the grouped-launch tests and benchmarks."""
from __future__ import annotations

import numpy as np

import paper_2310_20347_amd as mg
from paper_2310_20347_amd import inputs

from gemm_cases import encode, stored, to_device


class Batch:
    """count problems with device operands; keeps the host copies the oracle needs."""

    def __init__(self, dtype, shapes, seed, trans=None, alpha=1.0, beta=0.0, pad_to=16,
                 misalign_every=0, keep_host=True):
        import torch
        self.dtype = dtype
        self.problems = []
        self.host = []
        rng = np.random.default_rng(seed)
        is_int = dtype == mg.GEMM_I8
        for i, (m, n, k) in enumerate(shapes):
            ta, tb = trans[i] if trans else ("N", "N")
            if is_int:
                a = inputs.int8_uniform((m, k), seed * 7919 + 2 * i).astype(np.float32)
                b = inputs.int8_uniform((k, n), seed * 7919 + 2 * i + 1).astype(np.float32)
                c0 = rng.integers(-1000, 1000, size=(m, n)).astype(np.int32)
            else:
                a = inputs.uniform((m, k), seed * 7919 + 2 * i)
                b = inputs.uniform((k, n), seed * 7919 + 2 * i + 1)
                c0 = inputs.uniform((m, n), seed * 7919 + 100000 + i)
            es = {mg.GEMM_BF16: 2, mg.GEMM_F16: 2, mg.GEMM_F8E4M3: 1, mg.GEMM_I8: 1}.get(dtype, 4)
            q = max(1, pad_to // es)           # leading dims rounded up to 16-byte multiples

            def ld_of(cols):
                return -(-cols // q) * q
            lda = ld_of(m if ta == "T" else k)
            ldb = ld_of(k if tb == "T" else n)
            ldc = n
            mis = 1 if (misalign_every and i % misalign_every == 1) else 0
            if mis:
                lda += 1
            As = stored(encode(a, dtype), ta, lda)
            Bs = stored(encode(b, dtype), tb, ldb)
            Cs = stored(c0, "N", ldc)
            dA = to_device(np.concatenate([np.zeros(mis, As.dtype), As.reshape(-1)]))
            dB = to_device(Bs.reshape(-1))
            dC = to_device(Cs.reshape(-1).copy())
            al = float(alpha[i]) if hasattr(alpha, "__len__") else float(alpha)
            be = float(beta[i]) if hasattr(beta, "__len__") else float(beta)
            p = mg.Problem(ta, tb, m, n, k, al, dA.data_ptr() + mis * dA.element_size(), lda,
                           dB, ldb, be, dC, ldc)
            p._keep = (dA, dB, dC)
            self.problems.append(p)
            if keep_host:
                self.host.append(dict(a32=a, b32=b, As=As, Bs=Bs, C0=Cs, lda=lda, ldb=ldb,
                                      ldc=ldc))

    def reset_c(self):
        """Restores every C to its initial value (device copy of the host C0)."""
        import torch
        for p, h in zip(self.problems, self.host):
            dC = p._keep[2]
            dC.copy_(torch.from_numpy(np.ascontiguousarray(h["C0"]).reshape(-1)).to(dC.device))

    def results(self):
        import torch
        torch.cuda.synchronize()
        out = []
        for p in self.problems:
            c = p._keep[2].cpu().numpy().reshape(p.m, p.ldc)[:, :p.n]
            out.append(c)
        return out

    def flops(self):
        return sum(2.0 * p.m * p.n * p.k for p in self.problems)
