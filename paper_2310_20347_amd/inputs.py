"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random numbers and converts storage formats with library
routines (numpy / torch dtype casts); it contains none of the GEMM's own
arithmetic and imports neither the HIP binding nor the oracle.

Workload recipe (shapes and value distributions of the paper's workloads):

* squares m = n = k, entries U[-1, 1];
* im2col convolution shapes of ResNet50 v1.5 (paper section 8.1, Table 1),
  taken at batch 16 (m divided by 8): layer types 3, 12 and 7, plus a
  synthetic tall-k shape (196, 1024, 4608);
* precision inputs N(0, 1) and a badly scaled variant A = Dr A0 Dc with
  diagonal scales 2^U[-20, 20] (continuous exponent);
* batches of GEMMs with m, n, k independently log-uniform on [16, 4096];
* INT8 values uniform on the integers [-128, 127].

Seeds follow one rule: config c draws A with seed 1000c+1, B with 1000c+2,
C0 with 1000c+3 and the serving schedule with 1000c+9.
"""
from __future__ import annotations

import numpy as np

# Shapes (m, n, k) -----------------------------------------------------------

SQUARES = (1024, 2048, 4096, 8192)

# ResNet50 v1.5 im2col GEMMs of Table 1 at batch 128 for the three layer types
# used here; the benchmark runs them at batch 16 (m / 8).
RESNET50_TABLE1_BATCH128 = {3: (401408, 64, 576), 12: (25088, 256, 2304),
                            7: (100352, 128, 1152)}
CONV_SHAPES = ((50176, 64, 576), (3136, 256, 2304), (196, 1024, 4608),
               (12544, 128, 1152))


def seed_for(config: int, which: str) -> int:
    return 1000 * config + {"A": 1, "B": 2, "C": 3, "serve": 9}[which]


# Value draws -----------------------------------------------------------------

def uniform(shape, seed, lo=-1.0, hi=1.0, dtype=np.float32):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape).astype(dtype)


def normal(shape, seed, dtype=np.float32):
    return np.random.default_rng(seed).standard_normal(size=shape).astype(dtype)


def badly_scaled(rows, cols, seed, span=20.0, dtype=np.float32):
    """Dr * X0 * Dc with X0 ~ N(0,1) and diagonal entries 2^U[-span, span]."""
    rng = np.random.default_rng(seed)
    x0 = rng.standard_normal(size=(rows, cols))
    dr = np.exp2(rng.uniform(-span, span, size=(rows, 1)))
    dc = np.exp2(rng.uniform(-span, span, size=(1, cols)))
    return (dr * x0 * dc).astype(dtype)


def small_ints(shape, seed, lo=-8, hi=8, dtype=np.float32):
    """Integers in [lo, hi]; exact in every input format of the library."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=shape).astype(dtype)


def int8_uniform(shape, seed):
    return np.random.default_rng(seed).integers(-128, 128, size=shape).astype(np.int8)


def log_uniform_shapes(count, seed, lo=16, hi=4096):
    """count (m, n, k) triples, each dimension round(exp(U[ln lo, ln hi]))."""
    rng = np.random.default_rng(seed)
    v = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=(count, 3))))
    return [tuple(int(x) for x in row) for row in v.astype(np.int64)]


def poisson_arrivals(count, rate_per_s, seed):
    """Arrival times (seconds) of a Poisson process: cumulative exponential gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def categorical(count, probs, seed):
    rng = np.random.default_rng(seed)
    return rng.choice(len(probs), size=count, p=np.asarray(probs, dtype=np.float64))


# Storage formats (library casts) ----------------------------------------------

def to_bf16_bits(x):
    """FP32 -> bfloat16 bit patterns (uint16), round to nearest even (torch cast)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def to_f16_bits(x):
    """FP32 -> IEEE binary16 bit patterns (uint16), round to nearest even."""
    return np.ascontiguousarray(x, dtype=np.float32).astype(np.float16).view(np.uint16)


E4M3_MAX = 448.0


def to_e4m3_bits(x):
    """FP32 -> OCP E4M3FN codes (uint8), round to nearest even, saturating to
    +-448 (torch's cast turns overflow into NaN, so clamp first)."""
    import torch
    xf = np.clip(np.ascontiguousarray(x, dtype=np.float32), -E4M3_MAX, E4M3_MAX)
    t = torch.from_numpy(xf).to(torch.float8_e4m3fn)
    return t.view(torch.uint8).numpy()
