"""The synthetic workload recipe against the paper's own tables."""
import os

import numpy as np

from paper_2310_20347_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [list(map(float, ln.split())) for ln in f if ln.strip() and not ln.startswith("#")]


def test_conv_shapes_are_table1_rows_at_batch_16():
    rows = _rows("resnet50_table1.txt")
    table = {int(r[0]): tuple(int(x) for x in r[1:]) for r in rows}
    assert table == inputs.RESNET50_TABLE1_BATCH128
    batch16 = {(m // 8, n, k) for (m, n, k) in table.values()}
    assert batch16 <= set(inputs.CONV_SHAPES)
    assert len(set(inputs.CONV_SHAPES) - batch16) == 1   # the synthetic tall-k shape


def test_seeded_generators_are_deterministic():
    a = inputs.uniform((5, 7), inputs.seed_for(1, "A"))
    b = inputs.uniform((5, 7), inputs.seed_for(1, "A"))
    assert np.array_equal(a, b) and a.dtype == np.float32
    assert a.min() >= -1 and a.max() <= 1
    s = inputs.log_uniform_shapes(512, 0)
    assert len(s) == 512 and min(min(t) for t in s) >= 16 and max(max(t) for t in s) <= 4096
    q = inputs.int8_uniform((1000,), 3)
    assert q.dtype == np.int8 and q.min() == -128 and q.max() == 127


def test_badly_scaled_exponent_range():
    x = inputs.badly_scaled(256, 256, 7)
    e = np.log2(np.abs(x[x != 0]))
    assert e.max() > 30 and e.min() < -30     # product of two 2^U[-20,20] scales


def test_e4m3_cast_saturates():
    bits = inputs.to_e4m3_bits(np.array([1000.0, -1000.0, 448.0, 1.0], np.float32))
    assert list(bits) == [0x7E, 0xFE, 0x7E, 0x38]
