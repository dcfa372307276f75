"""Autotune the kernel family on this GPU and write the tuning table.

For every dtype class it times each compiled configuration (tile shape,
raster order, raster group) on representative shapes of each size bucket
(the library's gemm_tune) and writes paper_2310_20347_amd/mgemm_tune.json,
which the library loads by default.  Shapes: a coarse log grid of m, n, k
plus the benchmark workloads' own shapes.

    python -m paper_2310_20347_amd.tune [--quick] [--out PATH]
"""
import argparse
import itertools
import os
import sys
import time

import paper_2310_20347_amd as mg

HERE = os.path.dirname(os.path.abspath(__file__))

SWEEP = [(1024, 1024, 1024), (2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192),
         (50176, 64, 576), (3136, 256, 2304), (196, 1024, 4608), (12544, 128, 1152)]


def shapes_for(dtype, quick):
    grid = (16, 64, 256, 1024, 4096) if not quick else (64, 1024)
    shapes = list(itertools.product(grid, grid, grid))
    if dtype in (mg.GEMM_F32, mg.GEMM_F32_BF16X3):
        shapes += SWEEP
    if dtype != mg.GEMM_F32:
        shapes += [(8192, 8192, 8192)]
    # the split dtype resolves to two classes by k (< 64 uses six terms)
    if dtype == mg.GEMM_F32_BF16X3:
        shapes += [(m, n, 32) for m in grid for n in grid]
    seen, out = set(), []
    for s in shapes:
        if s not in seen:
            seen.add(s)
            out.append(s)
    return out


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--quick", action="store_true")
    p.add_argument("--reps", type=int, default=5)
    p.add_argument("--out", default=os.path.join(HERE, "mgemm_tune.json"))
    p.add_argument("--dtypes", default="0,1,2,3,4,5,7,8")
    a = p.parse_args()
    import torch
    torch.cuda.set_device(0)
    mg.gemm_init(None)
    for dt in [int(x) for x in a.dtypes.split(",")]:
        shapes = shapes_for(dt, a.quick)
        t0 = time.time()
        mg.gemm_tune(dt, shapes, reps=a.reps, out_path=a.out)
        print(f"tuned {mg.DTYPE_NAMES[dt]}: {len(shapes)} shapes in {time.time() - t0:.1f} s",
              flush=True)
    print(f"wrote {a.out}")


if __name__ == "__main__":
    sys.exit(main())
