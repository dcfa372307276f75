"""Autotune the kernel family on this GPU and write the tuning table.

For every dtype class it times each compiled configuration (tile shape,
raster order, raster group) on representative shapes of each size bucket
(the library's gemm_tune) and writes paper_2310_20347_amd/mgemm_tune.json,
which the library loads by default.  Shapes: a coarse log grid of m, n, k
plus the benchmark workloads' own shapes.

    python -m paper_2310_20347_amd.tune [--quick] [--out PATH] [--model-keep N]
    python -m paper_2310_20347_amd.tune --model-check [--dtypes 0,1,2]
    python -m paper_2310_20347_amd.tune --grouped [--dtypes 1,5] [--out PATH]

--grouped tunes the grouped kernel's tile body per size bucket instead
(gemm_tune_grouped: a batch of identical problems per bucket, every body).
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
    p.add_argument("--layouts", default="NN,NT,TN,TT",
                   help="layouts to tune (the table keeps the entries of the others)")
    p.add_argument("--chunk", type=int, default=16,
                   help="shapes per tuner call (progress is printed after each)")
    p.add_argument("--model-keep", type=int, default=0,
                   help="time only the analytical model's first N configurations per shape")
    p.add_argument("--grouped", action="store_true",
                   help="tune the grouped kernel's body per size bucket (m, n, k in 16..4096)")
    p.add_argument("--model-check", action="store_true",
                   help="measure the analytical model instead of tuning: time every "
                        "configuration on a sample of shapes and report how much slower the "
                        "model's first choice (and the shipped table's) is than the fastest")
    a = p.parse_args()
    import torch
    torch.cuda.set_device(0)
    mg.gemm_init(None)
    if a.model_check:
        return model_check([int(x) for x in a.dtypes.split(",")], a.reps, torch)
    if a.grouped:
        grid = [2 ** e for e in range(4, 13)]
        shapes = list(itertools.product(grid, grid, grid))
        dts = [int(x) for x in a.dtypes.split(",")] if a.dtypes != p.get_default("dtypes") \
            else [mg.GEMM_F32_BF16X3, mg.GEMM_I8]
        for dt in dts:
            t0 = time.time()
            mg.gemm_tune_grouped(dt, shapes, reps=a.reps, out_path=a.out)
            print(f"tuned grouped {mg.DTYPE_NAMES[dt]}: {len(shapes)} buckets in "
                  f"{time.time() - t0:.1f} s", flush=True)
        print(f"wrote {a.out}")
        return 0
    layouts = tuple(a.layouts.split(","))
    for dt in [int(x) for x in a.dtypes.split(",")]:
        shapes = shapes_for(dt, a.quick)
        t0 = time.time()
        for i in range(0, len(shapes), a.chunk):
            mg.gemm_tune(dt, shapes[i:i + a.chunk], reps=a.reps, out_path=a.out,
                         model_keep=a.model_keep, layouts=layouts)
            print(f"  {mg.DTYPE_NAMES[dt]}: {min(i + a.chunk, len(shapes))}/{len(shapes)} shapes, "
                  f"{time.time() - t0:.1f} s", flush=True)
        print(f"tuned {mg.DTYPE_NAMES[dt]}: {len(shapes)} shapes x {len(layouts)} layouts in "
              f"{time.time() - t0:.1f} s", flush=True)
    print(f"wrote {a.out}")


def model_check(dtypes, reps, torch):
    import numpy as np
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    rng = np.random.default_rng(5)
    grid = (64, 256, 1024, 4096)
    cube = list(itertools.product(grid, grid, grid))
    shapes = [cube[i] for i in rng.choice(len(cube), 20, replace=False)]
    shapes += [(8192, 8192, 8192), (196, 1024, 4608), (50176, 64, 576)]

    def operand(dt, r, c):
        if dt in (mg.GEMM_BF16, mg.GEMM_F16):
            return (torch.rand((r, c), device="cuda") * 2 - 1).to(torch.bfloat16).view(torch.int16)
        if dt in (mg.GEMM_F8E4M3, mg.GEMM_I8):
            return torch.randint(-8, 8, (r, c), device="cuda", dtype=torch.int8)
        if dt == mg.GEMM_F64:
            return torch.rand((r, c), device="cuda", dtype=torch.float64) * 2 - 1
        return torch.rand((r, c), device="cuda") * 2 - 1

    def timed(f):
        f()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            f()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    for dt in dtypes:
        model_loss, table_loss = [], []
        for (m, n, k) in shapes:
            A, B = operand(dt, m, k), operand(dt, k, n)
            ct = {mg.GEMM_I8: torch.int32, mg.GEMM_F64: torch.float64}.get(dt, torch.float32)
            C = torch.empty((m, n), device="cuda", dtype=ct)
            fam = mg.GEMM_F32_BF16X6 if (dt == mg.GEMM_F32_BF16X3 and k < 64) else dt
            times, model = {}, {}
            try:
                for cfg in range(mg.num_configs(fam)):
                    if not mg.config_supports(fam, cfg, "N", "N"):
                        continue
                    mg.force_config(dt, cfg, 0)
                    times[cfg] = timed(lambda: mg.gemm("N", "N", m, n, k, 1, A, k, B, n, 0, C, n, dt))
                    model[cfg] = mg.model_us(fam, cfg, m, n, k, cus)
            finally:
                mg.force_config(dt, -1, 0)
            table = timed(lambda: mg.gemm("N", "N", m, n, k, 1, A, k, B, n, 0, C, n, dt))
            best = min(times.values())
            model_loss.append(times[min(model, key=model.get)] / best)
            table_loss.append(table / best)
            del A, B, C
        ml, tl = np.array(model_loss), np.array(table_loss)
        print(f"{mg.DTYPE_NAMES[dt]:>7}: model's choice / fastest: mean {ml.mean():.3f}, median "
              f"{np.median(ml):.3f}, max {ml.max():.2f}, within 10% on {np.mean(ml <= 1.1):.0%} "
              f"of {len(ml)} shapes | shipped table: mean {tl.mean():.3f}, max {tl.max():.2f}",
              flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
