"""Calls from several host threads at once: each thread runs gemm() on its
own stream with its own workspace reservation (split-K and packed-split
configurations among the cases), concurrently with the others, and every
result equals the single-thread result bit for bit, from the same
configuration."""
import threading

import pytest

import paper_2310_20347_amd as mg

pytestmark = pytest.mark.gpu

CASES = [(mg.GEMM_F32, 196, 1024, 4608), (mg.GEMM_F32_BF16X3, 1024, 1024, 1024),
         (mg.GEMM_I8, 512, 768, 4096), (mg.GEMM_F32, 1000, 1000, 1000),
         (mg.GEMM_BF16, 777, 640, 960)]
THREADS = 4
ITERS = 5


def _operands(torch, g, dt, m, n, k):
    if dt == mg.GEMM_I8:
        A = torch.randint(-128, 128, (m, k), generator=g, dtype=torch.int8)
        B = torch.randint(-128, 128, (k, n), generator=g, dtype=torch.int8)
        return A.cuda(), B.cuda(), torch.int32, 1, 0
    A = torch.rand((m, k), generator=g) * 2 - 1
    B = torch.rand((k, n), generator=g) * 2 - 1
    if dt == mg.GEMM_BF16:
        A, B = A.bfloat16(), B.bfloat16()
    return A.cuda(), B.cuda(), torch.float32, 1.0, 0.0


def test_concurrent_threads_match_one_thread():
    import torch
    mg.gemm_init(None)
    g = torch.Generator().manual_seed(5)
    ops = [(dt, m, n, k) + _operands(torch, g, dt, m, n, k) for dt, m, n, k in CASES]
    needs = [mg.workspace_bytes("N", "N", m, n, k, dt) for dt, m, n, k in CASES]
    need = max(needs)
    assert sum(x > 0 for x in needs) >= 2, needs   # split-K / packed split among the cases
    ref = []
    for dt, m, n, k, A, B, ct, one, zero in ops:
        C = torch.zeros((m, n), dtype=ct, device="cuda")
        mg.gemm("N", "N", m, n, k, one, A, k, B, n, zero, C, n, dt)
        ref.append((C, mg.last_config()["cfg"]))
    torch.cuda.synchronize()
    errors = []

    def worker(tid):
        try:
            s = torch.cuda.Stream()
            mg.reserve_workspace(max(need, 1 << 20), 0, stream=s)
            outs = [torch.full((m, n), -1, dtype=ct, device="cuda")
                    for dt, m, n, k, A, B, ct, one, zero in ops]
            torch.cuda.synchronize()
            for it in range(ITERS):
                for i, (dt, m, n, k, A, B, ct, one, zero) in enumerate(ops):
                    mg.gemm("N", "N", m, n, k, one, A, k, B, n, zero, outs[i], n, dt, stream=s)
                    cfg = mg.last_config()["cfg"]
                    if cfg != ref[i][1]:
                        errors.append(f"thread {tid} case {i}: configuration {cfg}, not {ref[i][1]}")
            s.synchronize()
            for i, out in enumerate(outs):
                if not torch.equal(out, ref[i][0]):
                    errors.append(f"thread {tid} case {i}: result differs from one thread's")
            mg.release_workspace(stream=s)
        except Exception as e:  # reported below, with the thread
            errors.append(f"thread {tid}: {e!r}")

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(THREADS)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a thread did not finish"
    assert not errors, errors


def test_concurrent_grouped_launches_match_one_thread():
    """Grouped launches from several threads, each on its own stream (the
    library's rotating descriptor slots are shared), equal the one-thread
    launch bit for bit."""
    import torch
    mg.gemm_init(None)
    g = torch.Generator().manual_seed(9)
    shapes = [(37, 300, 64), (256, 128, 512), (16, 16, 16), (515, 97, 1024), (128, 640, 208),
              (1000, 24, 96), (64, 64, 4096), (300, 300, 304)]
    for dt in (mg.GEMM_I8, mg.GEMM_F32_BF16X3):
        ops = [(m, n, k) + _operands(torch, g, dt, m, n, k) for m, n, k in shapes]

        def problems(Cs):
            return [mg.Problem("N", "N", m, n, k, one, A, k, B, n, zero, C, n)
                    for (m, n, k, A, B, ct, one, zero), C in zip(ops, Cs)]

        ref = [torch.zeros((m, n), dtype=ct, device="cuda") for m, n, k, A, B, ct, one, zero in ops]
        mg.gemm_grouped(problems(ref), dt)
        torch.cuda.synchronize()
        errors = []

        def worker(tid):
            try:
                s = torch.cuda.Stream()
                Cs = [torch.full((m, n), -1, dtype=ct, device="cuda")
                      for m, n, k, A, B, ct, one, zero in ops]
                torch.cuda.synchronize()
                batch = problems(Cs)
                for it in range(ITERS):
                    mg.gemm_grouped(batch, dt, stream=s)
                s.synchronize()
                for i, C in enumerate(Cs):
                    if not torch.equal(C, ref[i]):
                        errors.append(f"{mg.DTYPE_NAMES[dt]} thread {tid} problem {i} differs")
            except Exception as e:  # reported below, with the thread
                errors.append(f"{mg.DTYPE_NAMES[dt]} thread {tid}: {e!r}")

        threads = [threading.Thread(target=worker, args=(t,)) for t in range(THREADS)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=120)
        assert not any(t.is_alive() for t in threads), "a thread did not finish"
        assert not errors, errors
