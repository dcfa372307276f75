"""The host-side code of the library (C ABI validation and dispatch, tuning
table, analytical model, serving scheduler on its simulated device) under
AddressSanitizer and UndefinedBehaviorSanitizer: the CPU tests of the ABI and
of the serving scheduler run in a child process against the sanitized build
(paper_2310_20347_amd/build.py build_sanitized) with the sanitizer runtime
preloaded; any report aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2310_20347_amd"))


def test_host_code_clean_under_asan_and_ubsan():
    import build
    if not build.sanitizer_runtime():
        pytest.skip("no AddressSanitizer runtime next to the compiler")
    if not os.path.exists(os.path.join(build.BUILD, "abi.cpp.o")):
        pytest.skip("the library is not built (build() makes the kernel objects)")
    build.build_sanitized()
    env = build.sanitizer_env()
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", os.path.join(ROOT, "tests", "test_abi_host.py"),
                        os.path.join(ROOT, "tests", "test_serve_sim.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-3000:] + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in tail and "runtime error" not in tail
