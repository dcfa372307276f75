"""Build the HIP library libmgemm.so (gfx950) in-tree with hipcc.

Every source under csrc/ is compiled in parallel to an object file, then
linked into paper_2310_20347_amd/libmgemm.so.  All device code is compiled
with packed-FP32 instructions disabled.

build_sanitized() makes a second library, _build_san/libmgemm_san.so, whose
host code (the C ABI, dispatch, tuning table, serving loop, model: the .cpp
sources) is compiled with AddressSanitizer and UndefinedBehaviorSanitizer
(host side only; the kernels' objects are the normal build's).  Load it with
MGEMM_LIBRARY and the sanitizer runtime preloaded (sanitizer_env()).
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libmgemm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", CSRC, "-I", INCLUDE,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


# Per-source flags.  The grouped persistent kernels claim their next tile
# with an atomic whose result is used only after the current tile; the
# compiler's atomic optimizer (which combines a wave's atomics) would wait for
# that result right after issuing it, at the start of every tile.
EXTRA = {"grouped_k_": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]}


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    extra = [f for k, v in EXTRA.items() if os.path.basename(src).startswith(k) for f in v]
    cmd = [HIPCC] + COMMON + extra + lang + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(ln for ln in r.stderr.splitlines() if noise not in ln)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip() and verbose:
        print(err, flush=True)
    return obj


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-ldl"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


SAN_DIR = os.path.join(HERE, "_build_san")
SAN_OUT = os.path.join(SAN_DIR, "libmgemm_san.so")
SAN_FLAGS = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def sanitizer_runtime():
    """The compiler's AddressSanitizer runtime (preloaded into the test process)."""
    rt = glob.glob(os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))),
                                "llvm", "lib", "clang", "*", "lib", "linux",
                                "libclang_rt.asan-x86_64.so"))
    if not rt:
        rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return rt[0] if rt else None


def sanitizer_env():
    env = dict(os.environ)
    env["MGEMM_LIBRARY"] = SAN_OUT
    env["LD_PRELOAD"] = sanitizer_runtime() or ""
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


def build_sanitized(verbose=False, jobs=None):
    """The host sources with ASan/UBSan, linked with the normal build's
    kernel objects (build() first)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    cpp = sorted(glob.glob(os.path.join(CSRC, "*.cpp")))
    hip = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def comp(src):
        obj = os.path.join(SAN_DIR, os.path.basename(src) + ".o")
        cmd = [HIPCC] + [f for f in COMMON if f != "-O3"] + SAN_FLAGS + ["-x", "hip", "-c", src,
                                                                        "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-4000:]}")
        return obj

    with cf.ThreadPoolExecutor(jobs or min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(comp, cpp))
    objs += [os.path.join(BUILD, os.path.basename(s) + ".o") for s in hip]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"run build() first: missing {missing[:3]}")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", SAN_OUT] + objs + ["-ldl"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return SAN_OUT


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
