"""ctypes binding of libmgemm.so: same names as the C ABI, marshalling only."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Any, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))

GEMM_F32 = 0
GEMM_F32_BF16X3 = 1
GEMM_BF16 = 2
GEMM_F16 = 3
GEMM_F8E4M3 = 4
GEMM_I8 = 5
GEMM_F32_BF16X3_ONLY = 6
GEMM_F32_BF16X6 = 7
GEMM_F64 = 8
GEMM_I16 = 9
GEMM_I32 = 10
GEMM_NUM_DTYPES = 11
DTYPE_NAMES = {GEMM_F32: "f32", GEMM_F32_BF16X3: "bf16x3", GEMM_BF16: "bf16", GEMM_F16: "f16",
               GEMM_F8E4M3: "e4m3", GEMM_I8: "i8", GEMM_F32_BF16X3_ONLY: "bf16x3_only",
               GEMM_F32_BF16X6: "bf16x6", GEMM_F64: "f64",
               GEMM_I16: "i16", GEMM_I32: "i32"}

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double
_C = ctypes.c_char
_INT = ctypes.c_int


class _Problem(ctypes.Structure):
    _fields_ = [("transA", _C), ("transB", _C), ("m", _I64), ("n", _I64), ("k", _I64),
                ("alpha", _D), ("A", _P), ("lda", _I64), ("B", _P), ("ldb", _I64),
                ("beta", _D), ("C", _P), ("ldc", _I64)]


class MGemmError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where} failed with code {code}: {strerror(code)}")


def lib_path() -> str:
    """The in-tree library, or the build named by MGEMM_LIBRARY (the
    sanitizer build of the host code uses this)."""
    return os.environ.get("MGEMM_LIBRARY") or os.path.join(_HERE, "libmgemm.so")


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2310_20347_amd/build.py "
                           "(or __graft_entry__.build())")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 under the
    # same soname, so load PyTorch first and this library binds to the runtime
    # that PyTorch's device memory and streams belong to.  (Loaded the other
    # way round, the library's runtime failed to find the device once PyTorch
    # had initialised it.)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    L.gemm.argtypes = [_C, _C, _I64, _I64, _I64, _D, _P, _I64, _P, _I64, _D, _P, _I64, _INT]
    L.gemm_scaled.argtypes = [_C, _C, _I64, _I64, _I64, _D, _P, _I64, _P, _I64, _D, _P, _I64, _INT]
    L.gemm_scaled.restype = _INT
    L.gemm.restype = _INT
    L.gemm_noalloc.argtypes = [_C, _C, _I64, _I64, _I64, _D, _P, _I64, _P, _I64, _D, _P, _I64,
                               _INT]
    L.gemm_noalloc.restype = _INT
    L.gemm_noalloc_scratch_bytes.argtypes = []
    L.gemm_noalloc_scratch_bytes.restype = _I64
    L.gemm_grouped.argtypes = [_I64, ctypes.POINTER(_Problem), _INT]
    L.gemm_grouped.restype = _INT
    L.gemm_grouped_num_bodies.argtypes = [_INT]
    L.gemm_grouped_num_bodies.restype = _INT
    L.gemm_grouped_body_info.argtypes = [_INT, _INT, ctypes.POINTER(_I64)]
    L.gemm_grouped_body_info.restype = _INT
    L.gemm_grouped_force_body.argtypes = [_INT]
    L.gemm_grouped_force_body.restype = _INT
    L.gemm_grouped_bodies.argtypes = [_I64, ctypes.POINTER(_Problem), _INT, ctypes.POINTER(_INT)]
    L.gemm_grouped_bodies.restype = _INT
    L.gemm_tune_grouped.argtypes = [_INT, _I64, ctypes.POINTER(_I64), _INT, ctypes.c_char_p]
    L.gemm_tune_grouped.restype = _INT
    L.gemm_grouped_capacity.argtypes = []
    L.gemm_grouped_capacity.restype = _I64
    L.gemm_grouped_slot_create.argtypes = [ctypes.POINTER(_P), _I64]
    L.gemm_grouped_slot_create.restype = _INT
    L.gemm_grouped_slot_write.argtypes = [_P, _I64, ctypes.POINTER(_Problem), _INT]
    L.gemm_grouped_slot_write.restype = _INT
    L.gemm_grouped_slot_launch.argtypes = [_P]
    L.gemm_grouped_slot_launch.restype = _INT
    L.gemm_grouped_slot_destroy.argtypes = [_P]
    L.gemm_grouped_slot_destroy.restype = None
    L.gemm_set_stream.argtypes = [_P]
    L.gemm_set_stream.restype = _INT
    L.gemm_init.argtypes = [ctypes.c_char_p]
    L.gemm_init.restype = _INT
    L.gemm_shutdown.argtypes = []
    L.gemm_shutdown.restype = None
    L.gemm_strerror.argtypes = [_INT]
    L.gemm_strerror.restype = ctypes.c_char_p
    L.gemm_last_hip_error.argtypes = []
    L.gemm_last_hip_error.restype = _INT
    L.gemm_num_configs.argtypes = [_INT]
    L.gemm_num_configs.restype = _INT
    L.gemm_config_info.argtypes = [_INT, _INT, ctypes.POINTER(_I64)]
    L.gemm_config_info.restype = _INT
    L.gemm_config_staging.argtypes = [_INT, _INT]
    L.gemm_config_staging.restype = _INT
    L.gemm_config_mfma.argtypes = [_INT, _INT]
    L.gemm_config_mfma.restype = _INT
    L.gemm_config_layouts.argtypes = [_INT, _INT]
    L.gemm_config_layouts.restype = _INT
    L.gemm_force_config.argtypes = [_INT, _INT, _INT]
    L.gemm_force_config.restype = _INT
    L.gemm_last_config.argtypes = [ctypes.POINTER(_I64)]
    L.gemm_last_config.restype = _INT
    L.gemm_debug_count.argtypes = [ctypes.c_void_p, _I64, _I64, _I64, _INT]
    L.gemm_debug_count.restype = _INT
    L.gemm_debug_unwritten.argtypes = []
    L.gemm_debug_unwritten.restype = _I64
    L.gemm_tune.argtypes = [_INT, _I64, ctypes.POINTER(_I64), _INT, ctypes.c_char_p]
    L.gemm_tune_pruned.argtypes = [_INT, _I64, ctypes.POINTER(_I64), _INT, ctypes.c_char_p, _INT]
    L.gemm_tune_pruned.restype = _INT
    L.gemm_tune_layouts.argtypes = [_INT, _I64, ctypes.POINTER(_I64), _INT, ctypes.c_char_p, _INT,
                                    _INT]
    L.gemm_tune_layouts.restype = _INT
    L.gemm_model_us.argtypes = [_INT, _INT, _I64, _I64, _I64, _INT]
    L.gemm_model_us.restype = ctypes.c_double
    L.gemm_tune.restype = _INT
    L.gemm_reserve_workspace.argtypes = [_I64, _I64]
    L.gemm_reserve_workspace.restype = _INT
    L.gemm_release_workspace.argtypes = []
    L.gemm_release_workspace.restype = _INT
    L.gemm_workspace_bytes.argtypes = [_C, _C, _I64, _I64, _I64, _INT]
    L.gemm_workspace_bytes.restype = _I64
    L.gemm_scaled_workspace_bytes.argtypes = [_C, _C, _I64, _I64, _I64, _D, _INT]
    L.gemm_scaled_workspace_bytes.restype = _I64
    L.gemm_panel_occupancy.argtypes = [_I64, _I64, _I64, _I64]
    L.gemm_panel_occupancy.restype = _D
    _lib = L
    return L


def strerror(code: int) -> str:
    return lib().gemm_strerror(int(code)).decode()


def _check(rc: int, where: str) -> int:
    if rc != 0:
        raise MGemmError(rc, where)
    return rc


def _ptr(x: Any) -> Optional[int]:
    """Device address of a torch tensor (or a raw int address)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if hasattr(x, "is_cuda") and not x.is_cuda:
            raise ValueError("gemm operands must be device tensors")
        return x.data_ptr()
    raise TypeError(f"cannot take the device address of {type(x)}")


def set_stream(stream: Any = None) -> None:
    """Stream for this thread's calls: a torch.cuda.Stream, a raw handle, or None
    for torch's current stream."""
    if stream is None:
        import torch
        handle = torch.cuda.current_stream().cuda_stream
    elif isinstance(stream, int):
        handle = stream
    else:
        handle = stream.cuda_stream
    _check(lib().gemm_set_stream(handle or None), "gemm_set_stream")


def _tc(t: str) -> bytes:
    return t.encode() if isinstance(t, str) else bytes(t)


def gemm(transA: str, transB: str, m: int, n: int, k: int, alpha: float, A, lda: int, B,
         ldb: int, beta: float, C, ldc: int, dtype: int, stream: Any = None,
         check: bool = True) -> int:
    """C = alpha*op(A)*op(B) + beta*C on the current (or given) stream."""
    set_stream(stream)
    rc = lib().gemm(_tc(transA), _tc(transB), m, n, k, float(alpha), _ptr(A), lda, _ptr(B),
                    ldb, float(beta), _ptr(C), ldc, int(dtype))
    return _check(rc, "gemm") if check else rc


def gemm_noalloc(transA: str, transB: str, m: int, n: int, k: int, alpha: float, A, lda: int, B,
                 ldb: int, beta: float, C, ldc: int, dtype: int, stream: Any = None,
                 check: bool = True) -> int:
    """gemm() whose workspace configurations use the library's fixed device
    scratch array: never allocates; GEMM_E_WORKSPACE when the chosen
    configuration needs more than noalloc_scratch_bytes()."""
    set_stream(stream)
    rc = lib().gemm_noalloc(_tc(transA), _tc(transB), m, n, k, float(alpha), _ptr(A), lda,
                            _ptr(B), ldb, float(beta), _ptr(C), ldc, int(dtype))
    return _check(rc, "gemm_noalloc") if check else rc


def noalloc_scratch_bytes() -> int:
    """Size of gemm_noalloc's fixed device scratch array."""
    return int(lib().gemm_noalloc_scratch_bytes())


def gemm_scaled(transA: str, transB: str, m: int, n: int, k: int, alpha: float, A, lda: int, B,
                ldb: int, beta: float, C, ldc: int, dtype: int, stream: Any = None,
                check: bool = True) -> int:
    """Power-of-two scaled low-precision GEMM on FP32 A, B, C (dtype: the
    format the product runs in: GEMM_BF16, GEMM_F16 or GEMM_F8E4M3)."""
    set_stream(stream)
    rc = lib().gemm_scaled(_tc(transA), _tc(transB), m, n, k, float(alpha), _ptr(A), lda,
                           _ptr(B), ldb, float(beta), _ptr(C), ldc, int(dtype))
    return _check(rc, "gemm_scaled") if check else rc


@dataclass
class Problem:
    transA: str
    transB: str
    m: int
    n: int
    k: int
    alpha: float
    A: Any
    lda: int
    B: Any
    ldb: int
    beta: float
    C: Any
    ldc: int


def _problems(problems: Sequence[Problem]):
    arr = (_Problem * max(1, len(problems)))()
    for i, p in enumerate(problems):
        arr[i] = _Problem(_tc(p.transA), _tc(p.transB), p.m, p.n, p.k, float(p.alpha), _ptr(p.A),
                          p.lda, _ptr(p.B), p.ldb, float(p.beta), _ptr(p.C), p.ldc)
    return arr


class PackedProblems:
    """A problem list marshalled once into the C array gemm_grouped reads, for
    callers that launch the same list repeatedly."""

    def __init__(self, problems: Sequence[Problem]):
        self.count = len(problems)
        self.array = _problems(problems)
        self._keep = list(problems)


def gemm_grouped(problems, dtype: int, stream: Any = None, check: bool = True) -> int:
    """All problems (a sequence of Problem, or PackedProblems) in one
    persistent launch on the current (or given) stream."""
    set_stream(stream)
    if not isinstance(problems, PackedProblems):
        problems = PackedProblems(problems)
    rc = lib().gemm_grouped(problems.count, problems.array, int(dtype))
    return _check(rc, "gemm_grouped") if check else rc


def grouped_bodies_info(dtype: int) -> list:
    """The grouped compact kernel's tile bodies of the dtype's family:
    [{"mc", "nc", "pieces"}, ...]."""
    n = int(lib().gemm_grouped_num_bodies(int(dtype)))
    if n < 0:
        raise MGemmError(-1, "gemm_grouped_num_bodies")
    out = []
    for b in range(n):
        v = (_I64 * 3)()
        _check(lib().gemm_grouped_body_info(int(dtype), b, v), "gemm_grouped_body_info")
        out.append({"mc": int(v[0]), "nc": int(v[1]), "pieces": int(v[2])})
    return out


def grouped_force_body(body: int) -> None:
    """Pin this thread's grouped tables to one body (-1 clears)."""
    _check(lib().gemm_grouped_force_body(int(body)), "gemm_grouped_force_body")


def grouped_bodies(problems, dtype: int) -> list:
    """The body each problem would run (-1: none), without launching."""
    if not isinstance(problems, PackedProblems):
        problems = PackedProblems(problems)
    out = (_INT * max(1, problems.count))()
    _check(lib().gemm_grouped_bodies(problems.count, problems.array, int(dtype), out),
           "gemm_grouped_bodies")
    return [int(out[i]) for i in range(problems.count)]


def gemm_tune_grouped(dtype: int, shapes, reps: int = 5, out_path: Optional[str] = None) -> None:
    """Times every body on a batch of each shape; stores the fastest per bucket."""
    flat = (_I64 * max(1, 3 * len(shapes)))(*[int(v) for s in shapes for v in s])
    p = out_path.encode() if out_path else None
    _check(lib().gemm_tune_grouped(int(dtype), len(shapes), flat, int(reps), p),
           "gemm_tune_grouped")


def gemm_grouped_capacity() -> int:
    return int(lib().gemm_grouped_capacity())


class GroupedSlot:
    """A library-owned descriptor slot whose launch can be captured in a HIP graph."""

    def __init__(self, capacity: int = 1024):
        h = _P()
        _check(lib().gemm_grouped_slot_create(ctypes.byref(h), int(capacity)),
               "gemm_grouped_slot_create")
        self.handle = h
        self.capacity = int(capacity)

    def write(self, problems: Sequence[Problem], dtype: int, check: bool = True) -> int:
        rc = lib().gemm_grouped_slot_write(self.handle, len(problems), _problems(problems),
                                           int(dtype))
        return _check(rc, "gemm_grouped_slot_write") if check else rc

    def launch(self, stream: Any = None) -> None:
        set_stream(stream)
        _check(lib().gemm_grouped_slot_launch(self.handle), "gemm_grouped_slot_launch")

    def destroy(self) -> None:
        if self.handle:
            lib().gemm_grouped_slot_destroy(self.handle)
            self.handle = None


def gemm_init(tune_table_path: Optional[str] = None) -> None:
    p = tune_table_path.encode() if tune_table_path else None
    _check(lib().gemm_init(p), "gemm_init")


def gemm_shutdown() -> None:
    lib().gemm_shutdown()


def reserve_workspace(nbytes: int, scaled_bytes: int = 0, stream: Any = None) -> None:
    """Reserve workspace for the current (or given) stream: `nbytes` for gemm()'s
    packed split / split-K configurations, `scaled_bytes` for gemm_scaled()."""
    set_stream(stream)
    _check(lib().gemm_reserve_workspace(int(nbytes), int(scaled_bytes)), "gemm_reserve_workspace")


def release_workspace(stream: Any = None) -> None:
    """Synchronise the current (or given) stream and free its reservations."""
    set_stream(stream)
    _check(lib().gemm_release_workspace(), "gemm_release_workspace")


def workspace_bytes(transA: str, transB: str, m: int, n: int, k: int, dtype: int) -> int:
    """Workspace bytes the configuration gemm() picks for these sizes needs."""
    return int(lib().gemm_workspace_bytes(_tc(transA), _tc(transB), m, n, k, int(dtype)))


def scaled_workspace_bytes(transA: str, transB: str, m: int, n: int, k: int, beta: float,
                           dtype: int) -> int:
    return int(lib().gemm_scaled_workspace_bytes(_tc(transA), _tc(transB), m, n, k, float(beta),
                                                 int(dtype)))


def num_configs(dtype: int) -> int:
    return int(lib().gemm_num_configs(int(dtype)))


def config_info(dtype: int, cfg: int) -> dict:
    out = (_I64 * 8)()
    _check(lib().gemm_config_info(int(dtype), int(cfg), out), "gemm_config_info")
    keys = ("mc", "nc", "kc", "mr", "nr", "threads", "lds_bytes", "kind")
    info = dict(zip(keys, [int(v) for v in out]))
    st = int(lib().gemm_config_staging(int(dtype), int(cfg)))
    info["staging"] = (("registers", "direct", "packed", "a_unpacked", "b_unpacked", "unpacked",
                        "digit_planes")[st]
                       if st >= 0 else None)
    info["layouts"] = int(lib().gemm_config_layouts(int(dtype), int(cfg)))
    info["mfma"] = int(lib().gemm_config_mfma(int(dtype), int(cfg)))
    return info


def config_supports(dtype: int, cfg: int, transA: str, transB: str, vec: bool = True) -> bool:
    """Whether configuration `cfg` has a kernel for this layout and staging."""
    t = 2 * (transA in "TtCc") + (transB in "TtCc")
    return bool(config_info(dtype, cfg)["layouts"] >> (2 * t + (1 if vec else 0)) & 1)


def force_config(dtype: int, cfg: int, order: int = 0) -> None:
    _check(lib().gemm_force_config(int(dtype), int(cfg), int(order)), "gemm_force_config")


def debug_count(C, m: int, n: int, ldc: int, dtype: int) -> None:
    """Enqueue a count of the debug sentinel in the m x n block of C."""
    _check(lib().gemm_debug_count(_ptr(C), m, n, ldc, int(dtype)), "gemm_debug_count")


def debug_unwritten() -> int:
    """Sentinel elements counted on this device since the last call (resets it)."""
    v = int(lib().gemm_debug_unwritten())
    if v < 0:
        _check(-v, "gemm_debug_unwritten")
    return v


def last_config() -> dict:
    out = (_I64 * 4)()
    _check(lib().gemm_last_config(out), "gemm_last_config")
    return {"dtype": int(out[0]), "cfg": int(out[1]), "order": int(out[2]), "terms": int(out[3])}


def gemm_tune(dtype: int, shapes: Sequence[Sequence[int]], reps: int = 10,
              out_path: Optional[str] = None, model_keep: int = 0,
              layouts: Sequence[str] = ("NN", "NT", "TN", "TT")) -> None:
    """Times the configurations on each shape in each layout (only the model's
    first model_keep when > 0) and stores the fastest per (layout, size bucket)."""
    flat = (_I64 * max(1, 3 * len(shapes)))(*[int(v) for s in shapes for v in s])
    p = out_path.encode() if out_path else None
    mask = 0
    for lay in layouts:
        mask |= 1 << (2 * (lay[0] in "TtCc") + (lay[1] in "TtCc"))
    _check(lib().gemm_tune_layouts(int(dtype), len(shapes), flat, int(reps), p, int(model_keep),
                                   mask), "gemm_tune")


def model_us(dtype: int, cfg: int, m: int, n: int, k: int, cus: int = 256) -> float:
    """The analytical model's time (microseconds) of configuration cfg."""
    return float(lib().gemm_model_us(int(dtype), int(cfg), m, n, k, int(cus)))


def panel_occupancy(rows: int, cols: int, elem_bytes: int, capacity_bytes: int) -> float:
    return float(lib().gemm_panel_occupancy(rows, cols, elem_bytes, capacity_bytes))
