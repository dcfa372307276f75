"""Blocked GEMM family for AMD Instinct MI355X (gfx950).

Python binding of ``libmgemm.so`` (C ABI declared in ``include/mgemm.h``).
The binding only marshals arguments: every step of the computation runs in
the library's HIP kernels.  PyTorch supplies device memory and streams.
If the built library is missing the import of any entry point raises; there
is no CPU fallback.
"""
from ._binding import (  # noqa: F401
    GEMM_BF16, GEMM_F16, GEMM_F32, GEMM_F32_BF16X3, GEMM_F32_BF16X3_ONLY, GEMM_F32_BF16X6,
    GEMM_F64, GEMM_F8E4M3, GEMM_I8, GEMM_I16, GEMM_I32, GEMM_NUM_DTYPES, DTYPE_NAMES, MGemmError, Problem, config_info, config_supports,
    debug_count, debug_unwritten, force_config,
    gemm, gemm_noalloc, noalloc_scratch_bytes, gemm_scaled, gemm_tune_grouped,
    grouped_bodies, grouped_bodies_info, grouped_force_body, gemm_grouped, gemm_grouped_capacity, gemm_init, gemm_shutdown, gemm_tune,
    GroupedSlot, PackedProblems, last_config, lib, lib_path, model_us, num_configs,
    panel_occupancy, release_workspace, reserve_workspace, scaled_workspace_bytes,
    set_stream, strerror, workspace_bytes,
)
