"""Randomized complete pivoting (RCP) block LDL^T on AMD MI355X (gfx950).

Thin Python binding of the C ABI in ``include/rcp.h`` (librcp.so, built
in-tree by ``paper_1710_00125_amd.build``).  The functions carry the C names
and only marshal arguments: torch tensors on the GPU supply device memory and
the current torch stream is handed to the library; every step of the
factorization, the solve and the refinement runs in the library's HIP
kernels.  There is no fallback: if librcp.so is missing or no GPU is present
the calls raise.
"""

from ._binding import (RCP_EABORT, RCP_ENOCONV, RCP_NOALLOC_MAX_N, RCP_PREC_BF16S, RCP_PREC_BF16X3,
                       RCP_PREC_FP64, RCP_PREC_FP32, RCPError, Batch,
                       Factors, exported_symbols, lib_path, load, pack_batch, rcp_batch_create,
                       rcp_batch_get_table, rcp_batch_set_table, rcp_factor, rcp_factor_ex, rcp_factor_mp, rcp_factor_q,
                       rcp_get_stats, rcp_launch_shape, rcp_omega, rcp_release,
                       rcp_set_grid_limit, rcp_set_overlap, rcp_set_profiling,
                       rcp_set_speculation, rcp_set_recompute,
                       rcp_set_stream,
                       rcp_solve, rcp_solve_ir, rcp_solve_mp, rcp_solve_noalloc)

__all__ = ["RCP_EABORT", "RCP_ENOCONV", "RCP_NOALLOC_MAX_N", "RCP_PREC_BF16S", "RCP_PREC_BF16X3",
           "RCP_PREC_FP64", "RCP_PREC_FP32", "RCPError", "Batch",
           "Factors", "exported_symbols", "lib_path", "load", "pack_batch", "rcp_batch_create",
           "rcp_batch_get_table", "rcp_batch_set_table", "rcp_factor", "rcp_factor_ex", "rcp_factor_mp", "rcp_factor_q",
           "rcp_get_stats", "rcp_launch_shape", "rcp_omega", "rcp_release", "rcp_set_grid_limit",
           "rcp_set_overlap", "rcp_set_profiling", "rcp_set_speculation", "rcp_set_recompute", "rcp_set_stream", "rcp_solve", "rcp_solve_ir",
           "rcp_solve_mp", "rcp_solve_noalloc"]
