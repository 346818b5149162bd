"""CPU checks of the C ABI library: it loads, and it exports every entry
point that include/rcp.h declares (no compute calls without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rcp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\bint\s+(rcp_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("rcp_factor", "rcp_solve", "rcp_omega", "rcp_set_stream",
                     "rcp_get_stats", "rcp_set_profiling", "rcp_release"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1710_00125_amd as pkg
    path = pkg.lib_path()
    if not os.path.exists(path):
        pytest.skip("librcp.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert all(pkg.exported_symbols().values())


def test_argument_errors_without_gpu():
    # argument validation happens before any device call
    import paper_1710_00125_amd as pkg
    if not os.path.exists(pkg.lib_path()):
        pytest.skip("librcp.so not built")
    lib = pkg.load()
    null = ctypes.c_void_p(0)
    one = ctypes.c_void_p(8)   # never dereferenced: validation fails first
    assert lib.rcp_factor(-1, null, 1, 4, 2, 0, null, null, null, null) == -1
    assert lib.rcp_factor(4, null, 4, 4, 2, 0, one, one, one, one) == -2
    assert lib.rcp_factor(4, one, 3, 4, 2, 0, one, one, one, one) == -3
    assert lib.rcp_factor(4, one, 4, 0, 2, 0, one, one, one, one) == -4
    assert lib.rcp_factor(4, one, 4, 4, -1, 0, one, one, one, one) == -5
    assert lib.rcp_factor(4, one, 4, 4, 2, 0, null, one, one, one) == -7
    assert lib.rcp_factor(4, one, 4, 4, 2, 0, one, null, one, one) == -8
    assert lib.rcp_factor(4, one, 4, 4, 2, 0, one, one, null, one) == -9
    assert lib.rcp_factor(4, one, 4, 4, 2, 0, one, one, one, null) == -10
    assert lib.rcp_factor(0, null, 1, 4, 2, 0, null, null, null, null) == 0
    assert lib.rcp_solve(-1, null, null, null, null, 1, null, 1) == -1
    assert lib.rcp_solve(4, one, one, one, one, 1, one, 3) == -8
    assert lib.rcp_solve(4, one, one, one, one, -1, one, 4) == -6
    assert lib.rcp_solve(0, null, null, null, null, 1, null, 1) == 0
    assert lib.rcp_solve_noalloc(-1, null, null, null, null, 1, null, 1) == -1
    assert lib.rcp_solve_noalloc(4, one, one, one, one, 1, one, 3) == -8
    big = pkg.RCP_NOALLOC_MAX_N + 1   # beyond the fixed scratch array
    assert lib.rcp_solve_noalloc(big, one, one, one, one, 1, one, big) == -1003
    assert lib.rcp_solve_noalloc(0, null, null, null, null, 1, null, 1) == 0
    assert lib.rcp_omega(0, -1, 4, null) == -2
    assert lib.rcp_omega(0, 2, -4, null) == -3
    assert lib.rcp_omega(0, 2, 4, null) == -4


def test_mixed_precision_argument_errors_without_gpu():
    import paper_1710_00125_amd as pkg
    if not os.path.exists(pkg.lib_path()):
        pytest.skip("librcp.so not built")
    lib = pkg.load()
    null = ctypes.c_void_p(0)
    one = ctypes.c_void_p(8)
    f = lib.rcp_factor_mp
    assert f(-1, null, 1, 4, 2, 0, 1, null, null, null, null) == -1
    assert f(4, one, 3, 4, 2, 0, 1, one, one, one, one) == -3
    assert f(4, one, 4, 4, 2, 0, 0, one, one, one, one) == -7
    assert f(4, one, 4, 4, 2, 0, 3, one, one, one, one) == -7
    assert f(4, one, 4, 4, 2, 0, 2, null, one, one, one) == -8
    assert f(4, one, 4, 4, 2, 0, 2, one, one, one, null) == -11
    assert f(0, null, 1, 4, 2, 0, 1, null, null, null, null) == 0
    assert lib.rcp_solve_mp(4, one, one, one, one, 1, one, 3) == -8
    ir = lib.rcp_solve_ir
    args = [4, one, 4, one, one, one, one, 1, one, 4, one, 4, 1e-13, 5, 20, None]
    for pos, val, code in [(0, -1, -1), (2, 3, -3), (7, -1, -8), (9, 3, -10), (11, 3, -12),
                           (12, 0.0, -13), (13, 0, -14), (14, 0, -15), (14, 65, -15)]:
        a = list(args)
        a[pos] = val
        assert ir(*a) == code, (pos, val)
    a = list(args)
    a[0] = 0
    assert ir(*a) == 0


def test_batch_table_set_and_get_without_gpu():
    # the block-size table is host state: set, read back, reject bad entries
    import paper_1710_00125_amd as pkg
    if not os.path.exists(pkg.lib_path()):
        pytest.skip("librcp.so not built")
    lib = pkg.load()
    saved = pkg.rcp_batch_get_table(0)
    try:
        pkg.rcp_batch_set_table([8, 16, 24, 32], 0)
        assert pkg.rcp_batch_get_table(0) == [8, 16, 24, 32]
        bad = (ctypes.c_int32 * 4)(8, 0, 16, 16)
        assert lib.rcp_batch_set_table(0, bad) == -2
        too_big = (ctypes.c_int32 * 4)(8, 16, 16, 33)
        assert lib.rcp_batch_set_table(0, too_big) == -2
        assert lib.rcp_batch_set_table(7, bad) == -1
        assert lib.rcp_batch_set_table(0, ctypes.POINTER(ctypes.c_int32)()) == -2
        assert pkg.rcp_batch_get_table(0) == [8, 16, 24, 32]   # unchanged by rejected calls
    finally:
        pkg.rcp_batch_set_table(saved, 0)


def test_column_major_view_is_passed_without_copy():
    # the binding hands the library a transposed view's own memory and
    # copies anything else (host logic only; CPU tensors)
    import torch
    from paper_1710_00125_amd._binding import _colmajor
    X = torch.arange(12.0, dtype=torch.float64).reshape(3, 4)
    view = X.t()                           # 4 x 3, its transpose is X
    cm = _colmajor(view)
    assert cm.data_ptr() == X.data_ptr()   # no copy
    assert torch.equal(cm.t(), view)
    row_major = torch.arange(9.0, dtype=torch.float64).reshape(3, 3)
    cm2 = _colmajor(row_major)
    assert cm2.data_ptr() != row_major.data_ptr() and cm2.is_contiguous()
    assert torch.equal(cm2.t(), row_major)    # memory[i + j n] = A[i, j]


def test_launch_shape_dispatch_without_gpu():
    # which selection kernel and grid each shape gets (host logic only)
    import paper_1710_00125_amd as pkg
    if not os.path.exists(pkg.lib_path()):
        pytest.skip("librcp.so not built")
    sh = pkg.rcp_launch_shape(16384, 128, 16, 256)
    assert (sh["select_grid"], sh["select_cols"], sh["select_regs"]) == (256, 64, 1)
    assert (sh["panel_grid"], sh["panel_rows"], sh["supported"]) == (256, 64, 1)
    # the selection takes 64 columns per workgroup wherever the grid allows:
    # 9000 gives 141 workgroups of 64 (the last one 40), 2000 gives 32 of 63
    # (the last 47)
    sh = pkg.rcp_launch_shape(9000, 128, 16, 256)
    assert (sh["select_grid"], sh["select_cols"], sh["select_regs"]) == (141, 64, 1)
    sh = pkg.rcp_launch_shape(2000, 128, 16, 256)
    assert (sh["select_grid"], sh["select_cols"]) == (32, 63)
    # the q = b panel takes 32 rows per workgroup below the full grid
    assert (sh["panel_grid"], sh["panel_rows"]) == (63, 32)
    # one more column than the register slab holds, or a taller sketch: LDS
    assert pkg.rcp_launch_shape(16385, 128, 16, 256)["select_regs"] == 0
    assert pkg.rcp_launch_shape(1300, 128, 24, 256)["select_regs"] == 0
    assert pkg.rcp_launch_shape(1300, 128, 16, 256)["select_regs"] == 1
    # the LDS budget bounds the order
    assert pkg.rcp_launch_shape(20000, 128, 16, 256)["supported"] == 1
    assert pkg.rcp_launch_shape(30000, 128, 16, 256)["supported"] == 0
    assert pkg.rcp_launch_shape(16384, 128, 200, 256)["supported"] == 0
    # grid limits give the large per-workgroup shapes at small orders
    try:
        pkg.rcp_set_grid_limit(32, 32)
        sh = pkg.rcp_launch_shape(2048, 128, 16, 256)
        assert (sh["select_grid"], sh["select_cols"], sh["select_regs"]) == (32, 64, 1)
        assert (sh["panel_grid"], sh["panel_rows"]) == (32, 64)
        pkg.rcp_set_grid_limit(24, 0)
        sh = pkg.rcp_launch_shape(2048, 128, 16, 256)
        assert (sh["select_cols"], sh["select_regs"], sh["supported"]) == (86, 0, 1)
        pkg.rcp_set_grid_limit(8, 8)
        assert pkg.rcp_launch_shape(2048, 128, 16, 256)["supported"] == 0
    finally:
        pkg.rcp_set_grid_limit(0, 0)
    lib = pkg.load()
    info = pkg._binding._LaunchInfo()
    assert lib.rcp_launch_shape(0, 128, 16, 256, ctypes.byref(info)) == -1
    assert lib.rcp_launch_shape(16, 129, 16, 256, ctypes.byref(info)) == -2
    assert lib.rcp_launch_shape(16, 128, 385, 256, ctypes.byref(info)) == -3
    assert lib.rcp_launch_shape(16, 128, 16, 0, ctypes.byref(info)) == -4
    assert lib.rcp_launch_shape(16, 128, 16, 256, None) == -5
    assert lib.rcp_set_grid_limit(-1, 0) == -1 and lib.rcp_set_grid_limit(0, -1) == -2


def test_release_without_device_work():
    # nothing allocated yet: releasing is a no-op and may be repeated
    import paper_1710_00125_amd as pkg
    if not os.path.exists(pkg.lib_path()):
        pytest.skip("librcp.so not built")
    assert pkg.rcp_release() == 0
    assert pkg.rcp_release() == 0


def test_mode_setters_validate_without_gpu():
    # pure setters: no device call; an unknown mode is refused and changes
    # nothing
    import paper_1710_00125_amd as pkg
    if not os.path.exists(pkg.lib_path()):
        pytest.skip("librcp.so not built")
    lib = pkg.load()
    for bad in (-1, 3):
        assert lib.rcp_set_profiling(bad) == -1
    for good in (1, 2, 0):
        assert lib.rcp_set_profiling(good) == 0
    for bad in (-2, 2):
        assert lib.rcp_set_speculation(bad) == -1
    for good in (0, 1, -1):
        assert lib.rcp_set_speculation(good) == 0
    with pytest.raises(ValueError):
        pkg.rcp_set_profiling(5)
    pkg.rcp_set_profiling(False)
