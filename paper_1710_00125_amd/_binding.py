"""ctypes marshalling for librcp.so (see include/rcp.h for the contract)."""

import atexit
import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

RCP_ENONFINITE = -1000
RCP_EDEVICE = -1001
RCP_ENOMEM = -1002
RCP_EUNSUPPORTED = -1003
RCP_ENOCONV = -1004
RCP_EABORT = -1005
RCP_PREC_FP64 = 0
RCP_PREC_FP32 = 1
RCP_PREC_BF16X3 = 2
RCP_PREC_BF16S = 3
RCP_NOALLOC_MAX_N = 16384


class RCPError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} returned {code}")
        self.code = code


class _Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nblocks", ctypes.c_int64), ("n2x2", ctypes.c_int64),
                ("ncase", ctypes.c_int64 * 4), ("ms_total", ctypes.c_double),
                ("ms_omega", ctypes.c_double), ("ms_sketch", ctypes.c_double),
                ("ms_select", ctypes.c_double), ("ms_panel", ctypes.c_double),
                ("ms_sketch_update", ctypes.c_double), ("ms_commit", ctypes.c_double),
                ("ms_update", ctypes.c_double), ("ms_finalize", ctypes.c_double),
                ("ms_solve", ctypes.c_double), ("launches_update", ctypes.c_int64),
                ("flops_update", ctypes.c_double), ("bytes_update", ctypes.c_double),
                ("max_abs_a", ctypes.c_double), ("max_abs_l", ctypes.c_double),
                ("max_abs_d", ctypes.c_double), ("rho_d", ctypes.c_double),
                ("min_margin", ctypes.c_double), ("near_ties", ctypes.c_int64),
                ("recomputes", ctypes.c_int64), ("rank", ctypes.c_int64)]


class _LaunchInfo(ctypes.Structure):
    _fields_ = [("select_grid", ctypes.c_int32), ("select_cols", ctypes.c_int32),
                ("select_regs", ctypes.c_int32), ("panel_grid", ctypes.c_int32),
                ("panel_rows", ctypes.c_int32), ("panel_lds", ctypes.c_int64),
                ("select_lds", ctypes.c_int64), ("supported", ctypes.c_int32)]


class _IrResult(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int32), ("inner", ctypes.c_int32), ("berr", ctypes.c_double),
                ("ms", ctypes.c_double)]


class _BatchInfo(ctypes.Structure):
    _fields_ = [("b", ctypes.c_int32), ("info", ctypes.c_int32), ("ir_iters", ctypes.c_int32),
                ("n2x2", ctypes.c_int32), ("berr", ctypes.c_double)]


_SIGS = {
    "rcp_set_stream": (ctypes.c_int, [ctypes.c_void_p]),
    "rcp_set_profiling": (ctypes.c_int, [ctypes.c_int32]),
    "rcp_set_overlap": (ctypes.c_int, [ctypes.c_int32]),
    "rcp_set_speculation": (ctypes.c_int, [ctypes.c_int32]),
    "rcp_set_recompute": (ctypes.c_int, [ctypes.c_int32]),
    "rcp_get_stats": (ctypes.c_int, [ctypes.POINTER(_Stats)]),
    "rcp_release": (ctypes.c_int, []),
    "rcp_set_grid_limit": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32]),
    "rcp_launch_shape": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.POINTER(_LaunchInfo)]),
    "rcp_omega": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_void_p]),
    "rcp_factor": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "rcp_factor_ex": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rcp_solve_ir64": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(_IrResult)]),
    "rcp_factor_q": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                    ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]),
    "rcp_solve": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_int64]),
    "rcp_solve_noalloc": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_void_p, ctypes.c_int64]),
    "rcp_factor_mp": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "rcp_solve_mp": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.c_int64]),
    "rcp_solve_ir": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(_IrResult)]),
    "rcp_batch_create": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "rcp_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "rcp_batch_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_BatchInfo)]),
    "rcp_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rcp_batch_get_table": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "rcp_batch_set_table": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
}


def lib_path():
    return os.path.join(_HERE, "librcp.so")


def load():
    """Load librcp.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        path = lib_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with "
                               "`python -m paper_1710_00125_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _LIB = lib
        # free the library's device resources before the interpreter (and
        # with it torch and the HIP runtime) shuts down
        atexit.register(_release_at_exit)
    return _LIB


def _release_at_exit():
    if _LIB is not None:
        try:
            _LIB.rcp_release()
        except Exception:
            pass


def exported_symbols():
    """Names of the C entry points the binding expects (all must resolve)."""
    lib = load()
    return {name: hasattr(lib, name) for name in _SIGS}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("librcp needs a GPU: torch.cuda.is_available() is False")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _check(fn, code, ok_positive=False):
    if code < 0 or (code > 0 and not ok_positive):
        raise RCPError(fn, code)
    return code


def rcp_set_stream(stream=None):
    """Hand a HIP stream (torch.cuda.Stream or raw handle) to the library."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    return load().rcp_set_stream(ctypes.c_void_p(handle))


def rcp_set_profiling(mode):
    """mode 1 (or True): time every kernel launch, 2: the trailing update's
    launches only, 0 (or False): none."""
    rc = load().rcp_set_profiling(int(mode))
    if rc != 0:
        raise ValueError(f"rcp_set_profiling: mode {mode} is not 0, 1 or 2")
    return rc


def rcp_set_overlap(on):
    return load().rcp_set_overlap(1 if on else 0)


def rcp_set_speculation(mode):
    """mode 1: speculate in the SBKP panels whenever the shape allows, 0: never,
    -1: the measured rule (the default)."""
    rc = load().rcp_set_speculation(int(mode))
    if rc != 0:
        raise ValueError(f"rcp_set_speculation: mode {mode} is not -1, 0 or 1")
    return rc


def rcp_set_recompute(r=1):
    """Algorithm 2 with recompute budget r for later factorizations (1 =
    Algorithm 1)."""
    _check("rcp_set_recompute", load().rcp_set_recompute(int(r)))


def rcp_release():
    return load().rcp_release()


def rcp_set_grid_limit(select_max=0, panel_max=0):
    """Bound the persistent selection / panel grids (0: one workgroup per CU)."""
    return _check("rcp_set_grid_limit",
                  load().rcp_set_grid_limit(int(select_max), int(panel_max)))


def rcp_launch_shape(n, b, p, num_cu=256):
    """Launch shape of the first block (host-only query), as a dict."""
    info = _LaunchInfo()
    _check("rcp_launch_shape", load().rcp_launch_shape(int(n), int(b), int(p), int(num_cu),
                                                       ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in _LaunchInfo._fields_}


def rcp_get_stats():
    st = _Stats()
    load().rcp_get_stats(ctypes.byref(st))
    out = {name: getattr(st, name) for name, _ in _Stats._fields_}
    out["ncase"] = list(st.ncase)
    return out


def rcp_omega(seed, l, n, device="cuda"):
    """Omega (l x n, row-major) as the factorization draws it for ``seed``."""
    torch = _torch()
    out = torch.empty((l, n), dtype=torch.float64, device=device)
    rcp_set_stream()
    _check("rcp_omega", load().rcp_omega(ctypes.c_uint64(seed & (2**64 - 1)), l, n, _ptr(out)))
    return out


@dataclass
class Factors:
    n: int
    perm: object     # int64[n]
    L: object        # n x n (logical view; storage is column-major), float64 or float32
    D: object        # float64[2n]
    ipiv: object     # int8[n]
    info: int
    precision: int = 0   # 0 = FP64, RCP_PREC_FP32, RCP_PREC_BF16X3


def _colmajor(A):
    """The column-major storage of A (memory[i + j n] = A[i, j]): A's own
    memory when A is a transposed view of a contiguous tensor, else a copy."""
    At = A.t()
    return At if At.is_contiguous() else At.contiguous()


def rcp_factor(A, b, p, seed):
    """P A P^T = L D L^T of the symmetric matrix whose lower triangle is A's.

    A: (n, n) float64 tensor on the GPU (logical indexing A[i, j]).
    Returns Factors; info > 0 flags an exactly zero 1x1 pivot.
    """
    torch = _torch()
    n = A.shape[0]
    assert A.dim() == 2 and A.shape[1] == n and A.dtype == torch.float64 and A.is_cuda
    Acm = _colmajor(A)                         # memory[i + j n] = A[i, j] (read only)
    dev = A.device
    perm = torch.empty(n, dtype=torch.int64, device=dev)
    Lbuf = torch.empty((n, n), dtype=torch.float64, device=dev)
    D = torch.empty(2 * n, dtype=torch.float64, device=dev)
    ipiv = torch.empty(n, dtype=torch.int8, device=dev)
    rcp_set_stream()
    info = load().rcp_factor(n, _ptr(Acm), max(1, n), int(b), int(p),
                             ctypes.c_uint64(int(seed) & (2**64 - 1)), _ptr(perm), _ptr(Lbuf),
                             _ptr(D), _ptr(ipiv))
    _check("rcp_factor", info, ok_positive=True)
    return Factors(n, perm, Lbuf.t(), D, ipiv, info)


def rcp_factor_q(A, b, p, seed, q):
    """rcp_factor with q pivots per sketch: q = b as rcp_factor, q = 1 one
    sketch argmax per step (sketch of 1 + p rows)."""
    torch = _torch()
    n = A.shape[0]
    assert A.dim() == 2 and A.shape[1] == n and A.dtype == torch.float64 and A.is_cuda
    Acm = _colmajor(A)
    dev = A.device
    perm = torch.empty(n, dtype=torch.int64, device=dev)
    Lbuf = torch.empty((n, n), dtype=torch.float64, device=dev)
    D = torch.empty(2 * n, dtype=torch.float64, device=dev)
    ipiv = torch.empty(n, dtype=torch.int8, device=dev)
    rcp_set_stream()
    info = load().rcp_factor_q(n, _ptr(Acm), max(1, n), int(b), int(p),
                               ctypes.c_uint64(int(seed) & (2**64 - 1)), int(q), _ptr(perm),
                               _ptr(Lbuf), _ptr(D), _ptr(ipiv))
    _check("rcp_factor_q", info, ok_positive=True)
    return Factors(n, perm, Lbuf.t(), D, ipiv, info)


def rcp_factor_ex(A, b, p, seed, q=None, precision=RCP_PREC_FP64):
    """The general factorization: q pivots per sketch (None = b) in a working
    precision (RCP_PREC_*); L is float64 for FP64 and BF16S, else float32."""
    torch = _torch()
    n = A.shape[0]
    assert A.dim() == 2 and A.shape[1] == n and A.dtype == torch.float64 and A.is_cuda
    Acm = _colmajor(A)
    dev = A.device
    ldt = torch.float64 if precision in (RCP_PREC_FP64, RCP_PREC_BF16S) else torch.float32
    perm = torch.empty(n, dtype=torch.int64, device=dev)
    Lbuf = torch.empty((n, n), dtype=ldt, device=dev)
    D = torch.empty(2 * n, dtype=torch.float64, device=dev)
    ipiv = torch.empty(n, dtype=torch.int8, device=dev)
    rcp_set_stream()
    info = load().rcp_factor_ex(n, _ptr(Acm), max(1, n), int(b), int(p),
                                ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                int(b if q is None else q), int(precision), _ptr(perm),
                                _ptr(Lbuf), _ptr(D), _ptr(ipiv))
    _check("rcp_factor_ex", info, ok_positive=True)
    return Factors(n, perm, Lbuf.t(), D, ipiv, info, int(precision))


def rcp_factor_mp(A, b, p, seed, precision=RCP_PREC_FP32):
    """Reduced-precision factorization (FP32 or BF16x3 update); L is float32."""
    torch = _torch()
    n = A.shape[0]
    assert A.dim() == 2 and A.shape[1] == n and A.dtype == torch.float64 and A.is_cuda
    Acm = _colmajor(A)
    dev = A.device
    perm = torch.empty(n, dtype=torch.int64, device=dev)
    Lbuf = torch.empty((n, n), dtype=torch.float32, device=dev)
    D = torch.empty(2 * n, dtype=torch.float64, device=dev)
    ipiv = torch.empty(n, dtype=torch.int8, device=dev)
    rcp_set_stream()
    info = load().rcp_factor_mp(n, _ptr(Acm), max(1, n), int(b), int(p),
                                ctypes.c_uint64(int(seed) & (2**64 - 1)), int(precision),
                                _ptr(perm), _ptr(Lbuf), _ptr(D), _ptr(ipiv))
    _check("rcp_factor_mp", info, ok_positive=True)
    return Factors(n, perm, Lbuf.t(), D, ipiv, info, int(precision))


def _rhs_cm(B):
    """(column-major n x nrhs buffer, vec flag): always a fresh copy so that
    the caller's B is never overwritten (B.t().contiguous() can alias B)."""
    torch = _torch()
    vec = B.dim() == 1
    Bm = B[:, None] if vec else B
    n, nrhs = Bm.shape
    Bcm = torch.empty((nrhs, n), dtype=torch.float64, device=Bm.device)
    Bcm.copy_(Bm.t())
    return Bcm, vec


def rcp_solve(f, B):
    """X with A X = B from the factors of rcp_factor or rcp_factor_mp;
    B is (n,) or (n, nrhs), float64."""
    torch = _torch()
    Bcm, vec = _rhs_cm(B)
    nrhs, n = Bcm.shape
    Lcm = f.L.t()                              # the column-major storage itself
    assert Lcm.is_contiguous()
    rcp_set_stream()
    fn = "rcp_solve_mp" if f.L.dtype != torch.float64 else "rcp_solve"
    code = getattr(load(), fn)(n, _ptr(Lcm), _ptr(f.D), _ptr(f.ipiv), _ptr(f.perm), nrhs,
                               _ptr(Bcm), max(1, n))
    _check(fn, code)
    X = Bcm.t()
    return X[:, 0] if vec else X


def rcp_solve_noalloc(f, B):
    """rcp_solve on the library's fixed scratch array (no device allocation
    inside the call; FP64 factors of rcp_factor, n <= RCP_NOALLOC_MAX_N).
    The right-hand sides are copied into a fresh column-major tensor here,
    as in rcp_solve; a caller that must not allocate at all calls the C entry
    point directly on buffers it already holds."""
    assert not f.precision, "rcp_solve_noalloc takes the FP64 factors of rcp_factor"
    Bcm, vec = _rhs_cm(B)
    nrhs, n = Bcm.shape
    Lcm = f.L.t()
    assert Lcm.is_contiguous()
    rcp_set_stream()
    code = load().rcp_solve_noalloc(n, _ptr(Lcm), _ptr(f.D), _ptr(f.ipiv), _ptr(f.perm), nrhs,
                                    _ptr(Bcm), max(1, n))
    _check("rcp_solve_noalloc", code)
    X = Bcm.t()
    return X[:, 0] if vec else X


def rcp_solve_mp(f, B):
    """rcp_solve for the float32 factors of rcp_factor_mp."""
    assert f.precision, "rcp_solve_mp needs the factors of rcp_factor_mp"
    return rcp_solve(f, B)


def rcp_solve_ir(A, f, B, tol=1e-13, max_outer=10, restart=30, raise_on_noconv=True):
    """FP64 solution of A X = B by GMRES-based refinement preconditioned by the
    reduced-precision factors f.  Returns (X, info dict)."""
    torch = _torch()
    n = A.shape[0]
    Acm = _colmajor(A)
    Bcm, vec = _rhs_cm(B)
    nrhs = Bcm.shape[0]
    Xcm = torch.empty_like(Bcm)
    Lcm = f.L.t()
    assert Lcm.is_contiguous()
    res = _IrResult()
    rcp_set_stream()
    fn = "rcp_solve_ir" if f.L.dtype == torch.float32 else "rcp_solve_ir64"
    code = getattr(load(), fn)(n, _ptr(Acm), max(1, n), _ptr(Lcm), _ptr(f.D), _ptr(f.ipiv),
                               _ptr(f.perm), nrhs, _ptr(Bcm), max(1, n), _ptr(Xcm), max(1, n),
                               float(tol), int(max_outer), int(restart), ctypes.byref(res))
    info = {"outer": res.outer, "inner": res.inner, "berr": res.berr, "ms": res.ms,
            "converged": code == 0}
    if code != RCP_ENOCONV or raise_on_noconv:
        _check(fn, code)
    X = Xcm.t()
    return (X[:, 0] if vec else X), info


# ---------------------------------------------------------------------------
# batched systems


def pack_batch(systems, nrhs, device="cuda"):
    """Pools for rcp_batch_create from a list of (A (n x n), B (n x nrhs))
    host arrays: column-major blocks laid end to end (see include/rcp.h)."""
    import numpy as np
    torch = _torch()
    ns = np.array([A.shape[0] for A, _ in systems], dtype=np.int32)
    a = np.concatenate([np.asarray(A, dtype=np.float64).T.ravel() for A, _ in systems])
    b = np.concatenate([np.asarray(B, dtype=np.float64).reshape(A.shape[0], nrhs).T.ravel()
                        for A, B in systems])
    return (ns, torch.from_numpy(a).to(device), torch.from_numpy(b).to(device))


class Batch:
    """A captured batch plan (rcp_batch_create); run() replays its graph."""

    def __init__(self, ns, Apool, Bpool, p, seed0, precision=0, nrhs=1, factors=False,
                 autotune=True):
        import numpy as np
        torch = _torch()
        self.ns = np.ascontiguousarray(ns, dtype=np.int32)
        self.count = len(self.ns)
        self.nrhs = nrhs
        self.precision = int(precision)
        dev = Apool.device
        n1 = int(self.ns.sum())
        self.Apool, self.Bpool = Apool, Bpool
        self.Xpool = torch.zeros(n1 * nrhs, dtype=torch.float64, device=dev)
        self.perm = self.L = self.D = self.ipiv = None
        if factors:
            n2 = int((self.ns.astype(np.int64) ** 2).sum())
            self.perm = torch.empty(n1, dtype=torch.int64, device=dev)
            self.L = torch.empty(n2, dtype=torch.float32 if precision else torch.float64,
                                 device=dev)
            self.D = torch.empty(2 * n1, dtype=torch.float64, device=dev)
            self.ipiv = torch.empty(n1, dtype=torch.int8, device=dev)
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        code = load().rcp_batch_create(
            self.count, self.ns.ctypes.data_as(ctypes.c_void_p), int(p),
            ctypes.c_uint64(int(seed0) & (2**64 - 1)), int(precision), int(nrhs),
            _ptr(Apool), _ptr(Bpool), _ptr(self.Xpool), _ptr(self.perm), _ptr(self.L),
            _ptr(self.D), _ptr(self.ipiv), 1 if autotune else 0, ctypes.byref(h))
        _check("rcp_batch_create", code)
        self._h = h

    def run(self):
        """Replay the captured launch once; returns its duration in ms."""
        ms = ctypes.c_float()
        _check("rcp_batch_run", load().rcp_batch_run(self._h, ctypes.byref(ms)))
        return ms.value

    def info(self):
        arr = (_BatchInfo * max(1, self.count))()
        _check("rcp_batch_get_info", load().rcp_batch_get_info(self._h, arr))
        return [{"b": r.b, "info": r.info, "ir_iters": r.ir_iters, "n2x2": r.n2x2,
                 "berr": r.berr} for r in arr[:self.count]]

    def close(self):
        if getattr(self, "_h", None):
            load().rcp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rcp_batch_create(ns, Apool, Bpool, p, seed0, precision=0, nrhs=1, factors=False,
                     autotune=True):
    return Batch(ns, Apool, Bpool, p, seed0, precision, nrhs, factors, autotune)


def rcp_batch_get_table(precision=0):
    arr = (ctypes.c_int32 * 4)()
    _check("rcp_batch_get_table", load().rcp_batch_get_table(int(precision), arr))
    return list(arr)


def rcp_batch_set_table(b_by_class, precision=0):
    """Block size per size class (n <= 64, 128, 256, 512) for plans created
    afterwards without autotuning."""
    arr = (ctypes.c_int32 * 4)(*[int(b) for b in b_by_class])
    _check("rcp_batch_set_table", load().rcp_batch_set_table(int(precision), arr))
