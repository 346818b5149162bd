"""GPU: the sliced-BF16 working precision (RCP_PREC_BF16S) and FP64 GMRES
refinement with its double L (rcp_solve_ir64), through the C ABI.

The trailing update multiplies 8-bit slices of the operand rows on the BF16
matrix cores, each slice-pair product exact in FP32 accumulation; the
products it leaves out are below about u_s = 2^-45 of the row maxima per
term, and storage stays FP64.  As for the other reduced forms the method's
decisions are unchanged and a refined run is judged on its solution:
  * the factors are a valid block LDL^T with reconstruction error
    <= 20 n u_s;
  * they agree with rcp_factor's FP64 factors of the same matrix: the same
    pivots (reported) and, where the pivots agree, L and D within
    1e3 n u_s max(1, |FP64 value|) (column-scaled like the other tests);
  * rcp_solve_ir64 reaches backward error <= 1e-13 at every condition
    number of the benchmark sweep, 1e10 included, and the solution lies
    within kappa_inf * 1e-12 of the FP64 oracle's.
"""

import sys

import numpy as np
import pytest

from oracle import rcp as orcp, textbook as tb
from workloads import gen

pytestmark = pytest.mark.gpu

U_S = 2.0 ** -45


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rcp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1710_00125_amd as pkg
    pkg.load()
    return pkg


def _dmat(D, ipiv):
    n = len(ipiv)
    Dm = np.diag(D[:n].copy())
    for i in np.nonzero(ipiv == 2)[0]:
        Dm[i + 1, i] = Dm[i, i + 1] = D[n + i]
    return Dm


CASES = [
    ("gaussian", 512, 32, 8, 1, 1e6),
    ("kkt", 400, 64, 10, 2, 1e6),
    ("householder", 1000, 64, 10, 41, 1e2),
    ("householder", 1000, 64, 10, 42, 1e6),
    ("householder", 1000, 64, 10, 43, 1e10),
    ("householder", 1500, 128, 16, 45, 1e10),
]


@pytest.mark.parametrize("kind,n,b,p,seed,cond", CASES)
def test_sliced_factor_and_refine(rcp, kind, n, b, p, seed, cond):
    import torch
    _say(f"sliced {kind} n={n} b={b} p={p} seed={seed} cond={cond:g}")
    if kind == "gaussian":
        A = gen.gaussian_sym(n, seed)
    elif kind == "kkt":
        A = gen.kkt(n, (3 * n) // 4, seed, nrefl=min(64, (3 * n) // 4))
    else:
        A = gen.householder_spectrum(n, seed, cond=cond, nrefl=64)
    nrhs = 4 if kind == "kkt" else 1
    rhs = gen.rhs(n, nrhs, seed)
    Ad = torch.from_numpy(A).cuda()
    f = rcp.rcp_factor_ex(Ad, b, p, seed, precision=rcp.RCP_PREC_BF16S)
    g = rcp.rcp_factor(Ad, b, p, seed)
    assert f.info == 0 and f.L.dtype == torch.float64
    perm, ipiv = f.perm.cpu().numpy(), f.ipiv.cpu().numpy()
    L, D = f.L.cpu().numpy(), f.D.cpu().numpy()
    pg, ig = g.perm.cpu().numpy(), g.ipiv.cpu().numpy()
    Lg, Dg = g.L.cpu().numpy(), g.D.cpu().numpy()
    rec = tb.reconstruction_error(A, perm, L, _dmat(D, ipiv))
    pd = np.nonzero(perm != pg)[0]
    idf = np.nonzero(ipiv != ig)[0]
    m = min(int(pd[0]) if pd.size else n, int(idf[0]) if idf.size else n)
    _say(f"  reconstruction {rec:.3e}; pivots agree with FP64 up to {m} of {n}")
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert rec <= 20 * n * U_S
    amax = np.max(np.abs(A))
    dk = np.abs(Dg[:n]) + np.abs(Dg[n:])
    dk = np.maximum(dk, np.roll(dk * (ig == 2), 1))
    colscale = np.maximum(1.0, amax / np.maximum(dk, 1e-300))[None, :m]
    tol = 1e3 * n * U_S
    assert np.all(np.abs(L[:m, :m] - Lg[:m, :m]) <=
                  tol * np.maximum(1.0, np.abs(Lg[:m, :m])) * colscale)
    assert np.all(np.abs(D[:m] - Dg[:m]) <= tol * np.maximum(amax, np.abs(Dg[:m])))
    rhs_d = torch.from_numpy(rhs).cuda()
    X, info = rcp.rcp_solve_ir(Ad, f, rhs_d, tol=1e-13, max_outer=10, restart=30)
    X = X.cpu().numpy()
    be = tb.backward_error(A, X, rhs)
    _say(f"  refined: backward error {np.max(be):.3e}, outer {info['outer']}, "
         f"inner {info['inner']}")
    assert info["converged"] and np.all(be <= 1e-13)
    ref = orcp.factor(A, b, p, seed=seed)
    xr = orcp.solve(ref, rhs)
    kappa = np.linalg.cond(tb.sym(A), p=np.inf)
    ferr = np.max(np.abs(X - xr)) / np.max(np.abs(xr))
    _say(f"  forward error vs the FP64 oracle {ferr:.3e} (kappa_inf {kappa:.2e})")
    assert ferr <= kappa * 1e-12


def test_sliced_rejects_bad_precision(rcp):
    import ctypes
    lib = rcp.load()
    one = ctypes.c_void_p(8)
    assert lib.rcp_factor_ex(4, one, 4, 4, 2, 0, 4, 9, one, one, one, one) == -8
    assert lib.rcp_factor_ex(4, one, 4, 4, 2, 0, 3, 0, one, one, one, one) == -7
