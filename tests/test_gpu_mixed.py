"""GPU: reduced-precision factorization and FP64 GMRES refinement.

The refinement is not part of the paper; its parity is judged on the
solution (the pivots of a reduced-precision run may differ from the FP64
oracle's wherever rounding in the narrower precision decides a comparison):
  * the refined solution has backward error ||A x - b||_inf /
    (||A||_inf ||x||_inf) <= 1e-13 (computed here in FP64 NumPy), and the
    library's own report of it agrees up to the rounding of the residual
    itself (10 n u);
  * it agrees with the FP64 oracle's solution to within
    kappa_inf(A) * 1e-13 * 10 (forward error of two backward-stable solutions);
  * the reduced-precision factors themselves are a valid block LDL^T: a
    permutation, unit lower L with zero entries inside 2x2 blocks, and a
    reconstruction error ||P A P^T - L D L^T||_inf / ||A||_inf <= 20 n u_w,
    u_w = 2^-24 (FP32) or 2^-16 (three BF16 products of split operands);
  * one application of the reduced-precision factors (rcp_solve_mp) already
    has backward error <= 1e3 * n * u_w.
Every case prints its name before running.
"""

import sys

import numpy as np
import pytest

from oracle import rcp as orcp, textbook as tb
from workloads import gen

pytestmark = pytest.mark.gpu

U_W = {1: 2.0 ** -24, 2: 2.0 ** -16}
NAMES = {1: "fp32", 2: "bf16x3"}


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
    Dm = np.diag(D[:n])
    for i in range(n - 1):
        if ipiv[i] == 2:
            Dm[i + 1, i] = Dm[i, i + 1] = D[n + i]
    return Dm


def _check_structure(perm, L, ipiv):
    n = len(perm)
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert np.all(np.diag(L) == 1.0)
    assert np.all(np.triu(L, 1) == 0.0)
    assert set(np.unique(ipiv)).issubset({0, 1, 2})
    for i in range(n):
        if ipiv[i] == 2:
            assert i + 1 < n and ipiv[i + 1] == 0 and L[i + 1, i] == 0.0
        if ipiv[i] == 0:
            assert i > 0 and ipiv[i - 1] == 2


def _matrix(kind, n, seed, cond=1e6):
    if kind == "gaussian":
        return gen.gaussian_sym(n, seed)
    if kind == "kkt":
        return gen.kkt(n, (3 * n) // 4, seed, nrefl=min(64, (3 * n) // 4))
    return gen.householder_spectrum(n, seed, cond=cond, nrefl=64)


CASES = [
    ("gaussian", 512, 32, 8, 1, 1e6),
    ("kkt", 400, 64, 10, 2, 1e6),
    ("householder", 1000, 64, 10, 41, 1e2),
    ("householder", 1000, 64, 10, 42, 1e6),
    ("householder", 1200, 128, 16, 44, 1e6),
]


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("kind,n,b,p,seed,cond", CASES)
def test_mixed_factor_and_refine(rcp, precision, kind, n, b, p, seed, cond):
    import torch
    _say(f"mixed {NAMES[precision]} {kind} n={n} b={b} p={p} seed={seed} cond={cond:g}")
    A = _matrix(kind, n, seed, cond)
    nrhs = 4 if kind == "kkt" else 1
    rhs = gen.rhs(n, nrhs, seed)
    dev = torch.device("cuda:0")
    Ad = torch.from_numpy(A).to(dev)
    f = rcp.rcp_factor_mp(Ad, b, p, seed, precision)
    assert f.info == 0
    perm, ipiv = f.perm.cpu().numpy(), f.ipiv.cpu().numpy()
    L = f.L.cpu().numpy().astype(np.float64)
    D = f.D.cpu().numpy()
    _check_structure(perm, L, ipiv)
    uw = U_W[precision]
    rec = tb.reconstruction_error(A, perm, L, _dmat(D, ipiv))
    _say(f"  reconstruction {rec:.3e}")
    assert rec <= 20 * n * uw

    rhs_d = torch.from_numpy(rhs).to(dev)
    x1 = rcp.rcp_solve_mp(f, rhs_d).cpu().numpy()
    be1 = np.max(tb.backward_error(A, x1, rhs))
    _say(f"  one low-precision solve: backward error {be1:.3e}")
    assert be1 <= 1e3 * n * uw

    X, info = rcp.rcp_solve_ir(Ad, f, rhs_d, tol=1e-13, max_outer=10, restart=30)
    X = X.cpu().numpy()
    assert np.array_equal(rhs_d.cpu().numpy(), rhs)   # B is not modified
    be = tb.backward_error(A, X, rhs)
    _say(f"  refined: backward error {np.max(be):.3e}, outer {info['outer']}, "
         f"inner {info['inner']}, reported {info['berr']:.3e}")
    assert info["converged"]
    assert np.all(be <= 1e-13)
    # the library's residual agrees with NumPy's up to the rounding of the
    # residual itself (different summation orders, about n u)
    assert abs(info["berr"] - np.max(be)) <= 1e-3 * np.max(be) + 10 * n * 2.0 ** -53
    ref = orcp.factor(A, b, p, seed=seed)
    xr = orcp.solve(ref, rhs)
    kappa = np.linalg.cond(tb.sym(A), p=np.inf)
    ferr = np.max(np.abs(X - xr)) / np.max(np.abs(xr))
    _say(f"  forward error vs the FP64 oracle {ferr:.3e} (kappa_inf {kappa:.2e})")
    assert ferr <= kappa * 1e-12


@pytest.mark.parametrize("precision", [1, 2])
def test_refine_reports_stagnation_at_cond_1e10(rcp, precision):
    """cond 1e10: rounding the trailing matrix to FP32 perturbs every
    eigen-direction below about 1e-7 ||A|| (a third of this log-uniform
    spectrum), so restarted GMRES cannot reach 1e-13 in a bounded number of
    iterations.  The call must say so (RCP_ENOCONV), report the backward
    error of the iterate it returns, and -- GMRES minimising the true
    residual over a space that contains d = 0 -- never leave a larger
    residual 2-norm than the first solve."""
    import torch
    n, b, p, seed = 1200, 128, 16, 43
    _say(f"stagnation {NAMES[precision]} householder n={n} cond=1e10")
    A = _matrix("householder", n, seed, 1e10)
    rhs = gen.rhs(n, 1, seed)
    dev = torch.device("cuda:0")
    Ad, bd = torch.from_numpy(A).to(dev), torch.from_numpy(rhs).to(dev)
    f = rcp.rcp_factor_mp(Ad, b, p, seed, precision)
    x0 = rcp.rcp_solve_mp(f, bd).cpu().numpy()
    X, info = rcp.rcp_solve_ir(Ad, f, bd, tol=1e-13, max_outer=3, restart=20,
                               raise_on_noconv=False)
    X = X.cpu().numpy()
    be = np.max(tb.backward_error(A, X, rhs))
    S = tb.sym(A)
    r0 = np.linalg.norm(S @ x0 - rhs)
    r1 = np.linalg.norm(S @ X - rhs)
    _say(f"  residual 2-norm {r0:.3e} -> {r1:.3e}, backward error {be:.3e}, {info}")
    assert not info["converged"] and info["outer"] == 3 and info["inner"] == 60
    assert abs(info["berr"] - be) <= 1e-3 * be
    assert r1 <= r0 * 1.01


# right-hand-side counts that exercise every residual kernel width (one,
# two, four at a time) and the refinement's groups of four
@pytest.mark.parametrize("nrhs", [2, 3, 6])
def test_refine_many_rhs(rcp, nrhs):
    import torch
    n, b, p, seed = 300, 32, 8, 12
    _say(f"refine fp32 n={n} nrhs={nrhs}")
    A = gen.gaussian_sym(n, seed)
    B = gen.rhs(n, nrhs, seed)
    dev = torch.device("cuda:0")
    Ad = torch.from_numpy(A).to(dev)
    f = rcp.rcp_factor_mp(Ad, b, p, seed, 1)
    X, info = rcp.rcp_solve_ir(Ad, f, torch.from_numpy(B).to(dev))
    x = X.cpu().numpy()
    be = tb.backward_error(A, x, B)
    _say(f"  backward errors {np.array2string(be, precision=2)}, {info}")
    assert info["converged"]
    assert np.all(be <= 1e-13)
    assert abs(info["berr"] - np.max(be)) <= 1e-3 * np.max(be) + 10 * n * np.finfo(float).eps / 2
    ref = orcp.factor(A, b, p, seed=seed)
    xr = orcp.solve(ref, B)
    kappa = np.linalg.cond(A, np.inf)
    assert np.max(np.abs(x - xr)) <= kappa * 1e-12 * max(1.0, np.max(np.abs(xr)))


def test_refine_already_converged(rcp):
    """A zero right-hand side: x0 = 0 is exact, no GMRES cycle runs."""
    import torch
    n = 200
    A = gen.gaussian_sym(n, 9)
    dev = torch.device("cuda:0")
    Ad = torch.from_numpy(A).to(dev)
    f = rcp.rcp_factor_mp(Ad, 32, 8, 9, 1)
    X, info = rcp.rcp_solve_ir(Ad, f, torch.zeros(n, dtype=torch.float64, device=dev))
    assert info["converged"] and info["outer"] == 0 and info["inner"] == 0
    assert np.all(X.cpu().numpy() == 0.0)


def test_fp32_pivots_mostly_match_oracle(rcp):
    """At moderate n the FP32 run takes the FP64 oracle's pivots except where
    a decision is within FP32 rounding: the permutations agree on most
    positions (recorded, with the first divergence)."""
    import torch
    n, b, p, seed = 256, 32, 8, 12
    A = gen.gaussian_sym(n, seed)
    f = rcp.rcp_factor_mp(torch.from_numpy(A).cuda(), b, p, seed, 1)
    perm = f.perm.cpu().numpy()
    ref = orcp.factor(A, b, p, seed=seed)
    same = np.mean(perm == ref.perm)
    first = int(np.argmax(perm != ref.perm)) if same < 1 else n
    _say(f"  fp32 vs oracle permutation agreement {same:.3f}, first divergence at {first}")
    assert first >= b   # the first block's QRCP and SBKP decisions agree
