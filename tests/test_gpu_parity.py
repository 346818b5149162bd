"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every case prints its name before running so that a failing GPU step can be
traced.  Tolerances:
  * permutation and block pattern: bit-exact (integer results) whenever the
    oracle's decision log has no near-tie (relative margin > 1e-9); the
    cases below are checked to have none;
  * L, D: |GPU - oracle| <= 1e3 * n * u * max(1, |oracle|) elementwise -- both
    are FP64 and differ only by summation order, amplified at most by the
    growth of the factorization (small for these inputs);
  * reconstruction ||P A P^T - L D L^T||_inf / ||A||_inf <= 50 n u;
  * solve backward error ||A x - b||_inf / (||A||_inf ||x||_inf) <= 1e-13.
"""

import sys

import numpy as np
import pytest

from oracle import omega as oomega, rcp as orcp, textbook as tb
from workloads import gen

pytestmark = pytest.mark.gpu

U = np.finfo(np.float64).eps / 2


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


def _dev():
    import torch
    return torch.device("cuda:0")


@pytest.mark.parametrize("seed,l,n", [(1, 40, 512), (3, 7, 13), (2**64 - 5, 144, 300), (0, 1, 1)])
def test_omega_bit_identical(rcp, seed, l, n):
    _say(f"omega seed={seed} l={l} n={n}")
    got = rcp.rcp_omega(seed, l, n).cpu().numpy()
    ref = oomega.omega(seed, l, n)
    assert got.shape == ref.shape
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def _factor_case(rcp, A, b, p, seed, check_margin=True):
    import torch
    n = A.shape[0]
    ref = orcp.factor(A, b, p, seed=seed)
    if check_margin:
        margin, _ = orcp.min_margin(ref, scale=np.max(np.abs(A)))
        assert margin > 1e-9, f"near-tie in the oracle run (margin {margin})"
    f = rcp.rcp_factor(torch.from_numpy(A).to(_dev()), b, p, seed)
    torch.cuda.synchronize()
    perm, ipiv = f.perm.cpu().numpy(), f.ipiv.cpu().numpy()
    assert np.array_equal(perm, ref.perm)
    assert np.array_equal(ipiv, ref.ipiv)
    L, D = f.L.cpu().numpy(), f.D.cpu().numpy()
    tol = 1e3 * n * U
    assert np.all(np.abs(L - ref.L) <= tol * np.maximum(1.0, np.abs(ref.L)))
    assert np.all(np.abs(D - ref.D) <= tol * np.maximum(1.0, np.abs(ref.D)))
    if np.any(A):
        assert tb.reconstruction_error(A, perm, L, _dmat(D, ipiv)) <= 50 * n * U
    else:                               # the relative error is 0/0; D itself is 0
        assert not np.any(D)
    return f, ref


def _dmat(D, ipiv):
    n = len(ipiv)
    Dm = np.diag(D[:n])
    for i in range(n - 1):
        if ipiv[i] == 2:
            Dm[i + 1, i] = Dm[i, i + 1] = D[n + i]
    return Dm


@pytest.mark.parametrize("n,b,p,seed", [
    (1, 4, 2, 1), (2, 4, 2, 2), (3, 2, 2, 3), (17, 4, 4, 6), (64, 8, 8, 8),
    (96, 16, 8, 7), (200, 32, 8, 10), (333, 32, 8, 11), (512, 32, 8, 1),
])
def test_factor_gaussian_matches_oracle(rcp, n, b, p, seed):
    _say(f"factor gaussian n={n} b={b} p={p} seed={seed}")
    A = gen.gaussian_sym(n, seed)
    _factor_case(rcp, A, b, p, seed)


@pytest.mark.parametrize("n,b,p,seed", [(1000, 64, 10, 5), (1300, 128, 16, 6)])
def test_factor_householder_matches_oracle(rcp, n, b, p, seed):
    _say(f"factor householder n={n} b={b} p={p} seed={seed}")
    A = gen.householder_spectrum(n, seed, cond=1e6, nrefl=64)
    _factor_case(rcp, A, b, p, seed)


@pytest.mark.parametrize("n,b,p,seed", [(700, 128, 40, 8), (450, 32, 140, 9)])
def test_factor_wide_sketch_matches_oracle(rcp, n, b, p, seed):
    """Sketches of more than 160 rows (l = 168 and 172): the sketch product
    covers them in two column blocks of at most 160, the last one narrower
    and staged with zero columns."""
    _say(f"factor wide sketch n={n} b={b} p={p} seed={seed}")
    A = gen.householder_spectrum(n, seed, cond=1e6, nrefl=64)
    _factor_case(rcp, A, b, p, seed)


@pytest.mark.parametrize("n,b,p,seed", [(128, 16, 4, 2), (400, 64, 10, 2), (1500, 64, 10, 3)])
def test_factor_kkt_matches_oracle(rcp, n, b, p, seed):
    _say(f"factor kkt n={n} b={b} p={p} seed={seed}")
    A = gen.kkt(n, (3 * n) // 4, seed, nrefl=min(64, (3 * n) // 4))
    _factor_case(rcp, A, b, p, seed)


# the chained triangular solves work on 64-row blocks and hold up to eight
# right-hand sides at once (two at a time going back): ragged orders, a single
# block, and counts that split into uneven groups
@pytest.mark.parametrize("n,nrhs", [(300, 1), (300, 4), (300, 3), (300, 11), (50, 2), (1000, 5)])
def test_solve_backward_error(rcp, n, nrhs):
    import torch
    b, p, seed = 32, 8, 4
    _say(f"solve n={n} nrhs={nrhs}")
    A = gen.gaussian_sym(n, seed)
    rhs = gen.rhs(n, nrhs, seed)
    f = rcp.rcp_factor(torch.from_numpy(A).to(_dev()), b, p, seed)
    rhs_dev = torch.from_numpy(rhs).to(_dev())
    X = rcp.rcp_solve(f, rhs_dev).cpu().numpy()
    # the right-hand side is not modified by the binding
    assert np.array_equal(rhs_dev.cpu().numpy(), rhs)
    ref = orcp.factor(A, b, p, seed=seed)
    xr = orcp.solve(ref, rhs)
    assert np.all(tb.backward_error(A, X, rhs) <= 1e-13)
    assert np.max(np.abs(X - xr)) <= 1e-9 * max(1.0, np.max(np.abs(xr)))


def test_column_major_view_reads_the_same_triangle(rcp):
    """A tensor whose transpose is contiguous is handed over without a copy;
    only the lower triangle is read either way (garbage above it here)."""
    import torch
    n, b, p, seed = 260, 32, 8, 6
    _say(f"column-major view n={n}")
    A = gen.gaussian_sym(n, seed)
    M = A.copy()
    M[np.triu_indices(n, 1)] = 1e30          # never read
    row_major = torch.from_numpy(M).to(_dev())
    col_major = torch.from_numpy(np.ascontiguousarray(M.T)).to(_dev()).t()
    assert not col_major.is_contiguous() and col_major.t().is_contiguous()
    assert torch.equal(row_major, col_major)
    f1 = rcp.rcp_factor(row_major, b, p, seed)
    f2 = rcp.rcp_factor(col_major, b, p, seed)
    assert torch.equal(f1.perm, f2.perm) and torch.equal(f1.ipiv, f2.ipiv)
    assert torch.equal(f1.L, f2.L) and torch.equal(f1.D, f2.D)
    ref = orcp.factor(A, b, p, seed=seed)
    assert np.array_equal(f2.perm.cpu().numpy(), ref.perm)


# the smallest sketches the interface allows: one column per block (b = 1),
# no oversampling (p = 0, l = b)
@pytest.mark.parametrize("n,b,p,seed", [(40, 1, 0, 21), (70, 8, 0, 22), (65, 1, 3, 23)])
def test_factor_minimal_sketch_matches_oracle(rcp, n, b, p, seed):
    _say(f"factor minimal sketch n={n} b={b} p={p}")
    A = gen.gaussian_sym(n, seed)
    _factor_case(rcp, A, b, p, seed)


def _block_singular(n, r, seed):
    """A Gaussian symmetric r x r block in the top corner, zeros elsewhere:
    the trailing Schur complement after r eliminations is exactly zero."""
    A = np.zeros((n, n))
    A[:r, :r] = gen.gaussian_sym(r, seed)
    return A


# exactly singular matrices: the selection runs out of nonzero sketch
# columns, SBKP takes case (0) pivots (zero multipliers, d = 0) and info
# reports the first exactly zero 1x1 pivot, as in the oracle; the solve
# refuses such factors
@pytest.mark.parametrize("name,n,r,b,p", [("zero", 12, 0, 4, 2), ("rank7", 40, 7, 8, 4),
                                          ("rank20", 100, 20, 16, 8)])
def test_factor_singular_reports_zero_pivot(rcp, name, n, r, b, p):
    import torch
    seed = 31
    _say(f"singular {name} n={n} b={b} p={p}")
    A = _block_singular(n, r, seed)
    f, ref = _factor_case(rcp, A, b, p, seed, check_margin=False)
    assert ref.info > 0
    assert f.info == ref.info
    with pytest.raises(rcp.RCPError):
        rcp.rcp_solve(f, torch.ones(n, dtype=torch.float64, device=_dev()))


# non-finite input: a NaN or an Inf in the lower triangle reaches the sketch
# and the factorization stops with RCP_ENONFINITE; the same entries in the
# strict upper triangle are never read
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_input(rcp, bad):
    import torch
    from paper_1710_00125_amd._binding import RCP_ENONFINITE
    n, b, p, seed = 150, 16, 8, 41
    _say(f"non-finite input {bad}")
    A = gen.gaussian_sym(n, seed)
    lower = A.copy()
    lower[97, 12] = bad
    with pytest.raises(rcp.RCPError) as e:
        rcp.rcp_factor(torch.from_numpy(lower).to(_dev()), b, p, seed)
    assert e.value.code == RCP_ENONFINITE
    upper = A.copy()
    upper[12, 97] = bad
    f = rcp.rcp_factor(torch.from_numpy(upper).to(_dev()), b, p, seed)
    ref = orcp.factor(A, b, p, seed=seed)
    assert np.array_equal(f.perm.cpu().numpy(), ref.perm)


# The persistent kernels' other shapes at sizes the oracle checks in
# seconds.  The selection keeps up to 64 sketch columns per workgroup in
# registers (l <= 144) and more, or taller sketches, in LDS.  It takes 64
# columns per workgroup where it can, so at every size the first block's
# workgroups own 64 or, ragged, fewer (n = 2000: 63, the last one 47), and
# later blocks run every width down to 33 as N shrinks.  A bounded grid gives
# more than 64 columns (LDS slab); grid limits (32, 32) give the q = b panel
# its full-size shape of 64 rows per workgroup at n = 2048.
@pytest.mark.parametrize("n,b,p,limits,regs,cols", [
    (2048, 128, 16, (32, 32), 1, 64),    # register slab, 64 columns; panel rows 64
    (2000, 128, 16, (0, 0), 1, 63),      # register slab, ragged 63 columns
    (1300, 128, 24, (0, 0), 0, 62),      # l = 152 > 144: LDS slab
    (2048, 128, 16, (24, 0), 0, 86),     # more than 64 columns: LDS slab
])
def test_factor_selection_shapes_match_oracle(rcp, n, b, p, limits, regs, cols):
    seed = 60 + n % 7
    _say(f"factor shapes n={n} b={b} p={p} grid limits={limits}")
    shape = None
    try:
        rcp.rcp_set_grid_limit(*limits)
        shape = rcp.rcp_launch_shape(n, b, p)
        assert shape["supported"] == 1
        assert shape["select_regs"] == regs and shape["select_cols"] == cols, shape
        A = gen.householder_spectrum(n, seed, cond=1e6, nrefl=64)
        _factor_case(rcp, A, b, p, seed)
    finally:
        rcp.rcp_set_grid_limit(0, 0)


def test_factor_reports_pivoting_statistics(rcp):
    """max|A|, max|L|, max|D| and rho_D in the call's statistics equal the
    same quantities computed from the inputs and outputs; the threshold
    margins are positive and no near-tie is reported for this input."""
    import torch
    n, b, p, seed = 700, 64, 10, 71
    _say(f"statistics n={n}")
    A = gen.kkt(n, (3 * n) // 4, seed, nrefl=64)
    f = rcp.rcp_factor(torch.from_numpy(A).to(_dev()), b, p, seed)
    st = rcp.rcp_get_stats()
    L, D, ipiv = f.L.cpu().numpy(), f.D.cpu().numpy(), f.ipiv.cpu().numpy()
    amax = np.max(np.abs(np.tril(A)))
    lmax = np.max(np.abs(np.tril(L, -1)))
    dmax = max(np.max(np.abs(D[:n])), np.max(np.abs(D[n:][ipiv == 2]), initial=0.0))
    assert st["max_abs_a"] == amax
    assert st["max_abs_l"] == lmax
    assert st["max_abs_d"] == dmax
    assert st["rho_d"] == pytest.approx(dmax / amax, rel=1e-15)
    assert st["n2x2"] == int(np.sum(ipiv == 2))
    assert 0.0 < st["min_margin"] < np.inf and st["near_ties"] == 0
    ref = orcp.factor(A, b, p, seed=seed)
    # the oracle's smallest threshold-test margin, relative to lambda
    marg = [min([abs(abs(e["akk"]) - orcp.ALPHA * e["lam"])] +
                ([abs(abs(e["arr"]) - orcp.ALPHA * e["lam"])] if e["arr"] is not None else []))
            / e["lam"] for e in ref.log if e["kind"] == "sbkp" and e["lam"] > 0]
    assert st["min_margin"] == pytest.approx(min(marg), rel=1e-6)
