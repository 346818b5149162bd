"""GPU parity on the paper's test-matrix types (Section 5), through the C ABI.

For every type the GPU factorization is compared with the oracle's run of the
same problem: the permutation and the block pattern bit for bit on the
positions no near-tie decides (oracle.rcp.near_tie_prefix: several types
have exactly equal entries, whose order two FP64 implementations may resolve
differently), L and D elementwise there (the tolerance of the other parity
tests), and, for the whole factorization, the reconstruction bound
||P A P^T - L D L^T||_inf / ||A||_inf <= 50 n u and the backward error of a
solve with the paper's right-hand side b = A x (eq. (5.1)) <= 1e-13.  Past a
near-tie the GPU's pivots are a valid run of the method for its own
decisions; the checks above hold for it all the same.
"""

import sys

import numpy as np
import pytest

from oracle import rcp as orcp, textbook as tb
from workloads import stress

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


def _dmat(D, ipiv):
    n = len(ipiv)
    Dm = np.diag(D[:n].copy())
    for i in np.nonzero(ipiv == 2)[0]:
        Dm[i + 1, i] = Dm[i, i + 1] = D[n + i]
    return Dm


@pytest.mark.parametrize("kind", [1, 2, 3, 4, 5, 6, 7, 8, 10])
@pytest.mark.parametrize("n,b,p,seed", [(200, 32, 4, 21), (1030, 64, 4, 22)])
def test_stress_type_matches_oracle(rcp, kind, n, b, p, seed):
    import torch
    _say(f"stress type {kind}: n={n} b={b} p={p} seed={seed}")
    A = stress.matrix(kind, n, seed=seed)
    f = rcp.rcp_factor(torch.from_numpy(A).cuda(), b, p, seed)
    st = rcp.rcp_get_stats()
    perm = f.perm.cpu().numpy()
    ipiv = f.ipiv.cpu().numpy()
    L = f.L.cpu().numpy()
    D = f.D.cpu().numpy()
    ref = orcp.factor(A, b, p, seed=seed)
    amax = np.max(np.abs(A))
    pre = orcp.near_tie_prefix(ref, amax)
    diff = np.nonzero(perm != ref.perm)[0]
    first = int(diff[0]) if diff.size else n
    rho_ref = np.max(np.abs(ref.D)) / amax
    _say(f"  info {f.info}/{ref.info}; near-tie prefix {pre}; first differing position {first}; "
         f"rho_D {st['rho_d']:.3g} (oracle {rho_ref:.3g}); 2x2 {int(np.sum(ipiv == 2))} "
         f"(oracle {int(np.sum(ref.ipiv == 2))})")
    assert f.info == ref.info == 0
    assert np.array_equal(perm[:pre], ref.perm[:pre])
    assert np.array_equal(ipiv[:pre], ref.ipiv[:pre])
    # L and D where the pivots agree: a multiplier of column k carries an
    # error of about n u max|A| / |d_k| and an entry of D one of n u max|A|
    # (the rank-deficient type has pivots far below max|A|)
    # (the positions before the first difference in perm or ipiv: their
    # rows and columns of L depend only on decisions both runs took alike)
    idiff = np.nonzero(ipiv != ref.ipiv)[0]
    m = min(first, int(idiff[0]) if idiff.size else n)
    tol = 1e3 * n * U
    dk = np.abs(ref.D[:n]) + np.abs(ref.D[n:])
    dk = np.maximum(dk, np.roll(dk * (ref.ipiv == 2), 1))   # a 2x2 block's second column
    colscale = np.maximum(1.0, amax / np.maximum(dk, 1e-300))[None, :m]
    assert np.all(np.abs(L[:m, :m] - ref.L[:m, :m]) <=
                  tol * np.maximum(1.0, np.abs(ref.L[:m, :m])) * colscale)
    assert np.all(np.abs(D[:m] - ref.D[:m]) <= tol * np.maximum(amax, np.abs(ref.D[:m])))
    assert np.all(np.abs(D[n:n + m] - ref.D[n:n + m]) <=
                  tol * np.maximum(amax, np.abs(ref.D[n:n + m])))
    # the whole GPU factorization is a valid block LDL^T of P A P^T
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert tb.reconstruction_error(A, perm, L, _dmat(D, ipiv)) <= 50 * n * U
    x = np.random.default_rng(seed).standard_normal((n, 1))
    rhs = A @ x
    X = rcp.rcp_solve(f, torch.from_numpy(rhs).cuda()).cpu().numpy()
    be = np.max(tb.backward_error(A, X, rhs))
    _say(f"  backward error {be:.2e}")
    assert be <= 1e-13
    # the growth factor the library reports is max|D| / max|A| of its own D
    assert st["rho_d"] == pytest.approx(np.max(np.abs(D)) / amax, rel=1e-12)
