"""CPU checks of the paper's test-matrix types (Section 5) and of the oracle
on them.

The generators are pinned by closed forms and structure the definitions
fix; the oracle is pinned on each type by the invariants that hold for any
correct block LDL^T (reconstruction, solve backward error, uniqueness of
L and D given the pivots) and by the qualitative results the paper reports
for RCP on these types (Section 5: bounded growth on the Bunch-Kaufman worst
case, growth factor 1 on the rank-deficient type, linear growth of ||L||_1).
"""

import numpy as np
import pytest

from oracle import rcp as orcp, textbook as tb
from workloads import stress

U = np.finfo(np.float64).eps / 2
ALL = (1, 2, 3, 4, 5, 6, 7, 8, 10)


@pytest.mark.parametrize("kind", ALL)
def test_types_are_symmetric(kind):
    for n in (6, 17, 64):
        if kind == 1 and n % 2:
            continue
        A = stress.matrix(kind, n, seed=4)
        assert A.shape == (n, n)
        assert np.array_equal(A, A.T)
        assert np.all(np.isfinite(A))


def test_type1_structure():
    n, m = 20, 10
    A = stress.type1(n)
    alpha = (1 + np.sqrt(17)) / 8
    q = 1 + 1 / alpha
    d = np.diag(A)[:m - 2]
    assert d[0] == pytest.approx(1 / (1 - q), rel=1e-15)
    assert np.allclose(d[1:] * q, d[:-1], rtol=1e-14, atol=0)      # d_{k+1} = d_k / q
    assert np.all(A[m - 2:m, :m] == 1.0) and np.all(A[:m, m - 2:m] == 1.0)
    off = A[:m - 2, :m - 2] - np.diag(d)
    assert not np.any(off)
    assert np.array_equal(A[m:, :m], (1 - stress.TYPE1_EPS) * np.eye(m))
    assert not np.any(A[m:, m:])


def test_type2_structure():
    n = 9
    A = stress.type2(n)
    assert A[0, n - 1] == 2.0 and A[1, 1] == n
    sup = [A[k - 1, k] for k in range(2, n)]           # 1-based (k, k+1), k = 2..n-1
    assert sup == [float(v) for v in range(n, 2, -1)]   # n, n-1, ..., 3
    mask = np.zeros((n, n), dtype=bool)
    mask[0, n - 1] = mask[n - 1, 0] = mask[1, 1] = True
    for k in range(1, n - 1):
        mask[k, k + 1] = mask[k + 1, k] = True
    assert not np.any(A[~mask])


def test_type3_is_hankel():
    A = stress.type3(12, seed=2)
    for i in range(11):
        for j in range(1, 12):
            assert A[i, j] == A[i + 1, j - 1]


def test_type4_is_an_orthogonal_involution():
    # the DST-I matrix scaled by sqrt(2/(n+1)) is symmetric and orthogonal
    for n in (5, 16, 33):
        S = stress.type4(n)
        assert np.max(np.abs(S @ S - np.eye(n))) < 1e-13


def test_type5_dct1_identity():
    # DCT-I: C W C W = (n-1)/2 I with W = diag(1/2, 1, ..., 1, 1/2)
    for n in (3, 9, 40):
        C = stress.type5(n)
        w = np.ones(n)
        w[0] = w[-1] = 0.5
        W = np.diag(w)
        assert np.max(np.abs(C @ W @ C @ W - (n - 1) / 2 * np.eye(n))) < 1e-12 * n
        assert np.all(C[0] == 1.0) and np.all(C[:, 0] == 1.0)


def test_type8_blocks():
    n = 40
    A = stress.type8(n, seed=3)
    n1 = n - n // 4
    assert np.array_equal(A[:n1, :n1], np.eye(n1))
    assert not np.any(A[n1:, n1:])


def test_type10_rank_and_sign():
    A = stress.type10(120, seed=5)
    ev = np.linalg.eigvalsh(A)
    top = np.max(np.abs(ev))
    assert np.max(ev) <= 1e-12 * top               # negative semidefinite (1 - q < 0)
    rank = int(np.sum(np.abs(ev) > 1e-13 * top))
    assert 25 <= rank <= 45                        # lambda_i decays by 1/(1 + sqrt 2)


@pytest.mark.parametrize("kind", ALL)
@pytest.mark.parametrize("n,b,p", [(64, 16, 4), (150, 32, 4)])
def test_oracle_invariants_on_each_type(kind, n, b, p):
    A = stress.matrix(kind, n, seed=9)
    f = orcp.factor(A, b, p, seed=12)
    assert f.info == 0
    assert tb.reconstruction_error(A, f.perm, f.L, f.dmatrix()) <= 50 * n * U
    # the right-hand side of the paper's experiments: b = A x, x random
    x = np.random.default_rng(kind).standard_normal((n, 1))
    rhs = A @ x
    xs = orcp.solve(f, rhs)
    assert np.max(tb.backward_error(A, xs, rhs)) <= 1e-13
    # L and D are unique given the pivots: the textbook elimination agrees.
    # On the rank-deficient type the entries of column k carry an error of
    # about u max|A| / |d_k| and past the numerical rank the Schur
    # complement is rounding noise, so there only the columns with
    # |d_k| > 1e-6 max|A| are compared
    Lt, Dt = tb.block_ldlt_given(A, f.perm, f.ipiv)
    Dm = f.dmatrix()
    r = n
    if kind == 10:
        dmag = np.abs(f.D[:n]) + np.abs(f.D[n:])
        small = np.nonzero(dmag <= 1e-6 * np.max(np.abs(A)))[0]
        r = int(small[0]) if small.size else n
        assert 10 <= r <= 45
    scale = max(1.0, np.max(np.abs(Dm)))
    assert np.max(np.abs(Lt[:, :r] - f.L[:, :r])) <= 1e4 * n * U * max(1.0, np.max(np.abs(f.L)))
    assert np.max(np.abs(Dt[:r, :r] - Dm[:r, :r])) <= 1e4 * n * U * scale


@pytest.mark.parametrize("n", [64, 128, 256])
def test_paper_growth_results(n):
    # Type 1 (the Bunch-Kaufman worst case): RCP's element growth stays
    # small; Type 10 (rank deficient): growth factor 1 (Section 5)
    A1 = stress.type1(n)
    f1 = orcp.factor(A1, 16, 4, seed=5, schedule="eager")
    assert f1.rho_elem <= 4.0
    A10 = stress.type10(n, seed=3)
    f10 = orcp.factor(A10, 16, 4, seed=5, schedule="eager")
    assert f10.rho_elem == pytest.approx(1.0, abs=1e-12)


def test_l_norm_grows_with_n_on_the_dct_type():
    # ||L||_1 grows about linearly with n on types 4, 5 (Section 5)
    vals = []
    for n in (64, 128, 256):
        f = orcp.factor(stress.type5(n), 16, 4, seed=5)
        vals.append(np.max(np.sum(np.abs(f.L), axis=0)))
    assert vals[0] < vals[1] < vals[2]
    assert vals[2] / vals[0] > 2.0
