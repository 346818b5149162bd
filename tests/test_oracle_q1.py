"""Pins for the q = 1 branch of Algorithm 1 in the oracle (one pivot chosen
per sketch, the sketch updated after every elimination step by eq. (3.3)).

  * with b = 1 the two branches are the same algorithm (one QRCP step is
    the argmax of the sketch column norms, and the block sketch update with
    L11 = I is eq. (3.3)): bit-identical results;
  * the sketch identity B^(k) = Omega~_2 A^(k) (Section 3.1) at every block
    start, against Schur complements from dense solves (pins the per-step
    update, 2x2 pivots included);
  * with Omega = I the choice at every step is the largest exact Schur
    column norm (brute force);
  * reconstruction, uniqueness of L and D given the pivots, the case-(1)
    multiplier bound and the 2x2 determinant range of Section 4, and growth
    within a small factor of Bunch-Parlett complete pivoting.
"""

import numpy as np
import pytest

from oracle import rcp, textbook as tb
from oracle.omega import omega as omega_matrix
from workloads import gen

U = np.finfo(np.float64).eps / 2


@pytest.mark.parametrize("n,p,seed", [(40, 4, 1), (75, 0, 2), (120, 6, 3)])
def test_b1_branches_agree(n, p, seed):
    A = gen.gaussian_sym(n, seed) if seed % 2 else gen.kkt(n, (3 * n) // 4, seed, nrefl=8)
    f1 = rcp.factor(A, 1, p, seed=seed, q=1)
    fb = rcp.factor(A, 1, p, seed=seed)
    assert np.array_equal(f1.perm, fb.perm) and np.array_equal(f1.ipiv, fb.ipiv)
    assert np.array_equal(f1.L.view(np.uint64), fb.L.view(np.uint64))
    assert np.array_equal(f1.D.view(np.uint64), fb.D.view(np.uint64))


@pytest.mark.parametrize("n,b,p,seed", [(60, 8, 4, 4), (90, 16, 4, 5), (64, 7, 2, 6)])
def test_sketch_identity_at_block_starts(n, b, p, seed):
    A = gen.gaussian_sym(n, seed) if seed != 5 else gen.kkt(n, 60, seed, nrefl=8)
    f = rcp.factor(A, b, p, seed=seed, q=1, record_sketch=True)
    Om = omega_matrix(seed, 1 + p, n)
    assert int(np.sum(f.ipiv == 2)) > 0
    for K0, perm, Bk in f.sketch_at_block_start[1:]:
        ref = Om[:, perm[K0:]] @ tb.schur_complement(tb.permuted(A, perm), K0)
        assert np.max(np.abs(Bk - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))


def test_exact_norm_mode_every_step():
    n = 30
    A = gen.gaussian_sym(n, 9)
    f = rcp.factor(A, 8, n - 1, omega=np.eye(n), q=1, trace=True)
    picks = [e for e in f.log if e["kind"] == "qrcp"]
    assert len(picks) == sum(1 for e in f.log if e["kind"] == "sbkp")
    for e in picks:
        k = e["K0"]
        S = tb.schur_complement(tb.permuted(A, e["perm"]), k)
        assert e["pos"] - k == int(np.argmax(np.linalg.norm(S, axis=0)))


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_invariants(seed):
    n, b, p = 130, 16, 4
    A = gen.gaussian_sym(n, seed) if seed % 2 else gen.kkt(n, 97, seed, nrefl=8)
    f = rcp.factor(A, b, p, seed=seed, q=1)
    assert f.info == 0
    assert tb.reconstruction_error(A, f.perm, f.L, f.dmatrix()) <= 50 * n * U
    Lt, Dt = tb.block_ldlt_given(A, f.perm, f.ipiv)
    assert np.allclose(Lt, f.L, atol=1e-10) and np.allclose(Dt, f.dmatrix(), atol=1e-10)
    for e in f.log:
        if e["kind"] == "sbkp" and e["case"] == 1:
            k = e["k"]
            assert np.max(np.abs(f.L[k + 1:, k]), initial=0) <= 1 / rcp.ALPHA * (1 + 1e-14)
    for i in range(n - 1):
        if f.ipiv[i] == 2:
            d11, d22, c = f.D[i], f.D[i + 1], abs(f.D[n + i])
            assert -1.5 * c * c < d11 * d22 - c * c < -0.5 * c * c
    rhs = gen.rhs(n, 2, seed)
    assert np.max(tb.backward_error(A, rcp.solve(f, rhs), rhs)) <= 1e-14


@pytest.mark.parametrize("seed", [1, 2])
def test_growth_against_bunch_parlett(seed):
    n = 48
    A = gen.gaussian_sym(n, seed)
    f = rcp.factor(A, 8, 4, seed=seed, q=1, schedule="eager")
    _, _, _, _, rho_bp = tb.bunch_parlett(A)
    assert f.rho_elem <= 10 * rho_bp


def test_delayed_and_eager_schedules_agree():
    n = 70
    A = gen.gaussian_sym(n, 11)
    f = rcp.factor(A, 16, 4, seed=11, q=1)
    fe = rcp.factor(A, 16, 4, seed=11, q=1, schedule="eager")
    assert np.array_equal(f.perm, fe.perm) and np.array_equal(f.ipiv, fe.ipiv)
    assert np.allclose(f.L, fe.L, atol=1e-12) and np.allclose(f.D, fe.D, atol=1e-12)
