"""Pins for Algorithm 2 in the oracle (Section 4.5: recomputed random
projections and the rank-deficiency exit), from inputs whose Schur
complements are known in closed form:

  * an r0 x r0 Gaussian block among exact zeros: after the block's columns
    the Schur complement is exactly zero, so every sketch of it is zero and
    the method must stop with rank r0;
  * a spectrum with a gap (r0 eigenvalues of size 1, the rest 1e-9): after
    r0 pivots the Schur complement is of order 1e-9, below EPS^(1/2) beta
    and above EPS beta, so with r = 2 the sketch is recomputed exactly once
    and the factorization goes on; with a gap of 1e-6 (above EPS^(1/2)) it
    is never recomputed;
  * the recomputed sketch equals a fresh Omega times the Schur complement
    computed independently by dense solves;
  * r = 1 is Algorithm 1 bit for bit.
"""

import numpy as np
import pytest

from oracle import rcp, textbook as tb
from oracle.omega import omega as omega_matrix
from workloads import gen

U = np.finfo(np.float64).eps / 2


@pytest.mark.parametrize("seed", [1, 2])
def test_r1_is_algorithm1(seed):
    A = gen.gaussian_sym(90, seed)
    f1 = rcp.factor(A, 16, 4, seed=seed)
    f2 = rcp.factor(A, 16, 4, seed=seed, recompute=1)
    assert np.array_equal(f1.perm, f2.perm) and np.array_equal(f1.ipiv, f2.ipiv)
    assert np.array_equal(f1.L.view(np.uint64), f2.L.view(np.uint64))
    assert np.array_equal(f1.D.view(np.uint64), f2.D.view(np.uint64))
    assert f2.recomputed == [] and f2.rank == 90


@pytest.mark.parametrize("r", [2, 3])
def test_exact_zero_schur_complement_stops(r):
    n, r0, b = 100, 32, 16
    A = gen.zero_padded(n, r0, 5)
    f = rcp.factor(A, b, 4, seed=3, recompute=r)
    assert f.rank == r0 and f.info == r0 + 1
    assert f.recomputed == [r0]
    assert not np.any(f.D[r0:n]) and not np.any(f.D[n + r0:])
    assert np.all(f.ipiv[r0:] == 1)
    assert np.array_equal(f.L[r0:, r0:], np.eye(n - r0))
    # the first r0 positions hold the nonzero block, and P A P^T = L D L^T
    nz = set(np.nonzero(np.any(A != 0, axis=0))[0])
    assert set(f.perm[:r0]) == nz
    assert tb.reconstruction_error(A, f.perm, f.L, f.dmatrix()) <= 50 * n * U
    # Algorithm 1 runs on through zero pivots instead
    g = rcp.factor(A, b, 4, seed=3)
    assert g.rank == n and g.info == r0 + 1 and g.recomputed == []


def test_gap_spectrum_recomputes_once_and_continues():
    n, r0, b, p, seed = 120, 32, 16, 4, 3
    A = gen.gap_spectrum(n, r0, 6, small=1e-9)
    f = rcp.factor(A, b, p, seed=seed, recompute=2, record_sketch=True)
    assert f.recomputed == [r0] and f.rank == n and f.info == 0
    assert tb.reconstruction_error(A, f.perm, f.L, f.dmatrix()) <= 50 * n * U
    # the sketch at that block start is the fresh Omega (stream 2) times the
    # Schur complement, computed here by dense solves
    K0, perm, B = [s for s in f.sketch_at_block_start if s[0] == r0][0]
    S = tb.schur_complement(tb.permuted(A, perm), r0)
    ref = omega_matrix(seed, b + p, n - r0, stream=2) @ S
    assert np.max(np.abs(B - ref)) <= 1e-6 * np.max(np.abs(ref))
    assert np.max(np.abs(ref)) < 1e-7 * f.sketch_scale
    # without Algorithm 2 the same matrix keeps the updated sketch
    g = rcp.factor(A, b, p, seed=seed)
    assert g.recomputed == [] and g.rank == n


def test_gap_above_the_first_threshold_is_not_recomputed():
    A = gen.gap_spectrum(120, 32, 6, small=1e-6)
    f = rcp.factor(A, 16, 4, seed=3, recompute=2)
    assert f.recomputed == [] and f.rank == 120


def test_three_thresholds():
    # r = 3: EPS^(1/3) ~ 6e-6, EPS^(2/3) ~ 4e-11; a gap of 1e-9 is recomputed
    # once (below the first) and then passes the second and every later check
    A = gen.gap_spectrum(120, 32, 6, small=1e-9)
    f = rcp.factor(A, 16, 4, seed=3, recompute=3)
    assert f.recomputed == [32] and f.rank == 120
