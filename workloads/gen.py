"""Seeded matrix and right-hand-side generators.

Every generator takes an integer seed and returns float64 NumPy arrays built
with NumPy's PCG64 generator.  Matrices are returned exactly symmetric (the
lower triangle is mirrored into the upper one), so row-major and column-major
readings of the array agree.

Matrix families (paper, Section 5):
  * gaussian_sym          Type 6: an n x n Gaussian matrix, symmetrised as
                          (G + G^T)/2.
  * kkt                   Type 7: the saddle-point matrix [[H, C^T], [C, 0]]
                          with H symmetric positive definite.
  * householder_spectrum  a dense symmetric indefinite matrix Q diag(s*lam) Q^T
                          with a prescribed log-uniform spectrum and random
                          signs, Q a product of Householder reflectors.
"""

import numpy as np

# stream ids inside one seed, so that the matrix, the right-hand side and the
# reflectors of one configuration never share random numbers
_STREAM_MATRIX = 0
_STREAM_RHS = 2
_STREAM_REFLECTORS = 3


def _rng(seed, stream):
    return np.random.default_rng(np.random.SeedSequence([int(seed), stream]))


def _mirror_lower(A):
    """Make A exactly symmetric by copying its lower triangle upward."""
    n = A.shape[0]
    blk = 2048
    for j0 in range(0, n, blk):
        j1 = min(n, j0 + blk)
        # rows j0:j1 of the upper part = columns j0:j1 of the lower part
        A[j0:j1, j0:] = np.where(
            np.arange(j0, j1)[:, None] <= np.arange(j0, n)[None, :],
            A[j0:, j0:j1].T, A[j0:j1, j0:])
    return A


def gaussian_sym(n, seed):
    """(G + G^T)/2 with G i.i.d. N(0, 1)."""
    G = _rng(seed, _STREAM_MATRIX).standard_normal((n, n))
    A = G + G.T
    A *= 0.5
    return A


def householder_product_wy(n, nrefl, rng):
    """Q = H_1 H_2 ... H_k as I - V T V^T (compact WY form, T upper triangular).

    H_i = I - tau_i v_i v_i^T with v_i ~ N(0, I_n) and tau_i = 2 / (v_i^T v_i).
    """
    V = rng.standard_normal((n, nrefl))
    tau = 2.0 / np.einsum("ij,ij->j", V, V)
    T = np.zeros((nrefl, nrefl))
    for i in range(nrefl):
        T[i, i] = tau[i]
        if i:
            T[:i, i] = -tau[i] * (T[:i, :i] @ (V[:, :i].T @ V[:, i]))
    return V, T


def _q_diag_qt(lam, V, T):
    """Q diag(lam) Q^T for Q = I - V T V^T, as diag(lam) plus a rank-2k term."""
    k = V.shape[1]
    U = V @ T
    LV = lam[:, None] * V
    M = V.T @ LV
    X = np.concatenate([U, LV], axis=1)
    C = np.zeros((2 * k, 2 * k))
    C[:k, :k] = M
    C[:k, k:] = -np.eye(k)
    C[k:, :k] = -np.eye(k)
    A = (X @ C) @ X.T
    A[np.diag_indices_from(A)] += lam
    return _mirror_lower(A)


def householder_spectrum(n, seed, cond=1e6, nrefl=64):
    """A = Q diag(s*lam) Q^T: lam log-uniform in [1/cond, 1], s = +-1 w.p. 1/2.

    Q is a product of ``nrefl`` random Householder reflectors.
    """
    rng = _rng(seed, _STREAM_MATRIX)
    lam = 10.0 ** (-np.log10(cond) * rng.random(n))
    s = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    V, T = householder_product_wy(n, min(nrefl, n), _rng(seed, _STREAM_REFLECTORS))
    return _q_diag_qt(s * lam, V, T)


def kkt(n, n1, seed, nrefl=64, lam_min=1e-3):
    """[[H, C^T], [C, 0]] with H = Q diag(lam) Q^T (n1 x n1, SPD, lam
    log-uniform in [lam_min, 1]) and C ((n - n1) x n1) i.i.d. N(0,1)/sqrt(n1).
    """
    rng = _rng(seed, _STREAM_MATRIX)
    lam = 10.0 ** (np.log10(lam_min) * rng.random(n1))
    V, T = householder_product_wy(n1, min(nrefl, n1), _rng(seed, _STREAM_REFLECTORS))
    H = _q_diag_qt(lam, V, T)
    C = rng.standard_normal((n - n1, n1)) / np.sqrt(n1)
    A = np.zeros((n, n))
    A[:n1, :n1] = H
    A[n1:, :n1] = C
    A[:n1, n1:] = C.T
    return A


def zero_padded(n, r0, seed):
    """An r0 x r0 Gaussian-symmetric block at r0 random positions of an
    n x n zero matrix: exactly rank r0 or less, with exactly zero rows and
    columns elsewhere."""
    rng = _rng(seed, _STREAM_MATRIX)
    where = np.sort(rng.permutation(n)[:r0])
    A = np.zeros((n, n))
    A[np.ix_(where, where)] = gaussian_sym(r0, seed)
    return A


def gap_spectrum(n, r0, seed, small=1e-9, nrefl=16):
    """Q diag(s lam) Q^T with lam = 1 for r0 eigenvalues and `small` for the
    others, random signs s, Q a product of `nrefl` Householder reflectors:
    after r0 well chosen pivots the Schur complement is of order `small`."""
    rng = _rng(seed, _STREAM_MATRIX)
    lam = np.full(n, float(small))
    lam[rng.permutation(n)[:r0]] = 1.0
    s = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    V, T = householder_product_wy(n, min(nrefl, n), _rng(seed, _STREAM_REFLECTORS))
    return _q_diag_qt(s * lam, V, T)


def rhs(n, nrhs, seed):
    """Right-hand sides, i.i.d. N(0, 1), shape (n, nrhs)."""
    return _rng(seed, _STREAM_RHS).standard_normal((n, nrhs))
