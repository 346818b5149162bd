"""The matrix types of the paper's numerical experiments (Section 5).

Inputs only: these functions build the symmetric test matrices the paper
defines and hold none of the factorization's arithmetic.  Random entries come
from NumPy's PCG64 (the paper used LAPACK's DLARNV), seeded per matrix.

  type1   the Bunch-Kaufman worst case for element growth:
          [[A1, (1 - eps) I], [(1 - eps) I, 0]], A1 = diag(d_1 .. d_{m-2})
          bordered by two rows and columns of ones, d_k = q^(1-k) / (1 - q),
          q = 1 + 1/alpha, alpha = (1 + sqrt(17)) / 8; order 2 m
  type2   the bounded Bunch-Kaufman worst case for work: zero except
          A(1, n) = 2, A(2, 2) = n and A(k, k+1) = n + 2 - k for k = 2 .. n-1
          (1-based, mirrored)
  type3   Hankel: A(i, j) = a_{i+j-1}, a_1 .. a_{2n-1} i.i.d. N(0, 1)
  type4   discrete sine transform: sqrt(2/(n+1)) sin(i j pi / (n+1))
  type5   discrete cosine transform: cos((i-1)(j-1) pi / (n-1))
  type6   Gaussian, symmetrised as (G + G^T)/2 (gen.gaussian_sym)
  type7   KKT [[H, C^T], [C, 0]] (gen.kkt)
  type8   augmented system [[I, W], [W^T, 0]], W i.i.d. N(0, 1)
  type10  rank deficient W Lambda W^T, W i.i.d. N(0, 1),
          lambda_i = q^(1-i) / (1 - q), q = 1 + sqrt(2)

Readings where the paper leaves a choice open: eps = 2^-10 in type 1; the
zero block of types 7 and 8 has order n2 = floor(n/4) (n1 = n - n2); type 7
uses the saddle-point generator of the benchmark workloads (H symmetric
positive definite with a log-uniform spectrum in [1e-3, 1], C i.i.d.
N(0, 1)/sqrt(n1)), the paper leaving its leading block unspecified.
"""

import numpy as np

from . import gen

TYPE1_EPS = 2.0 ** -10


def _rng(seed, stream):
    return np.random.default_rng(np.random.SeedSequence([int(seed), stream]))


def type1(n, eps=TYPE1_EPS):
    """Bunch-Kaufman worst case, order n (even, n >= 6)."""
    if n % 2 or n < 6:
        raise ValueError("type 1 needs an even order n >= 6")
    m = n // 2
    alpha = (1.0 + np.sqrt(17.0)) / 8.0
    q = 1.0 + 1.0 / alpha
    k = np.arange(1, m - 1, dtype=np.float64)
    d = q ** (1.0 - k) / (1.0 - q)
    A1 = np.zeros((m, m))
    A1[np.arange(m - 2), np.arange(m - 2)] = d
    A1[m - 2:, :] = 1.0
    A1[:, m - 2:] = 1.0
    A = np.zeros((n, n))
    A[:m, :m] = A1
    A[m:, :m] = (1.0 - eps) * np.eye(m)
    A[:m, m:] = (1.0 - eps) * np.eye(m)
    return A


def type2(n):
    """Bounded Bunch-Kaufman worst case, order n >= 3."""
    if n < 3:
        raise ValueError("type 2 needs n >= 3")
    A = np.zeros((n, n))
    A[0, n - 1] = A[n - 1, 0] = 2.0
    A[1, 1] = float(n)
    for k in range(2, n):              # 1-based k = 2 .. n-1
        A[k - 1, k] = A[k, k - 1] = float(n + 2 - k)
    return A


def type3(n, seed):
    """Hankel matrix with i.i.d. N(0, 1) anti-diagonals."""
    a = _rng(seed, 30).standard_normal(2 * n - 1)
    i = np.arange(n)
    return a[i[:, None] + i[None, :]]


def type4(n):
    """Discrete sine transform matrix (symmetric and orthogonal)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(i, i) * np.pi / (n + 1))


def type5(n):
    """Discrete cosine transform matrix, order n >= 2."""
    if n < 2:
        raise ValueError("type 5 needs n >= 2")
    i = np.arange(n, dtype=np.float64)
    return np.cos(np.outer(i, i) * np.pi / (n - 1))


def _blocks(n):
    n2 = n // 4
    return n - n2, n2


def type6(n, seed):
    return gen.gaussian_sym(n, seed)


def type7(n, seed):
    n1, _ = _blocks(n)
    return gen.kkt(n, n1, seed, nrefl=min(64, n1))


def type8(n, seed):
    """Augmented system [[I, W], [W^T, 0]], W (n1 x n2) i.i.d. N(0, 1)."""
    n1, n2 = _blocks(n)
    W = _rng(seed, 80).standard_normal((n1, n2))
    A = np.zeros((n, n))
    A[:n1, :n1] = np.eye(n1)
    A[:n1, n1:] = W
    A[n1:, :n1] = W.T
    return A


def type10(n, seed):
    """Rank-deficient W Lambda W^T (numerical rank about 42)."""
    q = 1.0 + np.sqrt(2.0)
    i = np.arange(1, n + 1, dtype=np.float64)
    lam = q ** (1.0 - i) / (1.0 - q)
    W = _rng(seed, 100).standard_normal((n, n))
    A = (W * lam[None, :]) @ W.T
    # exactly symmetric: mirror the lower triangle
    il = np.tril_indices(n, -1)
    A[il[1], il[0]] = A[il]
    return A


TYPES = {
    1: lambda n, seed: type1(n),
    2: lambda n, seed: type2(n),
    3: type3,
    4: lambda n, seed: type4(n),
    5: lambda n, seed: type5(n),
    6: type6,
    7: type7,
    8: type8,
    10: type10,
}


def matrix(kind, n, seed=0):
    """Type `kind` (1..8, 10) of order n."""
    return TYPES[kind](n, seed)
