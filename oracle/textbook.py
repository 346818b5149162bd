"""Independent comparators for the RCP oracle -- TEST INFRASTRUCTURE.

None of these functions shares arithmetic with ``oracle.rcp``; they compute
the same quantities from their textbook definitions (or by brute force), so
the tests can pin the oracle against them.
"""

import numpy as np

ALPHA_BP = (1.0 + np.sqrt(17.0)) / 8.0   # Bunch-Parlett / Bunch-Kaufman alpha (Section 2.3)


def sym(A):
    A = np.asarray(A, dtype=np.float64)
    return np.tril(A) + np.tril(A, -1).T


def permuted(A, perm):
    """P A P^T with (P A P^T)[i, j] = A[perm[i], perm[j]]."""
    perm = np.asarray(perm)
    return sym(A)[np.ix_(perm, perm)]


def schur_complement(M, k):
    """A22 - A21 A11^{-1} A21^T of a symmetric M after its first k rows and
    columns (Section 2.2), by a dense solve."""
    if k == 0:
        return M.copy()
    A11 = M[:k, :k]
    A21 = M[k:, :k]
    return M[k:, k:] - A21 @ np.linalg.solve(A11, A21.T)


def block_ldlt_given(A, perm, ipiv):
    """Block LDL^T of P A P^T with the block pattern given by ipiv and no
    pivoting: plain right-looking elimination of Section 2.2.  Returns
    (L, Dm) with Dm the block-diagonal matrix."""
    M = permuted(A, perm)
    n = M.shape[0]
    L = np.eye(n)
    Dm = np.zeros((n, n))
    k = 0
    while k < n:
        s = 2 if ipiv[k] == 2 else 1
        E = M[k:k + s, k:k + s].copy()
        Dm[k:k + s, k:k + s] = E
        if k + s < n:
            if s == 1 and E[0, 0] == 0.0:
                Lk = np.zeros((n - k - s, 1))
            else:
                Lk = M[k + s:, k:k + s] @ np.linalg.inv(E)
            L[k + s:, k:k + s] = Lk
            M[k + s:, k + s:] -= Lk @ E @ Lk.T
        k += s
    return L, Dm


def all_schur_complements(A, perm, ipiv):
    """A^{(k)} at every block boundary k of the pattern (dense solves)."""
    M = permuted(A, perm)
    n = M.shape[0]
    out = []
    k = 0
    while k < n:
        out.append((k, schur_complement(M, k)))
        k += 2 if ipiv[k] == 2 else 1
    return out


def growth_factors(A, perm, ipiv):
    """(rho_elem, rho_col) of Definitions 2.2 and 2.3 by brute force."""
    M = sym(A)
    e0 = np.max(np.abs(M))
    c0 = np.max(np.linalg.norm(M, axis=0))
    e, c = e0, c0
    for _, S in all_schur_complements(A, perm, ipiv):
        if S.size:
            e = max(e, np.max(np.abs(S)))
            c = max(c, np.max(np.linalg.norm(S, axis=0)))
    return e / e0, c / c0


def norm_12(M):
    """||M||_{1,2}: largest column 2-norm (Section 2.1)."""
    return np.max(np.linalg.norm(M, axis=0))


def norm_1inf(M):
    """||M||_{1,inf}: largest absolute entry (Section 2.1)."""
    return np.max(np.abs(M))


def greedy_columns_lstsq(B, q):
    """Greedy column selection: at step j pick the column whose residual,
    after least-squares projection onto the picked columns, has the largest
    norm (ties: smallest index).  Returns picked column indices of B."""
    B = np.asarray(B, dtype=np.float64)
    picks = []
    for _ in range(min(q, B.shape[0], B.shape[1])):
        best, arg = -1.0, -1
        for c in range(B.shape[1]):
            if c in picks:
                continue
            if picks:
                Q = B[:, picks]
                coef = np.linalg.lstsq(Q, B[:, c], rcond=None)[0]
                res = B[:, c] - Q @ coef
            else:
                res = B[:, c]
            v = res @ res
            if v > best:
                best, arg = v, c
        if best <= 0:
            break
        picks.append(arg)
    return picks


def transpositions_to_positions(picks, N):
    """Simulate moving pick j (an index into the original order) to slot j by
    one transposition with whatever occupies slot j.  Returns (found, order):
    the slot where each pick sat when it was taken, and the final order."""
    order = list(range(N))
    where = list(range(N))
    found = []
    for j, c in enumerate(picks):
        pc = where[c]
        found.append(pc)
        oj = order[j]
        order[j], order[pc] = order[pc], order[j]
        where[c], where[oj] = j, pc
    return found, order


def bunch_parlett(A):
    """Symmetric complete pivoting (Bunch and Parlett): at each step take the
    largest diagonal entry as a 1x1 pivot if it is >= alpha * (largest entry
    of the Schur complement), else the 2x2 pivot holding that largest entry.
    Returns (perm, L, Dm, ipiv, rho_elem)."""
    M = sym(A).copy()
    n = M.shape[0]
    perm = np.arange(n)
    L = np.zeros((n, n))
    Dm = np.zeros((n, n))
    ipiv = np.zeros(n, dtype=np.int8)
    a0 = np.max(np.abs(M)) if n else 1.0
    grow = a0

    def swap(i, j):
        if i == j:
            return
        M[[i, j], :] = M[[j, i], :]
        M[:, [i, j]] = M[:, [j, i]]
        L[[i, j], :] = L[[j, i], :]
        perm[[i, j]] = perm[[j, i]]

    k = 0
    while k < n:
        S = M[k:, k:]
        mu0 = np.max(np.abs(S))
        d = np.abs(np.diag(S))
        mu1 = np.max(d)
        if mu0 == 0.0 or mu1 >= ALPHA_BP * mu0:
            swap(k, k + int(np.argmax(d)))
            s = 1
        else:
            flat = int(np.argmax(np.abs(np.tril(S, -1))))
            i, j = divmod(flat, S.shape[0])
            swap(k, k + j)
            swap(k + 1, k + i)
            s = 2
        E = M[k:k + s, k:k + s].copy()
        Dm[k:k + s, k:k + s] = E
        if k + s < n:
            Lk = M[k + s:, k:k + s] @ np.linalg.inv(E) if np.any(E) else 0.0 * M[k + s:, k:k + s]
            L[k + s:, k:k + s] = Lk
            M[k + s:, k + s:] -= Lk @ E @ Lk.T
            grow = max(grow, np.max(np.abs(M[k + s:, k + s:])))
        ipiv[k] = 1 if s == 1 else 2
        if s == 2:
            ipiv[k + 1] = 0
        k += s
    return perm, np.tril(L, -1) + np.eye(n), Dm, ipiv, grow / a0


def backward_error(A, x, b):
    """||A x - b||_inf / (||A||_inf ||x||_inf) (eq. (5.1)), per column."""
    A = sym(A)
    x = np.atleast_2d(np.asarray(x).T).T
    b = np.atleast_2d(np.asarray(b).T).T
    r = A @ x - b
    anorm = np.max(np.sum(np.abs(A), axis=1))
    return np.max(np.abs(r), axis=0) / (anorm * np.max(np.abs(x), axis=0))


def reconstruction_error(A, perm, L, Dm):
    """||P A P^T - L D L^T||_inf / ||A||_inf."""
    M = permuted(A, perm)
    R = M - L @ Dm @ L.T
    return np.max(np.sum(np.abs(R), axis=1)) / np.max(np.sum(np.abs(M), axis=1))


def lemma31_p(n, eps, delta):
    """Oversampling required by Lemma 3.1: 4/(eps^2 - eps^3) ln(n(n+1)/delta)."""
    return 4.0 / (eps ** 2 - eps ** 3) * np.log(n * (n + 1) / delta)
