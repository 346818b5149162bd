"""Blocked randomized complete pivoting (RCP), FP64 -- TEST INFRASTRUCTURE.

Plain NumPy transcription of the paper's Algorithm 1 (Section 3), branch
q = b, written from the paper's description:

  * sketch            B = Omega A                              (Section 3)
  * per block         partial QRCP on B(:, k:n) picks b column pivots and
                      they are interchanged into positions k .. k+b-1
                      (Algorithm 1, q = b branch; Section 3.1)
  * per step          simplified Bunch-Kaufman pivoting (SBKP, Figure 2) on
                      the current column, then D and L columns as in a
                      SYTRF-style panel (Section 3.1, Section 2.2)
  * per block end     sketch update B(:,k:n) -= B~_1 L11^{-T} L21^T (block
                      form of eq. (3.3)) and the delayed Schur complement
                      update A22 -= L21 D1 L21^T (Algorithm 1, Section 3.1)
  * last pivot        D(n,n) = A(n,n) (Algorithm 1)

Positions (0-based) are used everywhere: ``perm[i]`` is the original index of
the row/column that sits at position i, so (P A P^T)[i, j] = A[perm[i],
perm[j]] and P A P^T = L D L^T.  Every interchange is applied at once to the
working matrix S, the sketch B, the computed rows of L and W = L D, and perm.

Readings of the paper that this file fixes (each is also listed in the design
notes of the repository):
  * the sketch has l = b + p rows, p the oversampling (Section 3.1, p = q+4);
  * QRCP is greedy: at step j the column of largest residual norm (squared
    norms compared, no downdating, recomputed each step) goes to position
    K0+j by one transposition; ties go to the smallest position; it stops
    early if the largest residual norm is 0;
  * SBKP: r is the smallest position attaining lambda (the tie rule of the
    Bunch-Kaufman footnote, Section 2.3); the tests are |a| >= fl(alpha *
    lambda) with alpha the double nearest sqrt(2)/2; lambda = 0 gives a 1x1
    pivot with a zero column of L ("nothing to do"), and a zero pivot value
    sets info to its 1-based position;
  * a 2x2 pivot may start at the last slot of a block, which then
    eliminates b+1 columns; the next block starts after it;
  * the block sketch update uses L11^{-T} (the derivation of eq. (3.3)
    applied to a block gives B~_2 - B~_1 L11^{-T} L21^T; for one column it is
    eq. (3.3) itself);
  * the multipliers of a 2x2 pivot use Cramer's rule exactly as written in
    the proof of Theorem 3.2 (Section 4.2).
"""

import numpy as np
from scipy.linalg import solve_triangular

from . import omega as omega_mod

ALPHA = np.sqrt(2.0) / 2.0   # Figure 2: alpha = sqrt(2)/2


class Factorization:
    """Result of :func:`factor` (all arrays in positions)."""

    def __init__(self, n):
        self.n = n
        self.perm = np.arange(n, dtype=np.int64)
        self.L = np.eye(n)
        self.D = np.zeros(2 * n)       # D[i] = d_ii, D[n+i] = d_{i+1,i}
        self.ipiv = np.zeros(n, dtype=np.int8)   # 1, or 2 then 0 for a 2x2
        self.info = 0
        self.log = []                  # decision log, one dict per decision
        self.rho_elem = None           # element growth (eager schedule only)
        self.block_starts = []
        self.sketch_at_block_start = []   # (K0, perm copy, B(:, K0:) copy) if recorded
        self.sketch_scale = 0.0        # largest column norm of the initial sketch
        self.rank = n                  # eliminated columns (< n: Algorithm 2 stopped)
        self.recomputed = []           # block starts where Algorithm 2 recomputed B

    def dmatrix(self):
        """D as an n x n block-diagonal matrix."""
        n = self.n
        Dm = np.diag(self.D[:n].copy())
        for i in range(n - 1):
            if self.ipiv[i] == 2:
                Dm[i + 1, i] = Dm[i, i + 1] = self.D[n + i]
        return Dm


def symmetric_from_lower(A):
    """The symmetric matrix whose lower triangle is that of A."""
    A = np.asarray(A, dtype=np.float64)
    return np.tril(A) + np.tril(A, -1).T


EPS = 2.0 ** -52   # machine precision of Algorithm 2 (the spacing of doubles at 1)


def factor(A, b, p, seed=0, omega=None, schedule="delayed", record_sketch=False,
           trace=False, recompute=1, q=None):
    """RCP block LDL^T of the symmetric matrix given by the lower triangle of A.

    A        n x n array; only A[i, j] with i >= j is read
    b        block size (number of QRCP pivots per block, q = b)
    p        oversampling; Omega has l = b + p rows
    seed     seed of Omega (see omega.omega); ignored when ``omega`` is given
    omega    optional explicit l x n sketching matrix (tests)
    schedule "delayed": Schur complement updated once per block, current
             columns built left-looking (Algorithm 1 as implemented in the
             paper); "eager": updated after every pivot (same result in
             exact arithmetic, also tracks the element growth factor)
    record_sketch  keep (K0, perm, B(:, K0:)) at every block start
    trace    keep a copy of perm in every decision-log entry (small n only)
    q        pivots chosen per sketch (Algorithm 1): None or b is the q = b
             branch (a b-step partial QRCP per block); 1 is the q = 1 branch:
             before every SBKP step the trailing column of largest sketch norm
             (ties: smallest position) is interchanged into position k, and
             after it the sketch is updated by the step's pivot columns,
             B(:, k+s:n) -= B(:, k:k+s-1) L(k+s:n, k:k+s-1)^T (eq. (3.3);
             inside a 2x2 block L11 = I).  The sketch then has l = 1 + p rows.
    recompute  r of Algorithm 2 (Section 4.5): with r = 1 this is Algorithm 1.
             With r >= 2, beta is the largest column norm of the first
             sketch and delta = (j+1)/r after j recomputations; while
             delta < 1, at every block start after the first the largest
             column norm t of the current sketch is compared with
             EPS^delta beta.  Below it, the sketch of the current Schur
             complement is recomputed with a fresh Omega (stream 1 + j of the
             seed, see omega.omega), j grows by one, and if the new t is still
             below EPS^delta beta the factorization stops there: the
             remaining Schur complement counts as zero (D = 0, 1x1 blocks,
             zero columns of L), ``f.rank`` is the number of eliminated
             columns and ``f.info`` the 1-based position after them.  The
             block starts that recomputed are in ``f.recomputed``.
    """
    S = symmetric_from_lower(A).copy()
    n = S.shape[0]
    f = Factorization(n)
    if n == 0:
        return f
    q1 = q == 1
    if omega is None:
        Om = omega_mod.omega(seed, (1 if q1 else b) + p, n)
    else:
        Om = np.asarray(omega, dtype=np.float64)
    l = Om.shape[0]
    B = Om @ S                       # the sketch B = Omega A
    # largest column norm of the first sketch: the scale of the absolute
    # errors of every later sketch value (used by decision_margins)
    f.sketch_scale = float(np.sqrt(np.max(np.einsum("ij,ij->j", B, B))))
    L = np.zeros((n, n))             # strictly lower part of L, by position
    W = np.zeros((n, n))             # W = L D for the current block's columns
    perm = f.perm
    amax = np.max(np.abs(S)) if n else 0.0
    growth = amax
    eager = schedule == "eager"

    def interchange(p1, p2):
        if p1 == p2:
            return
        ix, iy = [p1, p2], [p2, p1]
        S[ix, :] = S[iy, :]
        S[:, ix] = S[:, iy]
        B[:, ix] = B[:, iy]
        L[ix, :] = L[iy, :]
        W[ix, :] = W[iy, :]
        perm[ix] = perm[iy]

    def column(c, k, kd):
        """Current Schur column at position c, rows k..n-1 (left-looking over
        the not yet applied block columns kd..k-1)."""
        if k > kd:
            return S[k:, c] - L[k:, kd:k] @ W[c, kd:k]
        return S[k:, c].copy()

    def qrcp(K0, bb):
        """Greedy partial QR with column pivoting on B(:, K0:n)."""
        R = B[:, K0:].copy()
        N = n - K0
        for j in range(min(bb, l, N)):
            sub = R[j:, j:]
            nrm2 = np.einsum("ij,ij->j", sub, sub)
            c = int(np.argmax(nrm2))          # first maximum = smallest position
            best = nrm2[c]
            others = np.delete(nrm2, c)
            second = others.max() if others.size else 0.0
            f.log.append(dict(kind="qrcp", K0=K0, j=j, pos=K0 + j + c,
                              best=best, second=second))
            if trace:
                f.log[-1]["perm"] = perm.copy()
            if best == 0.0:
                break
            cj = j + c
            if cj != j:
                interchange(K0 + j, K0 + cj)
                R[:, [j, cj]] = R[:, [cj, j]]
            x = R[j:, j]
            v = x.copy()
            v[0] += np.copysign(np.sqrt(x @ x), x[0])
            vv = v @ v
            R[j:, j + 1:] -= np.outer(v, (2.0 / vv) * (v @ R[j:, j + 1:]))

    def sketch_argmax(k):
        """q = 1: the trailing column of largest sketch norm goes to k."""
        nrm2 = np.einsum("ij,ij->j", B[:, k:], B[:, k:])
        c = int(np.argmax(nrm2))              # first maximum = smallest position
        best = nrm2[c]
        others = np.delete(nrm2, c)
        second = others.max() if others.size else 0.0
        f.log.append(dict(kind="qrcp", K0=k, j=0, pos=k + c, best=best, second=second))
        if trace:
            f.log[-1]["perm"] = perm.copy()
        interchange(k, k + c)

    def sbkp(k, kd):
        """One step of Figure 2 at position k; returns s in {1, 2}."""
        col = column(k, k, kd)
        akk = col[0]
        rec = dict(kind="sbkp", k=k, akk=akk, r=None, lam=0.0, lam2=0.0, arr=None)
        if trace:
            rec["perm"] = perm.copy()
        if k < n - 1:
            off = np.abs(col[1:])
            j = int(np.argmax(off))           # smallest position on ties
            rec["r"] = r = k + 1 + j
            rec["lam"] = lam = off[j]
            rest = np.delete(off, j)
            rec["lam2"] = rest.max() if rest.size else 0.0
        else:
            lam = 0.0
        if lam == 0.0:
            case = 0                           # nothing to eliminate
        elif abs(akk) >= ALPHA * lam:
            case = 1
        else:
            colr = column(r, k, kd)
            arr = colr[r - k]
            rec["arr"] = arr
            if abs(arr) >= ALPHA * lam:
                case = 2
                interchange(k, r)
            else:
                case = 3
                interchange(k + 1, r)
        rec["case"] = case
        f.log.append(rec)
        if case in (0, 1, 2):
            col = column(k, k, kd)
            d = col[0]
            if d != 0.0:
                L[k + 1:, k] = col[1:] / d
            else:
                L[k + 1:, k] = 0.0
                if f.info == 0:
                    f.info = k + 1
            W[k, k] = d
            W[k + 1:, k] = L[k + 1:, k] * d
            f.D[k] = d
            f.ipiv[k] = 1
            return 1
        c0 = column(k, k, kd)
        c1 = column(k + 1, k, kd)
        e00, e10, e11 = c0[0], c0[1], c1[1]
        det = e00 * e11 - e10 * e10
        x, y = c0[2:], c1[2:]
        L[k + 2:, k] = (x * e11 - e10 * y) / det
        L[k + 2:, k + 1] = (e00 * y - e10 * x) / det
        W[k, k], W[k, k + 1], W[k + 1, k], W[k + 1, k + 1] = e00, e10, e10, e11
        W[k + 2:, k] = L[k + 2:, k] * e00 + L[k + 2:, k + 1] * e10
        W[k + 2:, k + 1] = L[k + 2:, k] * e10 + L[k + 2:, k + 1] * e11
        f.D[k], f.D[k + 1], f.D[n + k] = e00, e11, e10
        f.ipiv[k], f.ipiv[k + 1] = 2, 0
        return 2

    beta = f.sketch_scale
    nrec = 0

    def sketch_max(K0):
        return float(np.sqrt(np.max(np.einsum("ij,ij->j", B[:, K0:], B[:, K0:]))))

    k = 0
    while k < n:
        K0 = k
        bb = min(b, n - k)
        if recompute > 1 and K0 > 0 and nrec + 1 < recompute:
            # Algorithm 2: is the largest column norm of the sketch still
            # above EPS^delta beta?
            if sketch_max(K0) < EPS ** ((nrec + 1) / recompute) * beta:
                nrec += 1
                Om_j = omega_mod.omega(seed, l, n - K0, stream=omega_mod.STREAM_OMEGA + nrec)
                B[:, K0:] = Om_j @ S[K0:, K0:]
                f.recomputed.append(K0)
                if sketch_max(K0) < EPS ** ((nrec + 1) / recompute) * beta:
                    # rank deficient: the Schur complement is taken as zero
                    f.rank = K0
                    f.D[K0:n] = 0.0
                    f.D[n + K0:] = 0.0
                    f.ipiv[K0:] = 1
                    if f.info == 0:
                        f.info = K0 + 1
                    break
        f.block_starts.append(K0)
        if record_sketch:
            f.sketch_at_block_start.append((K0, perm.copy(), B[:, K0:].copy()))
        if not q1:
            qrcp(K0, bb)
        i = 0
        while i < bb and k < n:
            if q1:
                sketch_argmax(k)
            s = sbkp(k, K0 if not eager else k)
            if q1 and k + s < n:
                # eq. (3.3): the sketch of the new Schur complement
                t = slice(k, k + s)
                B[:, k + s:] -= B[:, t] @ L[k + s:, t].T
            if eager and k + s < n:
                t = slice(k, k + s)
                S[k + s:, k + s:] -= L[k + s:, t] @ W[k + s:, t].T
                growth = max(growth, np.max(np.abs(S[k + s:, k + s:])))
            k += s
            i += s
        if k < n and q1:
            if not eager:
                S[k:, k:] -= L[k:, K0:k] @ W[k:, K0:k].T
        elif k < n:
            # sketch update: B(:, k:n) -= B~_1 L11^{-T} L21^T
            L11 = np.tril(L[K0:k, K0:k], -1) + np.eye(k - K0)
            T = solve_triangular(L11, B[:, K0:k].T, lower=True, unit_diagonal=True).T
            B[:, k:] -= T @ L[k:, K0:k].T
            if not eager:
                # delayed Schur complement update A22 -= L21 D1 L21^T
                S[k:, k:] -= L[k:, K0:k] @ W[k:, K0:k].T
    f.L = np.tril(L, -1) + np.eye(n)
    if eager:
        f.rho_elem = growth / amax if amax > 0 else 1.0
    f.sketch = B
    return f


def solve(f, Bm):
    """x = P^T L^{-T} D^{-1} L^{-1} P b for every column b of Bm (Table 1,
    solution phase).  2x2 blocks of D use Cramer's rule."""
    Bm = np.asarray(Bm, dtype=np.float64)
    vec = Bm.ndim == 1
    if vec:
        Bm = Bm[:, None]
    n = f.n
    c = Bm[f.perm]
    y = solve_triangular(f.L, c, lower=True, unit_diagonal=True)
    w = y.copy()
    k = 0
    while k < n:
        if f.ipiv[k] == 2:
            e00, e11, e10 = f.D[k], f.D[k + 1], f.D[n + k]
            det = e00 * e11 - e10 * e10
            w[k] = (e11 * y[k] - e10 * y[k + 1]) / det
            w[k + 1] = (e00 * y[k + 1] - e10 * y[k]) / det
            k += 2
        else:
            w[k] = y[k] / f.D[k]
            k += 1
    z = solve_triangular(f.L, w, lower=True, trans="T", unit_diagonal=True)
    x = np.empty_like(z)
    x[f.perm] = z
    return x[:, 0] if vec else x


def min_margin(f, scale=None):
    """Smallest relative gap of any decision in the log (near-tie detector).

    QRCP picks: (best - second) / best of the squared residual norms.
    SBKP: (lam - lam2) / lam for the choice of r, and | |a| - alpha*lam | /
    lam for each threshold test that was evaluated.  A lambda that is zero
    or tiny relative to ``scale`` counts as a margin of lam / scale.
    Returns (margin, index into f.log).
    """
    if scale is None:
        scale = 1.0
    best = (np.inf, -1)
    for idx, e in enumerate(f.log):
        if e["kind"] == "qrcp":
            if e["best"] > 0 and e["second"] > 0:
                m = (e["best"] - e["second"]) / e["best"]
                best = min(best, (m, idx))
            continue
        lam = e["lam"]
        if e["r"] is None:
            continue
        ms = [lam / scale]
        if lam > 0:
            ms.append((lam - e["lam2"]) / lam)
            ms.append(abs(abs(e["akk"]) - ALPHA * lam) / lam)
            if e["arr"] is not None:
                ms.append(abs(abs(e["arr"]) - ALPHA * lam) / lam)
        best = min(best, (min(ms), idx))
    return best


def decision_margins(f, scale):
    """Margin of every logged decision, relative and absolute (near-tie data).

    A decision compares computed values; a second FP64 implementation that
    sums in another order gets each of them with an absolute error of order
    n u times the problem's scale, so a decision is fragile when its gap is
    small against that scale -- however large it is against the compared
    values themselves, which at the end of a factorization are far below the
    scale.  For every decision with at least one comparison this returns
    (kind, position, rel, abs):

      QRCP pick (kind 0, position K0 + j): the gap between the largest and
        the second largest residual norm, sqrt(best) - sqrt(second);
        rel = gap / sqrt(best), abs = gap / f.sketch_scale;
      SBKP step (kind 1, position k): the gaps lambda - lambda_2 (choice of
        r), | |a_kk| - alpha lambda | and, when it was evaluated,
        | |a_rr| - alpha lambda | (Figure 2's threshold tests), and lambda
        itself (the test lambda = 0); rel divides the smallest by lambda
        (lambda = 0 gives rel = 0), abs divides it by ``scale`` (max |A|).

    Decisions without a comparison (a lone candidate) are left out.  Returns
    four NumPy arrays.
    """
    kinds, pos, rel, ab = [], [], [], []
    sb = f.sketch_scale if f.sketch_scale > 0 else 1.0
    sa = scale if scale > 0 else 1.0
    for e in f.log:
        if e["kind"] == "qrcp":
            if e["best"] <= 0 or e["second"] <= 0:
                continue
            gap = np.sqrt(e["best"]) - np.sqrt(e["second"])
            kinds.append(0)
            pos.append(e["K0"] + e["j"])
            rel.append(gap / np.sqrt(e["best"]))
            ab.append(gap / sb)
            continue
        if e["r"] is None:
            continue
        lam = e["lam"]
        gaps = [lam, lam - e["lam2"], abs(abs(e["akk"]) - ALPHA * lam)]
        if e["arr"] is not None:
            gaps.append(abs(abs(e["arr"]) - ALPHA * lam))
        g = min(gaps)
        kinds.append(1)
        pos.append(e["k"])
        rel.append(g / lam if lam > 0 else 0.0)
        ab.append(g / sa)
    return (np.array(kinds, dtype=np.int8), np.array(pos, dtype=np.int64),
            np.array(rel, dtype=np.float64), np.array(ab, dtype=np.float64))


def near_tie_prefix(f, scale, tau=1e-9):
    """Length of the pivot sequence that no near-tie can change: the smallest
    position decided by a decision whose absolute margin (decision_margins)
    is <= tau, or n if there is none.  Positions before it are decided only
    by decisions with margins above tau, and the interchanges of a later
    decision never move an earlier position."""
    _, pos, _, ab = decision_margins(f, scale)
    bad = pos[ab <= tau]
    return int(bad.min()) if bad.size else f.n
