"""Pins for the RCP oracle (oracle/rcp.py) against things the paper and the
mathematics fix: hand-derived cases of Figure 2, brute-force Schur
complements, greedy column selection by least squares, the block sketch
identity, uniqueness of L and D given (Pi, Delta), textbook block LDL^T,
Bunch-Parlett complete pivoting, and the invariants of Section 4.
"""

import json
import os

import numpy as np
import pytest

from oracle import rcp, textbook as tb
from oracle.omega import omega as omega_matrix
from workloads import gen

U = np.finfo(np.float64).eps / 2
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cases():
    out = []
    for n, b, p, seed in [(1, 4, 2, 1), (2, 4, 2, 2), (3, 2, 2, 3), (5, 2, 3, 4),
                          (8, 3, 4, 5), (17, 4, 4, 6), (33, 8, 4, 7), (64, 8, 8, 8),
                          (64, 16, 2, 9), (100, 32, 8, 10)]:
        out.append((n, b, p, seed))
    return out


@pytest.mark.parametrize("n,b,p,seed", _cases())
def test_reconstruction_and_schedules(n, b, p, seed):
    A = gen.gaussian_sym(n, seed)
    f = rcp.factor(A, b, p, seed=seed)
    fe = rcp.factor(A, b, p, seed=seed, schedule="eager")
    # same decisions from the delayed and the eager Schur schedule
    assert np.array_equal(f.perm, fe.perm) and np.array_equal(f.ipiv, fe.ipiv)
    assert np.allclose(f.L, fe.L, atol=1e-12) and np.allclose(f.D, fe.D, atol=1e-12)
    assert tb.reconstruction_error(A, f.perm, f.L, f.dmatrix()) <= 50 * n * U
    assert sorted(f.perm) == list(range(n))
    # L unit lower, zero inside 2x2 blocks
    assert np.array_equal(np.triu(f.L, 1), np.zeros((n, n)))
    assert np.all(np.diag(f.L) == 1.0)
    for i in range(n - 1):
        if f.ipiv[i] == 2:
            assert f.L[i + 1, i] == 0.0 and f.ipiv[i + 1] == 0


def test_only_lower_triangle_is_read():
    A = gen.gaussian_sym(20, 3)
    junk = A + np.triu(np.random.default_rng(0).standard_normal((20, 20)), 1)
    f1, f2 = rcp.factor(A, 4, 4, seed=5), rcp.factor(junk, 4, 4, seed=5)
    assert np.array_equal(f1.perm, f2.perm) and np.array_equal(f1.L, f2.L)


def test_golden_sbkp_cases():
    cases = json.load(open(os.path.join(GOLDEN, "sbkp_cases.json")))["cases"]
    for c in cases:
        A = np.array(c["A"])
        n = A.shape[0]
        f = rcp.factor(A, 1, n - 1, omega=np.eye(n), trace=True)
        assert list(f.ipiv) == c["ipiv"], c["name"]
        assert np.allclose(f.D[:n], c["D_diag"], rtol=0, atol=1e-15), c["name"]
        assert np.allclose(f.D[n:], c["D_sub"], rtol=0, atol=1e-15), c["name"]
        if "perm" in c:
            assert list(f.perm) == c["perm"], c["name"]
            assert np.allclose(f.L, c["L"], rtol=0, atol=1e-15), c["name"]
        if "exact_case_sequence" in c:
            cs = [e["case"] for e in f.log if e["kind"] == "sbkp"]
            assert cs == c["exact_case_sequence"], c["name"]
        if "det" in c:
            assert f.D[0] * f.D[1] - f.D[n] ** 2 == c["det"]
        # the 2x2 examples do not depend on which column QRCP takes first
        f2 = rcp.factor(A, 2, 3, seed=17)
        assert list(f2.ipiv) == c["ipiv"] or "perm" in c


def test_diagonal_matrix_never_eliminates():
    d = np.array([3.0, -1.0, 0.5, 7.0, -2.0, 0.25])
    f = rcp.factor(np.diag(d), 2, 3, seed=1)
    assert np.array_equal(f.L, np.eye(6))
    assert np.all(f.ipiv == 1)
    assert np.array_equal(f.D[:6], d[f.perm])
    assert all(e["case"] == 0 for e in f.log if e["kind"] == "sbkp")


def test_zero_pivot_sets_info():
    A = np.diag([2.0, 0.0, 5.0])
    f = rcp.factor(A, 3, 2, omega=np.eye(3))
    # Omega = I: QRCP orders the columns by norm, 5, 2, 0
    assert list(f.perm) == [2, 0, 1]
    assert f.info == 3
    assert rcp.factor(np.zeros((4, 4)), 2, 2, seed=3).info == 1


def _rank_sbkp_check(A, f):
    """Audit every SBKP decision on the brute-force Schur complement."""
    n = f.n
    ipiv_so_far = []
    for e in f.log:
        if e["kind"] != "sbkp":
            continue
        k = e["k"]
        M = tb.permuted(A, e["perm"])
        S = tb.schur_complement(M, k)
        col = S[:, 0]
        scale = max(1.0, np.max(np.abs(S)))
        assert abs(col[0] - e["akk"]) <= 1e-9 * scale
        if k == n - 1:
            assert e["case"] == 0
            continue
        off = np.abs(col[1:])
        lam = off.max()
        assert abs(lam - e["lam"]) <= 1e-9 * scale
        if e["lam"] > 0:
            assert e["r"] == k + 1 + int(np.argmax(off))
        a = rcp.ALPHA
        if e["case"] == 0:
            assert e["lam"] == 0.0
        elif e["case"] == 1:
            assert abs(e["akk"]) >= a * e["lam"]
        else:
            assert abs(e["akk"]) < a * e["lam"]
            arr = S[e["r"] - k, e["r"] - k]
            assert abs(arr - e["arr"]) <= 1e-9 * scale
            if e["case"] == 2:
                assert abs(e["arr"]) >= a * e["lam"]
            else:
                assert abs(e["arr"]) < a * e["lam"]
        ipiv_so_far.append(e["case"])


@pytest.mark.parametrize("n,b,p,seed", [(12, 3, 3, 1), (25, 4, 4, 2), (40, 8, 2, 3)])
def test_sbkp_decisions_against_bruteforce_schur(n, b, p, seed):
    for A in (gen.gaussian_sym(n, seed), gen.kkt(n, (3 * n) // 4, seed, nrefl=4)):
        f = rcp.factor(A, b, p, seed=seed, trace=True)
        _rank_sbkp_check(A, f)


@pytest.mark.parametrize("n,b,p,seed", [(12, 3, 3, 1), (30, 5, 4, 2), (48, 8, 4, 3)])
def test_qrcp_and_sketch_identity_against_bruteforce(n, b, p, seed):
    A = gen.gaussian_sym(n, seed)
    Om = omega_matrix(seed, b + p, n)
    f = rcp.factor(A, b, p, seed=seed, record_sketch=True, trace=True)
    qlog = [e for e in f.log if e["kind"] == "qrcp"]
    for K0, perm, Bk in f.sketch_at_block_start:
        # sketch identity B^{(K0)} = Omega~_2 A^{(K0)} (eq. (3.3) in block form)
        S = tb.schur_complement(tb.permuted(A, perm), K0)
        Bref = Om[:, perm[K0:]] @ S
        assert np.max(np.abs(Bk - Bref)) <= 1e-10 * max(1.0, np.max(np.abs(Bref)))
        # greedy picks by least squares, replayed as transpositions
        bb = min(b, n - K0)
        picks = tb.greedy_columns_lstsq(Bref, bb)
        found, _ = tb.transpositions_to_positions(picks, n - K0)
        logged = [e["pos"] - K0 for e in qlog if e["K0"] == K0]
        assert logged[:len(found)] == found


def test_block_sketch_update_needs_inverse_transpose():
    # the reading L11^{-T}: with L11^{-1} instead the identity fails
    n, b, p, seed = 30, 6, 4, 4
    A = gen.gaussian_sym(n, seed)
    f = rcp.factor(A, b, p, seed=seed, record_sketch=True)
    K0, perm, B0 = f.sketch_at_block_start[0]
    K1, perm1, B1 = f.sketch_at_block_start[1]
    Om = omega_matrix(seed, b + p, n)
    ref = Om[:, perm1[K1:]] @ tb.schur_complement(tb.permuted(A, perm1), K1)
    assert np.allclose(B1, ref, atol=1e-10)
    # the same update with L11^{-1}
    P0 = perm1  # block-0 interchanges all happened before block 1 started
    Bstart = Om[:, P0] @ tb.sym(A)[np.ix_(P0, P0)]
    L11 = f.L[K0:K1, K0:K1]
    # rows of L21 as they stood when block 1 started (later blocks move rows)
    where = np.empty(n, dtype=int)
    where[f.perm] = np.arange(n)
    L21 = f.L[where[perm1[K1:]], K0:K1]
    wrong = Bstart[:, K1:] - Bstart[:, K0:K1] @ np.linalg.inv(L11) @ L21.T
    right = Bstart[:, K1:] - Bstart[:, K0:K1] @ np.linalg.inv(L11).T @ L21.T
    assert np.allclose(right, ref, atol=1e-10)
    if not np.allclose(L11, np.eye(K1 - K0)):
        assert not np.allclose(wrong, ref, atol=1e-6)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_uniqueness_given_pivot_pattern(seed):
    # (Pi, Delta) determines L and D (proof of Lemma 3.1)
    n = 50
    A = gen.gaussian_sym(n, seed)
    f = rcp.factor(A, 8, 4, seed=seed)
    L, Dm = tb.block_ldlt_given(A, f.perm, f.ipiv)
    assert np.allclose(L, f.L, atol=1e-11)
    assert np.allclose(Dm, f.dmatrix(), atol=1e-11)


def test_exact_norm_mode_picks_largest_schur_column():
    # with Omega = I the sketch of A^{(k)} has the exact column norms of A^{(k)}
    n = 24
    A = gen.gaussian_sym(n, 8)
    f = rcp.factor(A, 1, n - 1, omega=np.eye(n), record_sketch=True, trace=True)
    qlog = [e for e in f.log if e["kind"] == "qrcp"]
    for K0, perm, _ in f.sketch_at_block_start:
        S = tb.schur_complement(tb.permuted(A, perm), K0)
        norms = np.linalg.norm(S, axis=0)
        e = [q for q in qlog if q["K0"] == K0][0]
        assert e["pos"] - K0 == int(np.argmax(norms))


def test_invariants_case1_multipliers_and_2x2_blocks():
    for seed in range(1, 6):
        n = 120
        A = gen.gaussian_sym(n, seed) if seed % 2 else gen.kkt(n, 90, seed, nrefl=8)
        f = rcp.factor(A, 16, 8, seed=seed)
        for e in f.log:
            if e["kind"] == "sbkp" and e["case"] == 1:
                k = e["k"]
                # case (1): |l_jk| <= 1/alpha (proof of Theorem 3.2)
                assert np.max(np.abs(f.L[k + 1:, k]), initial=0) <= 1 / rcp.ALPHA * (1 + 1e-14)
        for i in range(n - 1):
            if f.ipiv[i] == 2:
                d11, d22, c = f.D[i], f.D[i + 1], abs(f.D[n + i])
                assert abs(d11) < rcp.ALPHA * c and abs(d22) < rcp.ALPHA * c
                det = d11 * d22 - c * c
                assert -1.5 * c * c < det < -0.5 * c * c


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_against_bunch_parlett(seed):
    n = 48
    A = gen.gaussian_sym(n, seed)
    f = rcp.factor(A, 8, 4, seed=seed, schedule="eager")
    perm, L, Dm, ipiv, rho_bp = tb.bunch_parlett(A)
    assert tb.reconstruction_error(A, perm, L, Dm) <= 50 * n * U
    b = gen.rhs(n, 1, seed)
    x_rcp = rcp.solve(f, b)
    x_ref = np.linalg.solve(tb.sym(A), b)
    assert tb.backward_error(A, x_rcp, b)[0] <= 1e-14
    assert np.allclose(x_rcp, x_ref, rtol=1e-9, atol=1e-9)
    # growth comparable to symmetric complete pivoting
    assert f.rho_elem <= 10 * rho_bp


@pytest.mark.parametrize("seed", [1, 2])
def test_growth_lemma22_and_theorem33(seed):
    n = 40
    A = gen.gaussian_sym(n, seed)
    f = rcp.factor(A, 4, 4, seed=seed, schedule="eager")
    re, rc = tb.growth_factors(A, f.perm, f.ipiv)
    assert abs(re - f.rho_elem) <= 1e-10 * re
    # Lemma 2.2
    assert re / np.sqrt(n) <= rc * (1 + 1e-12) and rc <= np.sqrt(n) * re * (1 + 1e-12)
    # Theorem 3.3 with eps = 1/2 (a loose bound, never binding here)
    eps = 0.5
    bound = (np.sqrt(2 * (1 + eps) / (1 - eps))) ** (3 + np.log(n - 1)) * \
        np.sqrt(n + 2) ** (2 + np.log(n - 1))
    assert rc <= bound


def test_lemma31_worked_number():
    # Section 4.1: n = 1000, eps = 0.5, delta = 0.05 gives p >= 538
    golden = json.load(open(os.path.join(GOLDEN, "lemma31_p.json")))
    for c in golden["cases"]:
        assert int(np.ceil(tb.lemma31_p(c["n"], c["eps"], c["delta"]))) == c["p"]


def test_lemma31_norm_preservation_rate():
    # with p from Lemma 3.1 every pivot column keeps sqrt((1-eps)/(1+eps)) of
    # the largest Schur column norm, in at least 1 - delta of the runs (b = 1)
    n, eps, delta = 10, 0.5, 0.2
    p = int(np.ceil(tb.lemma31_p(n, eps, delta)))
    fails = 0
    runs = 20
    for seed in range(runs):
        A = gen.gaussian_sym(n, 100 + seed)
        f = rcp.factor(A, 1, p, seed=seed, record_sketch=True, trace=True)
        qlog = [e for e in f.log if e["kind"] == "qrcp"]
        ok = True
        for K0, perm, _ in f.sketch_at_block_start:
            S = tb.schur_complement(tb.permuted(A, perm), K0)
            norms = np.linalg.norm(S, axis=0)
            pick = [q for q in qlog if q["K0"] == K0][0]["pos"] - K0
            if norms[pick] < np.sqrt((1 - eps) / (1 + eps)) * norms.max() * (1 - 1e-12):
                ok = False
        fails += not ok
    assert fails <= delta * runs


@pytest.mark.parametrize("nrhs", [1, 3])
def test_solve_matches_dense_solve(nrhs):
    n = 150
    A = gen.householder_spectrum(n, 5, cond=1e4, nrefl=16)
    f = rcp.factor(A, 16, 8, seed=5)
    b = gen.rhs(n, nrhs, 5)
    x = rcp.solve(f, b)
    xr = np.linalg.solve(A, b)
    assert np.all(tb.backward_error(A, x, b) <= 1e-15 * n)
    assert np.max(np.abs(x - xr)) <= 1e4 * n * U * np.max(np.abs(xr)) * 10


def test_min_margin_reports_ties():
    # a matrix with two equal off-diagonal magnitudes produces a 0 margin
    A = np.array([[0.1, 1.0, -1.0], [1.0, 0.2, 0.0], [-1.0, 0.0, 0.3]])
    f = rcp.factor(A, 3, 2, omega=np.eye(3))
    assert rcp.min_margin(f)[0] == 0.0


# ---- decision margins (near-tie detector) on hand-built cases where every
# compared quantity is known in closed form (Omega = I, so the sketch is A)

ALPHA_REF = 0.70710678118654752440   # sqrt(2)/2


def test_margins_threshold_test_and_qrcp_gap():
    # [[0.7, 1], [1, 0.5]]: QRCP compares column norms sqrt(1.49) and
    # sqrt(1.25) and takes column 0; SBKP then has a_kk = 0.7, lambda = 1,
    # r = 1, |0.7| < alpha so a_rr = 0.5 is tested too (also < alpha: a 2x2
    # pivot).  The smallest gap is | |a_kk| - alpha lambda | = alpha - 0.7.
    A = np.array([[0.7, 1.0], [1.0, 0.5]])
    f = rcp.factor(A, 1, 1, omega=np.eye(2))
    assert list(f.ipiv) == [2, 0]
    kind, pos, rel, ab = rcp.decision_margins(f, scale=1.0)
    assert list(kind) == [0, 1] and list(pos) == [0, 0]
    q_gap = np.sqrt(1.49) - np.sqrt(1.25)
    assert rel[0] == pytest.approx(q_gap / np.sqrt(1.49), rel=1e-12)
    assert ab[0] == pytest.approx(q_gap / np.sqrt(1.49), rel=1e-12)   # sketch scale = sqrt(1.49)
    assert rel[1] == pytest.approx(ALPHA_REF - 0.7, rel=1e-12)
    assert ab[1] == pytest.approx(ALPHA_REF - 0.7, rel=1e-12)
    # the relative detector agrees: (best - second) / best on squared norms
    m, at = rcp.min_margin(f, scale=1.0)
    assert m == pytest.approx(ALPHA_REF - 0.7, rel=1e-12) and f.log[at]["kind"] == "sbkp"
    assert rcp.near_tie_prefix(f, 1.0, tau=1e-3) == 2
    assert rcp.near_tie_prefix(f, 1.0, tau=1e-2) == 0


def test_margins_diagonal_test_of_the_candidate_row():
    # [[0.2, 1], [1, 0.7]]: QRCP takes column 1 (norm sqrt(1.49) against
    # sqrt(1.04)), so position 0 holds the 0.7 row: a_kk = 0.7 fails the
    # test, a_rr = 0.2 is tested (gap alpha - 0.2) and fails; the smallest
    # gap is still the a_kk one.  Scaled by max |A| = 1 and by lambda = 1.
    A = np.array([[0.2, 1.0], [1.0, 0.7]])
    f = rcp.factor(A, 1, 1, omega=np.eye(2))
    assert list(f.perm) == [1, 0]
    kind, pos, rel, ab = rcp.decision_margins(f, scale=2.0)
    e = [x for x in f.log if x["kind"] == "sbkp"][0]
    assert e["akk"] == 0.7 and e["arr"] == 0.2 and e["lam"] == 1.0
    assert rel[1] == pytest.approx(ALPHA_REF - 0.7, rel=1e-12)
    assert ab[1] == pytest.approx((ALPHA_REF - 0.7) / 2.0, rel=1e-12)


def test_margins_choice_of_r():
    # [[10, 3, 2.9], [3, 1, 0], [2.9, 0, 1]]: a_kk = 10 passes the test
    # (case 1); lambda = 3 at r = 1 against lambda_2 = 2.9: gap 0.1, the
    # smallest of {lambda, lambda - lambda_2, |10| - alpha 3}
    A = np.array([[10.0, 3.0, 2.9], [3.0, 1.0, 0.0], [2.9, 0.0, 1.0]])
    f = rcp.factor(A, 1, 2, omega=np.eye(3))
    kind, pos, rel, ab = rcp.decision_margins(f, scale=10.0)
    first_sbkp = int(np.nonzero(kind == 1)[0][0])
    assert pos[first_sbkp] == 0
    assert rel[first_sbkp] == pytest.approx(0.1 / 3.0, rel=1e-12)
    assert ab[first_sbkp] == pytest.approx(0.1 / 10.0, rel=1e-12)
    e = [x for x in f.log if x["kind"] == "sbkp"][0]
    assert e["case"] == 1 and e["lam2"] == 2.9


def test_margins_nearly_equal_columns():
    # diag(3, 2.9999, 1): QRCP's gap between the two largest column norms is
    # 1e-4 (relative 1e-4 / 3), and every SBKP step has lambda = 0 (a zero
    # off-diagonal: rel 0 and abs 0, a near-tie of the lambda = 0 test)
    A = np.diag([3.0, 2.9999, 1.0])
    f = rcp.factor(A, 3, 0, omega=np.eye(3))
    kind, pos, rel, ab = rcp.decision_margins(f, scale=3.0)
    assert kind[0] == 0 and pos[0] == 0
    assert rel[0] == pytest.approx(1e-4 / 3.0, rel=1e-9)
    assert ab[0] == pytest.approx(1e-4 / 3.0, rel=1e-9)
    sb = kind == 1
    assert np.all(rel[sb] == 0.0) and np.all(ab[sb] == 0.0)
    assert rcp.near_tie_prefix(f, 3.0) == 0


def test_near_tie_prefix_without_ties_is_n():
    A = gen.gaussian_sym(60, 12)
    f = rcp.factor(A, 8, 4, seed=12)
    kind, pos, rel, ab = rcp.decision_margins(f, scale=np.max(np.abs(A)))
    assert ab.min() > 1e-9
    assert rcp.near_tie_prefix(f, np.max(np.abs(A))) == 60
    # both margins of an SBKP step measure the same gap: abs * max|A| = rel * lambda
    lams = np.array([e["lam"] for e in f.log if e["kind"] == "sbkp" and e["r"] is not None])
    sb = kind == 1
    assert np.allclose(ab[sb] * np.max(np.abs(A)), rel[sb] * lams, rtol=1e-14, atol=0)
