"""GPU: Algorithm 2 (Section 4.5, rcp_set_recompute) against the oracle's
Algorithm 2, through the C ABI.

Inputs whose Schur complements are known in closed form make every
Algorithm 2 decision robust (far from its threshold):
  * an r0 x r0 Gaussian block among exact zeros: the Schur complement after
    the block is exactly zero, so the factorization stops with rank r0 and
    returns r0 + 1;
  * a spectral gap (eigenvalues 1 and 1e-9): the sketch is recomputed once,
    where the gap is reached, and the factorization completes.
Checked: the return value, the recomputation count and rank the library
reports, the permutation and block pattern bit for bit up to the first
disagreement with the oracle (which must come after the oracle's near-tie
prefix), L and D there, and P A P^T = L D L^T within 50 n u.
"""

import sys

import numpy as np
import pytest

from oracle import rcp as orcp, textbook as tb
from workloads import gen, stress

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
    yield pkg
    pkg.rcp_set_recompute(1)


def _dmat(D, ipiv):
    n = len(ipiv)
    Dm = np.diag(D[:n].copy())
    for i in np.nonzero(ipiv == 2)[0]:
        Dm[i + 1, i] = Dm[i, i + 1] = D[n + i]
    return Dm


def _run(rcp, A, b, p, seed, r):
    import torch
    n = A.shape[0]
    rcp.rcp_set_recompute(r)
    try:
        f = rcp.rcp_factor(torch.from_numpy(A).cuda(), b, p, seed)
        st = rcp.rcp_get_stats()
    finally:
        rcp.rcp_set_recompute(1)
    ref = orcp.factor(A, b, p, seed=seed, recompute=r)
    perm = f.perm.cpu().numpy()
    ipiv = f.ipiv.cpu().numpy()
    L = f.L.cpu().numpy()
    D = f.D.cpu().numpy()
    amax = np.max(np.abs(A))
    pre = orcp.near_tie_prefix(ref, amax)
    pd = np.nonzero(perm != ref.perm)[0]
    idf = np.nonzero(ipiv != ref.ipiv)[0]
    m = min(int(pd[0]) if pd.size else n, int(idf[0]) if idf.size else n)
    _say(f"  info {f.info}/{ref.info}; rank {st['rank']}/{ref.rank}; recomputes "
         f"{st['recomputes']}/{len(ref.recomputed)}; near-tie prefix {pre}; agree up to {m}")
    assert f.info == ref.info
    assert st["rank"] == ref.rank
    assert st["recomputes"] == len(ref.recomputed)
    assert m >= pre
    # a multiplier of column k carries an error of about n u max|A| / |d_k|
    # (past a spectral gap the pivots are far below max|A|)
    tol = 1e3 * n * U
    dk = np.abs(ref.D[:n]) + np.abs(ref.D[n:])
    dk = np.maximum(dk, np.roll(dk * (ref.ipiv == 2), 1))
    colscale = np.maximum(1.0, amax / np.maximum(dk, 1e-300))[None, :m]
    assert np.all(np.abs(L[:m, :m] - ref.L[:m, :m]) <=
                  tol * np.maximum(1.0, np.abs(ref.L[:m, :m])) * colscale)
    assert np.all(np.abs(D[:m] - ref.D[:m]) <= tol * np.maximum(amax, np.abs(ref.D[:m])))
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert tb.reconstruction_error(A, perm, L, _dmat(D, ipiv)) <= 50 * n * U
    return f, st, ref, m


@pytest.mark.parametrize("n,r0,b,p,r", [(100, 32, 16, 4, 2), (100, 32, 16, 4, 3),
                                        (1000, 256, 64, 8, 2)])
def test_exact_zero_schur_complement_stops(rcp, n, r0, b, p, r):
    _say(f"alg2 zero-padded n={n} r0={r0} b={b} p={p} r={r}")
    A = gen.zero_padded(n, r0, 5)
    f, st, ref, m = _run(rcp, A, b, p, 3, r)
    # the stop comes at the first block start past the nonzero block (a
    # block may have run on through zero pivots first)
    assert r0 <= ref.rank < r0 + b + 2 and f.info == r0 + 1
    assert m == n                      # the exit leaves the same order behind
    D = f.D.cpu().numpy()
    assert not np.any(D[r0:n]) and not np.any(D[n + r0:])


def test_algorithm1_runs_through_zero_pivots(rcp):
    _say("alg2 r=1 on the zero-padded matrix")
    A = gen.zero_padded(100, 32, 5)
    f, st, ref, m = _run(rcp, A, 16, 4, 3, 1)
    assert st["rank"] == 100 and st["recomputes"] == 0 and f.info == 33


@pytest.mark.parametrize("n,r0,b,p,r", [(120, 32, 16, 4, 2), (120, 32, 16, 4, 3),
                                        (1500, 256, 64, 8, 2)])
def test_spectral_gap_recomputes_once(rcp, n, r0, b, p, r):
    _say(f"alg2 gap n={n} r0={r0} b={b} p={p} r={r}")
    A = gen.gap_spectrum(n, r0, 6, small=1e-9)
    f, st, ref, m = _run(rcp, A, b, p, 3, r)
    assert ref.recomputed == [r0] and f.info == 0 and st["rank"] == n


def test_rank_deficient_type10(rcp):
    # type 10's Schur complement reaches rounding level after its numerical
    # rank; where Algorithm 2 then stops depends on rounding, so only the
    # validity of the GPU's own result is checked (and the solve refuses a
    # stopped factorization)
    import torch
    n = 300
    _say(f"alg2 type 10 n={n}")
    A = stress.type10(n, seed=8)
    rcp.rcp_set_recompute(2)
    try:
        f = rcp.rcp_factor(torch.from_numpy(A).cuda(), 32, 4, 9)
        st = rcp.rcp_get_stats()
    finally:
        rcp.rcp_set_recompute(1)
    perm = f.perm.cpu().numpy()
    ipiv = f.ipiv.cpu().numpy()
    L = f.L.cpu().numpy()
    D = f.D.cpu().numpy()
    _say(f"  info {f.info}; rank {st['rank']}; recomputes {st['recomputes']}")
    assert 32 <= st["rank"] <= n and st["recomputes"] >= 1
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert tb.reconstruction_error(A, perm, L, _dmat(D, ipiv)) <= 50 * n * U
