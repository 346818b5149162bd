"""GPU: the benchmark configurations at their full sizes, through the C ABI,
in the launch configuration the benchmark times (trailing update overlapped
with the next block's selection).

  * kkt4096 (n = 4096, b = 64, p = 10, nrhs = 4): the oracle factors it in
    seconds, so the check is the element-by-element one of the parity tests
    (the oracle run has no near-tie: min relative margin ~1e-5 > 1e-9):
    permutation and block pattern bit-exact, L and D within
    1e3 n u max(1, |oracle|), reconstruction <= 50 n u, solve backward error
    <= 1e-13 and the solution within 1e-9 of the oracle's;
  * householder16384 (n = 16384, b = 128, p = 16, cond 1e6, the headline):
    against the oracle's run stored in tests/golden/householder16384_oracle.npz
    (written by tests/golden/make_householder16384.py, which calls only the
    oracle): the permutation and the block pattern bit-exact on all n
    positions (the measured result, also past the stored near-tie prefix,
    the positions before the first decision whose gap is <= 1e-9 max|A|),
    D and the stored rows of L within 1e3 n u max(1, |oracle|), and the
    solution within cond * 1e-13 of the oracle's; then properties that hold at any size: perm a permutation;
    ipiv a valid pattern; L unit lower with L(i+1, i) = 0 inside every 2x2
    block; 4096 sampled entries (i >= j) of P A P^T - L D L^T each within
    50 n u ||A||_inf (the bound of the parity tests' norm check); solve
    backward error <= 1e-13; the same factors bit for bit with the update
    overlapped or not, and on a repeat.
Every case prints its name before running.
"""

import os
import sys

import numpy as np
import pytest

from oracle import rcp as orcp, textbook as tb
from workloads import CONFIGS

pytestmark = pytest.mark.gpu

U = np.finfo(np.float64).eps / 2
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "householder16384_oracle.npz")


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
    pkg.rcp_set_overlap(1)
    return pkg


def _dmat(D, ipiv):
    n = len(ipiv)
    Dm = np.diag(D[:n])
    for i in range(n - 1):
        if ipiv[i] == 2:
            Dm[i + 1, i] = Dm[i, i + 1] = D[n + i]
    return Dm


def _host(f):
    return (f.perm.cpu().numpy(), f.ipiv.cpu().numpy(), f.L.cpu().numpy(), f.D.cpu().numpy())


def test_kkt4096_full_size_matches_oracle(rcp):
    import torch
    cfg = CONFIGS["kkt4096"]
    _say(f"full size {cfg.name}: n={cfg.n} b={cfg.b} p={cfg.p} seed={cfg.seed}")
    A = cfg.matrix()
    n = cfg.n
    ref = orcp.factor(A, cfg.b, cfg.p, seed=cfg.seed)
    margin, _ = orcp.min_margin(ref, scale=np.max(np.abs(A)))
    _say(f"  oracle margin {margin:.2e}")
    assert margin > 1e-9
    Ad = torch.from_numpy(A).cuda()
    f = rcp.rcp_factor(Ad, cfg.b, cfg.p, cfg.seed)
    assert f.info == 0
    perm, ipiv, L, D = _host(f)
    assert np.array_equal(perm, ref.perm)
    assert np.array_equal(ipiv, ref.ipiv)
    tol = 1e3 * n * U
    assert np.all(np.abs(L - ref.L) <= tol * np.maximum(1.0, np.abs(ref.L)))
    assert np.all(np.abs(D - ref.D) <= tol * np.maximum(1.0, np.abs(ref.D)))
    assert tb.reconstruction_error(A, perm, L, _dmat(D, ipiv)) <= 50 * n * U
    B = cfg.rhs()
    X = rcp.rcp_solve(f, torch.from_numpy(B).cuda()).cpu().numpy()
    be = np.max(tb.backward_error(A, X, B))
    xr = orcp.solve(ref, B)
    _say(f"  backward error {be:.2e}")
    assert be <= 1e-13
    assert np.max(np.abs(X - xr)) <= 1e-9 * max(1.0, np.max(np.abs(xr)))


def _ldlt_entries(L, D, ipiv, I, J):
    """(L D L^T)(i, j) for the sampled pairs, one O(n) product each."""
    n = len(ipiv)
    two = np.nonzero(ipiv == 2)[0]
    out = np.empty(len(I))
    for s, (i, j) in enumerate(zip(I, J)):
        lj = L[j]
        y = D[:n] * lj
        y[two] += D[n + two] * lj[two + 1]
        y[two + 1] += D[n + two] * lj[two]
        out[s] = L[i] @ y
    return out


def test_householder16384_full_size(rcp):
    import torch
    cfg = CONFIGS["householder16384"]
    _say(f"full size {cfg.name}: n={cfg.n} b={cfg.b} p={cfg.p} seed={cfg.seed}")
    A = cfg.matrix()
    n = cfg.n
    Ad = torch.from_numpy(A).cuda()
    f = rcp.rcp_factor(Ad, cfg.b, cfg.p, cfg.seed)
    assert f.info == 0
    perm, ipiv, L, D = _host(f)
    L = np.ascontiguousarray(L)     # row-major: the sampled products read rows
    st = rcp.rcp_get_stats()
    # ---- against the oracle's run of the same problem
    gold = np.load(GOLDEN)
    assert int(gold["n"]) == n and int(gold["b"]) == cfg.b and int(gold["p"]) == cfg.p
    pre = int(gold["near_tie_prefix"])
    first = int(np.argmax(perm != gold["perm"])) if np.any(perm != gold["perm"]) else n
    _say(f"  oracle near-tie prefix {pre}; first differing position {first}; "
         f"GPU threshold margin min {st['min_margin']:.2e}, near-ties {st['near_ties']}")
    assert pre > n // 2
    assert np.array_equal(perm[:pre], gold["perm"][:pre])
    assert np.array_equal(ipiv[:pre], gold["ipiv"][:pre])
    # measured: the GPU takes every decision as the oracle does, also the
    # ones after the first decision the conservative near-tie reading flags
    # (absolute margin <= 1e-9 max|A|, at position 9105), so the whole
    # sequence is compared
    idiff = np.nonzero(ipiv != gold["ipiv"])[0]
    m = min(first, int(idiff[0]) if idiff.size else n)
    assert m == n, f"pivots differ from the oracle's from position {m}"
    tol = 1e3 * n * U
    Dg = gold["D"]
    assert np.all(np.abs(D[:m] - Dg[:m]) <= tol * np.maximum(1.0, np.abs(Dg[:m])))
    assert np.all(np.abs(D[n:n + m] - Dg[n:n + m]) <=
                  tol * np.maximum(1.0, np.abs(Dg[n:n + m])))
    for r, row in zip(gold["L_row_pos"], gold["L_rows"]):
        if r < m:
            assert np.all(np.abs(L[r] - row) <= tol * np.maximum(1.0, np.abs(row))), r
    # a permutation and a valid block pattern
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert set(np.unique(ipiv)).issubset({0, 1, 2})
    firsts = np.nonzero(ipiv == 2)[0]
    seconds = np.nonzero(ipiv == 0)[0]
    assert np.array_equal(firsts + 1, seconds)
    _say(f"  2x2 blocks {len(firsts)}")
    # unit lower L, zero inside 2x2 blocks
    assert np.all(np.diag(L) == 1.0)
    assert not np.any(np.triu(L, 1))
    assert np.all(L[firsts + 1, firsts] == 0.0)
    # sampled reconstruction entries
    rng = np.random.default_rng(7)
    I = rng.integers(0, n, 4096)
    J = rng.integers(0, n, 4096)
    I, J = np.maximum(I, J), np.minimum(I, J)
    I[:64] = np.arange(64)          # include the first diagonal entries
    J[:64] = np.arange(64)
    got = _ldlt_entries(L, D, ipiv, I, J)
    want = A[perm[I], perm[J]]
    anorm = np.max(np.sum(np.abs(A), axis=1))
    err = np.max(np.abs(got - want)) / anorm
    _say(f"  sampled reconstruction error {err:.2e} (bound {50 * n * U:.2e})")
    assert err <= 50 * n * U
    # the benchmark's right-hand side
    B = cfg.rhs()
    X = rcp.rcp_solve(f, torch.from_numpy(B).cuda()).cpu().numpy()
    be = np.max(tb.backward_error(A, X, B))
    xg = gold["x"]
    fwd = np.max(np.abs(X - xg)) / np.max(np.abs(xg))
    _say(f"  backward error {be:.2e}; difference from the oracle's solution {fwd:.2e}")
    assert be <= 1e-13
    assert fwd <= cfg.cond * 1e-13
    del f
    # bit-identical on a repeat, and with the update not overlapped
    for overlap in (1, 0):
        rcp.rcp_set_overlap(overlap)
        g = rcp.rcp_factor(Ad, cfg.b, cfg.p, cfg.seed)
        p2, i2, L2, D2 = _host(g)
        _say(f"  overlap={overlap}: identical factors")
        assert np.array_equal(p2, perm) and np.array_equal(i2, ipiv)
        assert np.array_equal(D2.view(np.uint64), D.view(np.uint64))
        assert np.array_equal(L2.view(np.uint64), L.view(np.uint64))
        del g, L2
    rcp.rcp_set_overlap(1)
