"""GPU: speculation in the SBKP panels (rcp_set_speculation) changes no result.

While a step's records are exchanged, each workgroup of the persistent panel
assumes SBKP case (0)/(1) (Figure 2) and forms the next step's column; cases
(2)/(3) restore what the assumption changed and redo the step.  The
decisions are those of the step-by-step method, so the factorization with
speculation forced on (mode 1) and forced off (mode 0) must agree exactly:
the permutation and block pattern bit for bit, L and D value for value.  The
inputs include many 2x2 pivots (KKT, types 2, 4 and 5), rank deficiency
(exactly zero pivots, case (0) with a_kk = 0) and both branches of Algorithm
1 (q = b and q = 1).  Each mode is also checked against the oracle on cases
without near-ties (tolerances of the other parity tests).
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
    pkg.rcp_set_speculation(-1)


def _run(rcp, A, b, p, seed, mode, q=None):
    import torch
    rcp.rcp_set_speculation(mode)
    try:
        At = torch.from_numpy(A).cuda()
        f = rcp.rcp_factor(At, b, p, seed) if q is None else rcp.rcp_factor_q(At, b, p, seed, q)
        st = rcp.rcp_get_stats()
        out = (f.perm.cpu().numpy(), f.ipiv.cpu().numpy(), f.L.cpu().numpy(), f.D.cpu().numpy(),
               f.info, st)
    finally:
        rcp.rcp_set_speculation(-1)
    return out


def _matrix(name, n, seed):
    if name == "gaussian":
        return gen.gaussian_sym(n, seed)
    if name == "householder":
        return gen.householder_spectrum(n, seed, cond=1e6, nrefl=64)
    if name == "kkt":
        return gen.kkt(n, (3 * n) // 4, seed, nrefl=min(64, (3 * n) // 4))
    if name == "zero_padded":
        return gen.zero_padded(n, n // 3, seed)
    return stress.matrix(int(name[4:]), n, seed=seed)


CASES = [
    ("gaussian", 1030, 64, 8, 31), ("householder", 1500, 128, 16, 32), ("kkt", 1100, 64, 10, 33),
    ("zero_padded", 700, 32, 8, 34), ("type2", 600, 32, 4, 35), ("type4", 600, 32, 4, 36),
    ("type5", 600, 32, 4, 37), ("type8", 600, 32, 4, 38), ("type10", 600, 32, 4, 39),
]


@pytest.mark.parametrize("q", [None, 1])
@pytest.mark.parametrize("name,n,b,p,seed", CASES)
def test_speculation_changes_nothing(rcp, name, n, b, p, seed, q):
    _say(f"speculation {name}: n={n} b={b} p={p} seed={seed} q={q}")
    A = _matrix(name, n, seed)
    on = _run(rcp, A, b, p, seed, 1, q)
    off = _run(rcp, A, b, p, seed, 0, q)
    for x, y in zip(on[:4], off[:4]):
        assert np.array_equal(x, y)
    assert on[4] == off[4]
    for key in ("n2x2", "ncase", "max_abs_l", "min_margin", "near_ties"):
        if key in on[5]:
            assert on[5][key] == off[5][key], key
    _say(f"  2x2 pivots: {on[5].get('n2x2')}, SBKP cases: {on[5].get('ncase')}")


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("name,n,b,p,seed", [("kkt", 1500, 64, 10, 3),
                                              ("householder", 1300, 128, 16, 6)])
def test_each_mode_matches_oracle(rcp, name, n, b, p, seed, mode):
    _say(f"speculation mode {mode} against the oracle: {name} n={n} b={b} p={p} seed={seed}")
    A = _matrix(name, n, seed)
    ref = orcp.factor(A, b, p, seed=seed)
    margin, _ = orcp.min_margin(ref, scale=np.max(np.abs(A)))
    assert margin > 1e-9
    perm, ipiv, L, D, info, _ = _run(rcp, A, b, p, seed, mode)
    assert np.array_equal(perm, ref.perm)
    assert np.array_equal(ipiv, ref.ipiv)
    tol = 1e3 * n * U
    assert np.all(np.abs(L - ref.L) <= tol * np.maximum(1.0, np.abs(ref.L)))
    assert np.all(np.abs(D - ref.D) <= tol * np.maximum(1.0, np.abs(ref.D)))
    Dm = np.diag(D[:n].copy())
    for i in np.nonzero(ipiv == 2)[0]:
        Dm[i + 1, i] = Dm[i, i + 1] = D[n + i]
    assert tb.reconstruction_error(A, perm, L, Dm) <= 50 * n * U


def test_mode_is_validated(rcp):
    with pytest.raises(ValueError):
        rcp.rcp_set_speculation(2)
    rcp.rcp_set_speculation(-1)
