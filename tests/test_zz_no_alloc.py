"""rcp_solve_noalloc (the solve on the library's fixed scratch array) against
rcp_solve (the solve on allocated scratch), through the C ABI.

Both run the same kernels with the same arguments, so the solutions must be
bit-identical; they are also checked against the solve tolerance (backward
error <= 1e-13).  Calls follow each other on the same array: the largest
order the array allows, then smaller orders with more right-hand sides, so
that what a previous call left in the array must not matter.
"""

import sys

import numpy as np
import pytest

from oracle import textbook as tb
from workloads import gen

pytestmark = pytest.mark.gpu


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
    return pkg


def _case(rcp, n, nrhs, b, p, seed):
    import torch
    dev = torch.device("cuda:0")
    A = gen.gaussian_sym(n, seed)
    B = gen.rhs(n, nrhs, seed)
    f = rcp.rcp_factor(torch.from_numpy(A).to(dev), b, p, seed)
    Bd = torch.from_numpy(B).to(dev)
    X_ref = rcp.rcp_solve(f, Bd)
    X_na = rcp.rcp_solve_noalloc(f, Bd)
    torch.cuda.synchronize()
    x_ref = X_ref.cpu().numpy()
    x_na = X_na.cpu().numpy()
    assert np.array_equal(x_na.view(np.uint64), x_ref.view(np.uint64)), \
        f"n={n} nrhs={nrhs}: max diff {np.max(np.abs(x_na - x_ref))}"
    berr = tb.backward_error(A, x_na, B)
    assert np.max(berr) <= 1e-13, berr
    return f


def test_noalloc_matches_solve_on_consecutive_calls(rcp):
    # largest order first, then smaller ones that leave most of the array as
    # the previous call wrote it
    for n, nrhs, b, p, seed in ((rcp.RCP_NOALLOC_MAX_N, 1, 128, 16, 61),
                                (1000, 3, 64, 10, 62),
                                (333, 11, 32, 8, 63)):
        _say(f"noalloc n={n} nrhs={nrhs} b={b} p={p} seed={seed}")
        _case(rcp, n, nrhs, b, p, seed)


def test_noalloc_rejects_orders_beyond_its_array(rcp):
    import torch
    _say("noalloc n=RCP_NOALLOC_MAX_N+1 rejected")
    one = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    ptr = one.data_ptr()
    n = rcp.RCP_NOALLOC_MAX_N + 1
    code = rcp.load().rcp_solve_noalloc(n, ptr, ptr, ptr, ptr, 1, ptr, n)
    assert code == -1003   # RCP_EUNSUPPORTED, before any device work
