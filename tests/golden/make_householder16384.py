"""Write the oracle's factorization of the n = 16384 headline matrix.

The headline workload is the dense symmetric indefinite matrix
A = Q diag(s lam) Q^T (64 Householder reflectors, lam log-uniform in
[1e-6, 1], random signs), block b = 128, oversampling p = 16, sketch seed 3,
one right-hand side.  This script runs the FP64 CPU oracle (Algorithm 1,
q = b) on it once and stores what a GPU parity test compares against:

  perm, ipiv          the pivot sequence and the block pattern (integers)
  D                   the block-diagonal factor, D[i] = d_ii, D[n+i] = d_{i+1,i}
  x                   the oracle's solution of A x = b
  L_rows, L_row_pos   a few full rows of L (by position)
  margin_*            every decision's margin, relative and absolute
                      (oracle.rcp.decision_margins), the position it decides,
                      and the near-tie prefix: the pivot positions no decision
                      with an absolute margin <= 1e-9 can change

It calls only ``oracle/`` and ``workloads/``.  Run from the repository root:

    python tests/golden/make_householder16384.py

(several minutes and about 14 GB of host memory).
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import rcp as orcp  # noqa: E402
from workloads import CONFIGS  # noqa: E402

OUT = os.path.join(HERE, "householder16384_oracle.npz")
ROW_POS = (0, 1, 127, 128, 129, 4095, 8191, 12287, 16254, 16383)


def main():
    cfg = CONFIGS["householder16384"]
    t0 = time.time()
    A = cfg.matrix()
    rhs = cfg.rhs()
    print(f"matrix generated in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    f = orcp.factor(A, cfg.b, cfg.p, seed=cfg.seed)
    print(f"oracle factorization in {time.time() - t0:.1f} s", flush=True)
    scale = float(np.max(np.abs(A)))
    margin, at = orcp.min_margin(f, scale=scale)
    kind, pos, rel, ab = orcp.decision_margins(f, scale)
    prefix = orcp.near_tie_prefix(f, scale, tau=1e-9)
    t0 = time.time()
    x = orcp.solve(f, rhs)
    print(f"oracle solve in {time.time() - t0:.1f} s", flush=True)
    rows = np.array(ROW_POS, dtype=np.int64)
    np.savez_compressed(
        OUT, n=cfg.n, b=cfg.b, p=cfg.p, seed=cfg.seed, perm=f.perm, ipiv=f.ipiv, D=f.D,
        x=x, info=f.info, L_row_pos=rows, L_rows=f.L[rows], min_margin=margin,
        margin_kind=kind, margin_pos=pos.astype(np.int32), margin_rel=rel, margin_abs=ab,
        near_tie_prefix=prefix, max_abs_a=scale, sketch_scale=f.sketch_scale,
        ncase=np.bincount([e["case"] for e in f.log if e["kind"] == "sbkp"], minlength=4))
    print(f"relative min margin {margin:.3e} at log entry {at}; near-tie prefix {prefix}; "
          f"2x2 blocks {int(np.sum(f.ipiv == 2))}; wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
