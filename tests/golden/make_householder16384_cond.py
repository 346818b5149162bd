"""Write the oracle's solutions of the three n = 16384 matrices of the
reduced-precision sweep (the headline generator with lambda log-uniform in
[1/cond, 1], cond 1e2, 1e6, 1e10, seeds 41, 42, 43; b = 128, p = 16, one
right-hand side), for the forward errors the benchmark reports.

It calls only ``oracle/`` and ``workloads/``.  Run from the repository root:

    python tests/golden/make_householder16384_cond.py

(several minutes per matrix and about 14 GB of host memory).
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

OUT = os.path.join(HERE, "householder16384_cond_oracle.npz")


def main():
    out = {}
    for c in ("1e+02", "1e+06", "1e+10"):
        cfg = CONFIGS[f"householder16384_cond{c}"]
        t0 = time.time()
        A = cfg.matrix()
        f = orcp.factor(A, cfg.b, cfg.p, seed=cfg.seed)
        x = orcp.solve(f, cfg.rhs())
        del f, A
        key = c.replace("+", "")
        out[f"x_{key}"] = x
        out[f"seed_{key}"] = cfg.seed
        print(f"{cfg.name}: oracle factor + solve in {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
