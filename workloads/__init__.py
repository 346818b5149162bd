"""Seeded synthetic inputs shaped like the paper's experiments.

This module only builds input matrices and right-hand sides.  It holds none
of the factorization's arithmetic, and it is the one piece of code that both
the oracle (``oracle/``) and the GPU path's tests and benchmark use.
"""

from .gen import (gaussian_sym, gap_spectrum, householder_spectrum, kkt, rhs,
                  householder_product_wy, zero_padded)
from .configs import CONFIGS, Config, batched_systems

__all__ = ["gaussian_sym", "gap_spectrum", "householder_spectrum", "kkt", "rhs", "zero_padded",
           "householder_product_wy", "CONFIGS", "Config", "batched_systems"]
