"""CPU oracle for randomized complete pivoting (RCP) -- TEST INFRASTRUCTURE.

This package is a plain, slow, FP64 NumPy implementation of what the GPU
library computes.  It exists only to check the GPU path: the tests under
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; nothing in the product package does, and it
imports nothing from the product package.  It shares no code with the HIP
path: the Gaussian sketch matrix is generated here by an independent
implementation of the same published counter-based generator.

Modules
  omega      Philox4x64-10 + Box-Muller, the random sketch matrix Omega
  rcp        Algorithm 1 (q = b branch): factorization, solve, decision log
  textbook   independent comparators: block LDL^T for a given pivot pattern,
             Bunch-Parlett complete pivoting, greedy column selection by
             least squares, Schur complements, norms and growth factors

Functions whose result is not pinned by the tests say "parity unpinned" in
their docstring; every other function is pinned by a ``-m "not gpu"`` test.
"""

from . import omega, rcp, textbook  # noqa: F401
