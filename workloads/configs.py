"""The benchmark and parity workloads, each a named, seeded configuration."""

from dataclasses import dataclass

import numpy as np

from . import gen


@dataclass(frozen=True)
class Config:
    name: str
    kind: str          # "gaussian_sym" | "kkt" | "householder"
    n: int
    b: int             # block size
    p: int             # oversampling: the sketch has l = b + p rows
    nrhs: int
    seed: int
    cond: float = 1e6  # householder only
    n1: int = 0        # kkt only: order of the SPD block H
    nrefl: int = 64    # number of Householder reflectors in Q

    @property
    def l(self):
        return self.b + self.p

    def matrix(self):
        if self.kind == "gaussian_sym":
            return gen.gaussian_sym(self.n, self.seed)
        if self.kind == "kkt":
            return gen.kkt(self.n, self.n1, self.seed, nrefl=self.nrefl)
        if self.kind == "householder":
            return gen.householder_spectrum(self.n, self.seed, cond=self.cond,
                                            nrefl=self.nrefl)
        raise ValueError(self.kind)

    def rhs(self):
        return gen.rhs(self.n, self.nrhs, self.seed)

    def scaled(self, n, b=None, p=None, name=None):
        """The same family at another size (used for parity-sized cases)."""
        kw = dict(self.__dict__)
        kw.update(n=n, name=name or f"{self.name}@{n}")
        if b is not None:
            kw["b"] = b
        if p is not None:
            kw["p"] = p
        if self.kind == "kkt":
            kw["n1"] = (3 * n) // 4
            kw["nrefl"] = min(self.nrefl, kw["n1"])
        return Config(**kw)


CONFIGS = {
    # Type 6 Gaussian-symmetric, small enough for the oracle in well under a second
    "gaussian512": Config("gaussian512", "gaussian_sym", n=512, b=32, p=8, nrhs=1, seed=1),
    # Type 7 saddle point: H 3072 x 3072 SPD, C 1024 x 3072
    "kkt4096": Config("kkt4096", "kkt", n=4096, b=64, p=10, nrhs=4, seed=2, n1=3072),
    # dense indefinite, cond ~ 1e6, the headline workload
    "householder16384": Config("householder16384", "householder", n=16384, b=128, p=16,
                               nrhs=1, seed=3, cond=1e6),
}

# the mixed-precision sweep: same generator, three condition numbers
for _cond, _seed in ((1e2, 41), (1e6, 42), (1e10, 43)):
    _name = f"householder16384_cond{_cond:.0e}"
    CONFIGS[_name] = Config(_name, "householder", n=16384, b=128, p=16, nrhs=1,
                            seed=_seed, cond=_cond)


def batched_systems(count=4096, nmin=16, nmax=512, seed=5, nrhs=4):
    """The batched workload: ``count`` independent systems of uneven order.

    Returns a list of (n, A, B, omega_seed).  Even indices are Gaussian
    symmetric, odd ones saddle-point with n1 = floor(3n/4).
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 99]))
    ns = rng.integers(nmin, nmax + 1, size=count)
    out = []
    for i, n in enumerate(ns):
        n = int(n)
        s = seed * 2**32 + i
        if i % 2 == 0:
            A = gen.gaussian_sym(n, s)
        else:
            n1 = (3 * n) // 4
            A = gen.kkt(n, n1, s, nrefl=min(16, n1))
        out.append((n, A, gen.rhs(n, nrhs, s), s))
    return out
