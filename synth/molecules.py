"""Seeded random molecules carrying contracted Cartesian Gaussian shells.

Recipe (all draws from numpy.random.default_rng(seed), in this order):
  1. atom positions uniform in [0, edge]^3, redrawn one at a time until the
     distance to every earlier atom is >= min_sep (if min_sep > 0);
  2. per atom, per shell in `shell_ls` order: K uniform in {kmin..kmax},
     then K exponents 10**U(log10 lo, log10 hi), then K coefficients
     U(0.1, 1).
The paper gives no benchmark molecules; these stand in for them with the
sizes and distributions of the workloads stated in the project's configs.
"""
from dataclasses import dataclass, field
import numpy as np


@dataclass(frozen=True)
class Factor:
    """Range-separated correlation factor parameters (c0, rho, B, mu, n)."""
    c0: float
    rho: float
    B: float
    mu: float
    n: int = 0


# Four parameter sets that between them exercise every S(alpha,beta,gamma)
# regime: P1 regular alpha > -1 (rho = 1/2), P2 non-integer alpha <= -1,
# P3 negative integer alpha with Tang-Toennies order n = 2, P4 integer rho.
FACTOR_SETS = {
    "P1": Factor(0.2, 0.5, 0.3, 0.8, 0),
    "P2": Factor(0.1, -1.5, 0.2, 1.2, 0),
    "P3": Factor(0.05, -3.0, 0.25, 1.0, 2),
    "P4": Factor(0.3, 1.0, 0.5, 0.5, 0),
}


# Correlation factors given by terms c r^alpha exp(b r - g r^2) instead of the
# range-separated parameters.  G5: three Gaussian geminals (the form of the
# usual Gaussian fits of an exponential correlation factor), a half-integer
# power and a growing term, so that every family of the term path is
# exercised.  STG: Ten-no's exponential exp(-gamma r), gamma = 1.2.  STG3: two
# decaying exponentials (one times r) and a Gaussian geminal.
GENERIC_FACTORS = {
    "G5": ((0.3, 0.0, 0.0, 0.2), (0.5, 0.0, 0.0, 1.1), (0.2, 0.0, 0.0, 5.0),
           (0.1, 1.0, 0.4, 0.7), (0.05, 0.5, 0.0, 0.9)),
    "STG": ((1.0, 0.0, -1.2, 0.0),),
    "STG3": ((0.8, 0.0, -1.0, 0.0), (0.3, 1.0, -1.5, 0.0), (-0.2, 0.0, 0.0, 0.6)),
}


@dataclass
class Shell:
    center: np.ndarray
    l: int
    exps: np.ndarray
    coefs: np.ndarray
    atom: int = 0

    def as_dict(self):
        return {"center": self.center, "l": self.l, "exps": self.exps, "coefs": self.coefs}


def molecule(seed, natoms, edge, min_sep, shell_ls, kmin, kmax, exp_lo, exp_hi,
             exp_range_by_l=None, forced_exps=None):
    rng = np.random.default_rng(seed)
    pos = []
    while len(pos) < natoms:
        x = rng.uniform(0.0, edge, 3)
        if min_sep > 0 and any(np.linalg.norm(x - y) < min_sep for y in pos):
            continue
        pos.append(x)
    shells = []
    for ia, c in enumerate(pos):
        for l in shell_ls:
            lo, hi = (exp_range_by_l or {}).get(l, (exp_lo, exp_hi))
            K = int(rng.integers(kmin, kmax + 1))
            ex = 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), K)
            co = rng.uniform(0.1, 1.0, K)
            shells.append(Shell(np.array(c, float), l, ex, co, ia))
    if forced_exps:
        # replace the first exponent of the first shells of the listed l by forced values
        for (l, value) in forced_exps:
            for s in shells:
                if s.l == l:
                    s.exps[0] = value
                    break
    return np.array(pos), shells


def tiny_config():
    """3 atoms in a 4 bohr cube, s and p shells of 3 primitives, exps in [0.1, 10]."""
    return molecule(1412, 3, 4.0, 0.0, (0, 1), 3, 3, 0.1, 10.0)


def config_plain():
    """20 atoms in a 12 bohr cube (min sep 1.5), shells s,s,p,p,d,f, K in 1..6, exps [0.05, 50]."""
    return molecule(5070, 20, 12.0, 1.5, (0, 0, 1, 1, 2, 3), 1, 6, 0.05, 50.0)


def config_batching_extra():
    """The two extra geometries of the batching workload (10 and 35 atoms)."""
    return (molecule(5071, 10, 9.5, 1.5, (0, 0, 1, 1, 2, 3), 1, 6, 0.05, 50.0),
            molecule(5072, 35, 14.4, 1.5, (0, 0, 1, 1, 2, 3), 1, 6, 0.05, 50.0))


def config_precision():
    return molecule(5072, 35, 14.4, 1.5, (0, 0, 1, 1, 2, 3), 1, 6, 0.05, 50.0)


def shells_to_arrays(shells):
    """Flatten shells into the arrays the C ABI takes.

    Returns (centers (nc,3), shell_table (ns,4) int32 [l, nprim, center, first],
    exps (np,), coefs (np,)).  Centers are the distinct shell centres in order.
    """
    centers, cidx = [], {}
    table, exps, coefs = [], [], []
    for s in shells:
        key = tuple(np.round(s.center, 15))
        if key not in cidx:
            cidx[key] = len(centers)
            centers.append(s.center)
        table.append([s.l, len(s.exps), cidx[key], len(exps)])
        exps.extend(s.exps.tolist())
        coefs.extend(s.coefs.tolist())
    return (np.array(centers, float).reshape(-1, 3), np.array(table, np.int32),
            np.array(exps, float), np.array(coefs, float))
