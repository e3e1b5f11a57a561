"""Writes the stored expected values used by the GPU parity tests.

Every value here comes from the CPU oracle (oracle/) on inputs from synth/;
nothing is read from the GPU library.  Run from the repository root:

    python tests/golden/make_golden.py [name ...]

Sets:
  df3      3 atoms (seed 77, 4 bohr cube, min. separation 1 bohr), s p d f
           shells with 1-2 primitives, exponents log-uniform in [0.1, 10];
           quartets that span every contraction path (same-centre (ff|ff)
           with R = 0, multi-centre (ff|ff), (dd|dd), mixed l, (ss|ff) and
           (ff|ss)), classes I1-I6 with the factor set P1.
  deep     deep contractions: 36 and 256 ket primitive pairs and a
           16-primitive bra shell (s and p shells); I3, I5, I6 with P1.
  plain20  quartets sampled from the 20-atom molecule (seed 5070), stratified
           by total angular momentum, restricted to at most 64 primitive
           quartets so that the oracle finishes; classes I2-I6, P1.
  tinyall  every unique quartet of the 3-atom s+p molecule (seed 1412): the 231
           quartets (bra pair index >= ket pair index) of I1-I4 and I6 and the
           441 (bra, ket) combinations of unordered pairs of I5, factor set P1.
  deephl   deep high-l contractions (deephl_shells): (dd|dd), (dd|ff), (fd|ff)
           and (ff|ff) with 36 ket primitive pairs, (ff|ff) and (fd|fd) with 36
           bra primitive pairs, and (sp|dd) with 1e4 exponents; I2-I6, P1.
  prec35   quartets sampled from the 35-atom molecule (seed 5072) of the
           precision workload, two per total angular momentum with at most 8
           primitive quartets each; I2-I6, P1.
  negpow   the 3-atom s+p molecule with kernels that have negative integer
           powers: P3 (rho = -3, n = 2) in I2-I6, P2 in I4/I6 (rho + rho' = -3),
           and the mixed pairs (P1, P3), (P3, P1); I3 beside the I5 entries.
  generic  the 3-atom s+p molecule with the factor G5 given by its terms
           (synth.GENERIC_FACTORS): I2-I6.
  factors  the 3-atom s+p molecule (seed 1412) with the other factor sets:
           P2 (non-integer rho < -1) for I2, I3, I5; P4 (integer rho >= 0)
           for I2-I6; the mixed pair (f, f') = (P1, P4) for I4 and I6; I3
           beside every I5 entry (the scale of its error).
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import integrals  # noqa: E402
from synth import FACTOR_SETS, config_plain, molecule  # noqa: E402

P1 = FACTOR_SETS["P1"]
HERE = os.path.dirname(os.path.abspath(__file__))


def df3_shells():
    return molecule(77, 3, 4.0, 1.0, (0, 1, 2, 3), 1, 2, 0.1, 10.0)[1]


# shells: atom k holds s=4k, p=4k+1, d=4k+2, f=4k+3
DF3_QUADS = [(3, 3, 3, 3), (7, 3, 11, 3), (6, 2, 10, 6), (3, 2, 7, 5), (0, 0, 7, 11), (11, 7, 0, 4),
             (9, 3, 2, 8), (10, 1, 4, 7), (5, 0, 9, 4), (6, 5, 2, 9), (7, 7, 6, 10), (1, 1, 1, 1)]
DF3_QUADS_I5 = [(3, 2, 6, 5), (2, 3, 6, 5), (7, 11, 1, 0), (0, 0, 11, 7), (6, 2, 10, 6), (5, 1, 9, 5),
                (2, 2, 9, 4), (3, 2, 7, 11)]


def deep_shells():
    """Five shells at seeded positions in a 3 bohr cube: p(16), s(2), s(6),
    p(6), s(16) primitives, exponents log-uniform in [0.1, 10]."""
    from synth.molecules import Shell
    ls, Ks = [1, 0, 0, 1, 0], [16, 2, 6, 6, 16]
    rng = np.random.default_rng(4242)
    pos = rng.uniform(0.0, 3.0, (len(ls), 3))
    out = []
    for i, (l, K) in enumerate(zip(ls, Ks)):
        ex = 10.0 ** rng.uniform(-1.0, 1.0, K)
        co = rng.uniform(0.1, 1.0, K)
        out.append(Shell(pos[i], l, ex, co, i))
    return out


def deephl_shells():
    """Six shells on three centres (seed 4343, 3 bohr cube): f(1) d(1) on the
    first, f(6) d(6) on the second (exponents log-uniform in [0.1, 10]), s(6)
    p(6) on the third with one exponent 1e4 each and the rest log-uniform in
    [0.1, 50]."""
    from synth.molecules import Shell
    rng = np.random.default_rng(4343)
    pos = rng.uniform(0.0, 3.0, (3, 3))
    spec = [(3, 1, 0), (2, 1, 0), (3, 6, 1), (2, 6, 1), (0, 6, 2), (1, 6, 2)]
    out = []
    for l, K, at in spec:
        hi = 50.0 if at == 2 else 10.0
        ex = 10.0 ** rng.uniform(-1.0, np.log10(hi), K)
        if at == 2:
            ex[0] = 1.0e4
        co = rng.uniform(0.1, 1.0, K)
        out.append(Shell(pos[at], l, ex, co, at))
    return out


# shells: 0 f(1), 1 d(1) | 2 f(6), 3 d(6) | 4 s(6), 5 p(6) with 1e4 exponents
DEEPHL_QUADS = [(1, 1, 3, 3), (1, 1, 2, 2), (0, 1, 2, 2), (0, 0, 2, 2), (2, 2, 0, 0), (2, 3, 0, 1), (4, 5, 3, 1)]


def tiny_pairs():
    return [(i, j) for i in range(6) for j in range(i + 1)]


def tinyall_quads(cls):
    """All unique quartets of the tiny molecule as f12_quartets_build lists them."""
    pr = tiny_pairs()
    if cls == 5:
        return [a + c for a in pr for c in pr]
    return [pr[b] + pr[k] for b in range(len(pr)) for k in range(b + 1)]


# (s2 s2|s6 p6): 36 ket primitive pairs; (s2 s2|s16 s16): 256; (p16 s2|s6 s6): 16-primitive bra shell
DEEP_QUADS = [(1, 1, 2, 3), (1, 1, 4, 4), (0, 1, 2, 2)]


def plain20_quads(n_per_L=2, max_prim=64, seed=99, shells=None):
    if shells is None:
        _, shells = config_plain()
    ls = np.array([s.l for s in shells])
    ks = np.array([len(s.exps) for s in shells])
    rng = np.random.default_rng(seed)
    by_L = {}
    ns = len(shells)
    tries = 0
    while tries < 200000 and sum(len(v) for v in by_L.values()) < 13 * n_per_L:
        tries += 1
        a, b, c, d = (int(x) for x in rng.integers(0, ns, 4))
        if b > a:
            a, b = b, a
        if d > c:
            c, d = d, c
        if a * (a + 1) // 2 + b < c * (c + 1) // 2 + d:
            a, b, c, d = c, d, a, b
        if ks[a] * ks[b] * ks[c] * ks[d] > max_prim:
            continue
        L = int(ls[a] + ls[b] + ls[c] + ls[d])
        lst = by_L.setdefault(L, [])
        if len(lst) < n_per_L and (a, b, c, d) not in lst:
            lst.append((a, b, c, d))
    return [q for L in sorted(by_L) for q in by_L[L]]


def prec35_quads():
    """Two quartets per total angular momentum from the 35-atom molecule, at
    most 8 primitive quartets each (seed 98)."""
    from synth import config_precision
    return plain20_quads(seed=98, max_prim=8, shells=config_precision()[1])


# the "factors" set: (class, f, f') and the tiny molecule's quartets
FACTOR_CASES = [(2, "P2", "P2"), (3, "P2", "P2"), (5, "P2", "P2"), (2, "P4", "P4"), (3, "P4", "P4"),
                (4, "P4", "P4"), (5, "P4", "P4"), (6, "P4", "P4"), (4, "P1", "P4"), (6, "P1", "P4")]
FACTOR_QUADS = [(0, 0, 0, 0), (1, 0, 2, 3), (3, 1, 4, 2), (3, 3, 5, 1)]

# first derivatives d/dA of the s-f molecule's blocks ([3][block] per quartet):
# every shape but (ff|ff), whose derivative form the library does not build
GRAD_QUADS = [(6, 2, 10, 6), (3, 2, 7, 5), (0, 0, 7, 11), (11, 7, 0, 4), (9, 3, 2, 8), (10, 1, 4, 7),
              (5, 0, 9, 4), (1, 1, 1, 1)]


# negative powers in the kernel terms: P3 (rho = -3, n = 2) in every class,
# P2 (rho = -3/2) in I4 and I6 (rho + rho' = -3)
NEGPOW_CASES = [(2, "P3", "P3"), (3, "P3", "P3"), (4, "P3", "P3"), (5, "P3", "P3"), (6, "P3", "P3"),
                (4, "P2", "P2"), (6, "P2", "P2"), (4, "P1", "P3"), (6, "P3", "P1")]


def factor_key(cls, f, fp, quad):
    return "c%d_%s_%s_%d_%d_%d_%d" % ((cls, f, fp) + tuple(quad))


def _job(args):
    setname, cls, quad = args[:3]
    if setname in ("generic", "stg"):
        from oracle.factor import TermFactor
        from synth import GENERIC_FACTORS, tiny_config
        G = TermFactor(GENERIC_FACTORS[args[3]])
        sh = [tiny_config()[1][i].as_dict() for i in quad]
        return args, np.asarray(integrals.contracted(cls, *sh, G, G), dtype=np.float64).ravel()
    if setname in ("factors", "negpow"):
        from synth import tiny_config
        f, fp = args[3], args[4]
        sh = [tiny_config()[1][i].as_dict() for i in quad]
        return args, np.asarray(integrals.contracted(cls, *sh, FACTOR_SETS[f], FACTOR_SETS[fp]),
                                dtype=np.float64).ravel()
    if setname == "grad":
        from oracle.gradient import grad_first_centre
        sh = [df3_shells()[i].as_dict() for i in quad]
        return args, np.asarray(grad_first_centre(cls, *sh, P1, P1), dtype=np.float64).ravel()
    if setname == "tinyall":
        from synth import tiny_config
        shells = tiny_config()[1]
    elif setname == "prec35":
        from synth import config_precision
        shells = config_precision()[1]
    else:
        shells = {"df3": df3_shells, "deep": deep_shells, "deephl": deephl_shells}.get(
            setname, lambda: config_plain()[1])()
    sh = [shells[i].as_dict() for i in quad]
    return args, np.asarray(integrals.contracted(cls, *sh, P1, P1), dtype=np.float64).ravel()


def build(setname):
    if setname == "df3":
        jobs = [(setname, c, q) for c in (1, 2, 3, 4, 6) for q in DF3_QUADS]
        jobs += [(setname, 5, q) for q in DF3_QUADS_I5]
        jobs += [(setname, 3, q) for q in DF3_QUADS_I5 if q not in DF3_QUADS]
    elif setname == "deep":
        jobs = [(setname, c, q) for c in (5, 3, 6) for q in DEEP_QUADS]
    elif setname == "tinyall":
        jobs = [(setname, c, q) for c in (5, 1, 2, 3, 4, 6) for q in tinyall_quads(c)]
    elif setname == "deephl":
        jobs = [(setname, c, q) for c in (5, 2, 3, 4, 6) for q in DEEPHL_QUADS]
    elif setname == "prec35":
        from synth import config_precision
        quads = prec35_quads()
        jobs = [(setname, c, q) for c in (5, 2, 3, 4, 6) for q in quads]
    elif setname == "generic":
        jobs = [(setname, c, q, "G5", "G5") for c in (5, 2, 3, 4, 6) for q in FACTOR_QUADS]
    elif setname == "grad":
        jobs = [(setname, c, q) for c in (2, 3, 4, 6) for q in GRAD_QUADS]
    elif setname == "stg":
        jobs = [(setname, c, q, f, f) for f in ("STG", "STG3") for c in (5, 2, 3, 4, 6) for q in FACTOR_QUADS]
    elif setname in ("factors", "negpow"):
        base = FACTOR_CASES if setname == "factors" else NEGPOW_CASES
        cases = list(base) + [(3, f, fp) for (c, f, fp) in base if c == 5 and (3, f, fp) not in base]
        jobs = [(setname, c, q, f, fp) for (c, f, fp) in cases for q in FACTOR_QUADS]
    else:
        quads = plain20_quads()
        jobs = [(setname, c, q) for c in (5, 2, 3, 4, 6) for q in quads]
    out = {}
    with Pool(int(os.environ.get("GOLDEN_PROCS", "6"))) as pool:
        for args, val in pool.imap_unordered(_job, jobs):
            sname, cls, quad = args[:3]
            if sname in ("factors", "negpow", "generic", "stg"):
                out[factor_key(cls, args[3], args[4], quad)] = val
            else:
                out["c%d_%d_%d_%d_%d" % ((cls,) + tuple(quad))] = val
            print(*args, flush=True)
    np.savez_compressed(os.path.join(HERE, setname + ".npz"), **out)


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["df3", "deep", "plain20", "factors"]):
        build(name)
