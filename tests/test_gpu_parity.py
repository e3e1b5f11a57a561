"""GPU parity against the CPU oracle (live, small cases).

The radial derivatives A_n (auxiliary functions and recursions) are compared
point by point over the T = xi R^2 range of the workloads; whole contracted
blocks of every class are compared on quartets of the tiny molecule.
"""
import math
import sys

import numpy as np
import pytest

from synth import FACTOR_SETS, tiny_config
from tests.gpu_common import (REL_TOL, block_rel_err, envelope_err, i5_block_err, i5_vanishes, run_list,
                              run_quads, vanishes_by_parity, zero_block_err)

pytestmark = pytest.mark.gpu

P1 = FACTOR_SETS["P1"]


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_5070_amd import f12int
    return f12int


def _radial_points():
    rng = np.random.default_rng(2024)
    pts = []
    for T in [0.0, 1e-6, 0.05, 0.5, 1.0, 1.9, 2.1, 3.0, 4.9, 5.1, 7.9, 8.1, 10.0, 12.4, 12.6, 20.0, 50.0,
              107.0, 109.0, 400.0, 3000.0]:
        for _ in range(2):
            p, q = 10 ** rng.uniform(-1, 2), 10 ** rng.uniform(-1, 2)
            xi = p * q / (p + q)
            pts.append((p, q, math.sqrt(T / xi)))
    return pts


P2, P3 = FACTOR_SETS["P2"], FACTOR_SETS["P3"]


@pytest.mark.parametrize("cls,fac,facp", [(1, P1, P1), (2, P1, P1), (3, P1, P1), (4, P1, FACTOR_SETS["P4"]),
                                          (6, P1, P1), (2, P2, None), (3, FACTOR_SETS["P4"], None),
                                          (2, P3, None), (3, P3, None), (4, P3, None), (6, P3, None),
                                          (4, P2, None), (6, P2, None), (4, P1, P3)])
@pytest.mark.parametrize("L", [0, 4, 8, 12, 14])
def test_radial_derivatives_vs_oracle(lib, cls, fac, facp, L):
    from oracle import radial
    pts = _radial_points()
    p = np.array([x[0] for x in pts])
    q = np.array([x[1] for x in pts])
    R = np.array([x[2] for x in pts])
    xi = p * q / (p + q)
    T = xi * R * R
    # the oracle's cost grows fast with cancellation: skip points needing > 40 digits
    keep = np.array([radial.cancellation_digits(t, L) < 13 for t in T])
    p, q, R, xi, T = p[keep], q[keep], R[keep], xi[keep], T[keep]
    print(f"radial cls={cls} L={L} npts={len(p)}", flush=True)
    k = lib.Kernel(cls, fac, facp if facp is not None else fac)
    A = lib.aux_radial(k, p, q, R, L).cpu().numpy()
    ref = radial.radial_auto(cls, xi, R, L, fac, facp if facp is not None else fac)
    refN = (ref * radial.n_prime(p, q)[:, None]).to_float()
    err = envelope_err(A.T, refN, xi)
    i, n = np.unravel_index(np.argmax(err), err.shape)
    print(f"  worst scaled err {err.max():.2e} at T={T[i]:.3g} n={n}", flush=True)
    assert err.max() < 1e-13, (T[i], n, A[n, i], refN[i, n])


def test_radial_routes_agree_in_overlap(lib):
    """Branch consistency: the DD small-T series and the large-T lowering
    route agree from the switch point of each L (1.5 for L = 4, 3 for L = 8,
    5 for L = 12) up to T = 12; for kernels with negative integer powers, which
    switch at T = 14, at T = 10, 12, 14."""
    rng = np.random.default_rng(11)
    for cls, fac in ((3, P1), (6, P1), (2, FACTOR_SETS["P4"]), (2, P3), (6, P3), (4, P2)):
        k = lib.Kernel(cls, fac, fac)
        negint = fac.rho < -2 or (cls in (4, 6) and 2 * fac.rho <= -3)
        for L, Tsw in ((4, 1.5), (8, 3.0), (12, 5.0)):
            pts = []
            # kernels with negative integer powers switch at T = 14
            for T in ((10.0, 12.0, 14.0) if negint else (Tsw, Tsw + 1.0, 9.0, 12.0)):
                for _ in range(4):
                    p, q = 10 ** rng.uniform(-1, 2), 10 ** rng.uniform(-1, 2)
                    pts.append((p, q, math.sqrt(T * (p + q) / (p * q))))
            p, q, R = (np.array([x[j] for x in pts]) for j in range(3))
            a1 = lib.aux_radial(k, p, q, R, L, route=1).cpu().numpy().T
            a2 = lib.aux_radial(k, p, q, R, L, route=2).cpu().numpy().T
            err = envelope_err(a2, a1, p * q / (p + q))
            print(f"overlap cls={cls} L={L} max {err.max():.2e}", flush=True)
            assert err.max() < 1e-13


def test_radial_small_T_binary64_series(lib):
    """The binary64 small-T series (used for L <= 5, T < 2) against the
    double-double series, to the 1e-13 bound of the scaled envelope that the
    radial derivatives meet against the oracle (the double-double series
    carries the kernel's coefficients in double-double, the binary64 one
    their rounded values)."""
    rng = np.random.default_rng(17)
    for cls, fac in ((3, P1), (6, P1), (4, P1), (2, FACTOR_SETS["P4"])):
        k = lib.Kernel(cls, fac, fac)
        for L in range(0, 6):
            pts = []
            for T in (0.0, 1e-4, 0.3, 0.9, 1.4, 1.99):
                for _ in range(6):
                    p, q = 10 ** rng.uniform(-1.3, 2), 10 ** rng.uniform(-1.3, 2)
                    pts.append((p, q, math.sqrt(T * (p + q) / (p * q))))
            p, q, R = (np.array([x[j] for x in pts]) for j in range(3))
            a1 = lib.aux_radial(k, p, q, R, L, route=1).cpu().numpy().T
            a3 = lib.aux_radial(k, p, q, R, L, route=3).cpu().numpy().T
            err = envelope_err(a3, a1, p * q / (p + q))
            print(f"f64 series cls={cls} L={L} max {err.max():.2e}", flush=True)
            assert err.max() < 1e-13


@pytest.mark.parametrize("cls", [1, 3, 6])
def test_radial_large_T_mp_oracle(lib, cls):
    """A few large-T points where the oracle needs its arbitrary-precision path."""
    from oracle import radial
    L = 4
    pts = [(3.0, 5.0, 25.0), (40.0, 60.0, 9.0), (0.5, 1.5, 40.0)]
    p = np.array([x[0] for x in pts]); q = np.array([x[1] for x in pts]); R = np.array([x[2] for x in pts])
    xi = p * q / (p + q)
    print(f"radial-mp cls={cls} T={xi * R * R}", flush=True)
    k = lib.Kernel(cls, P1, P1)
    A = lib.aux_radial(k, p, q, R, L).cpu().numpy()
    ref = (radial.radial_auto(cls, xi, R, L, P1, P1) * radial.n_prime(p, q)[:, None]).to_float()
    err = envelope_err(A.T, ref, xi)
    print(f"  worst scaled err {err.max():.2e}", flush=True)
    assert err.max() < 1e-13


def _tiny():
    pos, shells = tiny_config()
    return shells


@pytest.mark.parametrize("cls", [1, 2, 3, 4, 6, 5])
def test_tiny_blocks_vs_oracle(lib, cls):
    from oracle import integrals
    shells = _tiny()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 1)
    k = lib.Kernel(cls, P1, P1)
    # s0 p0 s1 p1 s2 p2 on atoms 0,1,2: a spread of shell-type classes
    quads = [(0, 0, 0, 0), (2, 0, 4, 0), (1, 0, 2, 3), (3, 1, 4, 2), (5, 3, 1, 1), (1, 3, 5, 5), (3, 3, 5, 1)]
    if cls == 5:
        quads = [(0, 0, 0, 0), (1, 0, 2, 3), (3, 1, 4, 2), (3, 3, 5, 1)]
    print(f"tiny cls={cls} quads={quads}", flush=True)
    got = run_quads(lib, basis, pairs, k, cls, quads)
    for qd in quads:
        sh = [shells[i].as_dict() for i in qd]
        ref = integrals.contracted(cls, *sh, P1, P1).ravel()
        if cls == 5:
            ref3 = integrals.contracted(3, *sh, P1, P1).ravel()
            e = i5_block_err(got[qd], ref, ref3, np.concatenate([sh[0]["exps"], sh[1]["exps"]]),
                             i5_vanishes(shells[qd[0]].l, qd[0] == qd[1]))
        else:
            e = block_rel_err(got[qd], ref)
        print(f"  {qd} err {e:.2e}", flush=True)
        assert e < REL_TOL, (qd, e)


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name + ".npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _check_golden_set(lib, shells, golden, cls, quads):
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 1)
    k = lib.Kernel(cls, P1, P1)
    print(f"golden cls={cls} nquads={len(quads)}", flush=True)
    got = run_quads(lib, basis, pairs, k, cls, quads)
    worst = 0.0
    for qd in quads:
        ref = golden["c%d_%d_%d_%d_%d" % ((cls,) + tuple(qd))]
        if cls == 5:
            ref3 = golden["c3_%d_%d_%d_%d" % tuple(qd)]
            bra_exps = np.concatenate([shells[qd[0]].exps, shells[qd[1]].exps])
            e = i5_block_err(got[qd], ref, ref3, bra_exps, i5_vanishes(shells[qd[0]].l, qd[0] == qd[1]))
        else:
            e = block_rel_err(got[qd], ref)
        worst = max(worst, e)
        print(f"  {qd} l={[shells[i].l for i in qd]} max|I| {np.max(np.abs(ref)):.1e} err {e:.2e}", flush=True)
        assert e < REL_TOL, (qd, e)
    return worst


@pytest.mark.parametrize("cls", [1, 2, 3, 4, 6, 5])
def test_df_blocks_vs_golden(lib, cls):
    """s-f shells: every contraction path (small-class and large-class
    launches, same-centre R = 0, mixed l on both sides)."""
    sys.path.insert(0, __import__("os").path.join(__import__("os").path.dirname(__file__), "golden"))
    from make_golden import DF3_QUADS, DF3_QUADS_I5, df3_shells
    quads = DF3_QUADS_I5 if cls == 5 else DF3_QUADS
    _check_golden_set(lib, df3_shells(), _golden("df3"), cls, quads)


@pytest.mark.parametrize("cls", [2, 3, 4, 6, 5])
def test_plain20_sampled_vs_golden(lib, cls):
    """The 20-atom workload at full size: the class's whole unique-quartet
    list is built as bench.py builds it, and the stored oracle values of
    quartets sampled from it (two per total angular momentum, at most 64
    primitive quartets each) are compared with f12_eval on those entries,
    block-relative.  The screened list at 1e-12 is built as well: every
    sampled block it keeps must meet the 1e-12 block-relative bound, and every
    block it drops must be below 1e-12."""
    import os
    import torch
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import plain20_quads
    from synth import config_plain
    golden = _golden("plain20")
    _, shells = config_plain()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 0)
    k = lib.Kernel(cls, P1, P1)
    ks = lib.Kernel(3, P1, P1) if cls == 5 else k
    Q = lib.Quartets.build(pairs, pairs, cls)
    quads = Q.quads().astype(np.int64)
    offs = Q.offsets()
    keys = ((quads[:, 0] * 128 + quads[:, 1]) * 128 + quads[:, 2]) * 128 + quads[:, 3]
    Qs = lib.Quartets.build(pairs, pairs, cls, screen_tol=1e-12, screen_kernel=ks)
    sq = Qs.quads().astype(np.int64)
    kept = set((((sq[:, 0] * 128 + sq[:, 1]) * 128 + sq[:, 2]) * 128 + sq[:, 3]).tolist())
    sample = plain20_quads()
    print(f"plain20 cls={cls} list={len(keys)} screened={len(sq)} samples={len(sample)}", flush=True)
    bad = []
    for qd in sample:
        key = ((qd[0] * 128 + qd[1]) * 128 + qd[2]) * 128 + qd[3]
        idx = np.nonzero(keys == key)[0]
        assert len(idx) == 1, qd
        i = int(idx[0])
        out = torch.empty(int(offs[i + 1] - offs[i]), dtype=torch.float64, device="cuda")
        lib.eval_into(Q, k, out, i, i + 1)
        lib.stream_status()
        got = out.cpu().numpy()
        ref = golden["c%d_%d_%d_%d_%d" % ((cls,) + tuple(qd))]
        if cls == 5:
            ref3 = golden["c3_%d_%d_%d_%d" % tuple(qd)]
            e = i5_block_err(got, ref, ref3, np.concatenate([shells[qd[0]].exps, shells[qd[1]].exps]),
                             i5_vanishes(shells[qd[0]].l, qd[0] == qd[1]))
        else:
            e = block_rel_err(got, ref)
        mx = float(np.max(np.abs(ref)))
        in_screen = key in kept
        print(f"  {qd} l={[shells[j].l for j in qd]} max|I| {mx:.1e} err {e:.2e} "
              f"{'kept' if in_screen else 'dropped'} by the 1e-12 screen", flush=True)
        if (in_screen and e >= REL_TOL) or (not in_screen and mx >= 1e-12):
            bad.append((qd, mx, e, in_screen))
    assert not bad, bad


@pytest.mark.parametrize("cls", [3, 5])
def test_screening_keeps_schwarz_and_equal_blocks(lib, cls):
    """f12_quartets_build with screen_tol keeps at least the quartets with
    Q_ab Q_cd >= tol (Q_ab = sqrt(max |(ab|k3|ab)|), diagonal blocks evaluated
    here through an explicit list), kept blocks equal the unscreened ones bit
    for bit, and every dropped block is below tol."""
    import os
    import torch
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import df3_shells
    shells = df3_shells()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 0)
    k = lib.Kernel(cls, P1, P1)
    k3 = lib.Kernel(3, P1, P1)
    ns = len(shells)
    upairs = [(i, j) for i in range(ns) for j in range(i + 1)]
    diag = [(i, j, i, j) for (i, j) in upairs]
    got = run_quads(lib, basis, lib.Pairs(basis, 1), k3, 3, diag)
    Qab = {(i, j): math.sqrt(float(np.max(np.abs(got[(i, j, i, j)])))) for (i, j) in upairs}
    prods = sorted(Qab[p] * Qab[q] for p in upairs for q in upairs)
    tol = prods[len(prods) // 3]
    full = lib.Quartets.build(pairs, pairs, cls)
    scr = lib.Quartets.build(pairs, pairs, cls, screen_tol=tol, screen_kernel=k3)
    fq = [tuple(int(v) for v in r) for r in full.quads()]
    sq = [tuple(int(v) for v in r) for r in scr.quads()]
    schwarz = [q for q in fq if Qab[(q[0], q[1])] * Qab[(q[2], q[3])] >= tol]
    print(f"screening cls={cls} tol={tol:.3e} full={len(fq)} kept={len(sq)} schwarz={len(schwarz)}", flush=True)
    assert set(schwarz) <= set(sq)
    assert 0 < len(sq) < len(fq)
    hf = run_list(lib, full, k)
    hs = run_list(lib, scr, k)
    for q in sq:
        assert np.array_equal(hs[q], hf[q]), q
    kept = set(sq)
    worst = max(float(np.max(np.abs(hf[q]))) for q in fq if q not in kept)
    print(f"  largest dropped block {worst:.3e}", flush=True)
    assert worst < tol


@pytest.mark.parametrize("cls", [2, 3, 4, 6, 5])
def test_screening_estimate_on_spread_molecule(lib, cls):
    """On 8 atoms spread through a 20 bohr cube (s, p, d shells, 1-3
    primitives, exponents log-uniform in [0.05, 50]) every quartet that the
    screen drops at tol = 1e-12, 1e-9, 1e-6 is below tol (all blocks computed
    unscreened).  The long-range part of the factor grows like e^{B r}, so the
    product Q_ab Q_cd alone would drop blocks far above tol: those are
    counted and printed."""
    from synth import molecule
    _, shells = molecule(6061, 8, 20.0, 1.5, (0, 1, 2), 1, 3, 0.05, 50.0)
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 0)
    k = lib.Kernel(cls, P1, P1)
    ks = lib.Kernel(3, P1, P1) if cls == 5 else k
    full = lib.Quartets.build(pairs, pairs, cls)
    hf = run_list(lib, full, k)
    mx = {q: float(np.max(np.abs(v))) for q, v in hf.items()}
    ns = len(shells)
    upairs = [(i, j) for i in range(ns) for j in range(i + 1)]
    dg = run_quads(lib, basis, lib.Pairs(basis, 1), ks, 3 if cls == 5 else cls, [(i, j, i, j) for (i, j) in upairs])
    Qab = {(i, j): math.sqrt(float(np.max(np.abs(dg[(i, j, i, j)])))) for (i, j) in upairs}
    for tol in (1e-12, 1e-9, 1e-6):
        scr = lib.Quartets.build(pairs, pairs, cls, screen_tol=tol, screen_kernel=ks)
        kept = set(tuple(int(v) for v in r) for r in scr.quads())
        dropped = [q for q in mx if q not in kept]
        worst = max((mx[q] for q in dropped), default=0.0)
        plain_bad = sum(1 for q in mx if Qab[q[:2]] * Qab[q[2:]] < tol and mx[q] >= tol)
        print(f"spread cls={cls} tol={tol:.0e}: {len(mx)} quartets, kept {len(kept)}, "
              f"largest dropped {worst:.2e}; Q_ab Q_cd alone would drop {plain_bad} blocks >= tol", flush=True)
        assert worst < tol, (tol, worst)


def _factor_cases():
    import os
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import FACTOR_CASES
    return FACTOR_CASES


@pytest.mark.parametrize("cls,f,fp", _factor_cases())
def test_factor_sets_vs_golden(lib, cls, f, fp):
    """Whole blocks with the other factor sets on the 3-atom s+p molecule:
    P2 (non-integer rho < -1, W orders below -1), P4 (integer rho >= 0) and
    the mixed pair (P1, P4) of I4/I6, against stored oracle values."""
    import os
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import FACTOR_QUADS, factor_key
    golden = _golden("factors")
    shells = _tiny()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 1)
    k = lib.Kernel(cls, FACTOR_SETS[f], FACTOR_SETS[fp])
    print(f"factors cls={cls} f={f} f'={fp} quads={FACTOR_QUADS}", flush=True)
    got = run_quads(lib, basis, pairs, k, cls, FACTOR_QUADS)
    for qd in FACTOR_QUADS:
        ref = golden[factor_key(cls, f, fp, qd)]
        if cls == 5:
            ref3 = golden[factor_key(3, f, fp, qd)]
            e = i5_block_err(got[qd], ref, ref3, np.concatenate([shells[qd[0]].exps, shells[qd[1]].exps]),
                             i5_vanishes(shells[qd[0]].l, qd[0] == qd[1]))
        else:
            e = block_rel_err(got[qd], ref)
        print(f"  {qd} max|I| {np.max(np.abs(ref)):.1e} err {e:.2e}", flush=True)
        assert e < REL_TOL, (qd, e)


@pytest.mark.parametrize("cls", [2, 3, 4, 6, 5])
def test_factor_from_terms_vs_golden(lib, cls):
    """A correlation factor given by its terms (f12_kernel_create_terms; G5:
    Gaussian geminals, a half-integer power and a growing term) on the 3-atom
    s+p molecule against stored oracle values, and its radial derivatives
    against the live oracle at L = 4 and 12."""
    import os
    from oracle import radial
    from oracle.factor import TermFactor
    from synth import GENERIC_FACTORS
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import FACTOR_QUADS, factor_key
    golden = _golden("generic")
    shells = _tiny()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 1)
    terms = np.array(GENERIC_FACTORS["G5"])
    k = lib.Kernel.from_terms(cls, terms, terms)
    got = run_quads(lib, basis, pairs, k, cls, FACTOR_QUADS)
    print(f"generic G5 cls={cls}", flush=True)
    for qd in FACTOR_QUADS:
        ref = golden[factor_key(cls, "G5", "G5", qd)]
        if cls == 5:
            ref3 = golden[factor_key(3, "G5", "G5", qd)]
            e = i5_block_err(got[qd], ref, ref3, np.concatenate([shells[qd[0]].exps, shells[qd[1]].exps]),
                             i5_vanishes(shells[qd[0]].l, qd[0] == qd[1]))
        else:
            e = block_rel_err(got[qd], ref)
        print(f"  {qd} max|I| {np.max(np.abs(ref)):.1e} err {e:.2e}", flush=True)
        assert e < REL_TOL, (qd, e)
    if cls == 5:
        return
    G = TermFactor(GENERIC_FACTORS["G5"])
    pts = _radial_points()
    p = np.array([x[0] for x in pts]); q = np.array([x[1] for x in pts]); R = np.array([x[2] for x in pts])
    xi = p * q / (p + q)
    for L in (4, 12):
        keep = np.array([radial.cancellation_digits(t, L) < 13 for t in xi * R * R])
        A = lib.aux_radial(k, p[keep], q[keep], R[keep], L).cpu().numpy()
        ref = (radial.radial_auto(cls, xi[keep], R[keep], L, G, G) * radial.n_prime(p[keep], q[keep])[:, None]).to_float()
        err = envelope_err(A.T, ref, xi[keep])
        print(f"  radial L={L} worst scaled err {err.max():.2e}", flush=True)
        assert err.max() < 1e-13


@pytest.mark.parametrize("cls", [2, 3, 6])
def test_radial_far_side_of_narrow_kernels(lib, cls):
    """Kernels much narrower than the pair Gaussian (g >> xi) at large T: the
    F(-R) side of the large-T route is damped only by exp(-xi T / (xi + g)),
    so it must be kept far beyond the T where it vanishes for g = 0.  Single
    terms, each scored on its own envelope, against the oracle."""
    from oracle import radial
    from oracle.factor import TermFactor
    rng = np.random.default_rng(77)
    pts = []
    for T in (30.0, 60.0, 107.0, 200.0, 400.0, 600.0):  # exp(-T) stays above the underflow
        for _ in range(3):
            xi = 10 ** rng.uniform(-2, -0.5)
            p = xi * (1 + 10 ** rng.uniform(-0.5, 0.5))
            q = p * xi / (p - xi)
            pts.append((p, q, math.sqrt(T / xi)))
    p = np.array([x[0] for x in pts]); q = np.array([x[1] for x in pts]); R = np.array([x[2] for x in pts])
    xi = p * q / (p + q)
    for term in ((1.0, 0.0, 0.0, 5.0), (0.7, 0.0, 0.0, 50.0), (0.4, 1.0, 0.3, 2.0), (0.2, 0.5, 0.0, 8.0)):
        k = lib.Kernel.from_terms(cls, [term])
        G = TermFactor((term,))
        for L in (0, 4, 12):
            keep = np.array([radial.cancellation_digits(t, L) < 13 for t in xi * R * R])
            A = lib.aux_radial(k, p[keep], q[keep], R[keep], L).cpu().numpy()
            ref = (radial.radial_auto(cls, xi[keep], R[keep], L, G, G)
                   * radial.n_prime(p[keep], q[keep])[:, None]).to_float()
            err = envelope_err(A.T, ref, xi[keep])
            # these values are exp(-w R^2) with w R^2 ~ T: a one-ulp change of
            # xi (which binary64 forms from p and q) moves them by ~T eps
            tol = 1e-13 + 4e-16 * (xi[keep] * R[keep] ** 2)
            print(f"far side cls={cls} term={term} L={L}: worst scaled err {err.max():.2e}, "
                  f"worst err/tol {(err.max(axis=1) / tol).max():.2f}", flush=True)
            assert np.all(err.max(axis=1) < tol), (term, L)


@pytest.mark.parametrize("cls", [2, 3, 4, 6])
def test_decaying_exponentials_radial_vs_oracle(lib, cls):
    """Ten-no's exponential exp(-1.2 r) and STG3 (two decaying exponentials
    and a Gaussian) through f12_kernel_create_terms: radial derivatives at
    L = 0, 4, 12 (STG) and 0, 8 (STG3) against the oracle, over T from 0 to 3000 and xi from
    0.01 to 30, so that both ladders of the small-T route (upward for
    |b|/sqrt(xi) <= 7, downward beyond), the table and the scaled far-side
    forms of the large-T route, and both signs of X_+ are reached."""
    from oracle import radial
    from oracle.factor import TermFactor
    from synth import GENERIC_FACTORS
    rng = np.random.default_rng(1225)
    pts = []
    for T in (0.0, 1e-4, 0.3, 1.0, 2.5, 4.0, 6.5, 9.0, 15.0, 30.0, 60.0, 150.0, 600.0, 3000.0):
        for lxi in (-2.0, -1.3, -0.5, 0.5, 1.5):
            xi = 10 ** (lxi + rng.uniform(-0.1, 0.1))
            p = xi * (1 + 10 ** rng.uniform(-0.5, 0.5))
            q = p * xi / (p - xi)
            pts.append((p, q, math.sqrt(T / xi)))
    p = np.array([x[0] for x in pts]); q = np.array([x[1] for x in pts]); R = np.array([x[2] for x in pts])
    xi = p * q / (p + q)
    for name in ("STG", "STG3"):
        terms = GENERIC_FACTORS[name]
        k = lib.Kernel.from_terms(cls, terms, terms)
        G = TermFactor(terms)
        for L in ((0, 4, 12) if name == "STG" else (0, 8)):
            keep = np.array([radial.cancellation_digits(t, L) < 13 for t in xi * R * R])
            A = lib.aux_radial(k, p[keep], q[keep], R[keep], L).cpu().numpy()
            ref = (radial.radial_auto(cls, xi[keep], R[keep], L, G, G)
                   * radial.n_prime(p[keep], q[keep])[:, None]).to_float()
            sc = (2.0 * xi[keep])[:, None] ** np.arange(L + 1)[None, :]
            live = np.max(np.abs(ref) / sc, axis=1) > 1e-290  # exp(-T) below the underflow: both zero
            err = envelope_err(A.T[live], ref[live], xi[keep][live])
            assert np.all(np.abs(A.T[~live]) < 1e-280)
            # binary64 forms xi from p and q: values ~exp(-T) move by ~T eps.  From
            # T = 14 on, where the series does not converge fast enough
            # (4 xi T / b^2 > ~0.35), the large-T route runs, whose lowering
            # form cancels by ~10 (|b| / (2 xi R))^L while 2 xi R < |b|: the
            # documented accuracy limit of decaying kernels with diffuse pairs
            Tl, xl, Rl = xi[keep][live] * R[keep][live] ** 2, xi[keep][live], R[keep][live]
            bmax = {2: 1.0, 3: 1.0, 4: 2.0, 6: 2.0}[cls] * max(-t[2] for t in terms)
            ratio = bmax / np.maximum(2 * xl * Rl, 1e-300)
            grow = np.where((Tl >= 14.0) & (ratio > 1.0), 10.0 * ratio ** L, 1.0)
            tol = (1e-13 + 4e-16 * Tl) * grow
            i = int(np.argmax(err.max(axis=1) / tol))
            print(f"{name} cls={cls} L={L}: {int(live.sum())} points, worst scaled err {err.max():.2e}, "
                  f"worst err/tol {(err.max(axis=1) / tol).max():.2f} at T={Tl[i]:.3g} xi={xl[i]:.3g} "
                  f"(tolerance factor {grow[i]:.3g})", flush=True)
            assert np.all(err.max(axis=1) < tol), (name, L)


@pytest.mark.parametrize("cls", [2, 3, 4, 6, 5])
def test_decaying_exponentials_vs_golden(lib, cls):
    """Blocks of the 3-atom s+p molecule with Ten-no's exponential and STG3
    (f12_kernel_create_terms) against stored oracle values."""
    import os
    from synth import GENERIC_FACTORS
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import FACTOR_QUADS, factor_key
    golden = _golden("stg")
    shells = _tiny()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 1)
    for name in ("STG", "STG3"):
        terms = np.array(GENERIC_FACTORS[name])
        k = lib.Kernel.from_terms(cls, terms, terms)
        got = run_quads(lib, basis, pairs, k, cls, FACTOR_QUADS)
        for qd in FACTOR_QUADS:
            ref = golden[factor_key(cls, name, name, qd)]
            if cls == 5:
                ref3 = golden[factor_key(3, name, name, qd)]
                e = i5_block_err(got[qd], ref, ref3, np.concatenate([shells[qd[0]].exps, shells[qd[1]].exps]),
                                 i5_vanishes(shells[qd[0]].l, qd[0] == qd[1]))
            else:
                e = block_rel_err(got[qd], ref)
            print(f"{name} cls={cls} {qd} max|I| {np.max(np.abs(ref)):.1e} err {e:.2e}", flush=True)
            assert e < REL_TOL, (name, qd, e)


def _negpow_cases():
    sys.path.insert(0, __import__("os").path.join(__import__("os").path.dirname(__file__), "golden"))
    from make_golden import NEGPOW_CASES
    return NEGPOW_CASES


@pytest.mark.parametrize("cls,f,fp", _negpow_cases())
def test_negative_powers_vs_golden(lib, cls, f, fp):
    """Kernels with negative integer powers of r in their terms (finite parts
    with log terms on the device): P3 (rho = -3, n = 2) in every class, P2 in
    I4 and I6 (rho + rho' = -3), and the mixed pairs with P3, on the 3-atom
    s+p molecule against stored oracle values."""
    import os
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import FACTOR_QUADS, factor_key
    golden = _golden("negpow")
    shells = _tiny()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 1)
    k = lib.Kernel(cls, FACTOR_SETS[f], FACTOR_SETS[fp])
    print(f"negpow cls={cls} f={f} f'={fp}", flush=True)
    got = run_quads(lib, basis, pairs, k, cls, FACTOR_QUADS)
    for qd in FACTOR_QUADS:
        ref = golden[factor_key(cls, f, fp, qd)]
        if cls == 5:
            ref3 = golden[factor_key(3, f, fp, qd)]
            e = i5_block_err(got[qd], ref, ref3, np.concatenate([shells[qd[0]].exps, shells[qd[1]].exps]),
                             i5_vanishes(shells[qd[0]].l, qd[0] == qd[1]))
        else:
            e = block_rel_err(got[qd], ref)
        print(f"  {qd} max|I| {np.max(np.abs(ref)):.1e} err {e:.2e}", flush=True)
        assert e < REL_TOL, (qd, e)


@pytest.mark.parametrize("cls", [1, 2, 3, 4, 6, 5])
def test_tiny_all_quartets_vs_golden(lib, cls):
    """Every unique quartet of the 3-atom s+p molecule (231 for I1-I4 and I6,
    441 for I5), evaluated as one list built by f12_quartets_build, against
    stored oracle values."""
    import os
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import tinyall_quads
    golden = _golden("tinyall")
    shells = _tiny()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 0)
    k = lib.Kernel(cls, P1, P1)
    Q = lib.Quartets.build(pairs, pairs, cls)
    got = run_list(lib, Q, k)
    expect = tinyall_quads(cls)
    print(f"tinyall cls={cls} quartets={len(got)}", flush=True)
    assert sorted(got) == sorted(expect)
    def diag(a, b):
        # max |(ab|ab)| of the class's kernel (I3 for I5, times the largest bra
        # exponent: the scale of the Laplacian terms)
        c = 3 if cls == 5 else cls
        v = float(np.max(np.abs(golden["c%d_%d_%d_%d_%d" % (c, a, b, a, b)])))
        if cls == 5:
            v *= float(max(np.max(shells[a].exps), np.max(shells[b].exps)))
        return v

    worst, worst_zero, bad, nzero = 0.0, 0.0, [], 0
    for qd in expect:
        ref = golden["c%d_%d_%d_%d_%d" % ((cls,) + tuple(qd))]
        a, b, c, d = qd
        if vanishes_by_parity(qd, shells) or (cls == 5 and i5_vanishes(shells[a].l, a == b)):
            e = zero_block_err(got[qd], diag(a, b), diag(c, d) if cls != 5 else diag(c, d) /
                               float(max(np.max(shells[c].exps), np.max(shells[d].exps))))
            worst_zero = max(worst_zero, e)
            nzero += 1
        else:
            e = block_rel_err(got[qd], ref)
            worst = max(worst, e)
        if e >= REL_TOL:
            bad.append((qd, e))
    print(f"  worst block-relative error {worst:.2e}; {nzero} blocks that vanish identically, "
          f"largest |I_gpu| on their pairs' scale {worst_zero:.2e}", flush=True)
    assert not bad, bad


@pytest.mark.parametrize("cls", [2, 3, 4, 6, 5])
def test_deep_high_l_vs_golden(lib, cls):
    """(dd|dd), (dd|ff), (fd|ff), (ff|ff) with 36 ket primitive pairs (more
    than one staging chunk of 32), (ff|ff) and (fd|fd) with 36 bra primitive
    pairs, and (sp|dd) with 1e4 exponents, against stored oracle values; for
    I5 these run both forms of the contraction (the Laplacian-folded bra and
    the four-component form of the largest shapes)."""
    import os
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import DEEPHL_QUADS, deephl_shells
    _check_golden_set(lib, deephl_shells(), _golden("deephl"), cls, DEEPHL_QUADS)


@pytest.mark.parametrize("cls", [3, 5, 6])
def test_deep_contractions_vs_golden(lib, cls):
    """Deep contractions: 36 and 256 ket primitive pairs (several staging
    chunks of ket primitives) and a 16-primitive bra shell (the ABI maximum)."""
    import os
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import DEEP_QUADS, deep_shells
    _check_golden_set(lib, deep_shells(), _golden("deep"), cls, DEEP_QUADS)


def test_eval_error_paths(lib):
    """Argument errors are reported before any launch: short output buffer,
    class mismatch, stage 2 without stage 1, empty range."""
    import torch
    shells = _tiny()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 0)
    k3, k2 = lib.Kernel(3, P1, P1), lib.Kernel(2, P1, P1)
    Q = lib.Quartets.build(pairs, pairs, 3)
    offs = Q.offsets()
    short = torch.empty(int(offs[2] - offs[0]) - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.F12Error) as e:
        lib.eval_into(Q, k3, short, 0, 2)
    assert e.value.status == -6
    buf = torch.empty(int(offs[-1]), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.F12Error) as e:
        lib.eval_into(Q, k2, buf)
    assert e.value.status == -1
    with pytest.raises(lib.F12Error) as e:
        lib.eval_stage(Q, k3, buf, 0, 1, 2)
    assert e.value.status == -1
    lib.eval_into(Q, k3, buf, 3, 3)  # empty range: nothing to do
    lib.stream_status()
