"""More pins of the CPU oracle: the factor derivative, the geminal kernels of
I2/I4/I6 with a long-range part, contraction over several primitives, the
d-shell Laplacian and the rank-2/rank-3 Cartesian bookkeeping.

Every reference here is computed by a route that shares nothing with the
oracle's: the factor of Eq. (rs12) written out in mpmath and differentiated
numerically, a two-dimensional (|v|, cos theta) quadrature of the convolution
that Eq. (bfinal) reduces to one dimension, single-primitive evaluations
recombined by hand, finite differences and rotations of the geometry.  Each
docstring names the mistake the pin catches.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import dd, integrals, radial
from oracle.factor import TermFactor, f_deriv, f_value
from synth import FACTOR_SETS, GENERIC_FACTORS

P1, P2, P3, P4 = (FACTOR_SETS[k] for k in ("P1", "P2", "P3", "P4"))


def _f_mp(fac):
    """f(r) of Eq. (rs12) with S_n of Eq. (ttdamp), in mpmath (working
    precision), or the sum of the terms of a TermFactor."""
    if isinstance(fac, TermFactor):
        return lambda r: mp.fsum(mp.mpf(c) * mp.power(r, a) * mp.exp(b * r - g * r * r) for (c, a, b, g) in fac.terms)

    def f(r):
        x = fac.mu * r * r
        head, t = mp.mpf(1), mp.mpf(1)
        for k in range(1, fac.n + 1):
            t = t * x / k
            head += t
        S = 1 - mp.exp(-x) * head
        return (1 + r / 2) * mp.exp(-x) + S * fac.c0 * mp.power(r, fac.rho) * mp.exp(fac.B * r)
    return f


@pytest.mark.parametrize("name", ["P1", "P2", "P3", "P4"])
def test_factor_and_derivative_vs_mpmath(name):
    """f (Eq. (rs12)) and df/dr at 50 radii in [1e-3, 30] against f written out
    at 60 digits and differentiated numerically by mpmath.  Catches a sign or
    a dropped term in dS_n/dr, in the (rho/r + B) factor of the long-range
    part or in the -mu r^2 terms of the short-range part: f'(0) = 1/2 alone
    does not see them, since they vanish at r = 0."""
    fac = FACTOR_SETS[name]
    r = np.geomspace(1e-3, 30.0, 50)
    fv = f_value(fac, dd.DD(r)).to_mp()
    fd = f_deriv(fac, dd.DD(r)).to_mp()
    with mp.workdps(60):
        f = _f_mp(fac)
        for i, ri in enumerate(r):
            x = mp.mpf(ri)
            ref = f(x)
            dref = mp.diff(f, x)
            assert abs(fv[i] - ref) <= 1e-28 * abs(ref), (ri, fv[i], ref)
            assert abs(fd[i] - dref) <= 1e-26 * (abs(dref) + abs(ref)), (ri, fd[i], dref)


def _fr_terms_mp(fac):
    """df/dr of a TermFactor by the product rule, term by term."""
    return lambda r: mp.fsum(mp.mpf(c) * mp.power(r, a) * mp.exp(b * r - g * r * r) * (a / r + b - 2 * g * r)
                             for (c, a, b, g) in fac.terms)


def _kernel_mp(cls, fac, facp):
    """k_i(r) for classes 2, 3, 4, 6 from the mpmath f; f_r by mp.diff for the
    factors of Eq. (rs12), by the product rule for factors given by terms."""
    f, fp = _f_mp(fac), _f_mp(facp)
    if cls == 6 and isinstance(fac, TermFactor) and isinstance(facp, TermFactor):
        fr, fpr = _fr_terms_mp(fac), _fr_terms_mp(facp)
        return lambda r: fr(r) * fpr(r)
    if cls == 2:
        return lambda r: f(r) / r
    if cls == 3:
        return f
    if cls == 4:
        return lambda r: f(r) * fp(r)
    if cls == 6:
        return lambda r: mp.diff(f, r) * mp.diff(fp, r)
    raise ValueError(cls)


def _convolution_derivatives(cls, fac, facp, xi, R, nmax=3):
    """A_n / N', n = 0..nmax, from the three-dimensional convolution
    B = (pi/(p+q))^{3/2} int d^3v k(|v|) exp(-xi |v - X|^2), |X| = R, written
    in (v, c = cos theta) and integrated numerically in both variables:
      A_n / N' = (xi/pi) 2^n int_0^inf 2 pi v^2 k(v) int_{-1}^{1} d^n/du^n G dc dv,
    with G = exp(-xi (v^2 + u - 2 v c sqrt(u))), u = R^2 (D = R^-1 d/dR = 2 d/du,
    and (pi/(p+q))^{3/2} = xi N'/pi).  The u-derivatives of G by the chain rule:
    phi = -xi (v^2 + u - 2 v c u^{1/2}), G' = phi' G, G'' = (phi'' + phi'^2) G,
    G''' = (phi''' + 3 phi' phi'' + phi'^3) G."""
    k = _kernel_mp(cls, fac, facp)
    xi, R = mp.mpf(xi), mp.mpf(R)
    u = R * R
    ts = mp.calculus.quadrature.TanhSinh(mp.mp)
    # full tanh-sinh rule of step 2^-5 on [-1, 1] (mpmath stores each level's
    # new abscissas separately and leaves the step factor to the caller); the
    # integrand is entire in c, so this step is exact to the working precision
    cnodes = []
    for lev in range(1, 6):
        cnodes += ts.get_nodes(-1, 1, lev, mp.mp.prec)
    cnodes = [(c, w * mp.mpf(2) ** -5) for (c, w) in cnodes]
    cache = {}

    def inner(v):
        if v in cache:
            return cache[v]
        acc = [mp.mpf(0)] * (nmax + 1)
        for (c, w) in cnodes:
            G = mp.exp(-xi * (v * v + u - 2 * v * c * R))
            p1 = -xi + xi * v * c / R
            p2 = -xi * v * c / (2 * R ** 3)
            p3 = 3 * xi * v * c / (4 * R ** 5)
            ders = [G, p1 * G, (p2 + p1 * p1) * G, (p3 + 3 * p1 * p2 + p1 ** 3) * G]
            for n in range(nmax + 1):
                acc[n] += w * ders[n]
        cache[v] = acc
        return acc

    B = max([0.0] + [b for (c, a, b, g) in fac.terms if b > 0]) if isinstance(fac, TermFactor) else max(fac.B, 0)
    peak = R + B / xi
    w = 1 / mp.sqrt(xi)
    pts = [0, max(peak - 8 * w, 0) / 2, max(peak - 8 * w, mp.mpf("0.01")), peak, peak + 8 * w, peak + 30 * w]
    # a factor given by its terms: each term's exp(b r - g r^2) (products of
    # two for I4/I6) times the pair Gaussian peaks at (2 xi R + b)/(2 (xi + g))
    if isinstance(fac, TermFactor):
        bgs = {(b, g) for (_, _, b, g) in fac.terms}
        if cls in (4, 6):
            bgs = {(b1 + b2, g1 + g2) for (b1, g1) in bgs for (_, _, b2, g2) in facp.terms}
        for (b, g) in bgs:
            ctr = (2 * xi * R + b) / (2 * (xi + g))
            sg = 1 / mp.sqrt(xi + g)
            pts += [max(ctr + k * sg, mp.mpf("0.01")) for k in (-8, -2, 0, 2, 8)]
    pts = sorted(set(pts))
    out = []
    for n in range(nmax + 1):
        val = mp.quad(lambda v: 2 * mp.pi * v * v * k(v) * inner(v)[n], pts + [mp.inf])
        out.append(xi / mp.pi * 2 ** n * val)
    return out


@pytest.mark.parametrize("cls,fa,fb,T", [(2, "P1", "P1", 5.0), (4, "P1", "P4", 0.3), (4, "P4", "P4", 40.0),
                                         (6, "P1", "P1", 5.0), (4, "P2", "P2", 0.3), (2, "P3", "P3", 5.0),
                                         (6, "P1", "P4", 40.0), (3, "P3", "P3", 40.0), (6, "G5", "G5", 0.3),
                                         (6, "STG", "STG", 0.3)])
def test_geminal_kernels_vs_convolution_quadrature(cls, fa, fb, T):
    """(ss|k_i|ss) radial derivatives n = 0..3 of the oracle (Eq. (bfinal) by
    its own panels and derivative forms) against the two-dimensional
    convolution quadrature above, for kernels with a long-range part
    (c0 != 0): I2, I4 with (P1, P4) and (P4, P4), I6, and the negative powers
    of P2 in I4 (rho + rho' = -3) and of P3 in I2 and I3, and a factor given
    by its terms (G5: Gaussian geminals, a half-integer power, a growing term).  Catches a wrong
    r k_i(r) for I4/I6 with c0 != 0 and quadrature panels placed without the
    exp((B + B') r) growth, which symmetry and invariance tests cannot see."""
    def get(name):
        return TermFactor(GENERIC_FACTORS[name]) if name in GENERIC_FACTORS else FACTOR_SETS[name]
    fac, facp = get(fa), get(fb)
    xi = 0.9
    R = math.sqrt(T / xi)
    A = radial.radial_auto(cls, [xi], [R], 3, fac, facp).to_mp()[0]
    with mp.workdps(23):
        ref = _convolution_derivatives(cls, fac, facp, xi, R)
    sc = [(2 * xi) ** n for n in range(4)]
    env = max(abs(ref[n]) / sc[n] for n in range(4))
    for n in range(4):
        err = abs(A[n] - ref[n]) / sc[n] / env
        assert err < 1e-16, (n, A[n], ref[n], err)


@pytest.mark.parametrize("cls,fa,T", [(2, "STG", 0.5), (3, "STG3", 30.0), (4, "STG3", 60.0), (6, "STG", 8.0)])
def test_decaying_exponentials_small_xi_vs_radial_quadrature(cls, fa, T):
    """Ten-no's exponential and other decaying terms (b < 0) with a diffuse
    pair Gaussian (xi = 0.02, so that b / sqrt(xi) ~ -8): the integrand of
    Eq. (bfinal) peaks at (2 xi R + b) / (2 xi), below R or at r = 0, far
    from the pair Gaussian's centre.  Oracle A_0..A_2 against mpmath's
    adaptive quadrature of the same radial integral,
      A_n / N' = int_0^inf r k(r) D^n g(r, R) dr,  g = [e^{-xi (r-R)^2} - e^{-xi (r+R)^2}] / R,
    with breaks at the powers of two up to 128 and at R and 2R (the peaks of
    these kernels lie below 1), and D^n g written out by hand.
    Catches quadrature panels that miss a decaying term's peak (the formula
    itself is pinned by the convolution quadrature above)."""
    fac = TermFactor(GENERIC_FACTORS[fa])
    xi = 0.02
    R = math.sqrt(T / xi)
    nmax = 2
    A = radial.radial_auto(cls, [xi], [R], nmax, fac, fac).to_mp()[0]
    with mp.workdps(40):
        k = _kernel_mp(cls, fac, fac)
        x = mp.mpf(xi)
        pts = sorted({mp.mpf(0), mp.mpf(R), mp.mpf(2 * R)} | {mp.mpf(2) ** j for j in range(-3, 8)}) + [mp.inf]

        Rm = mp.mpf(R)

        def dn(r, n):
            # g = h_- - h_+, h_s = e^{-xi (r + s R)^2} / R; with
            # q_s = -2 xi s r / R - 2 xi - 1/R^2:  D h_s = h_s q_s,
            # D^2 h_s = h_s (q_s^2 + q_s' / R),  q_s' = 2 xi s r / R^2 + 2 / R^3
            v = mp.mpf(0)
            for s_, sign in ((-1, 1), (1, -1)):
                h = mp.exp(-x * (r + s_ * Rm) ** 2) / Rm
                q = -2 * x * s_ * r / Rm - 2 * x - 1 / Rm ** 2
                dq = 2 * x * s_ * r / Rm ** 2 + 2 / Rm ** 3
                v += sign * h * (1 if n == 0 else (q if n == 1 else q * q + dq / Rm))
            return v

        ref = [mp.quad(lambda r: r * k(r) * dn(r, n), pts) for n in range(nmax + 1)]
    sc = [(2 * xi) ** n for n in range(nmax + 1)]
    env = max(abs(ref[n]) / sc[n] for n in range(nmax + 1))
    for n in range(nmax + 1):
        err = abs(A[n] - ref[n]) / sc[n] / env
        assert err < 1e-16, (n, A[n], ref[n], err)


def _one_prim(s, i):
    return dict(s, exps=np.asarray(s["exps"])[i:i + 1], coefs=np.ones(1))


def _shell(rng, l, K, spread=1.2):
    return {"center": rng.uniform(-spread, spread, 3), "l": l, "exps": 10 ** rng.uniform(-0.6, 0.6, K),
            "coefs": rng.uniform(0.1, 1.0, K)}


@pytest.mark.parametrize("cls", [3, 5])
def test_contraction_equals_sum_of_primitive_quartets(cls):
    """Contracted shells with K_a = 2, K_b = 3, K_c = 1, K_d = 2 against the sum
    of single-primitive evaluations weighted by c_a c_b c_c c_d.  Catches a
    mismatch between the flattened (K_a, K_b) primitive-pair order and the
    coefficient (or, for I5, Laplacian exponent) order in the contraction."""
    rng = np.random.default_rng(41 + cls)
    a, b, c, d = _shell(rng, 1, 2), _shell(rng, 0, 3), _shell(rng, 0, 1), _shell(rng, 1, 2)
    I = integrals.contracted(cls, a, b, c, d, P1, P1)
    ref = np.zeros_like(I)
    for i in range(2):
        for j in range(3):
            for k in range(1):
                for l in range(2):
                    w = a["coefs"][i] * b["coefs"][j] * c["coefs"][k] * d["coefs"][l]
                    ref += w * integrals.contracted(cls, _one_prim(a, i), _one_prim(b, j), _one_prim(c, k),
                                                    _one_prim(d, l), P1, P1)
    assert np.max(np.abs(I - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_symmetries_with_unequal_contraction_depths():
    """8-fold symmetry of I3 and the I5 antisymmetry (ab|cd) = -(ba|cd) with
    K_a = 2 != K_b = 3 > 1: swapping the bra shells must reorder both the
    primitive pairs and the coefficients consistently."""
    rng = np.random.default_rng(12)
    a, b, c, d = _shell(rng, 1, 2), _shell(rng, 0, 3), _shell(rng, 1, 2), _shell(rng, 0, 3)
    I = integrals.contracted(3, a, b, c, d, P1)
    sc = np.max(np.abs(I))
    assert np.max(np.abs(I - integrals.contracted(3, b, a, c, d, P1).transpose(1, 0, 2, 3))) <= 1e-15 * sc
    assert np.max(np.abs(I - integrals.contracted(3, c, d, a, b, P1).transpose(2, 3, 0, 1))) <= 1e-15 * sc
    I5 = integrals.contracted(5, a, b, c, d, P1)
    J5 = integrals.contracted(5, b, a, c, d, P1).transpose(1, 0, 2, 3)
    assert np.max(np.abs(I5 + J5)) <= 1e-15 * np.max(np.abs(I5))


@pytest.mark.slow
def test_i5_d_shell_bra_finite_difference():
    """Eq. (I5_) with a d shell in the bra: I5 = 1/2 (lap_A - lap_B) I3 by a
    5-point stencil on I3 over the centres A (d shell) and B (p shell).  The
    d shell's x^2, y^2, z^2 components are the only ones that reach the
    i (i-1) x^(i-2) branch of the oracle's bra Laplacian."""
    rng = np.random.default_rng(21)
    A0, B0, C, D = (rng.uniform(-1, 1, 3) for _ in range(4))
    sh = lambda l, e, x: {"center": x, "l": l, "exps": np.array([e]), "coefs": np.array([1.0])}
    ea, eb, ec, ed = 0.9, 0.6, 1.1, 0.7
    I5 = integrals.contracted(5, sh(2, ea, A0), sh(1, eb, B0), sh(0, ec, C), sh(0, ed, D), P1)
    h = 2e-3
    lap = np.zeros_like(I5)
    for which in (0, 1):
        for k in range(3):
            vals = []
            for m in (-2, -1, 0, 1, 2):
                A, B = A0.copy(), B0.copy()
                (A if which == 0 else B)[k] += m * h
                vals.append(integrals.contracted(3, sh(2, ea, A), sh(1, eb, B), sh(0, ec, C), sh(0, ed, D), P1))
            d2 = (-vals[0] + 16 * vals[1] - 30 * vals[2] + 16 * vals[3] - vals[4]) / (12 * h * h)
            lap += d2 if which == 0 else -d2
    assert np.max(np.abs(I5 - 0.5 * lap)) < 1e-7 * np.max(np.abs(I5))


def _tensor_of_shell_block(block, l):
    """Expand the canonical Cartesian components of one index of angular
    momentum l into a symmetric rank-l tensor index (3,)*l."""
    comps = integrals.cart(l)
    idx = np.zeros((3,) * l, dtype=int)
    for multi in np.ndindex(*((3,) * l)):
        cnt = [multi.count(0), multi.count(1), multi.count(2)]
        idx[multi] = comps.index(tuple(cnt))
    return idx


def _to_tensor(I, ls):
    """Block [a][b][c][d] -> tensor with each index of angular momentum l
    replaced by l Cartesian vector indices."""
    maps = [_tensor_of_shell_block(None, l) for l in ls]
    shape = sum(((3,) * l for l in ls), ())
    T = np.zeros(shape)
    for multi in np.ndindex(*shape):
        pos, ci = 0, []
        for l, mp_ in zip(ls, maps):
            sub = multi[pos:pos + l]
            ci.append(mp_[sub] if l else 0)
            pos += l
        T[multi] = I[tuple(ci)]
    return T


@pytest.mark.parametrize("ls", [(2, 0, 2, 1), (3, 0, 1, 2)])
def test_rotation_covariance_d_and_f_shells(ls):
    """Rotating every centre by an orthogonal Q turns each d index into a
    rank-2 and each f index into a rank-3 tensor index (x_i x_j -> Q_ik Q_jl
    x_k x_l).  Catches a wrong Cartesian component order or a wrong Hermite
    index t + t' in R_tuv beyond L = 3."""
    rng = np.random.default_rng(sum(ls) + 50)
    sh = [{"center": rng.uniform(-1, 1, 3), "l": l, "exps": 10 ** rng.uniform(-0.3, 0.3, 1),
           "coefs": np.array([1.0])} for l in ls]
    Qm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    I = integrals.contracted(2, *sh, P1)
    rot = [dict(s, center=Qm @ s["center"]) for s in sh]
    J = integrals.contracted(2, *rot, P1)
    TI, TJ = _to_tensor(I, ls), _to_tensor(J, ls)
    out = TI
    for ax in range(out.ndim):
        out = np.moveaxis(np.tensordot(Qm, out, axes=([1], [ax])), 0, ax)
    assert np.max(np.abs(TJ - out)) < 1e-13 * np.max(np.abs(TI))
