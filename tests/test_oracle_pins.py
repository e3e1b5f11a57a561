"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms (Boys function, Gaussian geminals), library routines (mpmath), the
paper's worked example, symmetries, invariances and finite differences.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import dd, integrals, radial
from oracle.factor import Factor, f_value, f_deriv, tang_toennies
from oracle.hermite import e_coefficients
from oracle.special import S_finite_part
from synth import FACTOR_SETS

P1 = FACTOR_SETS["P1"]
P4 = FACTOR_SETS["P4"]
SR = Factor(0.0, 0.5, 0.3, 0.8, 0)  # c0 = 0: short-range Gaussian part only


def boys(n, T):
    """Boys function F_n(T) = 1F1(n+1/2; n+3/2; -T)/(2n+1) (any real T)."""
    T = mp.mpf(T)
    return mp.hyp1f1(n + mp.mpf(1) / 2, n + mp.mpf(3) / 2, -T) / (2 * n + 1)


def shell(l, c, exps, coefs):
    return {"center": np.array(c, float), "l": l, "exps": np.array(exps, float), "coefs": np.array(coefs, float)}


# ---------------------------------------------------------------- radial part
@pytest.mark.parametrize("xi,T,nmax", [(0.05, 0.0, 6), (1.0, 0.3, 6), (1.0, 0.999, 6), (1.0, 1.001, 6),
                                       (3.0, 7.0, 10), (10.0, 40.0, 8), (0.3, 300.0, 4)])
def test_radial_coulomb_boys(xi, T, nmax):
    """Eq. (bfinal) with k1 = 1/r: A_n = 2 pi^(5/2)/(pq sqrt(p+q)) (-2 xi)^n F_n(T),
    i.e. A_n / N' = 2 (-2 xi)^n F_n(T) (Boys function via mpmath gammainc)."""
    R = math.sqrt(T / xi)
    A = radial.radial_auto(1, [xi], [R], nmax, P1, P1).to_mp()
    with mp.workdps(40):
        for n in range(nmax + 1):
            ref = 2 * (-2 * mp.mpf(xi)) ** n * boys(n, mp.mpf(xi) * mp.mpf(R) ** 2)
            assert abs(A[0, n] - ref) <= 1e-20 * abs(ref), (n, A[0, n], ref)


def test_radial_coulomb_mp_fallback():
    """Large T (cancellation beyond DD) goes through the arbitrary-precision path."""
    xi, T, nmax = 5.0, 3000.0, 4
    assert radial.cancellation_digits(T, nmax) > 13
    R = math.sqrt(T / xi)
    A = radial.radial_auto(1, [xi], [R], nmax, P1, P1).to_mp()
    with mp.workdps(40):
        for n in range(nmax + 1):
            ref = 2 * (-2 * mp.mpf(xi)) ** n * boys(n, mp.mpf(xi) * mp.mpf(R) ** 2)
            assert abs(A[0, n] - ref) <= 1e-20 * abs(ref)


@pytest.mark.parametrize("cls,fac,xi,T,n", [(2, "P1", 1.0, 40.0, 14), (6, "P1", 1.0, 40.0, 14),
                                            (4, "P4", 0.5, 60.0, 12)])
def test_radial_mp_route_agrees_with_dd_at_handover(cls, fac, xi, T, n):
    """radial_auto hands over from the DD quadrature to the mpmath one where the
    split form's cancellation exceeds 13 digits (T from about 40 at n = 14).
    Near that hand-over both quadratures must give the same A_n, on the
    (2 xi)^n-scaled envelope, for the geminal kernels too (the mpmath route
    is used at large T only; its panels are too coarse below T ~ 30)."""
    F = FACTOR_SETS[fac]
    assert radial.cancellation_digits(T, n) > 13 - 2  # at or near the hand-over
    R = math.sqrt(T / xi)
    a = radial.radial_derivatives(cls, [xi], [R], n, F, F).to_float().ravel()
    b = np.array([float(v) for v in radial.radial_derivatives_mp(cls, xi, R, n, F, F)])
    sc = (2 * xi) ** np.arange(n + 1)
    err = np.max(np.abs(a - b) / sc) / np.max(np.abs(b) / sc)
    assert err < 1e-13, (T, n, err)


def _geminal_B(mu, xi, u):
    """Short-range I2 kernel (1/r + 1/2) e^{-mu r^2}, as B/(pi/(p+q))^{3/2}:
    e^{-mu r^2}/r -> 2 pi/(mu+xi) e^{-mu xi u/(mu+xi)} F_0(xi^2 u/(mu+xi)),
    e^{-mu r^2}   -> (pi/(mu+xi))^{3/2} e^{-mu xi u/(mu+xi)}  (textbook)."""
    mu, xi, u = mp.mpf(mu), mp.mpf(xi), mp.mpf(u)
    e = mp.exp(-mu * xi * u / (mu + xi))
    return 2 * mp.pi / (mu + xi) * e * boys(0, xi * xi * u / (mu + xi)) + (mp.pi / (mu + xi)) ** 1.5 * e / 2


@pytest.mark.parametrize("xi,T", [(0.7, 0.0), (0.7, 0.5), (2.0, 3.0), (0.2, 12.0)])
def test_radial_geminal_closed_form(xi, T):
    """c0 = 0 reduces I2 to Gaussian-geminal kernels with closed forms; their
    radial derivatives A_n = 2^n d^n B/du^n (u = R^2) by mpmath differentiation."""
    nmax = 4
    R = math.sqrt(T / xi)
    p, q = 1.1, xi * 1.1 / (1.1 - xi) if xi < 1.1 else None
    A = radial.radial_auto(2, [xi], [R], nmax, SR, SR).to_mp()
    with mp.workdps(40):
        # A_n/N' with N' = sqrt(pi^5/(p+q))/(pq); (pi/(p+q))^{3/2}/N' = 4 xi / (4 pi)
        # because 4 xi N' = 4 pi (pi/(p+q))^{3/2}.
        scale = 4 * mp.mpf(xi) / (4 * mp.pi)
        for n in range(nmax + 1):
            ref = 2 ** n * mp.diff(lambda u: _geminal_B(SR.mu, xi, u), mp.mpf(R) ** 2, n) * scale
            assert abs(A[0, n] - ref) <= 1e-20 * abs(ref) + 1e-28, (n, A[0, n], ref)


@pytest.mark.parametrize("mu", [5.0, 50.0])
@pytest.mark.parametrize("xi,T", [(0.0135, 600.0), (0.013, 400.0), (0.0157, 107.0), (0.3, 200.0)])
def test_radial_narrow_geminal_closed_form(mu, xi, T):
    """Kernels much narrower than the pair Gaussian (mu >> xi) at large T put
    all the weight of the r-integral near r* = xi R / (mu + xi), far below R:
    the quadrature must resolve that peak on its own.  Closed forms (textbook
    Gaussian products, u = R^2): for e^{-mu r^2},
      B/(pi/(p+q))^{3/2} = (pi/(mu+xi))^{3/2} e^{-w u},  w = mu xi/(mu+xi),
    so A_n = (-2w)^n B exactly; for e^{-mu r^2}/r the F_0 form above."""
    from oracle.factor import TermFactor
    nmax = 3
    R = math.sqrt(T / xi)
    G = TermFactor(((1.0, 0.0, 0.0, mu),))
    A3 = radial.radial_auto(3, [xi], [R], nmax, G, G).to_mp()
    A2 = radial.radial_auto(2, [xi], [R], 0, G, G).to_mp()
    with mp.workdps(50):
        scale = mp.mpf(xi) / mp.pi
        m, x, u = mp.mpf(mu), mp.mpf(xi), mp.mpf(R) ** 2
        w = m * x / (m + x)
        b3 = (mp.pi / (m + x)) ** 1.5 * mp.exp(-w * u) * scale
        for n in range(nmax + 1):
            ref = (-2 * w) ** n * b3
            assert abs(A3[0, n] - ref) <= 1e-20 * abs(ref), (n, A3[0, n], ref)
        ref2 = 2 * mp.pi / (m + x) * mp.exp(-w * u) * boys(0, x * x * u / (m + x)) * scale
        assert abs(A2[0, 0] - ref2) <= 1e-20 * abs(ref2), (A2[0, 0], ref2)


def test_bfinal_vs_3d_convolution():
    """Eq. (bfinal) against the 2-D integral it comes from: B = (pi/(p+q))^{3/2}
    int d^3v k3(|v|) exp(-xi |v - X|^2), done in (v, cos theta) with mpmath."""
    p, q, R = 1.3, 0.7, 0.9
    xi = p * q / (p + q)
    A = radial.radial_auto(3, [xi], [R], 0, P1, P1)
    B_oracle = A.to_mp()[0, 0] * radial.n_prime(np.array([p]), np.array([q])).to_mp()[0]
    with mp.workdps(25):
        def k3(v):
            v = mp.mpf(v)
            return (1 + v / 2) * mp.exp(-P1.mu * v * v) + (1 - mp.exp(-P1.mu * v * v)) * P1.c0 * v ** P1.rho * mp.exp(P1.B * v)
        inner = lambda v: 2 * mp.pi * v * v * k3(v) * mp.quad(lambda c: mp.exp(-xi * (v * v + R * R - 2 * v * R * c)), [-1, 1])
        ref = (mp.pi / (p + q)) ** 1.5 * mp.quad(inner, [0, 1, 3, 8, 20])
    assert abs(B_oracle - ref) < 1e-15 * abs(ref)


def test_binary64_pointwise_route_fails_at_large_T():
    """Why the oracle works in double-double: the split-form pointwise
    derivative summed in binary64 (which is what the paper's H-recursion
    computes) loses digits like (2T)^n/(2n-1)!! at large T."""
    xi, T, n = 1.0, 100.0, 8
    R = math.sqrt(T / xi)
    r = np.linspace(R - 12, R + 12, 4001)
    wq = np.full_like(r, r[1] - r[0])
    wq[0] = wq[-1] = wq[0] / 2
    h = {}
    for s in (1, -1):
        E = np.exp(-xi * (r + s * R) ** 2)
        cur = {k: E / R ** k for k in range(1, 2 * n + 2)}
        for l in range(1, n + 1):
            cur = {k: -2 * s * xi * r * cur[k + 1] - 2 * xi * cur[k] - k * cur[k + 2] for k in range(1, 2 * (n - l) + 2)}
        h[s] = cur[1]
    v = float(np.sum(wq * (h[-1] - h[1])))
    ref = float(2 * (-2 * mp.mpf(xi)) ** n * boys(n, T))
    assert radial.cancellation_digits(T, n) > 8
    assert abs(v - ref) > 1e-6 * abs(ref)


# ----------------------------------------------------------- special functions
def test_worked_example_S_minus2():
    """The paper's worked example: S(-2, beta, 0) = -beta (gamma_E + ln(-beta) - 1), beta < 0."""
    for beta in (-0.8, -2.5):
        with mp.workdps(30):
            ref = -beta * (mp.euler + mp.log(-beta) - 1)
            # gamma = 0 needs the finite part with the exponential decay from beta alone
            val = S_finite_part(-2, beta, mp.mpf("1e-40"))
        assert abs(val - ref) < 1e-15 * abs(ref)


def test_S_beta_zero_closed_form():
    """S(alpha, 0, gamma) = Gamma((alpha+1)/2) / (2 gamma^((alpha+1)/2)) for
    non-integer alpha (finite part = analytic continuation)."""
    for a in (0.5, -1.5, -2.5):
        with mp.workdps(30):
            ref = mp.gamma((a + 1) / 2) / (2 * mp.mpf(0.7) ** ((a + 1) / 2))
            val = S_finite_part(a, 0, 0.7)
        assert abs(val - ref) < 1e-20 * abs(ref)


def test_tang_toennies_limits():
    """S_n(0) = 0, S_n(x) ~ x^(n+1)/(n+1)! as x -> 0, S_n(inf) = 1 (Eq. (ttdamp))."""
    for n in (0, 1, 2):
        x = dd.DD(np.array([0.0, 1e-6, 50.0]))
        s = tang_toennies(n, x).to_float()
        assert s[0] == 0.0
        assert abs(s[1] / (1e-6 ** (n + 1) / math.factorial(n + 1)) - 1) < 1e-5
        assert abs(s[2] - 1.0) < 1e-15


def test_factor_limits():
    """f(0) = 1, approached like r^(rho+2n+2); f'(0) = 1/2 (the cusp) when
    rho + 2n + 2 > 1; f -> c0 r^rho e^{B r} at large r (Eq. (rs12))."""
    for fac in (P1, FACTOR_SETS["P2"], FACTOR_SETS["P3"], P4):
        r0 = 1e-10
        r = dd.DD(np.array([r0, 40.0]))
        fv = f_value(fac, r).to_float()
        fd = f_deriv(fac, r).to_float()
        e = fac.rho + 2 * fac.n + 2
        lead = fac.c0 * fac.mu ** (fac.n + 1) / math.factorial(fac.n + 1) * r0 ** e
        assert abs(fv[0] - 1 - 0.5 * r0 - lead) < 1e-3 * abs(lead) + 1e-15
        if e > 1:
            assert abs(fd[0] - 0.5) < 1e-6
        lr = fac.c0 * 40.0 ** fac.rho * math.exp(fac.B * 40.0)
        assert abs(fv[1] / lr - 1) < 1e-12


# ------------------------------------------------------------- E coefficients
def test_e_coefficients_product_identity():
    """Eq. (AB) in 1-D: x_A^i x_B^j e^{-a x_A^2 - b x_B^2} = sum_t E_t^{ij} d^t/dP^t e^{-p x_P^2},
    with d^t/dP^t e^{-p (x-P)^2} = p^(t/2) H_t(sqrt(p)(x-P)) e^{-p (x-P)^2}."""
    a, b, A, B = 0.8, 1.7, -0.3, 0.9
    E = e_coefficients([a], [b], [A], [B], 3, 2).to_mp()[0]
    with mp.workdps(40):
        p = mp.mpf(a) + b
        P = (a * mp.mpf(A) + b * mp.mpf(B)) / p
        for x in (-1.2, 0.1, 0.77, 2.0):
            for i in range(4):
                for j in range(3):
                    xa, xb = x - mp.mpf(A), x - mp.mpf(B)
                    lhs = xa ** i * xb ** j * mp.exp(-a * xa ** 2 - b * xb ** 2)
                    rhs = sum(E[i, j, t] * p ** (mp.mpf(t) / 2) * mp.hermite(t, mp.sqrt(p) * (x - P))
                              * mp.exp(-p * (x - P) ** 2) for t in range(i + j + 1))
                    assert abs(lhs - rhs) < 1e-28 * abs(lhs)


def test_overlap_closed_form():
    """The overlap of two s Gaussians: E_0^{00} products times (pi/p)^{3/2} = (pi/p)^{3/2} e^{-ab/p |AB|^2}."""
    a, b = 0.6, 1.9
    A, B = np.array([0.1, -0.2, 0.3]), np.array([0.9, 0.4, -0.5])
    e = 1.0
    for k in range(3):
        e *= float(e_coefficients([a], [b], [A[k]], [B[k]], 0, 0).to_mp()[0, 0, 0, 0])
    assert abs(e - math.exp(-a * b / (a + b) * np.sum((A - B) ** 2))) < 1e-15


# -------------------------------------------------------- whole-integral pins
def test_ssss_coulomb_closed_form():
    """(ss|1/r12|ss) = 2 pi^(5/2) / (pq sqrt(p+q)) K_ab K_cd F_0(T)."""
    a, b, c, d = 0.9, 0.4, 1.3, 0.25
    A, B, C, D = ([0, 0, 0], [0.5, 0.1, 0], [1.0, 1.0, 0.3], [0.2, -0.8, 1.1])
    s = lambda e, x: shell(0, x, [e], [1.0])
    v = integrals.contracted(1, s(a, A), s(b, B), s(c, C), s(d, D))[0, 0, 0, 0]
    A, B, C, D = map(lambda x: np.array(x, float), (A, B, C, D))
    p, q = a + b, c + d
    P, Q = (a * A + b * B) / p, (c * C + d * D) / q
    xi = p * q / (p + q)
    ref = 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)) * math.exp(-a * b / p * np.sum((A - B) ** 2)) * \
        math.exp(-c * d / q * np.sum((C - D) ** 2)) * float(boys(0, xi * np.sum((P - Q) ** 2)))
    assert abs(v - ref) < 1e-15 * abs(ref)


def _rand_shells(rng, ls, spread=1.5, K=2):
    out = []
    for l in ls:
        out.append(shell(l, rng.uniform(-spread, spread, 3), 10 ** rng.uniform(-0.7, 0.7, K), rng.uniform(0.1, 1, K)))
    return out


@pytest.mark.parametrize("cls", [1, 2, 3, 4, 6])
def test_eightfold_symmetry(cls):
    """(ab|cd) = (ba|cd) = (ab|dc) = (cd|ab) for classes with a symmetric kernel."""
    rng = np.random.default_rng(10 + cls)
    a, b, c, d = _rand_shells(rng, (1, 0, 1, 1), K=1)
    I = integrals.contracted(cls, a, b, c, d, P1, P4)
    Iba = integrals.contracted(cls, b, a, c, d, P1, P4)
    Idc = integrals.contracted(cls, a, b, d, c, P1, P4)
    Icd = integrals.contracted(cls, c, d, a, b, P1, P4)
    scale = np.max(np.abs(I))
    assert np.max(np.abs(I - Iba.transpose(1, 0, 2, 3))) <= 1e-15 * scale
    assert np.max(np.abs(I - Idc.transpose(0, 1, 3, 2))) <= 1e-15 * scale
    assert np.max(np.abs(I - Icd.transpose(2, 3, 0, 1))) <= 1e-15 * scale


def test_i5_antisymmetry():
    """I5: (ab|cd) = -(ba|cd) and (ab|cd) = (ab|dc); no (cd|ab) relation."""
    rng = np.random.default_rng(5)
    a, b, c, d = _rand_shells(rng, (1, 0, 0, 1), K=1)
    I = integrals.contracted(5, a, b, c, d, P1)
    Iba = integrals.contracted(5, b, a, c, d, P1)
    Idc = integrals.contracted(5, a, b, d, c, P1)
    scale = np.max(np.abs(I))
    assert np.max(np.abs(I + Iba.transpose(1, 0, 2, 3))) <= 1e-15 * scale
    assert np.max(np.abs(I - Idc.transpose(0, 1, 3, 2))) <= 1e-15 * scale


def test_i5_equals_half_laplacian_difference_of_i3():
    """Eq. (I5_): I5 = 1/2 (lap_A - lap_B) I3, checked with a 5-point finite
    difference stencil on I3 over s-type primitives."""
    rng = np.random.default_rng(7)
    A0 = rng.uniform(-1, 1, 3)
    B0 = rng.uniform(-1, 1, 3)
    C, D = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
    ea, eb, ec, ed = 0.9, 0.5, 1.1, 0.7
    s = lambda e, x: shell(0, x, [e], [1.0])
    I5 = integrals.contracted(5, s(ea, A0), s(eb, B0), s(ec, C), s(ed, D), P1)[0, 0, 0, 0]
    h = 2e-3
    lap = 0.0
    for which in (0, 1):
        for k in range(3):
            vals = []
            for m in (-2, -1, 0, 1, 2):
                A, B = A0.copy(), B0.copy()
                (A if which == 0 else B)[k] += m * h
                vals.append(integrals.contracted(3, s(ea, A), s(eb, B), s(ec, C), s(ed, D), P1)[0, 0, 0, 0])
            d2 = (-vals[0] + 16 * vals[1] - 30 * vals[2] + 16 * vals[3] - vals[4]) / (12 * h * h)
            lap += d2 if which == 0 else -d2
    assert abs(I5 - 0.5 * lap) < 1e-7 * abs(I5)


def test_translation_invariance():
    rng = np.random.default_rng(3)
    a, b, c, d = _rand_shells(rng, (1, 1, 0, 1), K=1)
    I = integrals.contracted(3, a, b, c, d, P1)
    shift = np.array([0.37, -1.1, 2.3])
    sh = lambda s: dict(s, center=s["center"] + shift)
    J = integrals.contracted(3, sh(a), sh(b), sh(c), sh(d), P1)
    assert np.max(np.abs(I - J)) < 1e-14 * np.max(np.abs(I))


def test_rotation_covariance_p_shells():
    """Rotating every centre by an orthogonal matrix Q turns the (p s|p s) block
    into Q I Q^T: pins the Cartesian/Hermite bookkeeping of R_tuv."""
    rng = np.random.default_rng(4)
    a, b, c, d = _rand_shells(rng, (1, 0, 1, 0), K=1)
    Qm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    I = integrals.contracted(2, a, b, c, d, P1)[:, 0, :, 0]
    rot = lambda s: dict(s, center=Qm @ s["center"])
    J = integrals.contracted(2, rot(a), rot(b), rot(c), rot(d), P1)[:, 0, :, 0]
    assert np.max(np.abs(J - Qm @ I @ Qm.T)) < 1e-14 * np.max(np.abs(I))


def test_p_function_as_centre_derivative():
    """x_A e^{-a r_A^2} = (1/2a) d/dA_x e^{-a r_A^2}: the (p s|s s) block equals
    the A-gradient of (s s|s s) over 2a (5-point stencil)."""
    rng = np.random.default_rng(8)
    A0, B, C, D = (rng.uniform(-1, 1, 3) for _ in range(4))
    ea = 0.8
    s = lambda l, e, x: shell(l, x, [e], [1.0])
    Ip = integrals.contracted(4, s(1, ea, A0), s(0, 0.6, B), s(0, 1.2, C), s(0, 0.4, D), P1, P4)[:, 0, 0, 0]
    h = 2e-3
    for k in range(3):
        vals = []
        for m in (-2, -1, 1, 2):
            A = A0.copy()
            A[k] += m * h
            vals.append(integrals.contracted(4, s(0, ea, A), s(0, 0.6, B), s(0, 1.2, C), s(0, 0.4, D), P1, P4)[0, 0, 0, 0])
        g = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
        assert abs(Ip[k] - g / (2 * ea)) < 1e-8 * np.max(np.abs(Ip))


def test_i4_i6_swap_factors():
    """k4 = f f' and k6 = f_r f'_r are symmetric under f <-> f'."""
    rng = np.random.default_rng(9)
    a, b, c, d = _rand_shells(rng, (0, 1, 0, 0), K=1)
    for cls in (4, 6):
        I = integrals.contracted(cls, a, b, c, d, P1, P4)
        J = integrals.contracted(cls, a, b, c, d, P4, P1)
        assert np.max(np.abs(I - J)) <= 1e-15 * np.max(np.abs(I))
