"""Pins of the oracle's real solid harmonics (Sec. II.D, Eq. (Ylm) in real
form, Racah's normalisation), and the library's coefficient table against
them.  Each pin fixes something the construction could get wrong: a
polynomial that is not harmonic, a wrong norm or a lost orthogonality, a
flipped sign or swapped m, a wrong Cartesian column."""
import math
import os

import numpy as np
import pytest

from oracle import spherical as sp
from oracle.integrals import cart

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1412_5070_amd",
                   "libf12int.so")


def _sphere_moment(i, j, k):
    """int over the unit sphere of x^i y^j z^k (closed form)."""
    if i % 2 or j % 2 or k % 2:
        return 0.0
    g = math.gamma
    return 2.0 * g((i + 1) / 2) * g((j + 1) / 2) * g((k + 1) / 2) / g((i + j + k + 3) / 2)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 4])
def test_solid_harmonics_are_harmonic(l):
    """Every S_lm is a homogeneous polynomial of degree l with zero Laplacian."""
    for m in range(-l, l + 1):
        P = sp.solid_harmonic(l, m)
        assert all(sum(key) == l for key in P)
        lap = {}
        for (i, j, k), c in P.items():
            for d, e in ((0, i), (1, j), (2, k)):
                if e >= 2:
                    key = [i, j, k]
                    key[d] -= 2
                    lap[tuple(key)] = lap.get(tuple(key), 0.0) + c * e * (e - 1)
        assert all(abs(v) < 1e-12 for v in lap.values()), (l, m, lap)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 4])
def test_solid_harmonics_orthogonal_with_racah_norm(l):
    """int S_lm S_lm' dOmega = 4 pi / (2l+1) delta_mm' (Racah's normalisation
    of r^l Y_lm), by the closed-form sphere moments of the monomials."""
    for m in range(-l, l + 1):
        for mp in range(-l, l + 1):
            A, B = sp.solid_harmonic(l, m), sp.solid_harmonic(l, mp)
            v = sum(ca * cb * _sphere_moment(a[0] + b[0], a[1] + b[1], a[2] + b[2])
                    for a, ca in A.items() for b, cb in B.items())
            ref = 4 * math.pi / (2 * l + 1) if m == mp else 0.0
            assert abs(v - ref) < 1e-13, (l, m, mp, v)


@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_solid_harmonics_signs_and_axes(l):
    """S_l0 = 1 on the z axis; S_l,l and S_l,-l are positive multiples of
    Re (x + iy)^l and Im (x + iy)^l; the p set is (y, z, x) for m = -1, 0, 1."""
    rng = np.random.default_rng(l)

    def ev(P, x, y, z):
        return sum(c * x ** i * y ** j * z ** k for (i, j, k), c in P.items())

    assert abs(ev(sp.solid_harmonic(l, 0), 0.0, 0.0, 1.0) - 1.0) < 1e-14
    x, y = rng.normal(size=2)
    w = (x + 1j * y) ** l
    cp = ev(sp.solid_harmonic(l, l), x, y, 0.0) / w.real
    cm = ev(sp.solid_harmonic(l, -l), x, y, 0.0) / w.imag
    norm = math.sqrt(math.factorial(2 * l) * 2) / (2 ** l * math.factorial(l))  # |S_ll| / |(x+iy)^l|
    assert abs(cp - norm) < 1e-12 and abs(cm - norm) < 1e-12, (cp, cm, norm)
    if l == 1:
        assert np.allclose(sp.coefficients(1), [[0, 1, 0], [0, 0, 1], [1, 0, 0]])
    if l == 2:
        C = sp.coefficients(2)
        comps = cart(2)
        assert abs(C[4, comps.index((2, 0, 0))] - math.sqrt(3) / 2) < 1e-15
        assert abs(C[0, comps.index((1, 1, 0))] - math.sqrt(3)) < 1e-15


def test_block_transform_p_is_permutation():
    """For p shells the transform only reorders (x, y, z) to (y, z, x)."""
    rng = np.random.default_rng(3)
    B = rng.normal(size=(3, 1, 3, 1))
    S = sp.block_to_sph(B, 1, 0, 1, 0).reshape(3, 1, 3, 1)
    perm = [1, 2, 0]
    assert np.array_equal(S, B[perm][:, :, perm])


@pytest.mark.skipif(not os.path.exists(LIB), reason="libf12int.so not built")
@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_library_coefficients_equal_oracle(l):
    """The library builds its table by the recurrences of the real solid
    harmonics; it must equal the oracle's closed sum."""
    from paper_1412_5070_amd import f12int
    assert np.allclose(f12int.sph_coefficients(l), sp.coefficients(l), rtol=0, atol=2e-15)


def test_i5_same_shell_vanishes_over_solid_harmonics():
    """Over solid harmonics a shell is S_lm(r) G(r) with one radial G for all
    m, so lap phi_m = S_lm H(r) and (lap phi_m) phi_m' - phi_m (lap phi_m') = 0
    pointwise: the oracle's I5 block of a d shell taken twice as the bra,
    transformed to S_lm, vanishes, although its Cartesian block does not.
    Catches a wrong Laplacian term in the oracle's I5 for l >= 2, or a wrong
    solid harmonic."""
    from oracle import integrals
    from synth import FACTOR_SETS
    rng = np.random.default_rng(11)
    d = {"center": np.array([0.1, -0.2, 0.3]), "l": 2, "exps": np.array([0.9, 2.1]), "coefs": np.array([0.6, 0.4])}
    c = {"center": np.array([1.0, 0.4, -0.5]), "l": 1, "exps": np.array([0.7]), "coefs": np.array([1.0])}
    s = {"center": np.array([-0.6, 0.8, 0.2]), "l": 0, "exps": np.array([1.3]), "coefs": np.array([1.0])}
    P1 = FACTOR_SETS["P1"]
    I5 = np.asarray(integrals.contracted(5, d, d, c, s, P1, P1), dtype=float)
    I3 = np.asarray(integrals.contracted(3, d, d, c, s, P1, P1), dtype=float)
    S5 = sp.block_to_sph(I5, 2, 2, 1, 0)
    S3 = sp.block_to_sph(I3, 2, 2, 1, 0)
    assert np.max(np.abs(I5)) > 1e-3 * np.max(np.abs(I3))
    assert np.max(np.abs(S5)) < 1e-14 * 2.1 * np.max(np.abs(S3)), (np.max(np.abs(S5)), np.max(np.abs(S3)))


def test_i5_same_shell_vanishes_for_a_spherical_ket():
    """With the bra density difference written as a divergence,
    (lap phi_a) phi_b - phi_a (lap phi_b) = div(phi_b grad phi_a - phi_a grad phi_b),
    the I5 element is minus the integral of that flux against grad V, V the
    potential of the ket density.  When the ket is two s shells on the bra's
    centre, V is spherical about it and only the radial parts of the flux
    count; for two components P_a g, P_b g of one shell (P homogeneous of
    degree l, one radial g) those cancel pointwise.  So the oracle's Cartesian
    I5 block of a d shell taken twice, against s shells on the same centre,
    vanishes; moved off the centre, the ket gives a block of the size of its
    terms.  Catches a wrong or one-sided Laplacian term in the oracle's I5."""
    from oracle import integrals
    from synth import FACTOR_SETS
    A = np.array([0.2, -0.1, 0.4])
    d = {"center": A, "l": 2, "exps": np.array([0.8, 2.3]), "coefs": np.array([0.5, 0.7])}
    s1 = {"center": A, "l": 0, "exps": np.array([0.6, 1.9]), "coefs": np.array([0.3, 0.8])}
    s2 = {"center": A, "l": 0, "exps": np.array([1.4]), "coefs": np.array([1.0])}
    P1 = FACTOR_SETS["P1"]
    I5 = np.asarray(integrals.contracted(5, d, d, s1, s2, P1, P1), dtype=float)
    I3 = np.asarray(integrals.contracted(3, d, d, s1, s2, P1, P1), dtype=float)
    assert np.max(np.abs(I5)) < 1e-14 * 2.3 * np.max(np.abs(I3)), (np.max(np.abs(I5)), np.max(np.abs(I3)))
    s2_off = dict(s2, center=A + np.array([0.0, 0.9, -0.4]))
    J5 = np.asarray(integrals.contracted(5, d, d, s1, s2_off, P1, P1), dtype=float)
    J3 = np.asarray(integrals.contracted(3, d, d, s1, s2_off, P1, P1), dtype=float)
    assert np.max(np.abs(J5)) > 1e-3 * np.max(np.abs(J3))
