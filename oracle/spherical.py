"""Real solid harmonics and the Cartesian-to-spherical transform of integral
blocks (oracle).

Test infrastructure only.

Sec. II.D works with the regular solid harmonics r^l Y_lm (Eq. (Ylm)) and
notes that the real forms, the combinations of m and -m, serve equally.
Here the real solid harmonics are taken in Racah's normalisation,
S_lm(r) = sqrt(4 pi/(2l+1)) r^l Y_lm(r^) in real form (S_l0 = z^l + ...,
S_11 = x, S_1-1 = y), written out by the closed sum over Cartesian monomials
(t, u, v running over the terms of the expansion of r^l P_l^|m| cos / sin):
  S_lm = N_lm sum_t sum_u sum_v C_tuv x^(2t+|m|-2(u+v)) y^(2(u+v)) z^(l-2t-|m|),
  C_tuv = (-1)^(t+v-v_m) 4^-t binom(l,t) binom(l-t,|m|+t) binom(t,u) binom(|m|,2v),
  N_lm = sqrt(2 (l+|m|)! (l-|m|)! / 2^[m=0]) / (2^|m| l!),
with t = 0..floor((l-|m|)/2), u = 0..t, v = v_m, v_m + 1, ... <= |m|/2 and
v_m = 0 for m >= 0, 1/2 for m < 0.  A shell of unnormalised primitives
x^i y^j z^k exp(-e r^2) goes over to S_lm exp(-e r^2) = sum_c C[m, c] phi_c.
"""
import math
import numpy as np

from .integrals import cart


def solid_harmonic(l, m):
    """{(i, j, k): coefficient} of S_lm, the closed sum above."""
    am = abs(m)
    two_vm = 0 if m >= 0 else 1  # 2 v_m
    norm = math.sqrt(2.0 * math.factorial(l + am) * math.factorial(l - am) / (2.0 if m == 0 else 1.0))
    norm /= 2 ** am * math.factorial(l)
    poly = {}
    for t in range((l - am) // 2 + 1):
        for u in range(t + 1):
            two_v = two_vm
            while two_v <= am:
                sign = -1 if ((2 * t + two_v - two_vm) // 2) % 2 else 1
                c = sign * 0.25 ** t * math.comb(l, t) * math.comb(l - t, am + t) * math.comb(t, u) * math.comb(am, two_v)
                key = (2 * t + am - 2 * u - two_v, 2 * u + two_v, l - 2 * t - am)
                poly[key] = poly.get(key, 0.0) + norm * c
                two_v += 2
    return {k: v for k, v in poly.items() if v != 0.0}


def coefficients(l):
    """(2l+1, ncart(l)) matrix C[m + l, c] over the canonical Cartesian order."""
    comps = cart(l)
    C = np.zeros((2 * l + 1, len(comps)))
    for m in range(-l, l + 1):
        for key, v in solid_harmonic(l, m).items():
            C[m + l, comps.index(key)] = v
    return C


def block_to_sph(block, la, lb, lc, ld):
    """Cartesian block [a][b][c][d] (flat or 4-D) to [ma][mb][mc][md]."""
    dims = [len(cart(l)) for l in (la, lb, lc, ld)]
    X = np.asarray(block, dtype=np.float64).reshape(dims)
    for axis, l in enumerate((la, lb, lc, ld)):
        X = np.moveaxis(np.tensordot(coefficients(l), X, axes=([1], [axis])), 0, axis)
    return X.ravel()
