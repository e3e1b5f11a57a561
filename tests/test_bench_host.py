"""Host logic of bench.py: the method flop count behind roofline.achieved,
checked against the dense per-primitive-quartet counts and E^ab nonzero
fractions of the hot-path scope table (ket 2 H_ab H_cd n_cd and bra
2 n_ab H_ab n_cd flops: (pp|pp) 1,800 / 1,620, (dd|dd) 88,200 / 90,720,
(ff|ff) 1.41e6 / 1.68e6; E^ab 37 %, 27 %, 23 % nonzero for pp, dd, ff), and
the rule that marks I5 blocks vanishing identically."""
import math

import numpy as np
import pytest

import bench
from synth.molecules import Shell


@pytest.mark.parametrize("l, ket, bra", [(1, 1800, 1620), (2, 88200, 90720), (3, 1411200, 1680000)])
def test_method_count_dense_terms(l, ket, bra):
    L = 4 * l
    r = 3 * math.comb(L + 4, 4)
    assert bench.method_flops(l, l, l, l, False, 1, 0) == r + ket
    assert bench.method_flops(l, l, l, l, False, 0, 1) == pytest.approx(bra * bench.e_nonzero_fraction(l, l))
    # I5: four components of the ket and bra transforms, R at L + 2
    assert bench.method_flops(l, l, l, l, True, 1, 0) == 3 * math.comb(L + 6, 4) + 4 * ket


@pytest.mark.parametrize("l, frac", [(1, 0.37), (2, 0.27), (3, 0.23)])
def test_e_nonzero_fraction(l, frac):
    assert round(bench.e_nonzero_fraction(l, l), 2) == frac
    assert bench.e_nonzero_fraction(0, 0) == 1.0


def _sh(l, c, e=1.0):
    return Shell(np.array(c, float), l, np.array([e]), np.array([1.0]))


def test_i5_vanishing_rule():
    A, B = (0.0, 0.0, 0.0), (1.0, 0.5, -0.3)
    shells = [_sh(0, A), _sh(1, A), _sh(2, A), _sh(0, A, 2.5), _sh(0, B), _sh(1, A), _sh(2, B)]
    v = bench.i5_vanishes
    assert v((0, 0, 4, 6), shells)          # s shell twice
    assert v((1, 1, 6, 4), shells)          # p shell twice
    assert v((2, 2, 0, 3), shells)          # d twice, two s shells on its centre
    assert not v((2, 2, 0, 4), shells)      # an s shell off the centre
    assert not v((2, 2, 5, 0), shells)      # a p shell in the ket
    assert not v((2, 6, 0, 3), shells)      # two different shells
    assert not v((0, 3, 4, 4), shells)      # two different s shells
