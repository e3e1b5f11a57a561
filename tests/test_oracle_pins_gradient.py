"""Pins of the oracle's first derivatives with respect to a centre: centred
finite differences of the oracle's own integrals (an independent check of
the raised/lowered-shell formula), and translation invariance
d/dA + d/dB + d/dC + d/dD = 0 with each term from the formula applied to its
own centre (which fails for a wrong sign, factor 2e, or lowered-shell term)."""
import numpy as np
import pytest

from oracle import gradient, integrals
from synth import FACTOR_SETS


def _shells(seed, ls):
    rng = np.random.default_rng(seed)
    out = []
    for l in ls:
        K = 2
        out.append({"center": rng.uniform(-1.2, 1.2, 3), "l": l, "exps": 10 ** rng.uniform(-0.4, 0.4, K),
                    "coefs": rng.uniform(0.2, 1.0, K)})
    return out


@pytest.mark.parametrize("cls,ls", [(3, (1, 0, 1, 0)), (2, (2, 1, 0, 1)), (6, (1, 1, 1, 0)), (5, (2, 0, 1, 0))])
def test_gradient_against_finite_differences(cls, ls):
    sa, sb, sc, sd = _shells(7 + cls, ls)
    P1 = FACTOR_SETS["P1"]
    G = gradient.grad_first_centre(cls, sa, sb, sc, sd, P1, P1)
    h = 1e-3
    for d in range(3):
        vals = {}
        for k in (-2, -1, 1, 2):
            s2 = dict(sa, center=np.array(sa["center"], float) + k * h * np.eye(3)[d])
            vals[k] = integrals.contracted(cls, s2, sb, sc, sd, P1, P1)
        fd = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * h)  # error O(h^4)
        scale = np.max(np.abs(G[d])) + 1e-30
        assert np.max(np.abs(fd - G[d])) / scale < 1e-9, (d, np.max(np.abs(fd - G[d])) / scale)


@pytest.mark.parametrize("cls", [3, 4])
def test_gradient_translation_invariance(cls):
    sa, sb, sc, sd = _shells(21, (1, 2, 0, 1))
    P1, P4 = FACTOR_SETS["P1"], FACTOR_SETS["P4"]
    fp = P4 if cls == 4 else P1
    gA = gradient.grad_first_centre(cls, sa, sb, sc, sd, P1, fp)
    # d/dB of (ab|cd) is d/dA of (ba|cd) with a, b swapped back; C, D through (cd|ab)
    gB = np.transpose(gradient.grad_first_centre(cls, sb, sa, sc, sd, P1, fp), (0, 2, 1, 3, 4))
    gC = np.transpose(gradient.grad_first_centre(cls, sc, sd, sa, sb, fp, P1), (0, 3, 4, 1, 2))
    gD = np.transpose(gradient.grad_first_centre(cls, sd, sc, sa, sb, fp, P1), (0, 3, 4, 2, 1))
    tot = gA + gB + gC + gD
    scale = max(np.max(np.abs(g)) for g in (gA, gB, gC, gD))
    assert np.max(np.abs(tot)) / scale < 1e-13, np.max(np.abs(tot)) / scale
