"""Quadrature rules in double-double for the oracle (test infrastructure).

Gauss-Legendre nodes on [-1, 1] and tanh-sinh nodes on [0, 1], both
computed once with mpmath at 40 digits and rounded to DD, so that the
rule itself carries no binary64 error into sums with heavy cancellation.
"""
import functools
import numpy as np
import mpmath as mp
from . import dd


@functools.lru_cache(maxsize=None)
def gauss_legendre(n=48):
    """n-point Gauss-Legendre rule on [-1, 1] (nodes, weights) in DD."""
    with mp.workdps(45):
        xs, ws = [], []
        for k in range(1, n + 1):
            # Newton on P_n starting from the Chebyshev-like guess
            x = mp.cos(mp.pi * (k - mp.mpf(1) / 4) / (n + mp.mpf(1) / 2))
            for _ in range(100):
                p0, p1 = mp.mpf(1), x
                for j in range(2, n + 1):
                    p0, p1 = p1, ((2 * j - 1) * x * p1 - (j - 1) * p0) / j
                dp = n * (x * p1 - p0) / (x * x - 1)
                dx = p1 / dp
                x -= dx
                if abs(dx) < mp.mpf(10) ** -42:
                    break
            p0, p1 = mp.mpf(1), x
            for j in range(2, n + 1):
                p0, p1 = p1, ((2 * j - 1) * x * p1 - (j - 1) * p0) / j
            dp = n * (x * p1 - p0) / (x * x - 1)
            xs.append(x)
            ws.append(2 / ((1 - x * x) * dp * dp))
        return dd.DD.from_mp(xs), dd.DD.from_mp(ws)


@functools.lru_cache(maxsize=None)
def tanh_sinh(h=1.0 / 16, tmax=4.6):
    """tanh-sinh rule on [0, 1]: x = (1 + tanh(pi/2 sinh t)) / 2.

    Returns DD nodes x, DD weights w and DD complements 1 - x (so that the
    integrand can be evaluated without cancellation near the right end).
    """
    with mp.workdps(45):
        xs, ws, cs = [], [], []
        k = -int(tmax / h)
        while k * h <= tmax:
            t = k * mp.mpf(h)
            u = mp.pi / 2 * mp.sinh(t)
            ch = mp.cosh(u)
            # x = 1/(1+exp(-2u)), 1-x = 1/(1+exp(2u))
            x = 1 / (1 + mp.exp(-2 * u))
            c = 1 / (1 + mp.exp(2 * u))
            w = mp.mpf(h) * mp.pi / 2 * mp.cosh(t) / (2 * ch * ch)
            xs.append(x)
            cs.append(c)
            ws.append(w)
            k += 1
        return dd.DD.from_mp(xs), dd.DD.from_mp(ws), dd.DD.from_mp(cs)
