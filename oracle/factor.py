"""The range-separated correlation factor and the kernels k_i (oracle).

Test infrastructure only.

Eq. (rs12):  f(r) = (1 + r/2) exp(-mu r^2) + S_n(mu r^2) c0 r^rho exp(B r)
Eq. (ttdamp): S_n(x) = 1 - exp(-x) sum_{k<=n} x^k / k!
Kernels, Eqs. (k1)-(k6): k1 = 1/r, k2 = f/r, k3 = f, k4 = f f', k6 = f_r f'_r
where f_r = df/dr (Eq. (I6_) and the double-commutator identity above it).

Everything is evaluated pointwise in double-double on arrays of r > 0.
The oracle integrates K_i(r) = r k_i(r), the combination that appears in
the one-dimensional representation Eq. (bfinal).
"""
from dataclasses import dataclass
import math
import numpy as np
from . import dd


@dataclass(frozen=True)
class Factor:
    """Parameters (c0, rho, B, mu, n) of Eq. (rs12)/(ttdamp)."""
    c0: float
    rho: float
    B: float
    mu: float
    n: int = 0


@dataclass(frozen=True)
class TermFactor:
    """A factor given by its terms, f(r) = sum_t c_t r^alpha_t exp(b_t r - g_t r^2):
    the same family of functions that Eq. (rs12) expands into, for other
    correlation factors (Gaussian geminals, their products with powers of r).
    terms: tuple of (c, alpha, b, g)."""
    terms: tuple


def tang_toennies(n, x):
    """S_n(x) of Eq. (ttdamp) in DD for DD x >= 0.

    For x < 2 the tail form exp(-x) sum_{k>n} x^k/k! avoids the cancellation
    of 1 - exp(-x)(...) (the two expressions are identical).
    """
    x = dd.DD(x)
    ex = dd.exp(-x)
    # head: sum_{k<=n} x^k/k!
    term = dd.ones(x.shape)
    head = dd.ones(x.shape)
    for k in range(1, n + 1):
        term = term * x / float(k)
        head = head + term
    big = 1.0 - ex * head
    small_mask = x.hi < 0.5
    if not np.any(small_mask):
        return big
    # tail: sum_{k>n} x^k/k!, 28 terms give < 1e-34 relative for x < 0.5
    xs = dd.where(small_mask, x, 0.0)
    t = dd.ones(x.shape)
    for k in range(1, n + 1):
        t = t * xs / float(k)
    tail = dd.zeros(x.shape)
    for k in range(n + 1, n + 29):
        t = t * xs / float(k)
        tail = tail + t
    small = ex * tail
    return dd.where(small_mask, small, big)


def _terms_value(fac, r, deriv):
    """sum_t c_t r^alpha_t e^{b_t r - g_t r^2} (or its r-derivative) in DD."""
    out = dd.zeros(r.shape)
    lr = dd.log(r)
    for (c, a, b, g) in fac.terms:
        e = dd.exp(lr * float(a) + r * float(b) - r * r * float(g))
        if deriv:
            e = e * (float(a) / r + float(b) - 2.0 * float(g) * r)
        out = out + e * float(c)
    return out


def f_value(fac, r):
    """f(r) of Eq. (rs12) in DD (or of a TermFactor)."""
    r = dd.DD(r)
    if isinstance(fac, TermFactor):
        return _terms_value(fac, r, False)
    mr2 = fac.mu * r * r
    g = dd.exp(-mr2)
    short = (1.0 + 0.5 * r) * g
    if fac.c0 == 0.0:
        return short
    lr = dd.exp(dd.log(r) * fac.rho + r * fac.B)
    return short + tang_toennies(fac.n, mr2) * lr * fac.c0


def f_deriv(fac, r):
    """df/dr of Eq. (rs12) in DD.

    d/dr[(1 + r/2) e^{-mu r^2}] = (1/2 - 2 mu r - mu r^2) e^{-mu r^2};
    dS_n(x)/dx = e^{-x} x^n / n!, so d/dr S_n(mu r^2) = 2 mu r e^{-mu r^2}
    (mu r^2)^n / n!; and d/dr[r^rho e^{B r}] = (rho/r + B) r^rho e^{B r}.
    """
    r = dd.DD(r)
    if isinstance(fac, TermFactor):
        return _terms_value(fac, r, True)
    mr2 = fac.mu * r * r
    g = dd.exp(-mr2)
    short = (0.5 - 2.0 * fac.mu * r - fac.mu * r * r) * g
    if fac.c0 == 0.0:
        return short
    lr = dd.exp(dd.log(r) * fac.rho + r * fac.B)
    dS = 2.0 * fac.mu * r * g * dd.ipow(mr2, fac.n) / float(math.factorial(fac.n))
    S = tang_toennies(fac.n, mr2)
    return short + fac.c0 * lr * (dS + S * (fac.rho / r + fac.B))


def kernel_times_r(cls, fac, facp, r):
    """K_i(r) = r k_i(r) for class i in {1,2,3,4,6} (DD)."""
    r = dd.DD(r)
    if cls == 1:
        return dd.ones(r.shape)
    if cls == 2:
        return f_value(fac, r)
    if cls == 3:
        return r * f_value(fac, r)
    if cls == 4:
        return r * f_value(fac, r) * f_value(facp, r)
    if cls == 6:
        return r * f_deriv(fac, r) * f_deriv(facp, r)
    raise ValueError(f"class {cls} has no kernel of its own (I5 is built from I3)")


def _growth(fac):
    if isinstance(fac, TermFactor):
        return max([0.0] + [float(b) for (c, a, b, g) in fac.terms if g == 0 and b > 0])
    return max(fac.B, 0.0) if fac.c0 != 0 else 0.0


def gaussian_rates(cls, fac, facp):
    """Gaussian exponents mu of the kernel's geminal parts (used to place
    quadrature panels around their peaks)."""
    def rates(f):
        if isinstance(f, TermFactor):
            return sorted({float(g) for (c, a, b, g) in f.terms if g > 0})
        return [f.mu]
    if cls in (2, 3):
        return rates(fac)
    if cls in (4, 6):
        r1, r2 = rates(fac), rates(facp)
        return sorted({a + b for a in r1 for b in r2} | set(r1) | set(r2))
    return [0.0]


def term_peaks(cls, fac, facp):
    """(b, g) of the kernel's exponential factors e^{b r - g r^2} for factors
    given by their terms (used to place quadrature panels around the peak of
    each term's product with the pair Gaussian); [] for Eq. (rs12) factors."""
    def bg(f):
        return sorted({(float(b), float(g)) for (c, a, b, g) in f.terms})
    if not isinstance(fac, TermFactor) and not isinstance(facp, TermFactor):
        return []
    if cls in (2, 3, 5):
        return bg(fac) if isinstance(fac, TermFactor) else []
    if cls in (4, 6) and isinstance(fac, TermFactor) and isinstance(facp, TermFactor):
        return sorted({(b1 + b2, g1 + g2) for (b1, g1) in bg(fac) for (b2, g2) in bg(facp)})
    return []


def growth_rate(cls, fac, facp):
    """Largest exponential growth rate b of K_i (used to place quadrature panels)."""
    if isinstance(fac, TermFactor) or isinstance(facp, TermFactor):
        if cls in (2, 3):
            return _growth(fac)
        if cls in (4, 6):
            return _growth(fac) + _growth(facp)
        return 0.0
    b = 0.0
    if cls in (2, 3):
        b = max(fac.B, 0.0) if fac.c0 != 0 else 0.0
    elif cls in (4, 6):
        b1 = max(fac.B, 0.0) if fac.c0 != 0 else 0.0
        b2 = max(facp.B, 0.0) if facp.c0 != 0 else 0.0
        b = b1 + b2
    return b
