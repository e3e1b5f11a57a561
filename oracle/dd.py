"""Vectorised double-double ("DD") arithmetic on numpy arrays.

Test infrastructure only: part of the CPU oracle.

A DD number is an unevaluated sum hi + lo of two IEEE doubles with
|lo| <= ulp(hi)/2, giving about 32 significant decimal digits.  The oracle
evaluates the radial derivatives of the basic integrals and the Hermite
recurrences in DD because those quantities are computed from sums whose
terms are many orders of magnitude larger than the result (the cancellation
grows like (2T)^(n/2) with T = xi*R^2); in plain binary64 they would lose
most of their digits.

Algorithms: Dekker's splitting and Knuth's two-sum (error-free transforms),
the standard DD add / mul / div of Bailey's QD library (re-derived here from
the error-free transforms), and Taylor series with argument reduction for
exp and Newton iteration for log and sqrt.
"""
import numpy as np

_SPLIT = 134217729.0  # 2^27 + 1


def _two_sum(a, b):
    s = a + b
    bb = s - a
    err = (a - (s - bb)) + (b - bb)
    return s, err


def _quick_two_sum(a, b):
    s = a + b
    err = b - (s - a)
    return s, err


def _split(a):
    t = _SPLIT * a
    hi = t - (t - a)
    lo = a - hi
    return hi, lo


def _two_prod(a, b):
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    err = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, err


class DD:
    """Array of double-double numbers (hi, lo), broadcasting like numpy."""

    __slots__ = ("hi", "lo")
    __array_priority__ = 1000

    def __init__(self, hi, lo=None):
        if isinstance(hi, DD):
            self.hi, self.lo = hi.hi, hi.lo
            return
        self.hi = np.asarray(hi, dtype=np.float64)
        if lo is None:
            self.lo = np.zeros_like(self.hi)
        else:
            self.lo = np.asarray(lo, dtype=np.float64)

    # ---- construction helpers -------------------------------------------
    @staticmethod
    def from_mp(values):
        """Exact-to-DD rounding of mpmath numbers (or a nested list of them)."""
        import mpmath as mp
        arr = np.asarray(values, dtype=object)
        hi = np.empty(arr.shape)
        lo = np.empty(arr.shape)
        with mp.workprec(max(mp.mp.prec, 240)):
            for idx, v in np.ndenumerate(arr):
                h = float(v)
                hi[idx] = h
                lo[idx] = float(mp.mpf(v) - mp.mpf(h))
        return DD(hi, lo)

    def to_mp(self):
        import mpmath as mp
        out = np.empty(self.hi.shape, dtype=object)
        with mp.workprec(120):
            for idx in np.ndindex(self.hi.shape):
                out[idx] = mp.mpf(float(self.hi[idx])) + mp.mpf(float(self.lo[idx]))
        return out

    def __float__(self):
        return float(self.hi + self.lo)

    def to_float(self):
        return self.hi + self.lo

    @property
    def shape(self):
        return self.hi.shape

    def __getitem__(self, k):
        return DD(self.hi[k], self.lo[k])

    def __setitem__(self, k, v):
        v = _dd(v)
        self.hi[k] = v.hi
        self.lo[k] = v.lo

    def copy(self):
        return DD(self.hi.copy(), self.lo.copy())

    def __repr__(self):
        return f"DD(hi={self.hi!r}, lo={self.lo!r})"

    # ---- arithmetic -----------------------------------------------------
    def __neg__(self):
        return DD(-self.hi, -self.lo)

    def __add__(self, o):
        o = _dd(o)
        s, e = _two_sum(self.hi, o.hi)
        t, f = _two_sum(self.lo, o.lo)
        e = e + t
        s, e = _quick_two_sum(s, e)
        e = e + f
        s, e = _quick_two_sum(s, e)
        return DD(s, e)

    __radd__ = __add__

    def __sub__(self, o):
        return self + (-_dd(o))

    def __rsub__(self, o):
        return _dd(o) + (-self)

    def __mul__(self, o):
        o = _dd(o)
        p, e = _two_prod(self.hi, o.hi)
        e = e + (self.hi * o.lo + self.lo * o.hi)
        p, e = _quick_two_sum(p, e)
        return DD(p, e)

    __rmul__ = __mul__

    def __truediv__(self, o):
        if not isinstance(o, DD):
            d = np.asarray(o, dtype=np.float64)
            q1 = self.hi / d
            p, e = _two_prod(q1, d)
            s, f = _two_sum(self.hi, -p)
            f = f - e + self.lo
            q2 = (s + f) / d
            q1, q2 = _quick_two_sum(q1, q2)
            return DD(q1, q2)
        o = _dd(o)
        q1 = self.hi / o.hi
        r = self - o * q1
        q2 = r.hi / o.hi
        r = r - o * q2
        q3 = r.hi / o.hi
        q1, q2 = _quick_two_sum(q1, q2)
        return DD(q1, q2) + q3

    def __rtruediv__(self, o):
        return _dd(o) / self

    def __pow__(self, k):
        if isinstance(k, (int, np.integer)):
            return ipow(self, int(k))
        return dd_pow(self, k)

    # comparisons on the leading part are enough for branch selection
    def __lt__(self, o):
        o = _dd(o)
        return (self.hi < o.hi) | ((self.hi == o.hi) & (self.lo < o.lo))

    def __gt__(self, o):
        return _dd(o) < self

    def abs(self):
        neg = (self.hi < 0) | ((self.hi == 0) & (self.lo < 0))
        return DD(np.where(neg, -self.hi, self.hi), np.where(neg, -self.lo, self.lo))


def _dd(x):
    if isinstance(x, DD):
        return x
    return DD(x)


def where(cond, a, b):
    a, b = _dd(a), _dd(b)
    return DD(np.where(cond, a.hi, b.hi), np.where(cond, a.lo, b.lo))


def ipow(x, k):
    x = _dd(x)
    if k < 0:
        return 1.0 / ipow(x, -k)
    result = DD(np.ones_like(x.hi))
    base = x
    while k:
        if k & 1:
            result = result * base
        base = base * base
        k >>= 1
    return result


def sqrt(x):
    x = _dd(x)
    with np.errstate(invalid="ignore", divide="ignore"):
        y = np.sqrt(x.hi)
        safe = np.where(y > 0, y, 1.0)
        # one Newton step in DD: y + (x - y^2) / (2y)
        yy = DD(y)
        r = (x - yy * yy) / (2.0 * DD(safe))
        out = yy + r
    return where(y > 0, out, DD(np.zeros_like(y)))


_LN2 = None


def _ln2():
    global _LN2
    if _LN2 is None:
        import mpmath as mp
        with mp.workdps(40):
            _LN2 = DD.from_mp(mp.log(2))
    return _LN2


def exp(x):
    """DD exponential: x = k ln2 + r, r -> r / 2^8, Taylor, square back."""
    x = _dd(x)
    ln2 = _ln2()
    k = np.round(x.hi / ln2.hi)
    r = x - ln2 * k
    r = r * (1.0 / 256.0)
    # Taylor series of exp(r) - 1 with |r| < 0.0014: 12 terms give < 1e-40
    term = DD(np.ones_like(r.hi))
    s = DD(np.zeros_like(r.hi))
    for i in range(1, 14):
        term = (term * r) / float(i)
        s = s + term
    # (1 + s)^(256) computed as repeated squaring of (1 + s) keeping s small
    for _ in range(8):
        s = s * s + 2.0 * s
    e = s + 1.0
    with np.errstate(over="ignore", under="ignore", invalid="ignore"):
        scale = np.ldexp(1.0, np.clip(k, -1070, 1020).astype(np.int64))
        out = DD(e.hi * scale, e.lo * scale)
    underflow = x.hi < -740.0
    return where(underflow, DD(np.zeros_like(x.hi)), out)


def log(x):
    """DD natural log by two Newton steps on exp(y) = x."""
    x = _dd(x)
    with np.errstate(divide="ignore", invalid="ignore"):
        y = DD(np.log(x.hi))
        for _ in range(2):
            y = y + x * exp(-y) - 1.0
    return y


def dd_pow(x, p):
    """x**p for DD x > 0 and a binary64 exponent p (taken as exact)."""
    x = _dd(x)
    if float(p) == int(p) and abs(p) < 64:
        return ipow(x, int(p))
    return exp(log(x) * float(p))


def zeros(shape):
    return DD(np.zeros(shape), np.zeros(shape))


def ones(shape):
    return DD(np.ones(shape), np.zeros(shape))


def stack(items, axis=0):
    items = [_dd(i) for i in items]
    return DD(np.stack([i.hi for i in items], axis), np.stack([i.lo for i in items], axis))


def dsum(x, axis):
    """Sum along an axis by pairwise DD additions."""
    x = _dd(x)
    hi = np.moveaxis(x.hi, axis, 0)
    lo = np.moveaxis(x.lo, axis, 0)
    cur = DD(hi, lo)
    while cur.hi.shape[0] > 1:
        m = cur.hi.shape[0]
        h = m // 2
        s = DD(cur.hi[:h], cur.lo[:h]) + DD(cur.hi[h:2 * h], cur.lo[h:2 * h])
        if m % 2:
            s = DD(np.concatenate([s.hi, cur.hi[2 * h:]]), np.concatenate([s.lo, cur.lo[2 * h:]]))
        cur = s
    return DD(cur.hi[0], cur.lo[0])
