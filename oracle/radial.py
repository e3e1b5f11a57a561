"""Radial derivatives A_n = D^n B_i, D = R^-1 d/dR, by quadrature (oracle).

Test infrastructure only.

Eq. (bfinal): B_i(R) = N' int_0^inf K_i(r) g(r, R) dr with
  N' = sqrt(pi^5/(p+q)) / (p q),  K_i(r) = r k_i(r),
  g(r, R) = [exp(-xi (r-R)^2) - exp(-xi (r+R)^2)] / R,  xi = p q / (p+q).
Only g depends on R, so A_n = N' int_0^inf K_i(r) D^n g(r, R) dr, where
D^n g is evaluated pointwise in one of two exact forms:

  * split form (T = xi R^2 >= 1): D^n g = h^-_{1,n} - h^+_{1,n} with
    h^s_{k,l} = D^l [exp(-xi (r + s R)^2) / R^k]; applying D to the l = 0
    function gives the pointwise relation that the paper integrates into
    Eq. (finalrec):
      h^s_{k,l} = -2 s xi r h^s_{k+1,l-1} - 2 xi h^s_{k,l-1} - k h^s_{k+2,l-1}.
  * Bessel form (T < 1, including R = 0, where the split form cancels):
    g = 4 xi r exp(-xi (r^2 + R^2)) i_0(z), z = 2 xi r R (Eq. (qterm) with
    the factor 2 of the sinh identity restored), and
      D^n[e^{-xi R^2} i_0(cR)] = sum_j C(n,j) (-2 xi)^(n-j) c^(2j)
                                  e^{-xi R^2} i_j(z) / z^j,
    i_j(z)/z^j = sum_k (z^2/2)^k / (k! (2j+2k+1)!!)  (positive series).

The integral over r uses a tanh-sinh panel [0, a1] (it absorbs the r^rho
endpoint behaviour and the narrow exp(-xi (r+R)^2) peak) and Gauss-Legendre
panels over the region where the Gaussian bump and the kernel overlap.
Everything is double-double; the pointwise sums cancel by up to
(2T)^(n/2) and DD keeps about 32 digits.
"""
import math
import numpy as np
from . import dd
from .quadrature import gauss_legendre, tanh_sinh
from .factor import TermFactor, gaussian_rates, growth_rate, kernel_times_r, term_peaks

N_PEAK = 8  # Gauss-Legendre panels across each peak of the integrand


def _interior_edges(xi, R, lo, hi, c, w, b, mus, peaks=()):
    """Panel edges inside [lo, hi] (arrays over quartets, shape (P, M)).

    The integrand has up to two kinds of peaks: the pair Gaussian shifted by
    the kernel's growth, centred at c with width w = xi^-1/2 (14 widths each
    side), and, for each Gaussian rate mu of the kernel, the product of two
    Gaussians centred at r* = xi R / (mu + xi) (up to b / (2 (mu + xi)) further
    out for terms that also grow) with width (mu + xi)^-1/2 (12 widths each
    side).  Each peak gets N_PEAK panels of its own: a kernel much narrower
    than the pair Gaussian (mu >> xi) puts all its weight in a region far
    smaller than R, which a subdivision of [lo, hi] into equal panels would
    resolve poorly.  For a factor given by its terms, each term's
    exp(bt r - gt r^2) times the pair Gaussian peaks at
    (2 xi R + bt) / (2 (xi + gt)) with width (xi + gt)^-1/2 and gets panels
    as well (this places decaying terms, bt < 0, whose peak lies below R or
    at r = 0).  Edges are clipped to [lo, hi] and sorted; the gaps between
    peaks are single panels (the integrand there is below exp(-144) of its
    peaks)."""
    cand = [lo + 0.0 * xi, hi + 0.0 * xi]
    for k in range(N_PEAK + 1):
        cand.append(c - 14.0 * w + 28.0 * w * k / N_PEAK)
    for mu in mus:
        if mu > 0:
            sig = 1.0 / np.sqrt(mu + xi)
            rstar = xi * R / (mu + xi)
            a = rstar - 12.0 * sig
            e = rstar + b / (2.0 * (mu + xi)) + 12.0 * sig
            for k in range(N_PEAK + 1):
                cand.append(a + (e - a) * k / N_PEAK)
    for (bt, gt) in peaks:
        sig = 1.0 / np.sqrt(xi + gt)
        ctr = (2.0 * xi * R + bt) / (2.0 * (xi + gt))
        for k in range(N_PEAK + 1):
            cand.append(ctr - 14.0 * sig + 28.0 * sig * k / N_PEAK)
    E = np.stack(cand, axis=1)
    E = np.clip(E, lo[:, None], hi[:, None])
    E.sort(axis=1)
    return E


def _nodes(xi, R, cls, fac, facp):
    """Per-primitive-quartet quadrature nodes r and weights w (DD arrays)."""
    xi = np.asarray(xi, float)
    R = np.asarray(R, float)
    w = 1.0 / np.sqrt(xi)
    b = growth_rate(cls, fac, facp)
    mus = gaussian_rates(cls, fac, facp)
    c = R + b / (2.0 * xi)
    a1 = 0.5 * np.minimum(w, 1.0)
    hi = c + 14.0 * w
    lo = c - 14.0 * w
    for mu in mus:
        if mu > 0:
            rstar = xi * R / (mu + xi)
            lo = np.minimum(lo, rstar - 12.0 / np.sqrt(mu + xi))
    peaks = term_peaks(cls, fac, facp)
    for (bt, gt) in peaks:
        lo = np.minimum(lo, (2.0 * xi * R + bt) / (2.0 * (xi + gt)) - 14.0 / np.sqrt(xi + gt))
    lo = np.maximum(lo, a1)
    xg, wg = gauss_legendre(48)
    xt, wt, ct = tanh_sinh()
    parts_r, parts_w = [], []
    # tanh-sinh panel [0, a1]
    A1 = dd.DD(a1)[:, None]
    parts_r.append(A1 * dd.DD(xt.hi[None, :], xt.lo[None, :]))
    parts_w.append(A1 * dd.DD(wt.hi[None, :], wt.lo[None, :]))
    # gap panel [a1, lo] (usually negligible, kept for safety)
    def gl_panel(x0, x1):
        X0 = dd.DD(x0)[:, None]
        half = (dd.DD(x1) - dd.DD(x0)) * 0.5
        half = half[:, None]
        mid = X0 + half
        rr = mid + half * dd.DD(xg.hi[None, :], xg.lo[None, :])
        ww = half * dd.DD(wg.hi[None, :], wg.lo[None, :])
        return rr, ww
    rr, ww = gl_panel(a1, lo)
    parts_r.append(rr)
    parts_w.append(ww)
    E = _interior_edges(xi, R, lo, hi, c, w, b, mus, peaks)
    for k in range(E.shape[1] - 1):
        rr, ww = gl_panel(E[:, k], E[:, k + 1])
        parts_r.append(rr)
        parts_w.append(ww)
    r = dd.DD(np.concatenate([p.hi for p in parts_r], 1), np.concatenate([p.lo for p in parts_r], 1))
    wts = dd.DD(np.concatenate([p.hi for p in parts_w], 1), np.concatenate([p.lo for p in parts_w], 1))
    return r, wts


def _dn_split(xi, R, r, nmax):
    """D^n g, n = 0..nmax, split form.  xi, R: (P,1) DD; r: (P,N) DD."""
    out = []
    res = {}
    for s in (+1, -1):
        d = r + R * float(s)
        E = dd.exp(-(xi * d * d))
        invR = 1.0 / R
        kmax = 2 * nmax + 1
        h = [None] * (kmax + 2)
        p = E * invR
        for k in range(1, kmax + 1):
            h[k] = p
            p = p * invR
        levels = [h[1]]
        cur = h
        for l in range(1, nmax + 1):
            nxt = [None] * (kmax + 2)
            for k in range(1, 2 * (nmax - l) + 2):
                v = (-2.0 * s) * xi * r * cur[k + 1] - 2.0 * xi * cur[k] - float(k) * cur[k + 2]
                nxt[k] = v
            levels.append(nxt[1])
            cur = nxt
        res[s] = levels
    for n in range(nmax + 1):
        out.append(res[-1][n] - res[+1][n])
    return out


def _dn_bessel(xi, R, r, nmax):
    """D^n g, n = 0..nmax, Bessel form (valid for any R >= 0)."""
    z = 2.0 * xi * r * R
    y = z * z * 0.5
    # iota_j(z) = i_j(z)/z^j by its power series for j = nmax, nmax+1, then
    # the downward recurrence iota_{j-1} = (2j+1) iota_j + z^2 iota_{j+1}
    # (from i_{j-1} - i_{j+1} = (2j+1) i_j / z; all terms positive).
    ymax = float(np.max(y.hi)) if y.hi.size else 0.0
    nterms = 0
    tk, tmax_ = 1.0, 1.0
    while nterms < 600:
        nterms += 1
        tk = tk * ymax / (nterms * (2 * nterms + 1))
        tmax_ = max(tmax_, tk)
        if tk < 1e-36 * tmax_ and nterms > 10:
            break
    def series(j):
        term = dd.ones(r.shape)
        for m in range(3, 2 * j + 2, 2):
            term = term / float(m)  # 1/(2j+1)!! exactly in DD
        acc = term
        for k in range(1, nterms + 1):
            term = term * y / (float(k) * float(2 * j + 2 * k + 1))
            acc = acc + term
        return acc
    iota = [None] * (nmax + 2)
    iota[nmax + 1] = series(nmax + 1)
    iota[nmax] = series(nmax)
    z2 = z * z
    for j in range(nmax, 0, -1):
        iota[j - 1] = float(2 * j + 1) * iota[j] + z2 * iota[j + 1]
    pre = 4.0 * xi * r * dd.exp(-(xi * (r * r + R * R)))
    c2 = (2.0 * xi * r) * (2.0 * xi * r)
    out = []
    for n in range(nmax + 1):
        s = dd.zeros(r.shape)
        c2j = dd.ones(r.shape)
        for j in range(n + 1):
            coef = float(math.comb(n, j))
            s = s + coef * dd.ipow(-2.0 * xi, n - j) * c2j * iota[j]
            c2j = c2j * c2
        out.append(pre * s)
    return out


def _dfact(m):
    v = 1
    while m > 1:
        v *= m
        m -= 2
    return v


def radial_derivatives(cls, xi, R, nmax, fac, facp, chunk=256):
    """A_n / N' = int_0^inf K_i(r) D^n g(r, R) dr for n = 0..nmax.

    xi, R: 1-D float arrays (one entry per primitive quartet).
    Returns a DD array of shape (P, nmax+1).
    """
    xi = np.atleast_1d(np.asarray(xi, float))
    R = np.atleast_1d(np.asarray(R, float))
    P = xi.shape[0]
    hi = np.zeros((P, nmax + 1))
    lo = np.zeros((P, nmax + 1))
    for s0 in range(0, P, chunk):
        sl = slice(s0, min(P, s0 + chunk))
        xs, Rs = xi[sl], R[sl]
        T = xs * Rs * Rs
        for use_split in (False, True):
            m = (T >= 1.0) if use_split else (T < 1.0)
            if not np.any(m):
                continue
            xm, Rm = xs[m], Rs[m]
            r, w = _nodes(xm, Rm, cls, fac, facp)
            K = kernel_times_r(cls, fac, facp, r)
            XI = dd.DD(xm)[:, None]
            RR = dd.DD(Rm)[:, None]
            ders = (_dn_split if use_split else _dn_bessel)(XI, RR, r, nmax)
            KW = K * w
            idx = np.nonzero(m)[0] + s0
            for n in range(nmax + 1):
                v = dd.dsum(KW * ders[n], axis=1)
                hi[idx, n] = v.hi
                lo[idx, n] = v.lo
    return dd.DD(hi, lo)


def n_prime(p, q):
    """N' = sqrt(pi^5/(p+q)) / (p q) in DD (Eq. (bfinal))."""
    import mpmath as mp
    with mp.workdps(40):
        pi52 = dd.DD.from_mp(mp.pi ** mp.mpf(2.5))
    p = dd.DD(p)
    q = dd.DD(q)
    return pi52 / (dd.sqrt(p + q) * p * q)


# ---------------------------------------------------------------------------
# Arbitrary-precision path for quartets whose pointwise cancellation
# (2T)^n / (2n-1)!! exceeds what DD can absorb.  Same formulas (split form of
# D^n g, same panels), evaluated with mpmath at a precision chosen from the
# cancellation estimate.
# ---------------------------------------------------------------------------

def cancellation_digits(T, n):
    """log10 of the pointwise cancellation (2T)^n/(2n-1)!! of the split form."""
    if T < 1.0 or n == 0:
        return 0.0
    return n * math.log10(2.0 * T) - math.log10(_dfact(2 * n - 1))


def _kernel_mp(cls, fac, facp, r):
    import mpmath as mp

    def S(n, x):
        if x < 2:
            t = mp.mpf(1)
            for k in range(1, n + 1):
                t = t * x / k
            tail = mp.mpf(0)
            for k in range(n + 1, n + 200):
                t = t * x / k
                tail += t
                if abs(t) < abs(tail) * mp.mpf(10) ** (-mp.mp.dps - 5):
                    break
            return mp.exp(-x) * tail
        head, t = mp.mpf(1), mp.mpf(1)
        for k in range(1, n + 1):
            t = t * x / k
            head += t
        return 1 - mp.exp(-x) * head

    def terms(fc, deriv):
        v = mp.mpf(0)
        for (c, a, b, g) in fc.terms:
            e = mp.power(r, a) * mp.exp(b * r - g * r * r)
            v += c * (e * (a / r + b - 2 * g * r) if deriv else e)
        return v

    def f(fc):
        if isinstance(fc, TermFactor):
            return terms(fc, False)
        g = mp.exp(-fc.mu * r * r)
        v = (1 + r / 2) * g
        if fc.c0 != 0:
            v += S(fc.n, fc.mu * r * r) * fc.c0 * mp.power(r, fc.rho) * mp.exp(fc.B * r)
        return v

    def fr(fc):
        if isinstance(fc, TermFactor):
            return terms(fc, True)
        mr2 = fc.mu * r * r
        g = mp.exp(-mr2)
        v = (mp.mpf(1) / 2 - 2 * fc.mu * r - fc.mu * r * r) * g
        if fc.c0 != 0:
            lr = mp.power(r, fc.rho) * mp.exp(fc.B * r)
            dS = 2 * fc.mu * r * g * mr2 ** fc.n / mp.factorial(fc.n)
            v += fc.c0 * lr * (dS + S(fc.n, mr2) * (fc.rho / r + fc.B))
        return v

    if cls == 1:
        return mp.mpf(1)
    if cls == 2:
        return f(fac)
    if cls == 3:
        return r * f(fac)
    if cls == 4:
        return r * f(fac) * f(facp)
    if cls == 6:
        return r * fr(fac) * fr(facp)
    raise ValueError(cls)


def radial_derivatives_mp(cls, xi, R, nmax, fac, facp, extra_digits=None):
    """Same quantity as radial_derivatives for one (xi, R), T >= 1, in mpmath.

    Returns a list of mpf values A_n / N', n = 0..nmax.
    """
    import mpmath as mp
    T = xi * R * R
    dig = cancellation_digits(T, nmax)
    dps = int(36 + dig) if extra_digits is None else int(36 + extra_digits)
    with mp.workdps(dps):
        xi_m, R_m = mp.mpf(xi), mp.mpf(R)
        w = 1 / mp.sqrt(xi_m)
        b = growth_rate(cls, fac, facp)
        c = R_m + mp.mpf(b) / (2 * xi_m)
        a1 = min(w, mp.mpf(1)) / 2
        hi = c + 14 * w
        lo = c - 14 * w
        mus = gaussian_rates(cls, fac, facp)
        for mu in mus:
            if mu > 0:
                rstar = xi_m * R_m / (mu + xi_m)
                lo = min(lo, rstar - 12 / mp.sqrt(mu + xi_m))
        peaks = term_peaks(cls, fac, facp)
        for (bt, gt) in peaks:
            lo = min(lo, (2 * xi_m * R_m + bt) / (2 * (xi_m + gt)) - 14 / mp.sqrt(xi_m + gt))
        lo = max(lo, a1)
        gl = mp.calculus.quadrature.GaussLegendre(mp.mp)
        ts = mp.calculus.quadrature.TanhSinh(mp.mp)
        prec = mp.mp.prec
        degree = 6 if dig < 40 else 7
        gnodes = gl.get_nodes(-1, 1, degree, prec)
        # mpmath keeps each tanh-sinh level's new abscissas apart (level k
        # adds the odd multiples of 2^-k); the full rule of step h = 2^-D is
        # their union with every weight times h
        tlev = degree + 1
        tnodes = []
        for k in range(1, tlev + 1):
            tnodes += ts.get_nodes(-1, 1, k, prec)
        hstep = mp.mpf(2) ** (-tlev)
        tnodes = [(x, w * hstep) for (x, w) in tnodes]
        pts = [(mp.mpf(0), a1, tnodes), (a1, lo, gnodes)]
        # interior edges from the binary64 placement; the ends stay exact
        Ef = _interior_edges(np.array([float(xi_m)]), np.array([float(R_m)]), np.array([float(lo)]),
                             np.array([float(hi)]), np.array([float(c)]), np.array([float(w)]), float(b),
                             mus, peaks)[0]
        edges = [lo] + [mp.mpf(float(v)) for v in Ef[1:-1]] + [hi]
        edges = [min(max(v, lo), hi) for v in edges]
        pts += [(edges[k], edges[k + 1], gnodes) for k in range(len(edges) - 1)]
        acc = [mp.mpf(0)] * (nmax + 1)
        kmax = 2 * nmax + 1
        for (x0, x1, nodes) in pts:
            if x1 <= x0:
                continue
            half = (x1 - x0) / 2
            for (x, wq) in nodes:
                r = x0 + half * (x + 1)
                if r <= 0:
                    continue
                Kr = _kernel_mp(cls, fac, facp, r)
                ders = []
                res = {}
                for s in (1, -1):
                    E = mp.exp(-xi_m * (r + s * R_m) ** 2)
                    cur = [None] * (kmax + 3)
                    p = E / R_m
                    for k in range(1, kmax + 1):
                        cur[k] = p
                        p = p / R_m
                    lev = [cur[1]]
                    for l in range(1, nmax + 1):
                        nxt = [None] * (kmax + 3)
                        for k in range(1, 2 * (nmax - l) + 2):
                            nxt[k] = -2 * s * xi_m * r * cur[k + 1] - 2 * xi_m * cur[k] - k * cur[k + 2]
                        lev.append(nxt[1])
                        cur = nxt
                    res[s] = lev
                f = Kr * wq * half
                for n in range(nmax + 1):
                    acc[n] += f * (res[-1][n] - res[1][n])
        return [+a for a in acc]


def radial_auto(cls, xi, R, nmax, fac, facp, dd_digits=13.0):
    """A_n/N' for arrays (xi, R): DD where the cancellation fits, mpmath elsewhere.

    Returns (hi, lo) float arrays of shape (P, nmax+1) holding a DD value.
    """
    import mpmath as mp
    xi = np.atleast_1d(np.asarray(xi, float))
    R = np.atleast_1d(np.asarray(R, float))
    T = xi * R * R
    dig = np.array([cancellation_digits(t, nmax) for t in T])
    use_mp = dig > dd_digits
    out = dd.zeros((xi.shape[0], nmax + 1))
    if np.any(~use_mp):
        v = radial_derivatives(cls, xi[~use_mp], R[~use_mp], nmax, fac, facp)
        out.hi[~use_mp] = v.hi
        out.lo[~use_mp] = v.lo
    for i in np.nonzero(use_mp)[0]:
        vals = radial_derivatives_mp(cls, float(xi[i]), float(R[i]), nmax, fac, facp)
        d = dd.DD.from_mp(vals)
        out.hi[i] = d.hi
        out.lo[i] = d.lo
    return out
