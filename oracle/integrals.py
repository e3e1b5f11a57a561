"""Contracted F12 integrals (ab|k_i|cd), i = 1..6, over Cartesian shells (oracle).

Test infrastructure only.

Shells are dicts {"center": (3,), "l": int, "exps": (K,), "coefs": (K,)}.
Primitive functions are unnormalised, Eq. (basis): x_A^i y_A^k z_A^m
exp(-a r_A^2); contraction coefficients are used as given.  Cartesian
components of angular momentum l are ordered (i, k, m) with i from l down to
0, then k from l-i down to 0 (the paper does not fix an order).

Classes I1-I4 and I6 follow Eq. (ii):
  I = sum_tuv E^ab_tuv (-1)^(t+u+v) sum_t'u'v' E^cd_t'u'v' R^(t+t',u+u',v+v')
with X = Q - P.  I5 = (ab|[f, T1]|cd) follows Green's identity, Eq. (I5_):
  I5 = 1/2 [ (lap a, b|f|cd) - (a, lap b|f|cd) ],
  lap x^i e^{-a x^2} = [i(i-1) x^(i-2) - 2a(2i+1) x^i + 4a^2 x^(i+2)] e^{-a x^2}
summed over the three directions, i.e. I3 over shells of angular momentum
l-2, l and l+2.
"""
import itertools
import numpy as np
from . import dd
from .hermite import e_coefficients, hermite_r
from .radial import radial_auto, n_prime


def cart(l):
    """Canonical Cartesian components of angular momentum l."""
    out = []
    for i in range(l, -1, -1):
        for k in range(l - i, -1, -1):
            out.append((i, k, l - i - k))
    return out


def _pair_data(sa, sb):
    """Primitive-pair arrays over (Ka, Kb) flattened, plus E per direction."""
    ea = np.asarray(sa["exps"], float)
    eb = np.asarray(sb["exps"], float)
    A = np.asarray(sa["center"], float)
    B = np.asarray(sb["center"], float)
    a = np.repeat(ea, eb.size)
    b = np.tile(eb, ea.size)
    la, lb = sa["l"], sb["l"]
    Es = [e_coefficients(a, b, np.full(a.size, A[k]), np.full(a.size, B[k]), la, lb) for k in range(3)]
    return a, b, Es


def _pair_hermite(Es, la, lb):
    """E^ab[pp, comp_ab, t, u, v] as a dense DD array."""
    L = la + lb
    ca, cb = cart(la), cart(lb)
    P = Es[0].shape[0]
    out = dd.zeros((P, len(ca) * len(cb), L + 1, L + 1, L + 1))
    k = 0
    for (ix, iy, iz) in ca:
        for (jx, jy, jz) in cb:
            ex = Es[0][:, ix, jx, :]
            ey = Es[1][:, iy, jy, :]
            ez = Es[2][:, iz, jz, :]
            for t in range(ix + jx + 1):
                for u in range(iy + jy + 1):
                    exy = ex[:, t] * ey[:, u]
                    for v in range(iz + jz + 1):
                        out[:, k, t, u, v] = exy * ez[:, v]
            k += 1
    return out


def primitive_integrals(cls, sa, sb, sc, sd, fac=None, facp=None):
    """Uncontracted integrals for classes 1,2,3,4,6.

    Returns a DD array (Ka*Kb, Kc*Kd, n_ab, n_cd): bra primitive pairs in
    (a-major, b-minor) order, likewise for the ket.
    """
    la, lb, lc, ld = sa["l"], sb["l"], sc["l"], sd["l"]
    Lab, Lcd = la + lb, lc + ld
    L = Lab + Lcd
    a, b, Eab = _pair_data(sa, sb)
    c, d, Ecd = _pair_data(sc, sd)
    p = a + b
    q = c + d
    A = np.asarray(sa["center"], float)
    B = np.asarray(sb["center"], float)
    C = np.asarray(sc["center"], float)
    D = np.asarray(sd["center"], float)
    nb_, nk_ = p.size, q.size
    # primitive quartets: bra-major
    pp = np.repeat(p, nk_)
    qq = np.tile(q, nb_)
    aa = np.repeat(a, nk_)
    bb = np.repeat(b, nk_)
    cc = np.tile(c, nb_)
    dq = np.tile(d, nb_)
    # P and Q in DD, X = Q - P
    def centre(x, y, X, Y, k):
        x = dd.DD(x)
        y = dd.DD(y)
        return (x * float(X[k]) + y * float(Y[k])) / (x + y)
    Xc = [centre(cc, dq, C, D, k) - centre(aa, bb, A, B, k) for k in range(3)]
    R2 = Xc[0] * Xc[0] + Xc[1] * Xc[1] + Xc[2] * Xc[2]
    Rlen = dd.sqrt(R2)
    xi = dd.DD(pp) * dd.DD(qq) / (dd.DD(pp) + dd.DD(qq))
    # radial derivatives in DD; the quadrature takes (xi, R) rounded to binary64
    # only to place its panels and nodes: the integrand uses the DD values.
    An = _radial(cls, xi, Rlen, L, fac, facp)
    An = An * n_prime(pp, qq)[:, None]
    Rc = hermite_r(An, Xc[0], Xc[1], Xc[2], L)
    Hab = _pair_hermite(Eab, la, lb)  # (nb_, nab, Lab+1,...)
    Hcd = _pair_hermite(Ecd, lc, ld)
    nab = Hab.shape[1]
    ncd = Hcd.shape[1]
    Pq = nb_ * nk_
    # expand pair arrays to quartets
    Hab_q = dd.DD(np.repeat(Hab.hi, nk_, 0), np.repeat(Hab.lo, nk_, 0))
    Hcd_q = dd.DD(np.tile(Hcd.hi, (nb_, 1, 1, 1, 1)), np.tile(Hcd.lo, (nb_, 1, 1, 1, 1)))
    # ket transform W[q, cd, t, u, v] = sum_{t'u'v'} Ecd[q, cd, t',u',v'] R[q, t+t', u+u', v+v']
    W = dd.zeros((Pq, ncd, Lab + 1, Lab + 1, Lab + 1))
    for tp in range(Lcd + 1):
        for up in range(Lcd + 1 - tp):
            for vp in range(Lcd + 1 - tp - up):
                e = Hcd_q[:, :, tp, up, vp]
                if not np.any(e.hi):
                    continue
                r = Rc[:, tp:tp + Lab + 1, up:up + Lab + 1, vp:vp + Lab + 1]
                W = W + e[:, :, None, None, None] * r[:, None, :, :, :]
    # bra transform I[q, ab, cd] = sum_tuv (-1)^(t+u+v) Eab[q, ab, tuv] W[q, cd, tuv]
    I = dd.zeros((Pq, nab, ncd))
    for t in range(Lab + 1):
        for u in range(Lab + 1 - t):
            for v in range(Lab + 1 - t - u):
                e = Hab_q[:, :, t, u, v]
                if not np.any(e.hi):
                    continue
                sgn = -1.0 if (t + u + v) % 2 else 1.0
                I = I + (e * sgn)[:, :, None] * W[:, None, :, t, u, v]
    return DDQuartet(I.hi.reshape(nb_, nk_, nab, ncd), I.lo.reshape(nb_, nk_, nab, ncd))


class DDQuartet(dd.DD):
    pass


def _radial(cls, xi, R, L, fac, facp):
    """A_n/N' with DD (xi, R): evaluate at the binary64-rounded (xi, R) and
    correct to first order with A_{n+1} (dA_n/du = A_{n+1}/2 at fixed xi),
    which absorbs the DD residue of R^2."""
    xi_f = xi.to_float()
    R_f = R.to_float()
    A = radial_auto(cls, xi_f, R_f, L + 1, fac, facp)
    # u residue: (R_dd^2 - R_f^2)
    du = (R * R) - dd.DD(R_f) * dd.DD(R_f)
    out = A[:, : L + 1] + A[:, 1: L + 2] * du[:, None] * 0.5
    return out


def _contract(Ipr, sa, sb, sc, sd):
    ca = np.asarray(sa["coefs"], float)
    cb = np.asarray(sb["coefs"], float)
    cc = np.asarray(sc["coefs"], float)
    cd = np.asarray(sd["coefs"], float)
    wb = np.outer(ca, cb).ravel()
    wk = np.outer(cc, cd).ravel()
    w = dd.DD(wb)[:, None] * dd.DD(wk)[None, :]
    t = Ipr * w[:, :, None, None]
    t = dd.dsum(t, 0)
    t = dd.dsum(t, 0)
    return t


def _shift_shell(s, dl):
    s2 = dict(s)
    s2["l"] = s["l"] + dl
    return s2


def _laplacian_bra(cls_fn, side, sa, sb, sc, sd):
    """Primitive (lap a, b|cd) (side 0) or (a, lap b|cd) (side 1), DD (Kab, Kcd, nab, ncd)."""
    s_lap = sa if side == 0 else sb
    l = s_lap["l"]
    exps = np.asarray(s_lap["exps"], float)
    comps = cart(l)
    pieces = {}
    for dl in (-2, 0, 2):
        if l + dl < 0:
            continue
        sh = _shift_shell(s_lap, dl)
        args = [sh, sb, sc, sd] if side == 0 else [sa, sh, sc, sd]
        pieces[dl] = cls_fn(*args)
    Kab, Kcd = pieces[0].shape[0], pieces[0].shape[1]
    la, lb = sa["l"], sb["l"]
    na, nb = len(cart(la)), len(cart(lb))
    ncd = pieces[0].shape[3]
    out = dd.zeros((Kab, Kcd, na * nb, ncd))
    Ka, Kb = len(sa["exps"]), len(sb["exps"])
    # exponent of the Laplacian's orbital for each bra primitive pair
    if side == 0:
        alpha = np.repeat(exps, Kb)
    else:
        alpha = np.tile(exps, Ka)
    al = dd.DD(alpha)[:, None, None]
    for ci, (i, k, m) in enumerate(comps):
        for dirn in range(3):
            pw = (i, k, m)[dirn]
            for dl, coef_fn in ((-2, lambda p: float(p * (p - 1))), (0, None), (2, None)):
                if dl == -2 and pw < 2:
                    continue
                if l + dl < 0:
                    continue
                new = list((i, k, m))
                new[dirn] += dl
                j = cart(l + dl).index(tuple(new))
                if dl == -2:
                    cf = dd.DD(np.full(alpha.shape, float(pw * (pw - 1))))[:, None, None]
                elif dl == 0:
                    cf = al * (-2.0 * (2 * pw + 1))
                else:
                    cf = al * al * 4.0
                src = pieces[dl]
                # bra component index in the shifted shell
                for cb_ in range(nb if side == 0 else na):
                    if side == 0:
                        dst_idx = ci * nb + cb_
                        src_idx = j * nb + cb_
                    else:
                        dst_idx = cb_ * nb + ci
                        src_idx = cb_ * len(cart(l + dl)) + j
                    out[:, :, dst_idx, :] = out[:, :, dst_idx, :] + cf * src[:, :, src_idx, :]
    return out


def contracted(cls, sa, sb, sc, sd, fac=None, facp=None, as_dd=False):
    """Contracted integrals (ab|k_cls|cd) as float64 array [na, nb, nc, nd]."""
    if facp is None:
        facp = fac
    if cls == 5:
        fn = lambda w, x, y, z: primitive_integrals(3, w, x, y, z, fac, facp)
        left = _laplacian_bra(fn, 0, sa, sb, sc, sd)
        right = _laplacian_bra(fn, 1, sa, sb, sc, sd)
        Ipr = (left - right) * 0.5
    else:
        Ipr = primitive_integrals(cls, sa, sb, sc, sd, fac, facp)
    t = _contract(Ipr, sa, sb, sc, sd)
    na, nb, nc, nd = (len(cart(s["l"])) for s in (sa, sb, sc, sd))
    if as_dd:
        return t
    return t.to_float().reshape(na, nb, nc, nd)
