"""Hermite expansion coefficients and Hermite integrals (oracle).

Test infrastructure only.

E coefficients (Sec. II.B, Eq. (AB) and Eq. (Lambda)): the product of two
1-D Cartesian Gaussians x_A^i e^{-a x_A^2} x_B^j e^{-b x_B^2} equals
sum_t E_t^{ij} d^t/dP^t e^{-p x_P^2}.  The oracle uses the textbook
three-term form of the recursion (McMurchie-Davidson / Helgaker), which is a
different arrangement from the one printed in Eqs. (Ereci)-(Erect):
  E_0^{00} = exp(-(ab/p) X_AB^2)                                   (Erec0)
  E_t^{i+1,j} = E_{t-1}^{ij}/(2p) + X_PA E_t^{ij} + (t+1) E_{t+1}^{ij}
  E_t^{i,j+1} = E_{t-1}^{ij}/(2p) + X_PB E_t^{ij} + (t+1) E_{t+1}^{ij}

Hermite integrals (Eq. (ri)): R_tuv = d^t/dQx d^u/dQy d^v/dQz B(|Q - P|).
For a radial function h(|X|), d/dX_x h = X_x D h with D = R^-1 d/dR, which
gives the standard recurrence on R^(n)_tuv = d^tuv D^n B:
  R^(n)_{000} = A_n,  R^(n)_{t+1,u,v} = t R^(n+1)_{t-1,u,v} + X_x R^(n+1)_{tuv}.
"""
import numpy as np
from . import dd


def e_coefficients(a, b, Ax, Bx, la, lb):
    """E_t^{ij} for 0<=i<=la, 0<=j<=lb, 0<=t<=i+j along one direction.

    a, b, Ax, Bx: 1-D float arrays (one entry per primitive pair).
    Returns a DD array of shape (P, la+1, lb+1, la+lb+1).
    """
    a = dd.DD(np.asarray(a, float))
    b = dd.DD(np.asarray(b, float))
    Ax = dd.DD(np.asarray(Ax, float))
    Bx = dd.DD(np.asarray(Bx, float))
    p = a + b
    Px = (a * Ax + b * Bx) / p
    XAB = Ax - Bx
    XPA = Px - Ax
    XPB = Px - Bx
    inv2p = 0.5 / p
    P = a.shape[0]
    L = la + lb
    E = dd.zeros((P, la + 1, lb + 1, L + 2))
    E[:, 0, 0, 0] = dd.exp(-(a * b / p) * XAB * XAB)

    def get(i, j, t):
        if t < 0 or t > i + j:
            return dd.zeros((P,))
        return E[:, i, j, t]

    for i in range(la + 1):
        for j in range(lb + 1):
            if i == 0 and j == 0:
                continue
            if i > 0:
                for t in range(i + j + 1):
                    E[:, i, j, t] = inv2p * get(i - 1, j, t - 1) + XPA * get(i - 1, j, t) + float(t + 1) * get(i - 1, j, t + 1)
            else:
                for t in range(i + j + 1):
                    E[:, i, j, t] = inv2p * get(i, j - 1, t - 1) + XPB * get(i, j - 1, t) + float(t + 1) * get(i, j - 1, t + 1)
    return E[:, :, :, : L + 1]


def hermite_r(A, X, Y, Z, L):
    """Dense cube R[P, t, u, v] (t+u+v <= L, zero elsewhere) from A_n (DD (P, L+1))."""
    P = A.shape[0]
    # level n holds R^(n)_{tuv} for t+u+v <= L-n
    cur = None
    for n in range(L, -1, -1):
        m = L - n
        nxt = dd.zeros((P, m + 1, m + 1, m + 1))
        nxt[:, 0, 0, 0] = A[:, n]
        if cur is not None:
            for tot in range(1, m + 1):
                for t in range(tot + 1):
                    for u in range(tot - t + 1):
                        v = tot - t - u
                        if t > 0:
                            val = X * cur[:, t - 1, u, v]
                            if t > 1:
                                val = val + float(t - 1) * cur[:, t - 2, u, v]
                        elif u > 0:
                            val = Y * cur[:, t, u - 1, v]
                            if u > 1:
                                val = val + float(u - 1) * cur[:, t, u - 2, v]
                        else:
                            val = Z * cur[:, t, u, v - 1]
                            if v > 1:
                                val = val + float(v - 1) * cur[:, t, u, v - 2]
                        nxt[:, t, u, v] = val
        cur = nxt
    return cur
