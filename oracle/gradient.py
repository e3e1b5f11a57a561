"""First derivatives of the integrals with respect to a shell's centre (oracle).

Test infrastructure only.

The plain definition: moving centre A moves only the bra's first function,
and for one unnormalised primitive along x
  d/dA_x [(x - A_x)^i e^{-e (x - A_x)^2}] = 2e (x - A_x)^(i+1) e^{...} - i (x - A_x)^(i-1) e^{...},
so d/dA_x (ab|k|cd) over a contracted shell (coefficients c_k, exponents e_k)
is the block of the same shell raised to l + 1 with coefficients 2 e_k c_k,
at the component (i+1, j, k), minus i times the block of the shell lowered to
l - 1 at (i-1, j, k).  The same holds for I5, whose operator acts on the
functions and commutes with a translation of one of them.
"""
import numpy as np

from .integrals import cart, contracted


def grad_first_centre(cls, sa, sb, sc, sd, fac=None, facp=None):
    """[3, na, nb, nc, nd]: d/dA_x, d/dA_y, d/dA_z of (ab|k_cls|cd), A = sa's centre."""
    la = sa["l"]
    exps = np.asarray(sa["exps"], float)
    coefs = np.asarray(sa["coefs"], float)
    up = dict(sa, l=la + 1, coefs=2.0 * exps * coefs)
    I_up = contracted(cls, up, sb, sc, sd, fac, facp)
    I_dn = contracted(cls, dict(sa, l=la - 1), sb, sc, sd, fac, facp) if la > 0 else None
    comps, comps_up = cart(la), cart(la + 1)
    comps_dn = cart(la - 1) if la > 0 else []
    nb, nc, nd = I_up.shape[1:]
    out = np.zeros((3, len(comps), nb, nc, nd))
    for ci, c in enumerate(comps):
        for d in range(3):
            hi = list(c)
            hi[d] += 1
            out[d, ci] = I_up[comps_up.index(tuple(hi))]
            if c[d] > 0:
                lo = list(c)
                lo[d] -= 1
                out[d, ci] -= c[d] * I_dn[comps_dn.index(tuple(lo))]
    return out
