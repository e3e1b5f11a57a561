"""Shared helpers for the GPU tests (inputs from synth, the library through
its ctypes binding, the oracle for expected values)."""
import numpy as np

# Block-relative tolerance of the FP64 path: max |I_gpu - I_ref| / max |I_ref|
# over one contracted-quartet block.
REL_TOL = 1e-12


def block_rel_err(got, ref):
    """max |got - ref| / max |ref| over one contracted-quartet block."""
    scale = np.max(np.abs(ref))
    if scale == 0:
        return float(np.max(np.abs(got)))
    return float(np.max(np.abs(got - ref)) / scale)


def i5_vanishes(la, same_shell, spherical_ket=False):
    """An I5 block vanishes identically when the bra pair is one s or p shell
    taken twice: for l <= 1 the Laplacian of each component x_c e^{-a r^2} is
    x_c h(r) with one h for all components, so
    (lap phi_i) phi_j - phi_i (lap phi_j) = 0 pointwise.  For d and f shells
    the components are not harmonic and the block vanishes only against a
    spherical ket (two s shells on the bra's centre, spherical_ket): the
    difference is the divergence of phi_j grad phi_i - phi_i grad phi_j, whose
    radial part cancels for two components of one shell."""
    return same_shell and (la <= 1 or spherical_ket)


def vanishes_by_parity(quad, shells):
    """A block vanishes identically when its four shells sit on one centre and
    l_a + l_b + l_c + l_d is odd: inversion through that centre maps the
    integrand to minus itself (the kernel depends on r12 only)."""
    cs = {tuple(np.round(np.asarray(shells[i].center, float), 12)) for i in quad}
    return len(cs) == 1 and sum(shells[i].l for i in quad) % 2 == 1


def zero_block_err(got, diag_ab, diag_cd):
    """Error of a block that vanishes identically, on the scale
    sqrt(max |(ab|ab)| max |(cd|cd)|) of its pairs (Schwarz-like size of the
    terms that cancel): the GPU's rounding noise over that scale."""
    return float(np.max(np.abs(got))) / np.sqrt(diag_ab * diag_cd)


def i5_block_err(got, ref_i5, ref_i3, bra_exps, vanishes):
    """Block-relative error of an I5 block on its own scale max |I5|.  Only
    for a block that vanishes identically (i5_vanishes) is the GPU's rounding
    noise scored against the size of the terms that cancel, the largest bra
    exponent times max |I3| of the same quartet."""
    if vanishes:
        scale = float(np.max(bra_exps)) * float(np.max(np.abs(ref_i3)))
        return float(np.max(np.abs(got - ref_i5)) / scale)
    return block_rel_err(got, ref_i5)


def run_quads(f12int, basis, pairs, kernel, cls, quads):
    """Evaluate explicit shell quadruples on the GPU; returns {tuple(quad): block}."""
    import torch
    Q = f12int.Quartets.from_list(pairs, pairs, cls, quads)
    out = torch.empty(max(Q.n_out, 1), dtype=torch.float64, device="cuda")
    f12int.eval_into(Q, kernel, out)
    f12int.stream_status()
    host = out.cpu().numpy()
    offs = Q.offsets()
    order = Q.quads()
    res = {}
    for i, qd in enumerate(order):
        res[tuple(int(v) for v in qd)] = host[offs[i]:offs[i + 1]]
    return res


def run_list(f12int, Q, kernel):
    """Evaluate a whole quartet list; returns {tuple(quad): block}."""
    import torch
    out = torch.empty(max(Q.n_out, 1), dtype=torch.float64, device="cuda")
    f12int.eval_into(Q, kernel, out)
    f12int.stream_status()
    host = out.cpu().numpy()
    offs = Q.offsets()
    return {tuple(int(v) for v in qd): host[offs[i]:offs[i + 1]] for i, qd in enumerate(Q.quads())}


def envelope_err(A, ref, xi):
    """Errors of radial derivatives on their natural scale: |dA_n|/(2 xi)^n
    relative to max_k |A_k|/(2 xi)^k (A_n grows like (2 xi)^n; single A_n can
    pass near zero).  A, ref: (P, L+1); xi: (P,)."""
    L = A.shape[1] - 1
    sc = (2.0 * np.asarray(xi))[:, None] ** np.arange(L + 1)[None, :]
    env = np.max(np.abs(ref) / sc, axis=1)[:, None]
    return np.abs(A - ref) / sc / env
