"""Shared helpers for the GPU tests (inputs from synth, the library through
its ctypes binding, the oracle for expected values)."""
import numpy as np


def block_rel_err(got, ref):
    """max |got - ref| / max |ref| over one contracted-quartet block."""
    scale = np.max(np.abs(ref))
    if scale == 0:
        return float(np.max(np.abs(got)))
    return float(np.max(np.abs(got - ref)) / scale)


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


def envelope_err(A, ref, xi):
    """Errors of radial derivatives on their natural scale: |dA_n|/(2 xi)^n
    relative to max_k |A_k|/(2 xi)^k (A_n grows like (2 xi)^n; single A_n can
    pass near zero).  A, ref: (P, L+1); xi: (P,)."""
    L = A.shape[1] - 1
    sc = (2.0 * np.asarray(xi))[:, None] ** np.arange(L + 1)[None, :]
    env = np.max(np.abs(ref) / sc, axis=1)[:, None]
    return np.abs(A - ref) / sc / env


def i5_block_err(got, ref_i5, ref_i3, bra_exps):
    """I5 = 1/2 (lap_A - lap_B) I3 has the magnitude of (exponent x I3); a
    bra pair built from one shell gives a block that vanishes identically
    (lap x_c = x g(r), lap y_c = y g(r) with the same g), so the block is
    scored against max(max|I5|, max bra exponent * max|I3|)."""
    scale = max(np.max(np.abs(ref_i5)), float(np.max(bra_exps)) * np.max(np.abs(ref_i3)))
    return float(np.max(np.abs(got - ref_i5)) / scale)


# Blocks whose largest |integral| is below the workloads' screening threshold
# (1e-12) are negligible; there the MD sums in binary64 can cancel by 1e4 and
# more, so they are held to an absolute bound of 1e-12 of that threshold.
NEGLIGIBLE = 1e-12
ABS_FLOOR = 1e-24


def block_ok(got, ref, rel_tol=1e-12):
    """(passes, relative error, absolute error) under the rule above."""
    scale = float(np.max(np.abs(ref)))
    abs_err = float(np.max(np.abs(got - ref)))
    rel = abs_err / scale if scale > 0 else abs_err
    if scale >= NEGLIGIBLE:
        return rel < rel_tol, rel, abs_err
    return rel < rel_tol or abs_err < ABS_FLOOR, rel, abs_err
