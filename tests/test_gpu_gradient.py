"""First derivatives with respect to the bra's first centre (f12_eval_grad)
against stored oracle values (the plain definition: raised and lowered
shells), translation invariance on the GPU, and the error paths."""
import os
import sys

import numpy as np
import pytest

from synth import FACTOR_SETS
from tests.gpu_common import REL_TOL, block_rel_err

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
P1 = FACTOR_SETS["P1"]


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_5070_amd import f12int
    return f12int


def _grad_blocks(lib, pairs, k, cls, quads):
    import torch
    Q = lib.Quartets.from_list(pairs, pairs, cls, quads)
    offs = Q.offsets()
    out = {}
    for d in range(3):
        buf = torch.full((max(Q.n_out, 1),), np.nan, dtype=torch.float64, device="cuda")
        lib.eval_grad(Q, k, d, buf)
        h = buf.cpu().numpy()
        for i, qd in enumerate(Q.quads()):
            out.setdefault(tuple(int(v) for v in qd), [None] * 3)[d] = h[offs[i]:offs[i + 1]]
    lib.stream_status()
    return {q: np.stack(v) for q, v in out.items()}


@pytest.mark.parametrize("cls", [2, 3, 4, 6])
def test_gradient_vs_golden(lib, cls):
    from make_golden import GRAD_QUADS, df3_shells
    with np.load(os.path.join(HERE, "golden", "grad.npz"), allow_pickle=False) as z:
        golden = {k: z[k] for k in z.files}
    shells = df3_shells()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 1)
    k = lib.Kernel(cls, P1, P1)
    got = _grad_blocks(lib, pairs, k, cls, GRAD_QUADS)
    worst = 0.0
    for qd in GRAD_QUADS:
        ref = golden["c%d_%d_%d_%d_%d" % ((cls,) + qd)].reshape(3, -1)
        e = block_rel_err(got[qd].ravel(), ref.ravel())
        worst = max(worst, e)
        print(f"grad I{cls} {qd}: max|dI| {np.max(np.abs(ref)):.2e} err {e:.2e}", flush=True)
        assert e < REL_TOL, (qd, e)
    print(f"grad I{cls}: worst block-relative error {worst:.2e}", flush=True)


@pytest.mark.parametrize("cls", [3, 6])
def test_gradient_translation_invariance(lib, cls):
    """d/dA + d/dB + d/dC + d/dD = 0, with d/dB, d/dC, d/dD from the lists
    (ba|cd), (cd|ab), (dc|ab) of the same quartets."""
    from make_golden import GRAD_QUADS, df3_shells
    shells = df3_shells()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 1)
    k = lib.Kernel(cls, P1, P1)
    nc = [(s.l + 1) * (s.l + 2) // 2 for s in shells]
    qs = GRAD_QUADS
    gA = _grad_blocks(lib, pairs, k, cls, qs)
    gB = _grad_blocks(lib, pairs, k, cls, [(b, a, c, d) for (a, b, c, d) in qs])
    gC = _grad_blocks(lib, pairs, k, cls, [(c, d, a, b) for (a, b, c, d) in qs])
    gD = _grad_blocks(lib, pairs, k, cls, [(d, c, a, b) for (a, b, c, d) in qs])
    for (a, b, c, d) in qs:
        na, nb, ncc, nd = nc[a], nc[b], nc[c], nc[d]
        A = gA[(a, b, c, d)].reshape(3, na, nb, ncc, nd)
        B = gB[(b, a, c, d)].reshape(3, nb, na, ncc, nd).transpose(0, 2, 1, 3, 4)
        C = gC[(c, d, a, b)].reshape(3, ncc, nd, na, nb).transpose(0, 3, 4, 1, 2)
        D = gD[(d, c, a, b)].reshape(3, nd, ncc, na, nb).transpose(0, 3, 4, 2, 1)
        if len({tuple(np.round(shells[i].center, 12)) for i in (a, b, c, d)}) == 1 and \
                (shells[a].l + shells[b].l + shells[c].l + shells[d].l) % 2 == 0:
            continue  # one centre, even l sum: every derivative block vanishes by parity
        scale = max(np.max(np.abs(x)) for x in (A, B, C, D))
        err = np.max(np.abs(A + B + C + D)) / scale
        assert err < 1e-12, ((a, b, c, d), err)


def test_gradient_error_paths(lib):
    import torch
    from make_golden import df3_shells
    shells = df3_shells()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 1)
    out = torch.empty(200000, dtype=torch.float64, device="cuda")
    k3 = lib.Kernel(3, P1, P1)
    Qff = lib.Quartets.from_list(pairs, pairs, 3, [(3, 3, 3, 3)])  # (ff|ff): no derivative form
    with pytest.raises(lib.F12Error) as e:
        lib.eval_grad(Qff, k3, 0, out)
    assert e.value.status == -3
    Q = lib.Quartets.from_list(pairs, pairs, 3, [(1, 1, 1, 1)])
    with pytest.raises(lib.F12Error) as e:
        lib.eval_grad(Q, k3, 3, out)
    assert e.value.status == -1
    k5 = lib.Kernel(5, P1, P1)
    Q5 = lib.Quartets.from_list(pairs, pairs, 5, [(1, 1, 1, 1)])
    with pytest.raises(lib.F12Error) as e:
        lib.eval_grad(Q5, k5, 0, out)
    assert e.value.status == -1
    lib.stream_status()
