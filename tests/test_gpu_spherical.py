"""Blocks over real solid harmonics (f12_cart_to_sph) against the oracle:
the stored oracle Cartesian blocks of the 3-atom s-f molecule transformed by
the oracle's solid harmonics (Sec. II.D, Eq. (Ylm) in real form), and the
spherical offsets and sub-ranges of the entry point."""
import os
import sys

import numpy as np
import pytest

from synth import FACTOR_SETS
from tests.gpu_common import REL_TOL, block_rel_err, i5_block_err, vanishes_by_parity

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_5070_amd import f12int
    return f12int


@pytest.mark.parametrize("cls", [2, 3, 4, 6, 5])
def test_spherical_blocks_vs_oracle(lib, cls):
    import torch
    from make_golden import DF3_QUADS, DF3_QUADS_I5, df3_shells
    from oracle import spherical
    with np.load(os.path.join(HERE, "golden", "df3.npz"), allow_pickle=False) as z:
        golden = {k: z[k] for k in z.files}
    shells = df3_shells()
    quads = DF3_QUADS_I5 if cls == 5 else DF3_QUADS
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 1)
    P1 = FACTOR_SETS["P1"]
    k = lib.Kernel(cls, P1, P1)
    Q = lib.Quartets.from_list(pairs, pairs, cls, quads)
    cart = torch.empty(max(Q.n_out, 1), dtype=torch.float64, device="cuda")
    lib.eval_into(Q, k, cart)
    so = lib.offsets_sph(Q)
    sph = torch.full((int(so[-1]),), np.nan, dtype=torch.float64, device="cuda")
    lib.cart_to_sph(Q, cart, sph)
    lib.stream_status()
    h = sph.cpu().numpy()
    worst = 0.0
    for i, qd in enumerate(Q.quads()):
        qd = tuple(int(v) for v in qd)
        ls = [shells[j].l for j in qd]
        ref = spherical.block_to_sph(golden["c%d_%d_%d_%d_%d" % ((cls,) + qd)], *ls)
        got = h[so[i]:so[i + 1]]
        assert got.size == ref.size
        if vanishes_by_parity(qd, shells):
            continue
        if cls == 5:
            # over solid harmonics every shell is S_lm(r) G(r) with one radial G
            # for all m, so lap phi_m = S_lm H(r) and the I5 block of one shell
            # taken twice as the bra vanishes for any l (over Cartesians only for
            # l <= 1); such a block is scored against the size of the cancelling
            # terms, the bra exponent times the I3 block, as the Cartesian ones
            ref3 = spherical.block_to_sph(golden["c3_%d_%d_%d_%d" % qd], *ls)
            e = i5_block_err(got, ref, ref3, np.concatenate([shells[qd[0]].exps, shells[qd[1]].exps]),
                             qd[0] == qd[1])
            if qd[0] == qd[1]:
                assert np.max(np.abs(ref)) <= 1e-13 * np.max(np.abs(ref3)) * np.max(shells[qd[0]].exps)
        else:
            e = block_rel_err(got, ref)
        worst = max(worst, e)
        assert e < REL_TOL, (qd, e)
    print(f"spherical I{cls}: {Q.n_quartets} blocks, worst block-relative error vs oracle {worst:.2e}", flush=True)
    # a sub-range lands at offsets relative to its first block
    q0, q1 = 2, Q.n_quartets - 1
    sub = torch.full((int(so[q1] - so[q0]),), np.nan, dtype=torch.float64, device="cuda")
    offs = Q.offsets()
    lib.cart_to_sph(Q, cart[int(offs[q0]):int(offs[q1])].contiguous(), sub, q0, q1)
    torch.cuda.synchronize()
    assert torch.equal(sub, sph[int(so[q0]):int(so[q1])])
    with pytest.raises(lib.F12Error) as e:
        lib.cart_to_sph(Q, cart, sph[:-1])
    assert e.value.status == -6
