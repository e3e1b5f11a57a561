"""The batched path: quartet lists built on the device, and one class's
quartets from several lists evaluated by one captured graph (concurrent
branches, persistent contraction grids), against the plain path."""
import os
import sys

import numpy as np
import pytest

from synth import FACTOR_SETS, config_plain, molecule, tiny_config

pytestmark = pytest.mark.gpu
P1 = FACTOR_SETS["P1"]


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_5070_amd import f12int
    return f12int


def _same_list(A, B):
    qa, qb = A.quads(), B.quads()
    oa, ob = A.offsets(), B.offsets()
    return qa.shape == qb.shape and np.array_equal(qa, qb) and np.array_equal(oa, ob)


@pytest.mark.parametrize("cls", [3, 5])
def test_device_list_equals_host_list(lib, cls):
    """f12_quartets_build_device gives the host build's list (quartets, order,
    offsets): unscreened on the 20-atom molecule, and screened at 1e-12 and
    1e-6 (where the per-quartet growth term decides many quartets)."""
    _, shells = config_plain()
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 0)
    ks = lib.Kernel(3, P1, P1)
    for tol in (0.0, 1e-12, 1e-6):
        h = lib.Quartets.build(pairs, pairs, cls, screen_tol=tol, screen_kernel=ks if tol > 0 else None)
        d = lib.Quartets.build_device(pairs, pairs, cls, screen_tol=tol, screen_kernel=ks if tol > 0 else None)
        print(f"device list cls={cls} tol={tol:.0e}: host {h.n_quartets} device {d.n_quartets}", flush=True)
        assert h.n_quartets == d.n_quartets and h.n_out == d.n_out
        assert _same_list(h, d)
        assert h.n_prim() == d.n_prim()


def _parts(lib, cls, kern):
    """Three geometries: the 3-atom s+p molecule, a 3-atom s-f molecule and 5
    atoms of the 20-atom recipe; lists built on the device, screened at 1e-12."""
    import torch
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import df3_shells
    mols = [tiny_config()[1], df3_shells(), molecule(5071, 5, 6.0, 1.5, (0, 0, 1, 1, 2, 3), 1, 6, 0.05, 50.0)[1]]
    ks = lib.Kernel(3, P1, P1) if cls == 5 else kern
    keep = []
    parts = []
    for sh in mols:
        basis = lib.Basis.from_shells(sh)
        pairs = lib.Pairs(basis, 0)
        Q = lib.Quartets.build_device(pairs, pairs, cls, screen_tol=1e-12, screen_kernel=ks)
        out = torch.full((max(Q.n_out, 1),), np.nan, dtype=torch.float64, device="cuda")
        keep.append((basis, pairs))
        parts.append((Q, 0, Q.n_quartets, out))
    return parts, keep


@pytest.mark.parametrize("cls", [2, 5, 6])
def test_batch_equals_plain_eval(lib, cls, tmp_path):
    """A batch over three lists, tuned (the choices written to a file and read
    back by a second batch) and with every shape forced persistent (G = 256),
    replayed three times with eager work in between, gives f12_eval's blocks
    bit for bit."""
    import torch
    kern = lib.Kernel(cls, P1, P1)
    parts, keep = _parts(lib, cls, kern)
    refs = []
    for (Q, q0, q1, out) in parts:
        r = torch.empty_like(out)
        lib.eval_into(Q, kern, r)
        refs.append(r)
    lib.stream_status()
    path = str(tmp_path / "tune.txt")
    b1 = lib.Batch(parts, kern, nbranch=3, tune=True, tune_path=path)
    lines = open(path).read().split("\n")
    print(f"batch cls={cls}: {b1.n_quartets} quartets, {b1.n_chunks} chunks; tuned: "
          f"{[l for l in lines if l]}", flush=True)
    b2 = lib.Batch(parts, kern, nbranch=2, tune=True, tune_path=path)  # reads the file
    forced = str(tmp_path / "forced.txt")
    with open(forced, "w") as f:
        for l in lines:
            if l:
                a, b, c, _ = l.split()
                f.write(f"{a} {b} {c} 256\n")
    b3 = lib.Batch(parts, kern, nbranch=4, tune=False, tune_path=forced)
    for bt in (b1, b2, b3):
        for rep in range(3):
            for (_, _, _, out) in parts:
                out.fill_(np.nan)
            bt.launch()
            torch.cuda.synchronize()
            _ = (torch.ones(1000, device="cuda") * 2).sum().item()  # eager work between replays
            for (p, r) in zip(parts, refs):
                assert torch.equal(p[3], r), (cls, rep)
    lib.stream_status()
