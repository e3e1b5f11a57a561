"""f12_eval_noalloc (fixed library scratch, no device allocation) against
f12_eval on the same quartet list: two calls in a row, the second on a
smaller range, so the second call reads a scratch array that still holds the
first call's contents."""
import numpy as np
import pytest

from synth import FACTOR_SETS, config_plain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_5070_amd import f12int
    return f12int


@pytest.mark.parametrize("cls", [3, 5])
def test_noalloc_matches_eval(lib, cls):
    import torch
    _, shells = config_plain()
    rng = np.random.default_rng(31 + cls)
    ns = len(shells)
    ks = np.array([len(s.exps) for s in shells])
    quads = rng.integers(0, ns, (6000, 4)).astype(np.int32)
    nprim = int(ks[quads].prod(axis=1).sum())
    print(f"noalloc cls={cls} quartets={len(quads)} primitive quartets={nprim}", flush=True)
    # more primitive quartets than the fixed scratch holds: several chunks
    assert nprim > 262144
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 1)
    k = lib.Kernel(cls, FACTOR_SETS["P1"], FACTOR_SETS["P1"])
    Q = lib.Quartets.from_list(pairs, pairs, cls, quads)
    offs = Q.offsets()
    ref = torch.empty(Q.n_out, dtype=torch.float64, device="cuda")
    lib.eval_into(Q, k, ref)
    lib.stream_status()
    ref = ref.cpu().numpy()
    for (q0, q1) in ((0, Q.n_quartets), (17, 17 + 700)):
        out = torch.full((int(offs[q1] - offs[q0]),), np.nan, dtype=torch.float64, device="cuda")
        lib.eval_noalloc(Q, k, out, q0, q1)
        lib.stream_status()
        got = out.cpu().numpy()
        exp = ref[offs[q0]:offs[q1]]
        print(f"  range [{q0}, {q1}): max |diff| {np.max(np.abs(got - exp)):.2e}", flush=True)
        assert np.array_equal(got, exp)


def test_noalloc_argument_errors(lib):
    import torch
    _, shells = config_plain()
    basis = lib.Basis.from_shells(shells[:12])
    pairs = lib.Pairs(basis, 1)
    k3, k2 = lib.Kernel(3, FACTOR_SETS["P1"]), lib.Kernel(2, FACTOR_SETS["P1"])
    Q = lib.Quartets.from_list(pairs, pairs, 3, [(0, 1, 2, 3), (4, 5, 6, 7)])
    offs = Q.offsets()
    short = torch.empty(int(offs[-1]) - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.F12Error) as e:
        lib.eval_noalloc(Q, k3, short)
    assert e.value.status == -6
    buf = torch.empty(int(offs[-1]), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.F12Error) as e:
        lib.eval_noalloc(Q, k2, buf)
    assert e.value.status == -1
