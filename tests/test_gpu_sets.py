"""Several factor sets in one call (f12_eval_sets) and the device's
non-finite guard reported by f12_stream_status."""
import numpy as np
import pytest

from synth import FACTOR_SETS, GENERIC_FACTORS, tiny_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_5070_amd import f12int
    return f12int


@pytest.mark.parametrize("cls", [3, 5, 6])
def test_eval_sets_equal_one_set_at_a_time(lib, cls):
    """Three factor sets (P1, P3 and the term-list factor G5) over every
    quartet of the 3-atom s+p molecule: set s of f12_eval_sets equals f12_eval
    with that set's kernel bit for bit, and the layout is [set][block]."""
    import torch
    shells = tiny_config()[1]
    basis = lib.Basis.from_shells(shells)
    pairs = lib.Pairs(basis, 0)
    ks = [lib.Kernel(cls, FACTOR_SETS["P1"], FACTOR_SETS["P1"]), lib.Kernel(cls, FACTOR_SETS["P3"], FACTOR_SETS["P3"]),
          lib.Kernel.from_terms(cls, GENERIC_FACTORS["G5"], GENERIC_FACTORS["G5"])]
    Q = lib.Quartets.build(pairs, pairs, cls)
    n = Q.n_out
    print(f"eval_sets cls={cls}: {Q.n_quartets} quartets, {n} doubles per set", flush=True)
    out = torch.full((3 * n,), np.nan, dtype=torch.float64, device="cuda")
    lib.eval_sets(Q, ks, out)
    for s, k in enumerate(ks):
        ref = torch.empty(n, dtype=torch.float64, device="cuda")
        lib.eval_into(Q, k, ref)
        assert torch.equal(out[s * n:(s + 1) * n], ref), s
    # a sub-range: offsets relative to q_begin, sets n_range apart
    q0, q1 = 3, Q.n_quartets - 2
    offs = Q.offsets()
    nr = int(offs[q1] - offs[q0])
    sub = torch.full((3 * nr,), np.nan, dtype=torch.float64, device="cuda")
    lib.eval_sets(Q, ks, sub, q0, q1)
    for s, k in enumerate(ks):
        ref = torch.empty(nr, dtype=torch.float64, device="cuda")
        lib.eval_into(Q, k, ref, q0, q1)
        assert torch.equal(sub[s * nr:(s + 1) * nr], ref), s
    with pytest.raises(lib.F12Error) as e:
        lib.eval_sets(Q, ks, out[: 3 * n - 1])
    assert e.value.status == -6
    with pytest.raises(lib.F12Error) as e:
        lib.eval_sets(Q, [lib.Kernel(2 if cls != 2 else 3, FACTOR_SETS["P1"], FACTOR_SETS["P1"])], out)
    assert e.value.status == -1
    lib.stream_status()


def test_stream_status_reports_non_finite_values(lib):
    """Contraction coefficients of 1e200 overflow in c_a c_b: the blocks come
    out non-finite, and f12_stream_status says so (F12_ENONFINITE) once; the
    word is cleared, so a clean evaluation after it reports F12_OK."""
    import torch
    from synth import Shell
    shells = tiny_config()[1]
    lib.stream_status()  # start from a clear word
    big = [Shell(s.center, s.l, s.exps, s.coefs * 1e200, s.atom) for s in shells]
    for sh, bad in ((big, True), (shells, False)):
        basis = lib.Basis.from_shells(sh)
        pairs = lib.Pairs(basis, 1)
        k = lib.Kernel(3, FACTOR_SETS["P1"], FACTOR_SETS["P1"])
        Q = lib.Quartets.from_list(pairs, pairs, 3, [(0, 0, 1, 1), (2, 3, 4, 5)])
        out = torch.empty(Q.n_out, dtype=torch.float64, device="cuda")
        lib.eval_into(Q, k, out)
        torch.cuda.synchronize()
        print(f"coefficients x{1e200 if bad else 1.0:g}: finite outputs {bool(torch.isfinite(out).all())}", flush=True)
        if bad:
            assert not bool(torch.isfinite(out).all())
            with pytest.raises(lib.F12Error) as e:
                lib.stream_status()
            assert e.value.status == lib.ENONFINITE
        else:
            assert bool(torch.isfinite(out).all())
            lib.stream_status()
