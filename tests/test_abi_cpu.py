"""CPU-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol the header declares, validates arguments before touching the
device, and its host-side auxiliary-table builder matches mpmath."""
import ctypes
import os
import re

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1412_5070_amd", "libf12int.so")
HDR = os.path.join(ROOT, "include", "f12int.h")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libf12int.so not built")


def declared_functions():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(f12_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1412_5070_amd import f12int
    assert set(declared_functions()) == set(f12int.EXPORTS)


def test_strerror():
    from paper_1412_5070_amd import f12int
    assert f12int._lib.f12_strerror(0) == b"ok"
    assert b"factor" in f12int._lib.f12_strerror(-2)


def test_basis_validation():
    from paper_1412_5070_amd import f12int
    ok = ([[0, 0, 0]], [[1, 2, 0, 0]], [1.0, 0.5], [0.3, 0.7])
    f12int.Basis(*ok)
    with pytest.raises(f12int.F12Error) as e:
        f12int.Basis([[0, 0, 0]], [[4, 1, 0, 0]], [1.0], [1.0])  # g shell: above LMAX
    assert e.value.status == -3
    with pytest.raises(f12int.F12Error) as e:
        f12int.Basis([[0, 0, 0]], [[0, 1, 0, 0]], [-1.0], [1.0])  # negative exponent
    assert e.value.status == -1
    with pytest.raises(f12int.F12Error):
        f12int.Basis([[0, 0, np.nan]], [[0, 1, 0, 0]], [1.0], [1.0])
    with pytest.raises(f12int.F12Error):
        f12int.Basis([[0, 0, 0]], [[0, 2, 0, 0]], [1.0], [1.0])  # prims out of range


def test_factor_validation_before_device():
    from paper_1412_5070_amd import f12int
    from synth import Factor
    for bad in (Factor(0.2, 0.5, 0.3, 0.0, 0), Factor(0.2, 0.5, 0.3, -1.0, 0),
                Factor(np.inf, 0.5, 0.3, 0.8, 0), Factor(0.1, -3.0, 0.2, 1.0, 0)):
        with pytest.raises(f12int.F12Error) as e:
            f12int.Kernel(3, bad)
        assert e.value.status == -2
    with pytest.raises(f12int.F12Error) as e:
        f12int.Kernel(7, Factor(0.2, 0.5, 0.3, 0.8, 0))
    assert e.value.status == -1


def _w_ref(a, x):
    a, x = mp.mpf(a), mp.mpf(x)
    # R int_0^inf t^a e^{-(t-x)^2} dt = Gamma(a+1) e^{-x^2/2} 2^{-(a+1)/2} D_{-a-1}(-sqrt(2) x)
    return mp.gamma(a + 1) * mp.e ** (-x * x / 2) * mp.mpf(2) ** (-(a + 1) / 2) * mp.pcfd(-a - 1, -mp.sqrt(2) * x)


@pytest.mark.parametrize("alpha0,is_int,m_lo,m_hi", [(0.5, 0, -16, 24), (0.0, 1, 0, 24)])
@pytest.mark.parametrize("x", [-10.5, -6.2, -2.0, -0.6, -0.51, -0.3, 0.0, 0.2, 0.51, 1.5, 4.0, 9.0, 11.9, 12.1, 20.0, 35.9])
def test_aux_table_builder_vs_parabolic_cylinder(alpha0, is_int, m_lo, m_hi, x):
    """The host builder of W_a(x) (finite part for a < -1) against mpmath's
    parabolic cylinder function, to 3e-16 relative over the whole ladder."""
    from paper_1412_5070_amd import f12int
    col = f12int.aux_w_column(alpha0, is_int, m_lo, m_hi, x)
    with mp.workdps(30):
        for i, m in enumerate(range(m_lo, m_hi + 1)):
            ref = _w_ref(alpha0 + m, x)
            assert abs(col[i] - ref) <= 3e-16 * abs(ref), (m, col[i], ref)


def test_unsupported_kernel_terms_rejected_before_device():
    """Kernel terms the library does not evaluate return F12_EPARAM during
    term analysis, before any device work: negative integer powers (factor
    set P3 with rho = -3) and growing chains with b < 0 (B < 0)."""
    from paper_1412_5070_amd import f12int
    from synth import FACTOR_SETS, Factor
    for cls, f in ((3, FACTOR_SETS["P3"]), (2, FACTOR_SETS["P3"]), (3, Factor(0.2, 0.5, -0.3, 0.8, 0))):
        with pytest.raises(f12int.F12Error) as e:
            f12int.Kernel(cls, f, f)
        assert e.value.status == -2
