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
    assert b"non-finite" in f12int._lib.f12_strerror(-7)


def test_eval_sets_validation_before_device():
    """f12_eval_sets rejects null handles, nset < 1 and a null kernel array
    before any device work."""
    from paper_1412_5070_amd import f12int
    lib = f12int._lib
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.f12_eval_sets(None, arr, 1, 0, 0, None, 0, None) == -1
    assert lib.f12_eval_sets(None, None, 1, 0, 0, None, 0, None) == -1
    assert lib.f12_eval_sets(None, arr, 0, 0, 0, None, 0, None) == -1


def test_digest_validation_before_device():
    """f12_digest rejects a null list or a null digest pointer before any
    device work."""
    from paper_1412_5070_amd import f12int
    lib = f12int._lib
    dummy = ctypes.c_uint64(0)
    assert lib.f12_digest(None, 0, 0, None, ctypes.cast(ctypes.pointer(dummy), ctypes.c_void_p), None) == -1
    assert lib.f12_digest(None, 0, 1, None, None, None) == -1


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


def _w_negint_ref(n, x):
    """Finite part of int_0^inf t^(-n) e^{-(t-x)^2} dt written out in mpmath:
    on [0, 1] the Taylor series of the Gaussian integrated term by term (the
    finite part of int_eps^1 t^(j-n) is 1/(j-n+1), and 0 for j = n-1), plus
    the regular integral over [1, inf)."""
    x = mp.mpf(x)
    s, j = mp.mpf(0), 0
    # H_j = e^{-x^2} Hphys_j(x) / j!
    h0, h1 = mp.mpf(1), 2 * x
    hs = [h0, h1]
    for j in range(1, 400):
        hs.append((2 * x * hs[j] - 2 * hs[j - 1]) / (j + 1))
    for j, hj in enumerate(hs):
        if j != n - 1:
            s += hj / (j - n + 1)
    s *= mp.exp(-x * x)
    s += mp.quad(lambda t: t ** (-n) * mp.exp(-(t - x) ** 2), [1, max(1, x - 8), max(1, x), max(1, x) + 8, mp.inf])
    return s


@pytest.mark.parametrize("x", [-10.5, -6.2, -2.0, -0.6, 0.0, 0.7, 1.5, 4.0, 9.0, 20.0, 35.9])
def test_aux_table_negative_integer_orders(x):
    """The host builder's finite parts W_{-n}(x) (negative integer orders,
    used by kernels with negative powers of r) against the finite part
    written out in mpmath at 120 digits, n = 1..26."""
    from paper_1412_5070_amd import f12int
    col = f12int.aux_w_column(0.0, 1, -26, 2, x)
    # the Taylor series at t = 0 alternates with terms up to ~e^{x^2/2}: 120
    # digits keep the reference exact to double precision over the whole range
    with mp.workdps(120):
        for n in range(1, 27):
            ref = _w_negint_ref(n, x)
            assert abs(col[26 - n] - ref) <= 2e-15 * abs(ref) + 1e-300, (n, col[26 - n], ref)


def test_aux_table_negative_integer_orders_at_zero():
    """At x = 0 the finite parts are closed forms (Eq. (sila) at beta = 0):
    FP int t^(-2p-1) e^{-t^2} = (-1)^p psi(p+1) / (2 p!), and
    int t^(-2p) e^{-t^2} = Gamma(1/2 - p) / 2."""
    from paper_1412_5070_amd import f12int
    col = f12int.aux_w_column(0.0, 1, -26, 2, 0.0)
    with mp.workdps(30):
        for n in range(1, 27):
            if n % 2:
                p = (n - 1) // 2
                ref = (-1) ** p * mp.digamma(p + 1) / (2 * mp.factorial(p))
            else:
                ref = mp.gamma(mp.mpf(1) / 2 - n // 2) / 2
            assert abs(col[26 - n] - ref) <= 1e-15 * abs(ref), (n, col[26 - n], ref)


def test_unsupported_kernel_terms_rejected_before_device():
    """Kernel terms the library does not evaluate return F12_EPARAM during
    term analysis, before any device work: a negative integer power below
    -12 (rho = -13 with n = 6, a valid factor) and growing chains with b < 0
    (B < 0)."""
    from paper_1412_5070_amd import f12int
    from synth import Factor
    for cls, f in ((2, Factor(0.05, -13.0, 0.25, 1.0, 6)), (3, Factor(0.2, 0.5, -0.3, 0.8, 0))):
        with pytest.raises(f12int.F12Error) as e:
            f12int.Kernel(cls, f, f)
        assert e.value.status == -2


def test_factor_terms_validation_before_device():
    """f12_kernel_create_terms rejects, before any device work, terms it does
    not evaluate (a decaying exponential, b < 0, times a non-integer power, a
    negative Gaussian exponent, a negative integer or a non-integer power
    <= -1, non-finite values) and malformed lists."""
    from paper_1412_5070_amd import f12int
    for bad in ([[1.0, 0.5, -0.5, 0.0]], [[1.0, 0.0, 0.0, -1.0]], [[1.0, -1.0, 0.0, 1.0]],
                [[1.0, -1.5, 0.0, 1.0]], [[np.nan, 0.0, 0.0, 1.0]]):
        with pytest.raises(f12int.F12Error) as e:
            f12int.Kernel.from_terms(3, bad)
        assert e.value.status == -2, bad
    with pytest.raises(f12int.F12Error) as e:
        f12int.Kernel.from_terms(3, np.zeros((0, 4)))
    assert e.value.status == -1
