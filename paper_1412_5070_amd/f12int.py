"""ctypes binding of libf12int.so (argument marshalling only).

Every computation happens in the HIP library; this module converts numpy /
torch arguments to the pointers and sizes the C ABI takes.  Importing it
fails loudly if the library has not been built.
"""
import ctypes
import os

import numpy as np
# torch first: its HIP runtime (libamdhip64, same soname as /opt/rocm's) must be
# the one the library binds to, otherwise torch cannot initialise the device.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libf12int.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1412_5070_amd/build_lib.py "
                      "(or __graft_entry__.build())")
_lib = ctypes.CDLL(LIB_PATH)

_c_i32, _c_i64, _c_dbl, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
_P = ctypes.POINTER


class Factor(ctypes.Structure):
    _fields_ = [("c0", _c_dbl), ("rho", _c_dbl), ("B", _c_dbl), ("mu", _c_dbl),
                ("n", _c_i32), ("reserved", _c_i32)]

    @staticmethod
    def of(f):
        return Factor(float(f.c0), float(f.rho), float(f.B), float(f.mu), int(f.n), 0)


class ShellC(ctypes.Structure):
    _fields_ = [("l", _c_i32), ("nprim", _c_i32), ("center", _c_i32), ("first_prim", _c_i32)]


EXPORTS = {
    "f12_basis_create": (_c_i32, [_c_i32, _P(_c_dbl), _c_i32, _P(ShellC), _c_i32, _P(_c_dbl), _P(_c_dbl), _P(_vp)]),
    "f12_basis_destroy": (None, [_vp]),
    "f12_pairs_build": (_c_i32, [_vp, _c_i32, _vp, _P(_vp)]),
    "f12_pairs_count": (_c_i32, [_vp, _P(_c_i64), _P(_c_i64)]),
    "f12_pairs_destroy": (None, [_vp]),
    "f12_kernel_create": (_c_i32, [_c_i32, _P(Factor), _P(Factor), _P(_vp)]),
    "f12_kernel_create_terms": (_c_i32, [_c_i32, _c_i32, _P(_c_dbl), _c_i32, _P(_c_dbl), _P(_vp)]),
    "f12_kernel_terms": (_c_i32, [_vp, _P(_c_i32), _P(_c_dbl), _c_i32]),
    "f12_kernel_destroy": (None, [_vp]),
    "f12_quartets_build": (_c_i32, [_vp, _vp, _c_i32, _c_dbl, _vp, _vp, _P(_vp), _P(_c_i64), _P(_c_i64)]),
    "f12_quartets_build_device": (_c_i32, [_vp, _vp, _c_i32, _c_dbl, _vp, _vp, _P(_vp), _P(_c_i64), _P(_c_i64)]),
    "f12_quartets_from_list": (_c_i32, [_vp, _vp, _c_i32, _P(_c_i32), _c_i64, _P(_vp), _P(_c_i64)]),
    "f12_quartet_offsets": (_c_i32, [_vp, _P(_c_i64)]),
    "f12_quartet_list": (_c_i32, [_vp, _P(_c_i32)]),
    "f12_quartet_groups": (_c_i32, [_vp, _P(_c_i32), _P(_c_i64), _P(_c_i32), _c_i32]),
    "f12_quartets_prim_count": (_c_i32, [_vp, _P(_c_i64)]),
    "f12_quartets_destroy": (None, [_vp]),
    "f12_eval": (_c_i32, [_vp, _vp, _c_i64, _c_i64, _vp, _c_i64, _vp]),
    "f12_eval_precision": (_c_i32, [_vp, _vp, _c_i64, _c_i64, _vp, _c_i64, _c_i32, _vp]),
    "f12_eval_sets": (_c_i32, [_vp, _P(_vp), _c_i32, _c_i64, _c_i64, _vp, _c_i64, _vp]),
    "f12_eval_grad": (_c_i32, [_vp, _vp, _c_i32, _c_i64, _c_i64, _vp, _c_i64, _vp]),
    "f12_eval_noalloc": (_c_i32, [_vp, _vp, _c_i64, _c_i64, _vp, _c_i64, _vp]),
    "f12_eval_stage": (_c_i32, [_vp, _vp, _c_i64, _c_i64, _vp, _c_i64, _c_i32, _vp]),
    "f12_quartets_scratch_prims": (_c_i32, [_vp, _P(_c_i64)]),
    "f12_batch_create": (_c_i32, [_c_i32, _P(_vp), _P(_c_i64), _P(_c_i64), _vp, _P(_vp), _P(_c_i64), _c_i32,
                                  _c_i32, ctypes.c_char_p, _vp, _P(_vp)]),
    "f12_batch_launch": (_c_i32, [_vp, _vp]),
    "f12_batch_info": (_c_i32, [_vp, _P(_c_i64), _P(_c_i64), _P(_c_i64)]),
    "f12_batch_grid": (_c_i32, [_vp, _c_i32, _c_i32, _c_i32, _P(_c_i64)]),
    "f12_batch_destroy": (None, [_vp]),
    "f12_aux_radial": (_c_i32, [_vp, _c_i64, _vp, _vp, _vp, _c_i32, _c_i32, _vp, _vp]),
    "f12_aux_w_column": (_c_i32, [_c_dbl, _c_i32, _c_i32, _c_i32, _c_dbl, _P(_c_dbl)]),
    "f12_stream_status": (_c_i32, [_vp]),
    "f12_sph_coefficients": (_c_i32, [_c_i32, _P(_c_dbl)]),
    "f12_quartet_offsets_sph": (_c_i32, [_vp, _P(_c_i64)]),
    "f12_cart_to_sph": (_c_i32, [_vp, _c_i64, _c_i64, _vp, _vp, _c_i64, _vp]),
    "f12_hermite_hobson": (_c_i32, [_vp, _vp, _c_i64, _c_i32, _vp, _vp]),
    "f12_digest": (_c_i32, [_vp, _c_i64, _c_i64, _vp, _vp, _vp]),
    "f12_strerror": (ctypes.c_char_p, [_c_i32]),
}
for _name, (_res, _args) in EXPORTS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class F12Error(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {_lib.f12_strerror(status).decode()} (status {status})")
        self.status = status


def _check(status, where):
    if status != 0:
        raise F12Error(status, where)


def _dptr(a):
    return a.ctypes.data_as(_P(_c_dbl))


def _stream_ptr(stream):
    if stream is None:
        import torch
        return _vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _vp(stream)
    return _vp(stream.cuda_stream)


class Basis:
    """Contracted Cartesian shells on centres (copied into the library)."""

    def __init__(self, centers, shell_table, exps, coefs):
        centers = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
        st = np.ascontiguousarray(shell_table, dtype=np.int32).reshape(-1, 4)
        self.exps = np.ascontiguousarray(exps, dtype=np.float64)
        self.coefs = np.ascontiguousarray(coefs, dtype=np.float64)
        shells = (ShellC * len(st))(*[ShellC(*map(int, row)) for row in st])
        self.shell_l = st[:, 0].copy()
        self.handle = _vp()
        _check(_lib.f12_basis_create(len(centers), _dptr(centers), len(st), shells, len(self.exps),
                                     _dptr(self.exps), _dptr(self.coefs), ctypes.byref(self.handle)),
               "f12_basis_create")

    @staticmethod
    def from_shells(shells):
        from synth import shells_to_arrays
        return Basis(*shells_to_arrays(shells))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.f12_basis_destroy(h)
        self.handle = None


class Pairs:
    def __init__(self, basis, ordered, stream=None):
        self.basis = basis
        self.handle = _vp()
        _check(_lib.f12_pairs_build(basis.handle, int(ordered), _stream_ptr(stream), ctypes.byref(self.handle)),
               "f12_pairs_build")
        nsp, npp = _c_i64(), _c_i64()
        _lib.f12_pairs_count(self.handle, ctypes.byref(nsp), ctypes.byref(npp))
        self.n_shell_pairs, self.n_prim_pairs = nsp.value, npp.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.f12_pairs_destroy(h)
        self.handle = None


class Kernel:
    """Kernel k_i of class `cls` for factors f (and fp for I4/I6)."""

    def __init__(self, cls, f=None, fp=None):
        self.cls = int(cls)
        self.handle = _vp()
        fc = Factor.of(f) if f is not None else Factor(0, 0, 0, 1, 0, 0)
        fpc = Factor.of(fp) if fp is not None else None
        _check(_lib.f12_kernel_create(self.cls, ctypes.byref(fc), ctypes.byref(fpc) if fpc else None,
                                      ctypes.byref(self.handle)), "f12_kernel_create")

    @staticmethod
    def from_terms(cls, f_terms, fp_terms=None):
        """f12_kernel_create_terms: factors given as (c, alpha, b, g) rows of
        f(r) = sum c r^alpha exp(b r - g r^2)."""
        k = Kernel.__new__(Kernel)
        k.cls = int(cls)
        k.handle = _vp()
        ft = np.ascontiguousarray(f_terms, dtype=np.float64).reshape(-1, 4)
        fpt = None if fp_terms is None else np.ascontiguousarray(fp_terms, dtype=np.float64).reshape(-1, 4)
        _check(_lib.f12_kernel_create_terms(k.cls, len(ft), _dptr(ft), 0 if fpt is None else len(fpt),
                                            None if fpt is None else _dptr(fpt), ctypes.byref(k.handle)),
               "f12_kernel_create_terms")
        return k

    def terms(self):
        n = _c_i32()
        _check(_lib.f12_kernel_terms(self.handle, ctypes.byref(n), None, 0), "f12_kernel_terms")
        out = np.zeros(4 * n.value)
        _check(_lib.f12_kernel_terms(self.handle, ctypes.byref(n), _dptr(out), n.value), "f12_kernel_terms")
        return out.reshape(-1, 4)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.f12_kernel_destroy(h)
        self.handle = None


class Quartets:
    def __init__(self, handle, nq, nout, bra, ket, cls):
        self.handle, self.n_quartets, self.n_out, self.bra, self.ket, self.cls = handle, nq, nout, bra, ket, cls

    @staticmethod
    def build(bra, ket, cls, screen_tol=0.0, screen_kernel=None, stream=None):
        h, nq, nout = _vp(), _c_i64(), _c_i64()
        _check(_lib.f12_quartets_build(bra.handle, ket.handle, int(cls), float(screen_tol),
                                       screen_kernel.handle if screen_kernel else None, _stream_ptr(stream),
                                       ctypes.byref(h), ctypes.byref(nq), ctypes.byref(nout)),
               "f12_quartets_build")
        return Quartets(h, nq.value, nout.value, bra, ket, cls)

    @staticmethod
    def build_device(bra, ket, cls, screen_tol=0.0, screen_kernel=None, stream=None):
        """f12_quartets_build_device: the same list, generated, screened and sorted on the GPU."""
        h, nq, nout = _vp(), _c_i64(), _c_i64()
        _check(_lib.f12_quartets_build_device(bra.handle, ket.handle, int(cls), float(screen_tol),
                                              screen_kernel.handle if screen_kernel else None,
                                              _stream_ptr(stream), ctypes.byref(h), ctypes.byref(nq),
                                              ctypes.byref(nout)), "f12_quartets_build_device")
        return Quartets(h, nq.value, nout.value, bra, ket, cls)

    @staticmethod
    def from_list(bra, ket, cls, quads):
        q = np.ascontiguousarray(quads, dtype=np.int32).reshape(-1, 4)
        h, nout = _vp(), _c_i64()
        _check(_lib.f12_quartets_from_list(bra.handle, ket.handle, int(cls), q.ctypes.data_as(_P(_c_i32)),
                                           len(q), ctypes.byref(h), ctypes.byref(nout)), "f12_quartets_from_list")
        return Quartets(h, len(q), nout.value, bra, ket, cls)

    def offsets(self):
        o = np.zeros(self.n_quartets + 1, dtype=np.int64)
        _check(_lib.f12_quartet_offsets(self.handle, o.ctypes.data_as(_P(_c_i64))), "f12_quartet_offsets")
        return o

    def quads(self):
        q = np.zeros((self.n_quartets, 4), dtype=np.int32)
        _check(_lib.f12_quartet_list(self.handle, q.ctypes.data_as(_P(_c_i32))), "f12_quartet_list")
        return q

    def groups(self):
        """Shape groups of the public order: (starts int64[n+1], ls int32[n, 4])."""
        n = _c_i32()
        _check(_lib.f12_quartet_groups(self.handle, ctypes.byref(n), None, None, 0), "f12_quartet_groups")
        starts = np.zeros(n.value + 1, dtype=np.int64)
        ls = np.zeros((n.value, 4), dtype=np.int32)
        _check(_lib.f12_quartet_groups(self.handle, ctypes.byref(n), starts.ctypes.data_as(_P(_c_i64)),
                                       ls.ctypes.data_as(_P(_c_i32)), n.value), "f12_quartet_groups")
        if n.value == 0:
            starts[0] = 0
        return starts, ls

    def n_prim(self):
        n = _c_i64()
        _check(_lib.f12_quartets_prim_count(self.handle, ctypes.byref(n)), "f12_quartets_prim_count")
        return n.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.f12_quartets_destroy(h)
        self.handle = None


class Batch:
    """f12_batch_create: one class's quartets from several lists in one captured
    HIP graph (concurrent branches, tuned persistent contraction grids).
    parts: list of (Quartets, q_begin, q_end, out tensor)."""

    def __init__(self, parts, kernel, nbranch=4, tune=True, tune_path=None, stream=None):
        import torch
        n = len(parts)
        self.parts, self.kernel = parts, kernel
        for (_, _, _, out) in parts:
            assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        lists = (_vp * n)(*[p[0].handle for p in parts])
        qb = (_c_i64 * n)(*[int(p[1]) for p in parts])
        qe = (_c_i64 * n)(*[int(p[2]) for p in parts])
        outs = (_vp * n)(*[_vp(p[3].data_ptr()) for p in parts])
        caps = (_c_i64 * n)(*[p[3].numel() for p in parts])
        self.handle = _vp()
        _check(_lib.f12_batch_create(n, lists, qb, qe, kernel.handle, outs, caps, int(nbranch), int(bool(tune)),
                                     tune_path.encode() if tune_path else None, _stream_ptr(stream),
                                     ctypes.byref(self.handle)), "f12_batch_create")
        a, b, c = _c_i64(), _c_i64(), _c_i64()
        _check(_lib.f12_batch_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "f12_batch_info")
        self.n_quartets, self.n_prim, self.n_chunks = a.value, b.value, c.value

    def launch(self, stream=None):
        _check(_lib.f12_batch_launch(self.handle, _stream_ptr(stream)), "f12_batch_launch")

    def grid(self, lab, lcd, i5):
        g = _c_i64()
        _check(_lib.f12_batch_grid(self.handle, int(lab), int(lcd), int(i5), ctypes.byref(g)), "f12_batch_grid")
        return g.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.f12_batch_destroy(h)
        self.handle = None


def eval_into(quartets, kernel, out, q_begin=0, q_end=None, stream=None):
    """Enqueue f12_eval writing blocks [q_begin, q_end) into the float64 CUDA tensor `out`."""
    import torch
    if q_end is None:
        q_end = quartets.n_quartets
    assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
    _check(_lib.f12_eval(quartets.handle, kernel.handle, int(q_begin), int(q_end), _vp(out.data_ptr()),
                         out.numel(), _stream_ptr(stream)), "f12_eval")
    return out


def eval_grad(quartets, kernel, direction, out, q_begin=0, q_end=None, stream=None):
    """Enqueue f12_eval_grad: d/dA_direction of the blocks (A the bra's first centre)."""
    import torch
    if q_end is None:
        q_end = quartets.n_quartets
    assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
    _check(_lib.f12_eval_grad(quartets.handle, kernel.handle, int(direction), int(q_begin), int(q_end),
                              _vp(out.data_ptr()), out.numel(), _stream_ptr(stream)), "f12_eval_grad")
    return out


def eval_sets(quartets, kernels, out, q_begin=0, q_end=None, stream=None):
    """Enqueue f12_eval_sets: one kernel per factor set, output [set][quartet block]."""
    import torch
    if q_end is None:
        q_end = quartets.n_quartets
    assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
    arr = (_vp * len(kernels))(*[k.handle for k in kernels])
    _check(_lib.f12_eval_sets(quartets.handle, arr, len(kernels), int(q_begin), int(q_end), _vp(out.data_ptr()),
                              out.numel(), _stream_ptr(stream)), "f12_eval_sets")
    return out


FP64, SPLIT_FP32 = 0, 1
ENONFINITE = -7


def sph_coefficients(l):
    """f12_sph_coefficients: (2l+1, ncart(l)) matrix of the real solid harmonics."""
    nc = (l + 1) * (l + 2) // 2
    out = np.zeros((2 * l + 1) * nc)
    _check(_lib.f12_sph_coefficients(int(l), _dptr(out)), "f12_sph_coefficients")
    return out.reshape(2 * l + 1, nc)


def hermite_hobson(A, X, L, stream=None):
    """f12_hermite_hobson: R_tuv (Hermite order) from A (np, L+1) and X (np, 3), CUDA float64."""
    import torch
    A = A.contiguous(); X = X.contiguous()
    np_ = A.shape[0]
    R = torch.empty((np_, (L + 1) * (L + 2) * (L + 3) // 6), dtype=torch.float64, device=A.device)
    _check(_lib.f12_hermite_hobson(_vp(A.data_ptr()), _vp(X.data_ptr()), np_, int(L), _vp(R.data_ptr()),
                                   _stream_ptr(stream)), "f12_hermite_hobson")
    return R


def offsets_sph(quartets):
    o = np.zeros(quartets.n_quartets + 1, dtype=np.int64)
    _check(_lib.f12_quartet_offsets_sph(quartets.handle, o.ctypes.data_as(_P(_c_i64))), "f12_quartet_offsets_sph")
    return o


def cart_to_sph(quartets, cart, out, q_begin=0, q_end=None, stream=None):
    """Enqueue f12_cart_to_sph: Cartesian blocks (as eval_into writes them) to solid-harmonic blocks."""
    import torch
    if q_end is None:
        q_end = quartets.n_quartets
    assert cart.dtype == torch.float64 and cart.is_cuda and out.dtype == torch.float64 and out.is_cuda
    _check(_lib.f12_cart_to_sph(quartets.handle, int(q_begin), int(q_end), _vp(cart.data_ptr()),
                                _vp(out.data_ptr()), out.numel(), _stream_ptr(stream)), "f12_cart_to_sph")
    return out


def digest(quartets, out, d_digest, q_begin=0, q_end=None, stream=None):
    """Enqueue f12_digest: add the 64-bit digest of blocks [q_begin, q_end) in `out` (laid out as
    eval_into writes the range) to the int64 CUDA scalar `d_digest` (wrapping, mod 2^64)."""
    import torch
    if q_end is None:
        q_end = quartets.n_quartets
    assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
    assert d_digest.dtype == torch.int64 and d_digest.is_cuda
    _check(_lib.f12_digest(quartets.handle, int(q_begin), int(q_end), _vp(out.data_ptr()),
                           _vp(d_digest.data_ptr()), _stream_ptr(stream)), "f12_digest")
    return d_digest


def eval_precision(quartets, kernel, out, precision, q_begin=0, q_end=None, stream=None):
    """Enqueue f12_eval_precision: FP64 (0) or the split-FP32 ket transform (1)."""
    import torch
    if q_end is None:
        q_end = quartets.n_quartets
    assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
    _check(_lib.f12_eval_precision(quartets.handle, kernel.handle, int(q_begin), int(q_end),
                                   _vp(out.data_ptr()), out.numel(), int(precision), _stream_ptr(stream)),
           "f12_eval_precision")
    return out


def eval_noalloc(quartets, kernel, out, q_begin=0, q_end=None, stream=None):
    """Enqueue f12_eval_noalloc (no device allocation; fixed library scratch)."""
    import torch
    if q_end is None:
        q_end = quartets.n_quartets
    assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
    _check(_lib.f12_eval_noalloc(quartets.handle, kernel.handle, int(q_begin), int(q_end),
                                 _vp(out.data_ptr()), out.numel(), _stream_ptr(stream)), "f12_eval_noalloc")
    return out


def eval_stage(quartets, kernel, out, q_begin, q_end, stage, stream=None):
    """Enqueue one launch of f12_eval (stage 1: radial derivatives, stage 2:
    contraction) for a range inside one angular-momentum group."""
    import torch
    assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
    _check(_lib.f12_eval_stage(quartets.handle, kernel.handle, int(q_begin), int(q_end),
                               _vp(out.data_ptr()), out.numel(), int(stage), _stream_ptr(stream)),
           "f12_eval_stage")
    return out


def scratch_prims(quartets):
    n = _c_i64()
    _check(_lib.f12_quartets_scratch_prims(quartets.handle, ctypes.byref(n)), "f12_quartets_scratch_prims")
    return int(n.value)


def stream_status(stream=None):
    _check(_lib.f12_stream_status(_stream_ptr(stream)), "f12_stream_status")


def aux_radial(kernel, p, q, R, L, stream=None, route=0):
    """A_n, n = 0..L, on the device for (p, q, R) triples; returns a float64 CUDA tensor (L+1, n)."""
    import torch
    dev = torch.device("cuda")
    p = torch.as_tensor(p, dtype=torch.float64, device=dev).contiguous()
    q = torch.as_tensor(q, dtype=torch.float64, device=dev).contiguous()
    R = torch.as_tensor(R, dtype=torch.float64, device=dev).contiguous()
    n = p.numel()
    A = torch.empty((L + 1) * n, dtype=torch.float64, device=dev)
    _check(_lib.f12_aux_radial(kernel.handle, n, _vp(p.data_ptr()), _vp(q.data_ptr()), _vp(R.data_ptr()),
                               int(L), int(route), _vp(A.data_ptr()), _stream_ptr(stream)), "f12_aux_radial")
    return A.view(L + 1, n)


def aux_w_column(alpha0, is_int, m_lo, m_hi, x):
    """Host-side table builder's W_a(x), a = alpha0 + m_lo..m_hi (numpy)."""
    out = np.zeros(m_hi - m_lo + 1)
    _check(_lib.f12_aux_w_column(float(alpha0), int(is_int), int(m_lo), int(m_hi), float(x), _dptr(out)),
           "f12_aux_w_column")
    return out
