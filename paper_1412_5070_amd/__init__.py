"""MI355X-native evaluation of F12 two-electron integral classes I1-I6 with
the range-separated correlation factor (arXiv:1412.5070).

The computation runs in ``libf12int.so`` (HIP kernels for gfx950 behind a C
ABI, see include/f12int.h); ``f12int`` is a thin ctypes binding.
"""
from . import f12int  # noqa: F401
