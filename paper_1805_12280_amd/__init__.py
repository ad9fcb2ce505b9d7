"""MI355X-native FT convolution (FDAS) hot path: overlap-save FDFIR over a
template bank with a |y|^2 power plane, and a direct TDFIR baseline.

The compute runs in hand-written HIP kernels inside libfdas.so; `Plan` is a
thin ctypes binding over its C ABI (include/fdas.h).  The library is loaded
on first use, and using it without the built library raises.
"""

__all__ = ["Plan", "FdasError", "load_library"]


def __getattr__(name):
    if name in ("Plan", "FdasError", "load_library", "PlanInfo"):
        from . import fdas
        return getattr(fdas, name)
    raise AttributeError(name)
