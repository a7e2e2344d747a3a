"""Differentiable direct N-body engine for one AMD Instinct MI355X (gfx950).

The compute lives in libdnb.so (HIP kernels behind the C ABI of include/dnb.h);
this package only binds it.  Importing the package does not load the library;
the first Context does, and fails loudly if it has not been built.
"""
from .units import G, TIME_UNIT_MYR, gyr, myr  # noqa: F401

__all__ = ["Context", "Potential", "G", "TIME_UNIT_MYR", "gyr", "myr"]


def __getattr__(name):
    if name in ("Context", "Potential"):
        from . import engine
        return getattr(engine, name)
    raise AttributeError(name)
