"""Convolution gridding of single-dish spectra on AMD Instinct MI355X.

The library (``libhegrid.so``, C ABI in ``include/hegrid.h``) bins, sorts and
searches the samples once per field and then grids any number of channels
with hand-written gfx950 kernels.  ``api`` is its ctypes binding; ``synth``
draws seeded synthetic observations.  Nothing is loaded at import time.
"""
__all__ = ["api", "synth"]


def __getattr__(name):
    if name in ("api", "synth", "build"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    if name in ("Plan", "ang2pix_ring", "HegridError"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
