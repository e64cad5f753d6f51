"""MI355X (gfx950) implementation of the incremental-stencil WENO finite-volume
right-hand side for compressible two-phase flow (arXiv:1707.00592).

The compute path lives in the HIP library ``libisweno.so`` (sources under
``csrc/``, C ABI in ``include/isweno.h``); ``isweno`` is its thin ctypes
binding.  ``workloads`` builds seeded synthetic inputs and is importable
without the library.
"""
import importlib

__all__ = ["isweno", "workloads"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
