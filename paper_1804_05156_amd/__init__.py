"""MI355X (gfx950) library for linear finite element assembly of the Poisson problem.

The compute path lives in the HIP C-ABI library ``libfemhip.so`` (sources under
``csrc/``, declarations in ``include/femhip.h``); :mod:`.femhip` is its thin ctypes
binding and :mod:`.meshgen` builds seeded synthetic meshes.
"""
import importlib

__all__ = ["femhip", "meshgen"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
