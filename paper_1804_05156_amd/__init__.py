"""MI355X (gfx950) library for linear finite element assembly of the Poisson problem.

The compute path lives in the HIP C-ABI library ``libfemhip.so`` (sources under
``csrc/``, declarations in ``include/femhip.h``); :mod:`.femhip` is its thin ctypes
binding, :mod:`.batch` batches many meshes into one graph launch (with the
autotuner of its persistent solve), and :mod:`.meshgen` builds seeded synthetic
meshes.
"""
import importlib

__all__ = ["femhip", "batch", "meshgen"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
