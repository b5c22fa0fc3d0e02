"""MI355X-native CTU + PPMC + exact-Riemann timestep for the 3D Euler equations.

The compute path is the HIP library ``libctu.so`` (C ABI declared in include/ctu.h); the
Python layer is marshalling only.  Submodules:

* :mod:`.ctu` -- ctypes binding over the C ABI (``Grid``, ``Batch``); needs the built library
  and a GPU, and raises if either is missing.
* :mod:`.workloads` -- seeded synthetic initial conditions.
"""
import importlib

__all__ = ["ctu", "workloads"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
