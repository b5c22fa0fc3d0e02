"""MI355X-native CTU timestep for the 3D Euler equations: PPMC or PPMP reconstruction, the
exact or the Roe (HLLE fallback, optional H correction) Riemann solver, FP64 or FP32.

The compute path is the HIP library ``libctu.so`` (C ABI declared in include/ctu.h); the
Python layer is marshalling and scheduling only.  Submodules:

* :mod:`.ctu` -- ctypes binding over the C ABI (``Grid``, ``Batch``); needs the built library
  and a GPU, and raises if either is missing.
* :mod:`.serve` -- continuous-batching request loop (HBM-budget admission, two policies).
* :mod:`.autotune` -- tile-shape tuner for the marching sweeps.
* :mod:`.workloads` -- seeded synthetic initial conditions.
"""
import importlib

__all__ = ["ctu", "serve", "autotune", "workloads"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
