"""MI355X-native BDIM projection solver step (WaterLily.jl method, arXiv 2407.16032).

The compute path is the HIP library ``libwlmi.so`` (hand-written gfx950
kernels behind the C ABI of include/wlmi.h); this package only marshals
arguments.  Importing ``Simulation`` loads the library and raises if it has
not been built.
"""
from ._lib import WlError, load  # noqa: F401


def __getattr__(name):
    if name == "Simulation":
        from .sim import Simulation
        return Simulation
    raise AttributeError(name)


__all__ = ["Simulation", "WlError", "load"]
