"""MI355X-native spectral kinetic simulation of the ideal Multipole Resonance Probe.

The simulation itself lives in the HIP library built from csrc/mrpsim.hip
(C ABI: include/mrpsim.h); `sim` is its ctypes binding and `workload` holds
the seeded synthetic inputs.
"""
from . import workload  # noqa: F401

__all__ = ["workload", "sim"]


def __getattr__(name):
    if name == "sim":
        import importlib

        return importlib.import_module(__name__ + ".sim")
    raise AttributeError(name)
