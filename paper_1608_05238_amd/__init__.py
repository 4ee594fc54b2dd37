"""MI355X-native forward/adjoint radiance Monte Carlo with a harmonic angular tally.

Method: Hochuli, Powell, Arridge & Cox, "Quantitative photoacoustic tomography
using forward and adjoint Monte Carlo models of radiance" (arXiv:1608.05238).
The compute lives in librmc.so (HIP, gfx950) behind the C ABI of
include/mcrad.h; ``rmc`` is its Python binding.
"""
from . import _lib  # noqa: F401

__all__ = ["rmc", "autograd", "_lib"]


def __getattr__(name):
    if name in ("rmc", "autograd"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
