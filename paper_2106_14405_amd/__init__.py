"""MI355X-native batched rigid-body step (HIP for gfx950) behind a C ABI.

The physics runs only in librbsim.so; this package marshals arguments and
lets torch own device memory and streams.  Importing `Sim` requires the
built library and raises otherwise: there is no CPU fallback.
"""
from . import scenes  # noqa: F401
from ._lib import COLD, JACOBI, LEARNED, PGS, PREV, SimError  # noqa: F401


def __getattr__(name):
    if name == "Sim":
        from .sim import Sim
        return Sim
    raise AttributeError(name)
