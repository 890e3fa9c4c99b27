"""gfx950 (MI355X) implementation of the explicit 1D heat-equation update of
Lee and Bhattacharya (arXiv:1510.08982), synchronous (Eq.3) and asynchronous
with bounded staleness (Eq.4), plus batched ragged rods and a discrete adjoint.

The kernels live in libheat1d.so (C ABI, include/heat1d.h).  ``abi`` is the
one-to-one ctypes binding; ``heat`` adds PyTorch device-memory helpers and the
``HeatFn`` autograd function.  Importing this package does not load the
library; the first call does, and fails loudly if it is not built.
"""
from . import abi  # noqa: F401

__all__ = ["abi", "heat"]


def __getattr__(name):
    if name == "heat":
        import importlib
        return importlib.import_module(".heat", __name__)
    raise AttributeError(name)
