"""MI355X (gfx950) library for the explicit interfacial system C u = r of the
overlapping-circle stochastic substructuring method (arXiv 2311.08946).

The compute path is the HIP library ``libpdd.so`` (C ABI in include/pdd.h);
``binding`` marshals arguments to it with ctypes and uses PyTorch only for
device memory and streams.
"""
from .binding import Cover, PddError, System, lib  # noqa: F401

__all__ = ["Cover", "System", "PddError", "lib"]
