"""Tiled sparse-geometry D3Q19 lattice Boltzmann for AMD Instinct MI355X (gfx950).

The compute path is the HIP library ``libtiledlbm.so`` (C ABI in
``include/lbm.h``); this package holds its thin Python binding, the
checkpointed adjoint driver and seeded input generators.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "Tiling", "Lattice", "LbmError"]


def __getattr__(name):
    if name in ("Tiling", "Lattice"):
        from . import lattice
        return getattr(lattice, name)
    if name == "LbmError":
        from ._abi import LbmError
        return LbmError
    raise AttributeError(name)
