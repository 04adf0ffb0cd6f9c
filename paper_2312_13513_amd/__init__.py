"""MI355X (gfx950) per-cell stiff chemistry integration.

The HIP library ``libchem.so`` (C ABI in include/chem.h) integrates every CFD
cell over a flow step as an adiabatic constant-pressure reactor; ``chem`` is
its ctypes binding over torch device tensors and streams.  Importing ``chem``
fails loudly when the library has not been built (there is no CPU fallback).
"""


def __getattr__(name):
    if name in ("Mechanism", "ChemError"):
        from . import chem
        return getattr(chem, name)
    raise AttributeError(name)
