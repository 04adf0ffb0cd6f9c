"""MI355X (gfx950) per-cell stiff chemistry integration.

The HIP library ``libchem.so`` (C ABI in include/chem.h) integrates every CFD
cell over a flow step as an adiabatic constant-pressure reactor; ``chem`` is
its ctypes binding over torch device tensors and streams.
"""
from . import chem  # noqa: F401  (fails loudly if the library is not built)
from .chem import Mechanism, ChemError  # noqa: F401
