"""MI355X (gfx950) tensor-product operators for hexahedral spectral elements.

BP1.0 (mass), BP3.5 (collocated stiffness) and BP3.0 (de-aliased stiffness) of
arXiv 1711.00903 as hand-written HIP kernels behind the C ABI of
``include/fem.h`` (``libfem.so``); :mod:`.fem` is the ctypes binding and
:mod:`.mesh` keeps a mesh's tables and geometric data on the device.
"""
from . import fem  # noqa: F401

__all__ = ["fem"]
