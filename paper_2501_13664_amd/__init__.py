"""MI355X-native 3D multiscale discrete Radon (planes) and John (lines) transforms.

The transforms run in the HIP library ``libdrt3d.so`` (C ABI: include/drt3d.h);
this package is its Python binding (``api``) and a differentiable wrapper
(``autograd``). Importing the package does not load the library; the first call
does, and raises if it was not built.
"""
from ._lib import DRT3D_ALL, DRT3D_F32, DRT3D_I32, Drt3dError  # noqa: F401

__all__ = ["api", "autograd", "DRT3D_ALL", "DRT3D_I32", "DRT3D_F32", "Drt3dError"]
