"""MI355X-native (gfx950) relativistic lattice Boltzmann step on a Gaussian
quadrature (massless particles, third order, 48 populations per site).

The compute path is the in-tree HIP library ``librlbm.so`` behind the C ABI
of ``include/rlbm.h``; this package only marshals arguments to it.  Importing
``Lattice`` or calling any function loads the library and raises if it has
not been built: there is no CPU fallback.
"""
from ._binding import (EDGE, F16DEV, F32, F64, Batch, Lattice, NotFound, RlbmError, UNet, Unstable, check,
                       conv3x3_backward_data, conv3x3_backward_weight, conv3x3_forward, force_matrices, lib, mj_moment,
                       quadrature, quadrature_massive, quadrature_massless)

__all__ = ["Lattice", "Batch", "UNet", "conv3x3_forward", "conv3x3_backward_data", "conv3x3_backward_weight",
           "RlbmError", "Unstable", "NotFound", "quadrature", "force_matrices", "mj_moment", "quadrature_massive",
           "quadrature_massless", "lib", "check", "F64", "F32", "F16DEV", "EDGE"]
