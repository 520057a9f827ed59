"""MI355X (gfx950) library for the regularized fluctuating lattice Boltzmann
method on D3Q27 (Lauricella et al., arXiv:2507.08820).

The compute path is librflbm.so (HIP kernels behind the C interface of
include/rflbm.h); this package is its Python binding.
"""
from ._binding import (FIELDS, M_J, M_PI, M_RHO, MODEL, STORAGE, Batch, Lattice, Params, RFLBMError,
                       Stats, check, copy, load_library, make_params, rng_normals)

__all__ = ["FIELDS", "M_J", "M_PI", "M_RHO", "MODEL", "STORAGE", "Batch", "Lattice", "Params",
           "RFLBMError", "Stats", "check", "copy", "load_library", "make_params", "rng_normals"]
