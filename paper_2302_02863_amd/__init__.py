"""MI355X-native library for the decomposed variable-order fractional stiffness operator.

The product is libfpde.so (HIP kernels for gfx950 behind the C ABI in
include/fpde.h); this package only marshals arguments to it.
"""
from ._abi import (FpdeError, PART_ALL, PART_B, PART_M, PART_KNEAR, PART_KFAR, PART_FP64, PREC_FP64,  # noqa: F401
                   PREC_MIXED, lib)
from .operator import Operator, gauss_legendre, opts_struct  # noqa: F401
