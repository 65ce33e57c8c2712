"""MI355X (gfx950) local SpGEMM of the sparsity-aware 1D algorithm.

C_i = A * B_i for one column partition: H_i, Alg. 2 block selection, the
gather of A~, and a column-wise Gustavson product (flop binning, symbolic
count, scan, numeric) in hand-written HIP kernels behind the C ABI of
include/spgemm.h.  This package is the thin Python binding.
"""

from ._lib import SpgemmError, load  # noqa: F401
from . import tune  # noqa: F401
from .api import (DeviceCsc, HostCsc, Plan, SpGEMM, Batch, batched, default_tuning, spgemm,  # noqa: F401
                  tuning, galerkin_chain, BIN_NAMES, row_block, sum_parts, outer_product)

__all__ = ["DeviceCsc", "HostCsc", "Plan", "SpGEMM", "Batch", "batched", "SpgemmError", "default_tuning",
           "spgemm", "tuning", "galerkin_chain", "load", "BIN_NAMES", "tune", "row_block",
           "sum_parts", "outer_product"]
