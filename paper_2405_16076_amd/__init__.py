"""MI355X streaming randomized interpolative decomposition.

The HIP library (librid.so, built from csrc/) implements the single-pass
randomized ID of Alg. 3 with the coefficients of Alg. 4 and the NA-Hutch++
error estimate of Alg. 8 behind the C ABI of include/rid.h.  This package is
its thin Python binding.
"""
from .stream import OnlineRID, StreamBatch, StreamConfig, omega_block, sketch_columns  # noqa: F401
from ._lib import RIDError  # noqa: F401
