"""MI355X-native total least squares by Rayleigh quotient iteration.

RQI-PCGTLS and its mixed-precision variant RQI-PCGTLS-MP (Oktay & Carson,
"Mixed Precision Rayleigh Quotient Iteration for Total Least Squares
Problems"): hand-written CDNA4 HIP kernels behind the C ABI of
``include/tls.h`` (library ``lib/libtls.so``), with a thin ctypes binding in
:mod:`paper_2305_19028_amd.tls`.
"""
from . import tls  # noqa: F401

__all__ = ["tls"]
