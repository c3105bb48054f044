"""MI355X (gfx950) FFT-based block lower-triangular Toeplitz matvec.

``Operator(F).matvec(m)`` computes ``d = F m`` and ``.rmatvec(d)`` computes
``F^T d`` through the HIP library ``libftm.so`` (C ABI in ``include/ftm.h``).
There is no CPU fallback: without the built library every call raises.
"""
from ._lib import BF16, F16, F32, F64, FtmError  # noqa: F401
from .api import Operator, Precision, Server, round_values, sbgemv  # noqa: F401
