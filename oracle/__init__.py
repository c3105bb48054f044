"""CPU oracle (test infrastructure only; never imported by the product path).

Parity: every function is pinned by ``tests/test_oracle_pins.py`` (the
Toeplitz matvec) or ``tests/test_sbgemv_oracle.py`` (the batched product).
"""
from .toeplitz import (adjoint, adjoint_entries, exact_dot, forward,  # noqa: F401
                       forward_entries, hessian_data_space, relative_l2, spectrum)
from .sbgemv import sbgemv  # noqa: F401
