"""CPU oracle for the strided-batched matrix-vector product.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
module; only the tests and the benchmark use it.  It shares no code with the
GPU path.

The operation is the per-frequency product of phase 3 (Section 2.4) in its
standalone form (Section 3.1.1): for every matrix of a batch,
``y_b = alpha op(A_b) x_b + beta y_b`` with ``op`` the identity (N), the
transpose (T) or the conjugate transpose (C), and BLAS's column-major
storage.  Storage convention (the one the library's Python binding uses):
``A_cols[b, j, :m]`` is column ``j`` of the ``m x n`` matrix ``A_b``.  The
arithmetic is float64 / complex128, one library matrix product per batch
entry, nothing reordered.

Pins (checked by ``tests/test_sbgemv_oracle.py`` against things other than
this module): identity, diagonal, permutation and all-ones matrices (closed
forms), the adjoint identity ``<A x, y> = <x, A^H y>`` linking op N to op C,
op C equal to op T on real data and to ``conj(A^T conj(x))`` on complex data,
linearity in alpha and beta, and ``y`` left unread when ``beta`` is zero.
"""
from __future__ import annotations

import numpy as np


def sbgemv(op: str, A_cols: np.ndarray, m: int, x: np.ndarray, alpha=1.0, beta=0.0,
           y: np.ndarray | None = None) -> np.ndarray:
    """``alpha op(A_b) x_b + beta y_b`` for every ``b`` (see the module docstring)."""
    if op not in ("N", "T", "C"):
        raise ValueError("op must be 'N', 'T' or 'C'")
    cplx = np.iscomplexobj(A_cols) or np.iscomplexobj(x) or (y is not None and np.iscomplexobj(y))
    wide = np.complex128 if cplx else np.float64
    A = np.asarray(A_cols, dtype=wide)[:, :, :m]        # A[b, j, i] = A_b(i, j)
    xb = np.asarray(x, dtype=wide)
    out = []
    for b in range(A.shape[0]):
        Ab = A[b].T                                      # m x n
        if op == "N":
            r = Ab @ xb[b]
        elif op == "T":
            r = Ab.T @ xb[b]
        else:
            r = Ab.conj().T @ xb[b]
        out.append(r)
    r = alpha * np.stack(out)
    if beta != 0:
        r = r + beta * np.asarray(y, dtype=wide)
    return r
