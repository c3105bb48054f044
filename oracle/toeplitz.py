"""CPU oracle for the block lower-triangular Toeplitz matvec and its adjoint.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
module; only the tests, the package smoke check and the benchmark's CPU
baseline use it.  It shares no code with the GPU path.

Everything here is plain float64 NumPy written from the definitions in the
paper (Section 2.3, the block matrix of eq. (ShiftInvariance); Section 2.4 for
the adjoint and the Fourier-side objects).  Notation, 0-based: the first block
column is ``F_0 .. F_{Nt-1}`` (the paper's ``F_{11} .. F_{Nt,1}``), stored
``F[t][r][c]`` with lag ``t``, sensor row ``r < Nd`` and parameter column
``c < Nm``.  Parameter vectors are ``m[j][c]`` and data vectors ``d[i][r]``,
optionally with leading batch axes.

Pins (checked by ``tests/test_oracle_pins.py`` against things other than this
module): the dense block matrix assembled as printed in eq. (ShiftInvariance),
the adjoint identity, identity/delay blocks, the scalar case as a truncated
causal convolution (``numpy.convolve``), the geometric kernel's recursion,
``Nt = 1`` as a plain matrix-vector product, time-shift invariance, the
spectrum against closed forms and ``numpy.fft.rfft``, and the data-space
Hessian against the dense ``A A^T``, its symmetry and positive
semidefiniteness.
"""
from __future__ import annotations

import math

import numpy as np


def _check(F: np.ndarray) -> tuple[int, int, int]:
    if F.ndim != 3:
        raise ValueError("F must be [Nt][Nd][Nm]")
    return F.shape


def forward(F: np.ndarray, m: np.ndarray) -> np.ndarray:
    """``d_i = sum_{j<=i} F_{i-j} m_j`` for ``i = 0..Nt-1``.

    This is the product with the block lower-triangular Toeplitz matrix of
    eq. (ShiftInvariance), written as a sum over lags ``t = i - j``: every lag
    contributes ``F_t m_{i-t}`` to each output block ``i >= t``.  Each
    per-lag block product is a library matmul; nothing else is reordered.
    ``m`` is ``[..., Nt, Nm]``; the result is ``[..., Nt, Nd]``.
    """
    Nt, Nd, Nm = _check(F)
    m = np.asarray(m, dtype=np.float64)
    if m.shape[-2:] != (Nt, Nm):
        raise ValueError(f"m has shape {m.shape}, expected [..., {Nt}, {Nm}]")
    d = np.zeros(m.shape[:-2] + (Nt, Nd))
    for t in range(Nt):
        d[..., t:, :] += m[..., : Nt - t, :] @ F[t].T
    return d


def adjoint(F: np.ndarray, d: np.ndarray) -> np.ndarray:
    """``m_j = sum_{i>=j} F_{i-j}^T d_i`` for ``j = 0..Nt-1``.

    The adjoint of the real operator is its transpose (Section 2.1 defines the
    adjoint map; Section 2.4 applies it with the conjugate transpose in
    Fourier space, which is the transpose for real ``F``).  ``d`` is
    ``[..., Nt, Nd]``; the result is ``[..., Nt, Nm]``.
    """
    Nt, Nd, Nm = _check(F)
    d = np.asarray(d, dtype=np.float64)
    if d.shape[-2:] != (Nt, Nd):
        raise ValueError(f"d has shape {d.shape}, expected [..., {Nt}, {Nd}]")
    m = np.zeros(d.shape[:-2] + (Nt, Nm))
    for t in range(Nt):
        m[..., : Nt - t, :] += d[..., t:, :] @ F[t]
    return m


def hessian_data_space(F: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Data-space Hessian action ``F Gamma F^T x`` with ``Gamma = I``.

    The outer-loop problems of Section 3.2 assemble the dense data-space
    Hessian ``F Gamma F^*`` column by column (``Nd Nt`` actions); with the
    identity prior each action is the adjoint product followed by the forward
    one, by definition.  ``x`` is ``[..., Nt, Nd]``; so is the result.
    """
    return forward(F, adjoint(F, x))


# --- single entries, computed exactly and rounded once ----------------------

_SPLIT = 134217729.0  # 2**27 + 1, Veltkamp's splitting constant for float64


def _two_product(a: np.ndarray, b: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Dekker's exact product ``a*b = p + e`` (Dekker 1971), no FMA needed."""
    ca = _SPLIT * a
    ah = ca - (ca - a)
    al = a - ah
    cb = _SPLIT * b
    bh = cb - (cb - b)
    bl = b - bh
    p = a * b
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def exact_dot(a: np.ndarray, b: np.ndarray) -> float:
    """Correctly rounded ``sum(a*b)``: exact products, then ``math.fsum``."""
    p, e = _two_product(np.ravel(a).astype(np.float64), np.ravel(b).astype(np.float64))
    return math.fsum(np.concatenate([p, e]).tolist())


def forward_entries(F: np.ndarray, m: np.ndarray, ii, rr, exact: bool = True) -> np.ndarray:
    """Entries ``d_i[r] = sum_{j<=i} sum_c F_{i-j}[r, c] m_j[c]`` one by one.

    ``m`` is ``[Nt, Nm]`` (one right-hand side).  With ``exact`` the value is
    the correctly rounded float64 of the exact sum; otherwise a plain dot.
    """
    Nt, Nd, Nm = _check(F)
    out = np.empty(len(ii))
    for n, (i, r) in enumerate(zip(ii, rr)):
        a = F[i::-1, r, :]          # lags i, i-1, .., 0 pair with m_0 .. m_i
        b = m[: i + 1, :]
        out[n] = exact_dot(a, b) if exact else float(np.dot(a.ravel(), b.ravel()))
    return out


def adjoint_entries(F: np.ndarray, d: np.ndarray, jj, cc, exact: bool = True) -> np.ndarray:
    """Entries ``m_j[c] = sum_{i>=j} sum_r F_{i-j}[r, c] d_i[r]`` one by one."""
    Nt, Nd, Nm = _check(F)
    out = np.empty(len(jj))
    for n, (j, c) in enumerate(zip(jj, cc)):
        a = F[: Nt - j, :, c]       # lags 0 .. Nt-1-j pair with d_j .. d_{Nt-1}
        b = d[j:, :]
        out[n] = exact_dot(a, b) if exact else float(np.dot(a.ravel(), b.ravel()))
    return out


# --- Fourier-side objects (Section 2.4, Section 3.2.1) ----------------------

def spectrum(F: np.ndarray, L: int | None = None, ks=None) -> np.ndarray:
    """``Fhat_k = sum_{t<Nt} F_t exp(-2 pi i k t / L)`` by the DFT definition.

    This is the transform of the zero-padded first block column (padded to
    ``L = 2 Nt`` by default) that block-diagonalises the block-circulant
    embedding; bins ``k = 0 .. L/2`` are returned (the rest follow by
    conjugate symmetry because ``F`` is real).  The exponent ``k t`` is
    reduced modulo ``L`` in integers and the twiddles are evaluated in long
    double.  Returns complex128 ``[len(ks)][Nd][Nm]``.
    """
    Nt, Nd, Nm = _check(F)
    L = 2 * Nt if L is None else int(L)
    ks = np.arange(L // 2 + 1) if ks is None else np.asarray(ks)
    t = np.arange(Nt)
    e = np.outer(ks, t) % L
    ang = (2 * np.pi * e.astype(np.longdouble)) / L
    W = (np.cos(ang) - 1j * np.sin(ang)).astype(np.complex128)  # [k][t]
    return (W @ F.reshape(Nt, Nd * Nm)).reshape(len(ks), Nd, Nm)


def relative_l2(y: np.ndarray, ref: np.ndarray) -> float:
    """``||y - ref||_2 / ||ref||_2`` over the whole output (the paper's relative error)."""
    cplx = np.iscomplexobj(y) or np.iscomplexobj(ref)
    y = np.asarray(y, dtype=np.complex128 if cplx else np.float64)
    ref = np.asarray(ref, dtype=np.complex128 if cplx else np.float64)
    den = float(np.linalg.norm(ref.ravel()))
    num = float(np.linalg.norm((y - ref).ravel()))
    return num / den if den > 0 else num
