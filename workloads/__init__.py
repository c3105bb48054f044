"""Seeded synthetic inputs for the block lower-triangular Toeplitz matvec.

This module is shared by the CPU oracle and the GPU path.  It holds only
shapes and random draws: none of the method's arithmetic lives here.

Recipe (the paper uses no dataset, all inputs are synthetic):

* ``F`` is the first block column ``F_0 .. F_{Nt-1}``, stored ``[Nt][Nd][Nm]``
  (lag-major, then sensor row, then parameter column), float64.
  Entries are iid N(0, 1), optionally multiplied by ``1/sqrt(Nm)`` and by
  ``exp(-t/decay)`` at lag ``t``.
* Parameter vectors ``m`` are ``[nrhs][Nt][Nm]`` and data vectors ``d`` are
  ``[nrhs][Nt][Nd]`` (time-outer, space-inner block-vector order), iid N(0, 1).
* Every value is nudged, if needed, so that it is *not* exactly representable
  in float32: a float32 rounding of an input must incur an error, otherwise a
  single-precision memory phase would look error free (Section 4.2.1 of the
  paper makes the same point about its inputs).
* Seeds: ``2508_10202 + 100 * config + stream`` with stream 0 = F, 1 = m,
  2 = d, 3.. = extra right-hand sides or requests.  NumPy PCG64.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 2508_10202


@dataclasses.dataclass(frozen=True)
class Shape:
    """One operator shape: ``Nt`` time blocks, each block ``Nd x Nm``."""

    Nt: int
    Nd: int
    Nm: int
    scale_by_sqrt_nm: bool = True   # multiply F by 1/sqrt(Nm)
    decay: float | None = 200.0     # multiply F_t by exp(-t/decay)

    @property
    def L(self) -> int:
        return 2 * self.Nt

    @property
    def K(self) -> int:
        return self.Nt + 1


# Named workloads (the paper's single-GPU shape is "paper").
TINY = Shape(64, 16, 256, scale_by_sqrt_nm=False, decay=None)      # plain iid F
PAPER = Shape(1000, 100, 5000)                                       # Section 4.1.2 shape
MULTI_RHS = Shape(512, 128, 4096)                                    # 64 right-hand sides
MULTI_RHS_NRHS = 64
SERVING_OPS = (Shape(256, 32, 1000), Shape(512, 64, 2000),
               Shape(1000, 100, 5000), Shape(1000, 32, 8000))

CONFIG_ID = {"tiny": 1, "paper": 2, "mixed": 3, "multi_rhs": 4, "serving": 5}


def seed_for(config: int, stream: int) -> int:
    return SEED_BASE + 100 * config + stream


def _not_f32(x: np.ndarray) -> np.ndarray:
    """Move every float32-representable value one float64 ulp away from zero."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    flat = x.reshape(-1)
    exact = flat.astype(np.float32).astype(np.float64) == flat
    if exact.any():
        idx = np.nonzero(exact)[0]
        flat[idx] = np.nextafter(flat[idx], np.copysign(np.inf, flat[idx]))
    return x


def normal(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _not_f32(rng.standard_normal(size=shape, dtype=np.float64))


def make_F(s: Shape, seed: int) -> np.ndarray:
    """First block column ``F[t][r][c]`` following the recipe above."""
    F = np.random.default_rng(seed).standard_normal(size=(s.Nt, s.Nd, s.Nm), dtype=np.float64)
    if s.scale_by_sqrt_nm or s.decay is not None:
        w = np.ones(s.Nt)
        if s.decay is not None:
            w = np.exp(-np.arange(s.Nt) / s.decay)
        if s.scale_by_sqrt_nm:
            w = w / math.sqrt(s.Nm)
        F *= w[:, None, None]
    return _not_f32(F)


def make_m(s: Shape, seed: int, nrhs: int = 1) -> np.ndarray:
    return normal((nrhs, s.Nt, s.Nm), seed)


def make_d(s: Shape, seed: int, nrhs: int = 1) -> np.ndarray:
    return normal((nrhs, s.Nt, s.Nd), seed)


def config_inputs(name: str, s: Shape | None = None, nrhs: int = 1):
    """(shape, F, m, d) for a named workload, seeded by its config number."""
    cfg = CONFIG_ID[name]
    if s is None:
        s = {"tiny": TINY, "paper": PAPER, "mixed": PAPER, "multi_rhs": MULTI_RHS}[name]
    return s, make_F(s, seed_for(cfg, 0)), make_m(s, seed_for(cfg, 1), nrhs), make_d(s, seed_for(cfg, 2), nrhs)
