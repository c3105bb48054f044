"""Python facade over the C ABI: argument checks and marshalling only.

Every step of a matvec runs in the HIP library; torch provides device memory
(``torch.empty`` for outputs) and the current stream.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib
from ._lib import (BF16, F16, F32, F64, OP_C, OP_N, OP_T, TYPE_C, TYPE_D, TYPE_S, TYPE_Z, FtmPrecision, FtmTuning,
                   check, lib)

_CODE = {"d": F64, "s": F32, "h": F16, "b": BF16}
_CHAR = {v: k for k, v in _CODE.items()}


@dataclasses.dataclass(frozen=True)
class Precision:
    """Per-phase precision of one direction, in execution order (Section 3.2).

    Each field is one of ``F64, F32, F16, BF16``.  ``accum`` is the phase-3
    accumulation type (``F64`` or ``F32``).
    """

    pad: int = F64
    fft: int = F64
    gemv: int = F64
    ifft: int = F64
    unpad: int = F64
    accum: int = F64

    @classmethod
    def parse(cls, s: str) -> "Precision":
        """``"dssdd"`` style: one of d/s/h/b per phase (pad, fft, gemv, ifft,
        unpad), optionally ``"+a64"`` / ``"+a32"`` for the accumulation.
        Default accumulation: FP64 for an FP64 product, FP32 otherwise."""
        body, _, acc = s.partition("+")
        if len(body) != 5 or any(c not in _CODE for c in body):
            raise ValueError(f"precision string {s!r}: need 5 of d/s/h/b")
        codes = [_CODE[c] for c in body]
        if acc:
            if acc not in ("a64", "a32"):
                raise ValueError(f"precision string {s!r}: accumulation is +a64 or +a32")
            accum = F64 if acc == "a64" else F32
        else:
            accum = F64 if codes[2] == F64 else F32
        return cls(*codes, accum)

    def __str__(self) -> str:
        body = "".join(_CHAR[c] for c in (self.pad, self.fft, self.gemv, self.ifft, self.unpad))
        default = F64 if self.gemv == F64 else F32
        return body if self.accum == default else body + ("+a64" if self.accum == F64 else "+a32")

    def c(self) -> FtmPrecision:
        return FtmPrecision(self.pad, self.fft, self.gemv, self.ifft, self.unpad, self.accum)


def _prec(p) -> Precision | None:
    if p is None or isinstance(p, Precision):
        return p
    return Precision.parse(p)


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Operator:
    """Block lower-triangular Toeplitz operator held on the GPU as its spectrum.

    ``F`` is the first block column, a float64 CUDA tensor ``[Nt, Nd, Nm]``;
    any strided view works (e.g. ``G.permute(2, 0, 1)`` of a ``[Nd, Nm, Nt]``
    array): the setup transform reads the strides directly.
    ``spectra`` lists extra storage formats to keep for later
    :meth:`set_precision` calls (e.g. ``("s", "h")``).
    """

    def __init__(self, F: torch.Tensor, fwd=None, adj=None, spectra=(), max_rhs: int = 1,
                 stream=None):
        if not isinstance(F, torch.Tensor) or not F.is_cuda or F.dtype != torch.float64:
            raise TypeError("F must be a float64 CUDA (HIP) tensor")
        if F.dim() != 3:
            raise ValueError("F must be [Nt, Nd, Nm]")
        self.Nt, self.Nd, self.Nm = (int(x) for x in F.shape)
        self.device = F.device
        self.max_rhs = int(max_rhs)
        fwd, adj = _prec(fwd) or Precision(), _prec(adj) or Precision()
        mask = 0
        for s in spectra:
            mask |= 1 << (_CODE[s] if isinstance(s, str) else int(s))
        L = lib()
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = _stream_ptr(stream)
            st_t, st_r, st_c = F.stride()
            check(L.ftm_setup_operator_strided(ctypes.byref(h), F.data_ptr(), self.Nt, self.Nd, self.Nm, st_t, st_r,
                                               st_c, ctypes.byref(fwd.c()), ctypes.byref(adj.c()), mask,
                                               self.max_rhs, st), "ftm_setup_operator_strided")
        self._h = h
        self.fwd, self.adj = fwd, adj
        Lc = ctypes.c_int64()
        check(L.ftm_operator_info(h, None, None, None, ctypes.byref(Lc), None), "ftm_operator_info")
        self.L = int(Lc.value)           # pad length (2 Nt, or the next 7-smooth even length)
        self.K = self.L // 2 + 1         # kept frequencies

    # -- properties -------------------------------------------------------------
    @property
    def handle(self) -> int:
        if not self._h:
            raise RuntimeError("operator was closed")
        return self._h.value

    def device_bytes(self) -> int:
        n = ctypes.c_size_t()
        check(lib().ftm_operator_info(self.handle, None, None, None, None, ctypes.byref(n)),
              "ftm_operator_info")
        return int(n.value)

    def set_precision(self, fwd=None, adj=None) -> None:
        fwd, adj = _prec(fwd), _prec(adj)
        check(lib().ftm_set_precision(self.handle, ctypes.byref(fwd.c()) if fwd else None,
                                      ctypes.byref(adj.c()) if adj else None), "ftm_set_precision")
        self.fwd, self.adj = fwd or self.fwd, adj or self.adj

    # -- products -----------------------------------------------------------------
    def _apply(self, x: torch.Tensor, adjoint: bool, out, stream) -> torch.Tensor:
        n_in, n_out = (self.Nd, self.Nm) if adjoint else (self.Nm, self.Nd)
        x = _dev_f64(x, "x")
        single = x.dim() == 2
        xb = x.unsqueeze(0) if single else x
        if xb.dim() != 3 or tuple(xb.shape[1:]) != (self.Nt, n_in):
            raise ValueError(f"input must be [nrhs,] {self.Nt} x {n_in}, got {tuple(x.shape)}")
        nrhs = xb.shape[0]
        if out is None:
            out = torch.empty((nrhs, self.Nt, n_out), dtype=torch.float64, device=x.device)
        else:
            out = _dev_f64(out, "out")
            if out.numel() != nrhs * self.Nt * n_out:
                raise ValueError("out has the wrong size")
        fn = lib().ftm_rmatvec if adjoint else lib().ftm_matvec
        with torch.cuda.device(x.device):
            check(fn(self.handle, xb.data_ptr(), out.data_ptr(), nrhs, _stream_ptr(stream)),
                  "ftm_rmatvec" if adjoint else "ftm_matvec")
        return out[0] if single and out.dim() == 3 else out

    def matvec(self, m: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """``d = F m``; ``m`` is ``[Nt, Nm]`` or ``[nrhs, Nt, Nm]``."""
        return self._apply(m, False, out, stream)

    def rmatvec(self, d: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """``m = F^T d``; ``d`` is ``[Nt, Nd]`` or ``[nrhs, Nt, Nd]``."""
        return self._apply(d, True, out, stream)

    def workspace_size(self, nrhs: int = 1, adjoint: bool = False) -> int:
        """Workspace bytes one :meth:`apply` call of ``nrhs`` vectors needs at the
        current precision (``ftm_workspace_size``)."""
        n = ctypes.c_size_t()
        check(lib().ftm_workspace_size(self.handle, 1 if adjoint else 0, int(nrhs), ctypes.byref(n)),
              "ftm_workspace_size")
        return int(n.value)

    def apply(self, x: torch.Tensor, workspace: torch.Tensor, adjoint: bool = False, out=None,
              stream=None) -> torch.Tensor:
        """``F x`` (or ``F^T x``) on a caller-owned workspace (``ftm_apply``):
        calls with distinct workspaces may run concurrently on different
        streams.  ``workspace`` is a CUDA tensor of at least
        :meth:`workspace_size` bytes; ``nrhs`` is not limited by ``max_rhs``."""
        n_in, n_out = (self.Nd, self.Nm) if adjoint else (self.Nm, self.Nd)
        x = _dev_f64(x, "x")
        single = x.dim() == 2
        xb = x.unsqueeze(0) if single else x
        if xb.dim() != 3 or tuple(xb.shape[1:]) != (self.Nt, n_in):
            raise ValueError(f"input must be [nrhs,] {self.Nt} x {n_in}, got {tuple(x.shape)}")
        if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or not workspace.is_contiguous():
            raise TypeError("workspace must be a contiguous CUDA tensor")
        nrhs = xb.shape[0]
        if out is None:
            out = torch.empty((nrhs, self.Nt, n_out), dtype=torch.float64, device=x.device)
        else:
            out = _dev_f64(out, "out")
            if out.numel() != nrhs * self.Nt * n_out:
                raise ValueError("out has the wrong size")
        nbytes = workspace.numel() * workspace.element_size()
        with torch.cuda.device(x.device):
            check(lib().ftm_apply(self.handle, 1 if adjoint else 0, xb.data_ptr(), out.data_ptr(), nrhs,
                                  workspace.data_ptr(), nbytes, _stream_ptr(stream)), "ftm_apply")
        return out[0] if single and out.dim() == 3 else out

    def apply_scratch(self, x: torch.Tensor, adjoint: bool = False, out=None, stream=None) -> torch.Tensor:
        """``F x`` (or ``F^T x``) on the library's static per-GPU scratch
        (``ftm_apply_scratch``): the call allocates no device memory.  ``out``
        must be given by callers that cannot allocate.  Calls that overlap on
        one GPU race on the shared scratch."""
        n_in, n_out = (self.Nd, self.Nm) if adjoint else (self.Nm, self.Nd)
        x = _dev_f64(x, "x")
        single = x.dim() == 2
        xb = x.unsqueeze(0) if single else x
        if xb.dim() != 3 or tuple(xb.shape[1:]) != (self.Nt, n_in):
            raise ValueError(f"input must be [nrhs,] {self.Nt} x {n_in}, got {tuple(x.shape)}")
        nrhs = xb.shape[0]
        if out is None:
            out = torch.empty((nrhs, self.Nt, n_out), dtype=torch.float64, device=x.device)
        else:
            out = _dev_f64(out, "out")
            if out.numel() != nrhs * self.Nt * n_out:
                raise ValueError("out has the wrong size")
        with torch.cuda.device(x.device):
            check(lib().ftm_apply_scratch(self.handle, 1 if adjoint else 0, xb.data_ptr(), out.data_ptr(), nrhs,
                                          _stream_ptr(stream)), "ftm_apply_scratch")
        return out[0] if single and out.dim() == 3 else out

    def select_precision(self, tolerance: float, adjoint: bool = False, probe: torch.Tensor | None = None,
                         reps: int = 3, stream=None) -> dict:
        """Make the fastest configuration whose relative error (against the
        all-FP64 result on ``probe``) is at most ``tolerance`` the direction's
        configuration (``ftm_select_precision``).  Candidates use the spectrum
        copies kept at setup.  ``probe`` defaults to a seeded N(0,1) input.
        Returns ``{"prec": ..., "err": ..., "ms": ...}``."""
        n_in = self.Nd if adjoint else self.Nm
        if probe is None:
            g = torch.Generator(device=self.device)
            g.manual_seed(2508_10202)
            probe = torch.randn((self.Nt, n_in), dtype=torch.float64, device=self.device, generator=g)
        probe = _dev_f64(probe, "probe")
        if probe.numel() != self.Nt * n_in:
            raise ValueError("probe has the wrong size")
        p, err, ms = FtmPrecision(), ctypes.c_double(), ctypes.c_double()
        with torch.cuda.device(self.device):
            check(lib().ftm_select_precision(self.handle, 1 if adjoint else 0, float(tolerance), probe.data_ptr(),
                                             int(reps), ctypes.byref(p), ctypes.byref(err), ctypes.byref(ms),
                                             _stream_ptr(stream)), "ftm_select_precision")
        chosen = Precision(p.pad, p.fft, p.gemv, p.ifft, p.unpad, p.accum)
        if adjoint:
            self.adj = chosen
        else:
            self.fwd = chosen
        return {"prec": str(chosen), "err": err.value, "ms": ms.value}

    def hessian_workspace_size(self, nrhs: int = 1) -> int:
        """Workspace bytes of one :meth:`hessian` call of ``nrhs`` vectors."""
        n = ctypes.c_size_t()
        check(lib().ftm_hessian_workspace_size(self.handle, int(nrhs), ctypes.byref(n)),
              "ftm_hessian_workspace_size")
        return int(n.value)

    def hessian(self, x: torch.Tensor, workspace: torch.Tensor | None = None, out=None,
                stream=None) -> torch.Tensor:
        """Data-space Hessian actions ``F F^T x`` (``ftm_hessian_apply``) for
        ``x`` of shape ``[Nt, Nd]`` or ``[nrhs, Nt, Nd]``.  ``workspace`` (a
        contiguous CUDA tensor of at least :meth:`hessian_workspace_size`
        bytes) is allocated here when not given."""
        x = _dev_f64(x, "x")
        single = x.dim() == 2
        xb = x.unsqueeze(0) if single else x
        if xb.dim() != 3 or tuple(xb.shape[1:]) != (self.Nt, self.Nd):
            raise ValueError(f"input must be [nrhs,] {self.Nt} x {self.Nd}, got {tuple(x.shape)}")
        nrhs = xb.shape[0]
        if workspace is None:
            workspace = torch.empty(((self.hessian_workspace_size(nrhs) + 255) // 256 * 32,),
                                    dtype=torch.float64, device=x.device)
        if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or not workspace.is_contiguous():
            raise TypeError("workspace must be a contiguous CUDA tensor")
        if out is None:
            out = torch.empty_like(xb)
        else:
            out = _dev_f64(out, "out")
            if out.numel() != xb.numel():
                raise ValueError("out has the wrong size")
        nbytes = workspace.numel() * workspace.element_size()
        with torch.cuda.device(x.device):
            check(lib().ftm_hessian_apply(self.handle, xb.data_ptr(), out.data_ptr(), nrhs, workspace.data_ptr(),
                                          nbytes, _stream_ptr(stream)), "ftm_hessian_apply")
        return out[0] if single and out.dim() == 3 else out

    def spectrum(self, which="d", k0: int = 0, nk: int | None = None, stream=None) -> torch.Tensor:
        """Stored ``Fhat_k`` for ``k0 <= k < k0 + nk`` as complex128 ``[nk, Nd, Nm]``."""
        nk = (self.K - k0) if nk is None else nk
        code = _CODE[which] if isinstance(which, str) else int(which)
        out = torch.empty((nk, self.Nd, self.Nm, 2), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            check(lib().ftm_get_spectrum(self.handle, code, k0, nk, out.data_ptr(), _stream_ptr(stream)),
                  "ftm_get_spectrum")
        return torch.view_as_complex(out)

    def set_rhs_mode(self, mode: str) -> None:
        """Phase 3 for several right-hand sides: "auto", "gemv" (one product per
        vector) or "gemm" (matrix cores whenever the configuration allows)."""
        code = {"auto": _lib.RHS_AUTO, "gemv": _lib.RHS_GEMV, "gemm": _lib.RHS_GEMM}[mode]
        check(lib().ftm_set_rhs_mode(self.handle, code), "ftm_set_rhs_mode")

    def set_gemm_crossover(self, min_rhs: int) -> None:
        check(lib().ftm_set_gemm_crossover(self.handle, int(min_rhs)), "ftm_set_gemm_crossover")

    def autotune(self, reps: int = 10, cache: str | None = None, stream=None) -> dict:
        """Pick the phase-3 tile variants by timing them on this operator at its
        current precision (``ftm_autotune``).  With ``cache`` (a JSON file),
        an earlier choice for the same device, shape and precision is reused
        instead of timing again, and new choices are stored."""
        import json
        import os
        key = f"{torch.cuda.get_device_name(self.device)}|{self.Nt}x{self.Nd}x{self.Nm}|{self.fwd}|{self.adj}"
        db = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                db = json.load(fh)
        if key in db:
            self.set_tuning(**{k: v for k, v in db[key].items() if k != "ms"})
            return dict(db[key], cached=True)
        with torch.cuda.device(self.device):
            check(lib().ftm_autotune(self.handle, int(reps), _stream_ptr(stream)), "ftm_autotune")
        rec = self.tuning()
        if cache:
            db[key] = rec
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(db, fh, indent=1)
            os.replace(tmp, cache)
        return dict(rec, cached=False)

    def tuning(self) -> dict:
        """The kernel and tile choices for the current precision (``ftm_get_tuning``):
        per direction [forward, adjoint] the product's tile variant, the input
        and output transforms' kernels, the GEMM tile, the FP32-storage GEMM
        instructions, the GEMM crossover and the autotuned matvec time."""
        t = FtmTuning()
        check(lib().ftm_get_tuning(self.handle, ctypes.byref(t)), "ftm_get_tuning")
        return {"gemv_variant": list(t.gemv_variant), "fft_shape": [list(r) for r in t.fft_shape],
                "gemm_tile": list(t.gemm_tile), "gemm_kind": list(t.gemm_kind),
                "gemm_min_rhs": list(t.gemm_min_rhs), "ms": list(t.ms)}

    def set_tuning(self, gemv_variant=None, fft_shape=None, gemm_tile=None, gemm_min_rhs=None,
                   gemm_kind=None) -> None:
        """Set some of the choices (``ftm_set_tuning``); each argument is a
        [forward, adjoint] pair (``fft_shape``: a pair of [input, output])."""
        t = FtmTuning()
        check(lib().ftm_get_tuning(self.handle, ctypes.byref(t)), "ftm_get_tuning")
        for d in range(2):
            if gemv_variant is not None:
                t.gemv_variant[d] = int(gemv_variant[d])
            if fft_shape is not None:
                t.fft_shape[d][0], t.fft_shape[d][1] = int(fft_shape[d][0]), int(fft_shape[d][1])
            if gemm_tile is not None:
                t.gemm_tile[d] = int(gemm_tile[d])
            if gemm_kind is not None:
                t.gemm_kind[d] = int(gemm_kind[d])
            if gemm_min_rhs is not None:
                t.gemm_min_rhs[d] = int(gemm_min_rhs[d])
        check(lib().ftm_set_tuning(self.handle, ctypes.byref(t)), "ftm_set_tuning")

    def graph(self, x: torch.Tensor, adjoint: bool = False, out=None) -> "Graph":
        """Capture one matvec with fixed buffers into a HIP graph (``ftm_graph_create``)."""
        n_in, n_out = (self.Nd, self.Nm) if adjoint else (self.Nm, self.Nd)
        x = _dev_f64(x, "x")
        xb = x.unsqueeze(0) if x.dim() == 2 else x
        if tuple(xb.shape[1:]) != (self.Nt, n_in):
            raise ValueError("input has the wrong shape")
        y = out if out is not None else torch.empty((xb.shape[0], self.Nt, n_out), dtype=torch.float64,
                                                    device=x.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().ftm_graph_create(ctypes.byref(h), self.handle, 1 if adjoint else 0, xb.data_ptr(),
                                         y.data_ptr(), xb.shape[0]), "ftm_graph_create")
        return Graph(h, self, xb, y)

    def profile(self, enable: bool = True) -> None:
        """Record HIP events around each kernel of every following call."""
        check(lib().ftm_profile_enable(self.handle, 1 if enable else 0), "ftm_profile_enable")

    def profile_read(self, reset: bool = True) -> dict:
        """Average kernel times in ms: {"fwd": [fft, product, ifft], "adj": [...], "n": (nf, na)}."""
        ms = (ctypes.c_double * 6)()
        cnt = (ctypes.c_int64 * 2)()
        check(lib().ftm_profile_read(self.handle, ms, cnt, 1 if reset else 0), "ftm_profile_read")
        out = {"n": (int(cnt[0]), int(cnt[1]))}
        for d, name in enumerate(("fwd", "adj")):
            n = max(int(cnt[d]), 1)
            out[name] = [ms[3 * d + i] / n for i in range(3)]
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            lib().ftm_destroy_operator(self._h.value)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Graph:
    """A captured matvec; ``launch()`` replays it on a stream, ``y`` is its output."""

    def __init__(self, h, op, x, y):
        self._h, self.op, self.x, self.y = h, op, x, y

    def launch(self, stream=None) -> torch.Tensor:
        with torch.cuda.device(self.op.device):
            check(lib().ftm_graph_launch(self._h, _stream_ptr(stream)), "ftm_graph_launch")
        return self.y

    def close(self) -> None:
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.op.device)
            lib().ftm_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop over device-resident operators.

    ``submit`` returns at once with a ticket; the library's worker thread
    admits requests by workspace budget, coalesces queued requests for the
    same operator and direction into one multi-right-hand-side matvec, and
    runs batches of different operators concurrently on ``n_slots`` streams.
    """

    def __init__(self, workspace_budget: int, n_slots: int = 4, max_batch_rhs: int = 64):
        h = ctypes.c_void_p()
        check(lib().ftm_server_create(ctypes.byref(h), int(workspace_budget), int(n_slots), int(max_batch_rhs)),
              "ftm_server_create")
        self._h = h
        self.max_batch_rhs = int(max_batch_rhs)
        self._live = {}  # ticket -> (x, y, event): kept alive until completion

    def submit(self, op: Operator, x: torch.Tensor, adjoint: bool = False, out=None):
        """Queue ``F x`` (or ``F^T x``); returns ``(ticket, y)``.  ``y`` is
        written when the ticket completes.  ``x`` may still be in production on
        the current stream: an event recorded there is waited for on the device."""
        n_in, n_out = (op.Nd, op.Nm) if adjoint else (op.Nm, op.Nd)
        x = _dev_f64(x, "x")
        xb = x.unsqueeze(0) if x.dim() == 2 else x
        if xb.dim() != 3 or tuple(xb.shape[1:]) != (op.Nt, n_in):
            raise ValueError(f"input must be [nrhs,] {op.Nt} x {n_in}")
        nrhs = xb.shape[0]
        y = out if out is not None else torch.empty((nrhs, op.Nt, n_out), dtype=torch.float64, device=x.device)
        ev = torch.cuda.Event()
        ev.record()
        t = ctypes.c_uint64()
        check(lib().ftm_server_submit(self._h, op.handle, 1 if adjoint else 0, xb.data_ptr(), y.data_ptr(), nrhs,
                                      ctypes.c_void_p(ev.cuda_event), ctypes.byref(t)), "ftm_server_submit")
        self._live[t.value] = (xb, y, ev)
        return t.value, y

    def poll(self, ticket: int):
        done, lat = ctypes.c_int32(), ctypes.c_double()
        check(lib().ftm_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(lat)), "ftm_server_poll")
        if done.value:
            self._live.pop(ticket, None)
        return bool(done.value), lat.value

    def wait(self, ticket: int, timeout: float = 0.0) -> float:
        lat = ctypes.c_double()
        check(lib().ftm_server_wait(self._h, ticket, ctypes.byref(lat), float(timeout)), "ftm_server_wait")
        self._live.pop(ticket, None)
        return lat.value

    def latencies(self, first: int, n: int):
        import numpy as np
        out = np.empty(n, dtype=np.float64)
        check(lib().ftm_server_latencies(self._h, first, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
              "ftm_server_latencies")
        return out

    def release_done(self) -> None:
        """Drop references to tensors of completed requests."""
        for t in list(self._live):
            self.poll(t)

    def stats(self) -> dict:
        st = _lib.FtmServerStats()
        check(lib().ftm_server_get_stats(self._h, ctypes.byref(st)), "ftm_server_get_stats")
        return {name: getattr(st, name) for name, _ in st._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().ftm_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


_SB_TYPES = {torch.float32: (TYPE_S, ctypes.c_float, 1), torch.float64: (TYPE_D, ctypes.c_double, 1),
             torch.complex64: (TYPE_C, ctypes.c_float, 2), torch.complex128: (TYPE_Z, ctypes.c_double, 2)}
_SB_OPS = {"N": OP_N, "T": OP_T, "C": OP_C}


def sbgemv(A: torch.Tensor, x: torch.Tensor, m: int | None = None, op: str = "N", alpha=1.0, beta=0.0,
           y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Strided-batched y_b = alpha op(A_b) x_b + beta y_b (``ftm_sbgemv``), BLAS
    column-major semantics.  ``A`` is a CUDA tensor of shape (batch, n, lda)
    whose row j holds column j of the m x n matrix A_b (m = lda unless given);
    ``x`` is (batch, n) for op "N" and (batch, m) for "T" / "C"; ``y`` (batch,
    m) or (batch, n) is written in place (allocated when None, then beta must
    be zero).  dtype float32, float64, complex64 or complex128, all the same."""
    if op not in _SB_OPS:
        raise ValueError("op must be 'N', 'T' or 'C'")
    if A.dtype not in _SB_TYPES or x.dtype != A.dtype or (y is not None and y.dtype != A.dtype):
        raise ValueError("A, x and y must share one of float32, float64, complex64, complex128")
    if A.dim() != 3 or x.dim() != 2 or not A.is_cuda or not x.is_cuda:
        raise ValueError("A must be a CUDA (batch, n, lda) tensor and x a CUDA (batch, len) tensor")
    if not A.is_contiguous() or not x.is_contiguous():
        raise ValueError("A and x must be contiguous")
    batch, n, lda = A.shape
    m = lda if m is None else int(m)
    nx, ny = (n, m) if op == "N" else (m, n)
    if tuple(x.shape) != (batch, nx):
        raise ValueError(f"x must have shape {(batch, nx)}")
    if y is None:
        if beta != 0:
            raise ValueError("beta must be zero when y is allocated here")
        y = torch.empty((batch, ny), dtype=A.dtype, device=A.device)
    elif tuple(y.shape) != (batch, ny) or not y.is_contiguous():
        raise ValueError(f"y must be a contiguous tensor of shape {(batch, ny)}")
    code, ctype, ncomp = _SB_TYPES[A.dtype]

    def scalar(v):
        v = complex(v)
        if ncomp == 1 and v.imag != 0:
            raise ValueError("alpha and beta must be real for real types")
        return (ctype * 2)(v.real, v.imag) if ncomp == 2 else (ctype * 1)(v.real)
    al, be = scalar(alpha), scalar(beta)
    with torch.cuda.device(A.device):
        check(lib().ftm_sbgemv(code, _SB_OPS[op], m, n, ctypes.cast(al, ctypes.c_void_p), A.data_ptr(), lda,
                               n * lda, x.data_ptr(), nx, ctypes.cast(be, ctypes.c_void_p), y.data_ptr(), ny,
                               batch, _stream_ptr(stream)), "ftm_sbgemv")
    return y


def round_values(x: torch.Tensor, fmt: str, from_f32: bool = False, stream=None) -> torch.Tensor:
    """Round a float64 CUDA tensor into storage format ``fmt`` (one of d/s/h/b)
    exactly as the kernels do (``ftm_round``); returns float64 values."""
    x = _dev_f64(x, "x")
    y = torch.empty_like(x)
    with torch.cuda.device(x.device):
        check(lib().ftm_round(_CODE[fmt], 1 if from_f32 else 0, x.data_ptr(), y.data_ptr(), x.numel(),
                              _stream_ptr(stream)), "ftm_round")
    return y
