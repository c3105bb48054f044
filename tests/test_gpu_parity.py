"""Parity of the HIP path against the CPU oracle (run on an MI355X).

Every product goes through the C ABI (``libftm.so`` via ``Operator``); the
expected values come only from ``oracle/``.  Sizes span several tiles of
every kernel and ragged tails (odd Nm, Nd not a multiple of the 8-row block,
Nm not a multiple of the 8-column padding, L with radices 2, 3, 5, 7, 8).
"""
import math
import sys

import numpy as np
import pytest

import oracle
from workloads import PAPER, Shape, config_inputs, make_F, make_d, make_m

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12  # relative L2, float64 path


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _rel(a, b):
    return oracle.relative_l2(a, b)


def _prime_factors(v):
    out, p = [], 2
    while v > 1:
        while v % p == 0:
            out.append(p)
            v //= p
        p += 1
    return out


def _run(F, m=None, d=None, **kw):
    import torch
    from paper_2508_10202_amd import Operator
    op = Operator(torch.from_numpy(F).cuda(), **kw)
    out = {"L": op.L}
    if m is not None:
        out["d"] = op.matvec(torch.from_numpy(m).cuda()).cpu().numpy()
    if d is not None:
        out["m"] = op.rmatvec(torch.from_numpy(d).cuda()).cpu().numpy()
    op.close()
    return out


def test_tiny_config_fp64(gpu):
    """Nt=64, Nd=16, Nm=256, iid N(0,1): forward and adjoint vs the oracle."""
    s, F, m, d = config_inputs("tiny")
    _say("case tiny", s)
    out = _run(F, m[0], d[0])
    ref_d, ref_m = oracle.forward(F, m[0]), oracle.adjoint(F, d[0])
    assert _rel(out["d"], ref_d) <= FP64_TOL
    assert _rel(out["m"], ref_m) <= FP64_TOL
    assert np.max(np.abs(out["d"] - ref_d)) <= FP64_TOL * np.max(np.abs(ref_d))
    assert np.max(np.abs(out["m"] - ref_m)) <= FP64_TOL * np.max(np.abs(ref_m))
    # adjoint identity on the GPU's own outputs
    lhs, rhs = float(np.dot(out["d"].ravel(), d[0].ravel())), float(np.dot(m[0].ravel(), out["m"].ravel()))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


RAGGED = [
    Shape(45, 13, 301, decay=30.0),   # L = 90 = 2*3*3*5, odd Nm, Nd not a multiple of 8
    Shape(7, 3, 5, decay=None),       # L = 14 = 2*7
    Shape(1, 1, 1, decay=None),       # L = 2, a single block
    Shape(2048, 2, 9, decay=500.0),   # largest supported Nt, L = 4096
    Shape(100, 37, 1000),             # L = 200, several column tiles
    Shape(12, 9, 24, scale_by_sqrt_nm=False, decay=None),  # L = 24 = 8*3
    # 2 Nt with a prime factor above 7: the next 7-smooth even length is used
    Shape(11, 3, 7, decay=None),      # 2 Nt = 22 -> L = 24
    Shape(23, 5, 40, decay=10.0),     # 46 -> 48
    Shape(97, 4, 33, decay=40.0),     # 194 -> 196 = 4*7*7
    Shape(2047, 2, 5, decay=500.0),   # 4094 -> 4096
    # lengths with fixed-plan transform kernels: partial column tiles, a single
    # column, odd column counts, and Nt below L/2 (L padded to the fixed length)
    Shape(64, 3, 33, decay=None),     # L = 128
    Shape(127, 5, 17, decay=50.0),    # 254 -> 256
    Shape(199, 9, 45, decay=60.0),    # 398 -> 400
    Shape(512, 2, 1, decay=200.0),    # L = 1024, one parameter column
    Shape(256, 17, 23, decay=100.0),  # L = 512
    Shape(997, 3, 37, decay=300.0),   # 1994 -> 2000
]


@pytest.mark.parametrize("s", RAGGED, ids=lambda s: f"Nt{s.Nt}_Nd{s.Nd}_Nm{s.Nm}")
def test_ragged_shapes_fp64(gpu, s):
    _say("case ragged", s)
    F, m, d = make_F(s, 11), make_m(s, 12)[0], make_d(s, 13)[0]
    out = _run(F, m, d)
    assert out["L"] >= 2 * s.Nt and out["L"] % 2 == 0
    if all(p in (2, 3, 5, 7) for p in _prime_factors(2 * s.Nt)):
        assert out["L"] == 2 * s.Nt                     # the paper's length whenever it factors
    assert _rel(out["d"], oracle.forward(F, m)) <= FP64_TOL
    assert _rel(out["m"], oracle.adjoint(F, d)) <= FP64_TOL


# float32 transforms run their own plans (radix-16 passes for the factor 2^e):
# the ragged shapes again, plus lengths whose plans are 16, 16*5 and 16*16*8
RAGGED_F32 = RAGGED + [
    Shape(8, 3, 11, decay=None),      # L = 16
    Shape(40, 5, 70, decay=20.0),     # L = 80 = 16*5
    Shape(1024, 3, 17, decay=300.0),  # L = 2048 = 16*16*8
]


@pytest.mark.parametrize("prec", ["dsdsd", "sssss"])
@pytest.mark.parametrize("s", RAGGED_F32, ids=lambda s: f"Nt{s.Nt}_Nd{s.Nd}_Nm{s.Nm}")
def test_ragged_shapes_fp32_transforms(gpu, s, prec):
    _say("case ragged float32 transforms", s, prec)
    F, m, d = make_F(s, 14), make_m(s, 15)[0], make_d(s, 16)[0]
    out = _run(F, m, d, fwd=prec, adj=prec)
    e_f, e_a = _rel(out["d"], oracle.forward(F, m)), _rel(out["m"], oracle.adjoint(F, d))
    _, hi_f = mp_bounds(prec, s.L, s.Nm)
    _, hi_a = mp_bounds(prec, s.L, s.Nd)
    _say(f"  {prec}: fwd {e_f:.3e} <= {hi_f:.1e}, adj {e_a:.3e} <= {hi_a:.1e}")
    assert e_f <= hi_f and e_a <= hi_a


def test_identity_and_delay_blocks_exact(gpu):
    """F_0 = I gives d = m, F_2 = I a two-block delay (up to float64 rounding of the FFTs)."""
    Nt, n = 30, 8
    for lag in (0, 2):
        F = np.zeros((Nt, n, n))
        F[lag] = np.eye(n)
        m = make_m(Shape(Nt, n, n), 21)[0]
        out = _run(F, m, m)
        want_f = np.zeros_like(m)
        want_f[lag:] = m[:Nt - lag]
        want_a = np.zeros_like(m)
        want_a[:Nt - lag] = m[lag:]
        assert np.max(np.abs(out["d"] - want_f)) <= 1e-14
        assert np.max(np.abs(out["m"] - want_a)) <= 1e-14


def test_spectrum_fp64_vs_oracle(gpu):
    import torch
    from paper_2508_10202_amd import Operator
    for s in (Shape(64, 5, 33, scale_by_sqrt_nm=False, decay=None), Shape(45, 3, 17, decay=None),
              Shape(7, 2, 3, decay=None)):
        _say("case spectrum", s)
        F = make_F(s, 31)
        op = Operator(torch.from_numpy(F).cuda())
        got = op.spectrum("d").cpu().numpy()
        op.close()
        ref = oracle.spectrum(F)
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def _rne(x, p):
    """Round float64 x to p significand bits, nearest-even (normal range only)."""
    mant, e = np.frexp(x)
    return np.ldexp(np.rint(np.ldexp(mant, p)), e - p)


def test_spectrum_storage_formats(gpu):
    """The FP32/FP16/BF16 copies are the float64 spectrum rounded to nearest even."""
    import torch
    from paper_2508_10202_amd import Operator
    s = Shape(50, 6, 40, scale_by_sqrt_nm=False, decay=None)
    F = make_F(s, 41)
    op = Operator(torch.from_numpy(F).cuda(), spectra=("d", "s", "h", "b"))
    ref = op.spectrum("d").cpu().numpy()
    got = {w: op.spectrum(w).cpu().numpy() for w in "shb"}
    op.close()
    for part in (np.real, np.imag):
        r = part(ref)
        assert np.array_equal(part(got["s"]), r.astype(np.float32).astype(np.float64))
        assert np.array_equal(part(got["h"]), r.astype(np.float16).astype(np.float64))
        assert np.array_equal(part(got["b"]), _rne(r, 8))


def test_multi_rhs_matches_single_bitwise(gpu):
    """One vector at a time (FTM_RHS_GEMV): a batch equals its vectors run
    alone, bitwise.  The matrix-core path (the default for batches, float64
    accumulation here) is batch invariant: a vector's result does not depend
    on the batch around it or on the right-hand-side tile, bitwise; both
    within 1e-12 of the oracle."""
    import torch
    from paper_2508_10202_amd import Operator
    s = Shape(40, 10, 200)
    F, M, D = make_F(s, 51), make_m(s, 52, nrhs=40), make_d(s, 53, nrhs=40)
    op = Operator(torch.from_numpy(F).cuda(), max_rhs=40)
    Mt, Dt = torch.from_numpy(M).cuda(), torch.from_numpy(D).cuda()
    op.set_rhs_mode("gemv")
    batch_d, batch_m = op.matvec(Mt[:3]).cpu().numpy(), op.rmatvec(Dt[:3]).cpu().numpy()
    for b in range(3):
        assert np.array_equal(batch_d[b], op.matvec(Mt[b]).cpu().numpy())
        assert np.array_equal(batch_m[b], op.rmatvec(Dt[b]).cpu().numpy())
    assert _rel(batch_d, oracle.forward(F, M[:3])) <= FP64_TOL
    assert _rel(batch_m, oracle.adjoint(F, D[:3])) <= FP64_TOL
    op.set_rhs_mode("auto")
    ref_d, ref_m = oracle.forward(F, M), oracle.adjoint(F, D)
    g3d, g3m = op.matvec(Mt[:3]).cpu().numpy(), op.rmatvec(Dt[:3]).cpu().numpy()
    for n, tile in ((40, 0), (40, 16), (17, 32), (5, 64)):
        op.set_tuning(gemm_tile=(tile, tile))
        gd, gm = op.matvec(Mt[:n]).cpu().numpy(), op.rmatvec(Dt[:n]).cpu().numpy()
        assert np.array_equal(gd[:3], g3d) and np.array_equal(gm[:3], g3m), (n, tile)
        assert _rel(gd, ref_d[:n]) <= FP64_TOL and _rel(gm, ref_m[:n]) <= FP64_TOL
    op.close()


@pytest.mark.parametrize("shape", [1, 2, 3])
def test_fft_tiles_zero_the_padding_columns(gpu, shape):
    """Every transform kernel writes the workspace columns between Nm (and Nd)
    and their padded widths as zeros: with Nm = 4 mod 8 and Nd = 4 mod 8 the
    smaller column tile ends exactly at Nm, and a NaN-filled caller workspace
    must still give the oracle's result."""
    import torch
    from paper_2508_10202_amd import Operator
    s = Shape(64, 20, 500)
    F, M, D = make_F(s, 61), make_m(s, 62, nrhs=3), make_d(s, 63, nrhs=3)
    op = Operator(torch.from_numpy(F).cuda(), spectra=("s",), max_rhs=3)
    Mt, Dt = torch.from_numpy(M).cuda(), torch.from_numpy(D).cuda()
    want_d = np.stack([oracle.forward(F, M[b]) for b in range(3)])
    want_m = np.stack([oracle.adjoint(F, D[b]) for b in range(3)])
    for prec in ("ddddd", "sssss"):
        op.set_precision(fwd=prec, adj=prec)
        op.set_tuning(fft_shape=((shape, shape), (shape, shape)))
        nb = max(op.workspace_size(3, adjoint=a) for a in (False, True))
        ws = torch.full((nb // 8 + 1,), float("nan"), dtype=torch.float64, device="cuda")
        yd = op.apply(Mt, ws).cpu().numpy()
        ws.fill_(float("nan"))
        ym = op.apply(Dt, ws, adjoint=True).cpu().numpy()
        tol = 1e-12 if prec == "ddddd" else 1e-5
        assert np.isfinite(yd).all() and np.isfinite(ym).all(), (prec, shape)
        assert oracle.relative_l2(yd, want_d) < tol, (prec, shape)
        assert oracle.relative_l2(ym, want_m) < tol, (prec, shape)
    op.close()


@pytest.mark.parametrize("s", [Shape(512, 3, 40, decay=200.0), Shape(1000, 3, 40, decay=300.0)])
def test_long_transforms_every_tile_several_vectors(gpu, s):
    """The fixed-plan transforms of lengths 1024 and 2000 (twiddles held in
    registers one pass ahead) with 3 right-hand sides, in float64, float32 and
    with BF16 rounding: each transform kernel matches the oracle, and the
    larger and smaller column tiles give bitwise the same result (the tile
    decides only which workgroup transforms a column)."""
    import torch
    from paper_2508_10202_amd import Operator
    F, M, D = make_F(s, 71), make_m(s, 72, nrhs=3), make_d(s, 73, nrhs=3)
    op = Operator(torch.from_numpy(F).cuda(), spectra=("s", "b"), max_rhs=3)
    Mt, Dt = torch.from_numpy(M).cuda(), torch.from_numpy(D).cuda()
    want_d, want_m = oracle.forward(F, M), oracle.adjoint(F, D)
    for prec in ("ddddd", "sssss", "dbbbd"):
        op.set_precision(fwd=prec, adj=prec)
        got = {}
        for shape in (0, 1, 2):
            op.set_tuning(fft_shape=((shape, shape), (shape, shape)))
            got[shape] = (op.matvec(Mt).cpu().numpy(), op.rmatvec(Dt).cpu().numpy())
            _say(f"case long transforms {s.Nt} {prec} tile {shape}")
            e_f, e_a = _rel(got[shape][0], want_d), _rel(got[shape][1], want_m)
            if prec == "ddddd":
                assert e_f <= FP64_TOL and e_a <= FP64_TOL, (prec, shape, e_f, e_a)
            else:
                lo_f, hi_f = mp_bounds(prec, s.L, s.Nm)
                lo_a, hi_a = mp_bounds(prec, s.L, s.Nd)
                assert lo_f <= e_f <= hi_f and lo_a <= e_a <= hi_a, (prec, shape, e_f, e_a)
        assert np.array_equal(got[1][0], got[2][0]) and np.array_equal(got[1][1], got[2][1]), prec
    op.close()


def test_unaligned_vectors_match_aligned(gpu):
    """Input and output vectors 8 bytes past a 16-byte boundary take the
    transforms' per-column loads and stores, while whole tiles of aligned
    rows take the 16-byte loads and stores of column pairs: both give bitwise
    the same result, in float64, float32 and with BF16 rounding."""
    import torch
    from paper_2508_10202_amd import Operator
    s = Shape(512, 16, 48)
    F, M, D = make_F(s, 81), make_m(s, 82, nrhs=2), make_d(s, 83, nrhs=2)
    op = Operator(torch.from_numpy(F).cuda(), spectra=("s", "b"), max_rhs=2)
    Mt, Dt = torch.from_numpy(M).cuda(), torch.from_numpy(D).cuda()

    def shifted(a):
        buf = torch.empty(a.numel() + 1, dtype=torch.float64, device="cuda")
        v = buf[1:].view(a.shape)
        v.copy_(a)
        assert v.data_ptr() % 16 == 8
        return v

    for prec in ("ddddd", "sssss", "dbbbd"):
        _say(f"case unaligned vectors {prec}")
        op.set_precision(fwd=prec, adj=prec)
        want_d, want_m = op.matvec(Mt), op.rmatvec(Dt)
        out_d, out_m = shifted(torch.zeros_like(want_d)), shifted(torch.zeros_like(want_m))
        op.matvec(shifted(Mt), out=out_d)
        op.rmatvec(shifted(Dt), out=out_m)
        assert torch.equal(out_d, want_d) and torch.equal(out_m, want_m), prec
    op.close()


def test_apply_on_caller_workspaces_concurrently(gpu):
    """ftm_apply on two NaN-filled caller workspaces, on two streams at once:
    both results equal the operator's own-workspace call bitwise."""
    import torch
    from paper_2508_10202_amd import FtmError, Operator
    s = Shape(64, 20, 500)
    F, M, D = make_F(s, 57), make_m(s, 58, nrhs=3), make_d(s, 59, nrhs=3)
    op = Operator(torch.from_numpy(F).cuda(), spectra=("s",), max_rhs=3)
    Mt, Dt = torch.from_numpy(M).cuda(), torch.from_numpy(D).cuda()
    for prec in ("ddddd", "dssdd"):
        op.set_precision(fwd=prec, adj=prec)
        want_d, want_m = op.matvec(Mt).clone(), op.rmatvec(Dt).clone()
        nb = max(op.workspace_size(5, adjoint=a) for a in (False, True))
        ws = [torch.full((nb // 8 + 1,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(2)]
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        torch.cuda.synchronize()
        outs = []
        for rep in range(3):
            with torch.cuda.stream(streams[0]):
                yd = op.apply(Mt, ws[0], stream=streams[0])
            with torch.cuda.stream(streams[1]):
                ym = op.apply(Dt, ws[1], adjoint=True, stream=streams[1])
            outs.append((yd, ym))
        torch.cuda.synchronize()
        for yd, ym in outs:
            assert torch.equal(yd, want_d) and torch.equal(ym, want_m), prec
    # a workspace one byte short, or misaligned, is refused
    ws = torch.empty(op.workspace_size(3) + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(FtmError) as ei:
        op.apply(Mt, ws[: op.workspace_size(3) - 1])
    assert ei.value.status == 1
    with pytest.raises(FtmError) as ei:
        op.apply(Mt, ws[8:])
    assert ei.value.status == 1
    op.close()
    assert _rel(want_d.cpu().numpy(), oracle.forward(F, M)) <= 1e-6


def test_repeat_is_bitwise_deterministic(gpu):
    import torch
    from paper_2508_10202_amd import Operator
    s = Shape(64, 16, 256)
    F, m = make_F(s, 61), make_m(s, 62)[0]
    op = Operator(torch.from_numpy(F).cuda(), fwd="sssss", adj="dhhhd", spectra=("d",))
    mt = torch.from_numpy(m).cuda()
    dt = torch.from_numpy(make_d(s, 63)[0]).cuda()
    a1, a2 = op.matvec(mt).cpu(), op.matvec(mt).cpu()
    b1, b2 = op.rmatvec(dt).cpu(), op.rmatvec(dt).cpu()
    op.close()
    assert torch.equal(a1, a2) and torch.equal(b1, b2)


def test_abi_errors_on_gpu(gpu):
    import torch
    from paper_2508_10202_amd import FtmError, Operator
    s = Shape(16, 4, 8)
    op = Operator(torch.from_numpy(make_F(s, 71)).cuda(), max_rhs=2)
    m = torch.zeros((3, s.Nt, s.Nm), dtype=torch.float64, device="cuda")
    with pytest.raises(FtmError) as ei:
        op.matvec(m)                  # nrhs 3 > max_rhs 2
    assert ei.value.status == 1
    with pytest.raises(FtmError) as ei:
        op.set_precision(fwd="ddsdd")  # FP32 spectrum not kept
    assert ei.value.status == 2
    buf = torch.zeros(s.Nt * max(s.Nm, s.Nd) * 2, dtype=torch.float64, device="cuda")
    from paper_2508_10202_amd._lib import lib
    rc = lib().ftm_matvec(op.handle, buf.data_ptr(), buf.data_ptr() + 8, 1, None)
    assert rc == 1                    # input and output overlap
    op.close()


# --- mixed precision ---------------------------------------------------------------

U = {"d": 2.0 ** -53, "s": 2.0 ** -24, "h": 2.0 ** -11, "b": 2.0 ** -8}


def mp_bounds(prec: str, L: int, n: int):
    """Tolerance window for one precision string, shaped after eq. (error):
    pad/unpad rounding once, FFT/IFFT growing like log2 L, the product's
    storage rounding of Fhat and of its input, and its accumulation error
    (float32 accumulation: log2 n).  ``hi`` = 4x that budget; ``lo`` = the
    largest unit roundoff present / 64, so a phase that silently skips its
    rounding fails too."""
    from paper_2508_10202_amd import Precision
    p = Precision.parse(prec)
    ch = prec.split("+")[0]
    acc = U["d"] if p.accum == 0 else U["s"]
    lg = math.log2(L)
    budget = (U[ch[0]] + U[ch[1]] * lg + 2 * U[ch[2]] + acc * math.log2(max(n, 2))
              + U[ch[3]] * lg + U[ch[4]] + U["d"] * lg)
    lo = max(U[c] for c in ch) / 64 if ch != "ddddd" else 0.0
    return lo, 4 * budget + 1e-14


MP_CONFIGS = ["sdddd", "dsddd", "ddsdd", "ddsdd+a64", "dddsd", "dddds", "dssdd", "ddssd", "sssss",
              "ddhdd", "ddbdd", "dhddd", "dbddd", "dddhd", "dddbd", "hdddd", "ddddb",
              "dhhhd", "dbbbd", "hhhhh", "bbbbb", "shsbs"]


@pytest.fixture(scope="module")
def mp_case():
    s = Shape(200, 24, 1000)
    F, m, d = make_F(s, 81), make_m(s, 82)[0], make_d(s, 83)[0]
    return s, F, m, d, oracle.forward(F, m), oracle.adjoint(F, d)


@pytest.mark.parametrize("prec", MP_CONFIGS)
def test_mixed_precision_within_tolerance(gpu, mp_case, prec):
    s, F, m, d, ref_d, ref_m = mp_case
    _say("case mixed", prec)
    out = _run(F, m, d, fwd=prec, adj=prec)
    e_f, e_a = _rel(out["d"], ref_d), _rel(out["m"], ref_m)
    lo_f, hi_f = mp_bounds(prec, s.L, s.Nm)
    lo_a, hi_a = mp_bounds(prec, s.L, s.Nd)
    _say(f"  {prec}: fwd {e_f:.3e} in [{lo_f:.1e}, {hi_f:.1e}], adj {e_a:.3e} in [{lo_a:.1e}, {hi_a:.1e}]")
    assert lo_f <= e_f <= hi_f
    assert lo_a <= e_a <= hi_a


# --- the paper's shape at full size -----------------------------------------------------

@pytest.fixture(scope="module")
def paper_case():
    s, F, m, d = config_inputs("paper")
    return s, F, m[0], d[0]


def test_paper_shape_fp64_full_vectors(gpu, paper_case):
    """Nt=1000, Nd=100, Nm=5000 in float64: whole outputs vs the oracle, plus
    exactly rounded single entries."""
    import torch
    from paper_2508_10202_amd import Operator
    s, F, m, d = paper_case
    _say("case paper fp64")
    op = Operator(torch.from_numpy(F).cuda())
    got_d = op.matvec(torch.from_numpy(m).cuda()).cpu().numpy()
    got_m = op.rmatvec(torch.from_numpy(d).cuda()).cpu().numpy()
    op.close()
    ref_d, ref_m = oracle.forward(F, m), oracle.adjoint(F, d)
    e_f, e_a = _rel(got_d, ref_d), _rel(got_m, ref_m)
    _say(f"  paper fp64 rel err fwd {e_f:.3e} adj {e_a:.3e}")
    assert e_f <= FP64_TOL and e_a <= FP64_TOL
    rng = np.random.default_rng(5)
    ii, rr = rng.integers(0, s.Nt, 12), rng.integers(0, s.Nd, 12)
    ii[0], rr[0] = s.Nt - 1, s.Nd - 1                  # the longest sum
    ex = oracle.forward_entries(F, m, ii, rr)
    assert _rel(got_d[ii, rr], ex) <= FP64_TOL
    jj, cc = rng.integers(0, s.Nt, 12), rng.integers(0, s.Nm, 12)
    jj[0], cc[0] = 0, s.Nm - 1
    ea = oracle.adjoint_entries(F, d, jj, cc)
    assert _rel(got_m[jj, cc], ea) <= FP64_TOL


def test_paper_shape_mixed(gpu, paper_case):
    """The paper's optimum (FFT(m) and the product in FP32) and the all-FP32
    and half-storage configurations at the full shape."""
    import torch
    from paper_2508_10202_amd import Operator
    s, F, m, d = paper_case
    ref_d, ref_m = oracle.forward(F, m), oracle.adjoint(F, d)
    op = Operator(torch.from_numpy(F).cuda(), spectra=("s", "h", "b"))
    mt, dt = torch.from_numpy(m).cuda(), torch.from_numpy(d).cuda()
    for fwd, adj in (("dssdd", "ddssd"), ("sssss", "sssss"), ("ddsdd+a64", "ddsdd+a64"),
                     ("dhhhd", "dhhhd"), ("dbbbd", "dbbbd")):
        _say("case paper mixed", fwd, adj)
        op.set_precision(fwd=fwd, adj=adj)
        e_f = _rel(op.matvec(mt).cpu().numpy(), ref_d)
        e_a = _rel(op.rmatvec(dt).cpu().numpy(), ref_m)
        lo_f, hi_f = mp_bounds(fwd, s.L, s.Nm)
        lo_a, hi_a = mp_bounds(adj, s.L, s.Nd)
        _say(f"  {fwd}/{adj}: fwd {e_f:.3e} [{lo_f:.1e},{hi_f:.1e}] adj {e_a:.3e} [{lo_a:.1e},{hi_a:.1e}]")
        assert lo_f <= e_f <= hi_f and lo_a <= e_a <= hi_a
    op.close()


# --- many right-hand sides: the matrix-core GEMM path ---------------------------------

GEMM_PRECS = ["ddsdd", "sssss", "ddhdd", "ddbdd", "dhhhd", "dbbbd", "ddddd", "ddsdd+a64", "sdsds+a64"]


@pytest.fixture(scope="module")
def gemm_case():
    s = Shape(64, 40, 300, decay=50.0)       # Nd and Nm not multiples of the 16/64 tiles
    F = make_F(s, 91)
    M, D = make_m(s, 92, nrhs=70), make_d(s, 93, nrhs=70)
    return s, F, M, D, oracle.forward(F, M), oracle.adjoint(F, D)


def _gemm_bounds(prec, L, n):
    lo, hi = mp_bounds(prec, L, n)
    return (lo, FP64_TOL) if prec == "ddddd" else (lo, hi)


@pytest.mark.parametrize("prec", GEMM_PRECS)
@pytest.mark.parametrize("nrhs", [2, 17, 33, 70])
def test_gemm_path_vs_oracle(gpu, gemm_case, prec, nrhs):
    """Forced GEMM path (ragged in every tile dimension) for every right-hand-side
    tile (16, 32, 64, and the default for the batch) against the oracle, every
    right-hand side checked, and against the one-vector-at-a-time path of the
    same configuration.  float64 products and +a64 ones accumulate in float64
    on the matrix cores."""
    import torch
    from paper_2508_10202_amd import Operator
    s, F, M, D, ref_d, ref_m = gemm_case
    op = Operator(torch.from_numpy(F).cuda(), fwd=prec, adj=prec, max_rhs=nrhs)
    Mt, Dt = torch.from_numpy(M[:nrhs].copy()).cuda(), torch.from_numpy(D[:nrhs].copy()).cuda()
    op.set_rhs_mode("gemv")
    vd, vm = op.matvec(Mt).cpu().numpy(), op.rmatvec(Dt).cpu().numpy()
    op.set_rhs_mode("gemm")
    lo_f, hi_f = _gemm_bounds(prec, s.L, s.Nm)
    lo_a, hi_a = _gemm_bounds(prec, s.L, s.Nd)
    # FP32-storage products with float32 accumulation: both instruction kinds
    kinds = (0, 1, 2) if prec[2] == "s" and "+a64" not in prec else (0,)
    for tile in (0, 16, 32, 64):
        for kind in kinds:
            _say("case gemm", prec, nrhs, "tile", tile, "kind", kind)
            op.set_tuning(gemm_tile=(tile, tile), gemm_kind=(kind, kind))
            gd, gm = op.matvec(Mt).cpu().numpy(), op.rmatvec(Dt).cpu().numpy()
            e_f, e_a = _rel(gd, ref_d[:nrhs]), _rel(gm, ref_m[:nrhs])
            _say(f"  gemm {prec} nrhs={nrhs} tile={tile} kind={kind}: fwd {e_f:.3e} adj {e_a:.3e}; "
                 f"gemv fwd {_rel(vd, ref_d[:nrhs]):.3e}")
            assert lo_f <= e_f <= hi_f and lo_a <= e_a <= hi_a
            for b in range(nrhs):                 # every right-hand side, not just the norm
                assert _rel(gd[b], ref_d[b]) <= hi_f and _rel(gm[b], ref_m[b]) <= hi_a
            assert _rel(gd, vd) <= 2 * hi_f and _rel(gm, vm) <= 2 * hi_a
    op.close()


@pytest.mark.parametrize("Nd", [9, 24, 32])
def test_gemm_few_sensors(gpu, Nd):
    """Forward GEMM with at most 32 sensors, where half or more of each
    workgroup's waves own only rows past Nd and skip their spectrum loads and
    matrix-core work: every product kind and tile against the oracle and
    against the one-vector path, every right-hand side checked."""
    import torch
    from paper_2508_10202_amd import Operator
    s = Shape(64, Nd, 300, decay=50.0)
    nrhs = 37
    F, M, D = make_F(s, 95), make_m(s, 96, nrhs=nrhs), make_d(s, 97, nrhs=nrhs)
    ref_d = oracle.forward(F, M)
    op = Operator(torch.from_numpy(F).cuda(), spectra=("s", "b"), max_rhs=nrhs)
    Mt = torch.from_numpy(M).cuda()
    for prec in ("ddsdd", "dbbbd", "ddddd", "ddsdd+a64"):
        op.set_precision(fwd=prec, adj=prec)
        op.set_rhs_mode("gemv")
        vd = op.matvec(Mt).cpu().numpy()
        op.set_rhs_mode("gemm")
        lo_f, hi_f = _gemm_bounds(prec, s.L, s.Nm)
        kinds = (1, 2) if prec == "ddsdd" else (0,)
        for tile in (16, 64):
            for kind in kinds:
                _say("case gemm few sensors", Nd, prec, "tile", tile, "kind", kind)
                op.set_tuning(gemm_tile=(tile, tile), gemm_kind=(kind, kind))
                gd = op.matvec(Mt).cpu().numpy()
                e_f = _rel(gd, ref_d)
                assert lo_f <= e_f <= hi_f, (prec, tile, kind, e_f)
                for b in range(nrhs):
                    assert _rel(gd[b], ref_d[b]) <= hi_f, (prec, tile, kind, b)
                assert _rel(gd, vd) <= 2 * hi_f
    op.close()


def test_gemm_multi_rhs_shape(gpu):
    """Nt=512, Nd=128, Nm=4096 with 64 right-hand sides, FP32 and BF16 products on
    the matrix cores; four of the right-hand sides checked against the oracle."""
    import torch
    from paper_2508_10202_amd import Operator
    from workloads import MULTI_RHS, MULTI_RHS_NRHS, config_inputs
    s, F, M, D = config_inputs("multi_rhs", nrhs=MULTI_RHS_NRHS)
    pick = [0, 21, 42, 63]
    ref_d, ref_m = oracle.forward(F, M[pick]), oracle.adjoint(F, D[pick])
    op = Operator(torch.from_numpy(F).cuda(), fwd="ddsdd", adj="ddsdd", spectra=("b", "d"), max_rhs=64)
    Mt, Dt = torch.from_numpy(M).cuda(), torch.from_numpy(D).cuda()
    for prec, kind in (("ddsdd", 1), ("ddsdd", 2), ("dbbbd", 0), ("ddddd", 0), ("ddsdd+a64", 0)):
        _say("case multi-rhs", prec, "kind", kind)
        op.set_precision(fwd=prec, adj=prec)
        op.set_tuning(gemm_kind=(kind, kind))
        gd, gm = op.matvec(Mt).cpu().numpy(), op.rmatvec(Dt).cpu().numpy()
        e_f, e_a = _rel(gd[pick], ref_d), _rel(gm[pick], ref_m)
        lo_f, hi_f = _gemm_bounds(prec, s.L, s.Nm)
        lo_a, hi_a = _gemm_bounds(prec, s.L, s.Nd)
        _say(f"  multi-rhs {prec}: fwd {e_f:.3e} [{lo_f:.1e},{hi_f:.1e}] adj {e_a:.3e} [{lo_a:.1e},{hi_a:.1e}]")
        assert lo_f <= e_f <= hi_f and lo_a <= e_a <= hi_a
    op.close()


# --- data-space Hessian actions F F^T ----------------------------------------------------

@pytest.mark.parametrize("prec,nrhs,s", [
    ("ddddd", 3, Shape(64, 16, 256)),
    ("ddddd", 1, Shape(45, 13, 301, decay=30.0)),
    ("ddddd", 5, Shape(100, 37, 1000)),        # float64 matrix-core path for both directions
    ("dssdd", 20, Shape(100, 37, 1000)),       # float32 matrix-core path
    ("ddsdd+a64", 20, Shape(64, 40, 300, decay=50.0)),
])
def test_hessian_actions_vs_oracle(gpu, prec, nrhs, s):
    """y = F F^T x through ftm_hessian_apply against the oracle's definition,
    every right-hand side, plus the symmetry <Hx, z> = <x, Hz> on the GPU's own
    outputs."""
    import torch
    from paper_2508_10202_amd import Operator
    _say("case hessian", prec, nrhs, s)
    F = make_F(s, 121)
    X, Z = make_d(s, 122, nrhs=nrhs), make_d(s, 123, nrhs=nrhs)
    op = Operator(torch.from_numpy(F).cuda(), fwd=prec, adj=prec, max_rhs=nrhs)
    Xt, Zt = torch.from_numpy(X).cuda(), torch.from_numpy(Z).cuda()
    ws = torch.full(((op.hessian_workspace_size(nrhs) + 7) // 8,), float("nan"), dtype=torch.float64, device="cuda")
    hx = op.hessian(Xt, workspace=ws).cpu().numpy()
    hz = op.hessian(Zt).cpu().numpy()
    ref = oracle.hessian_data_space(F, X)
    tol = FP64_TOL if prec == "ddddd" else mp_bounds(prec, s.L, s.Nd)[1] + mp_bounds(prec, s.L, s.Nm)[1]
    e = _rel(hx, ref)
    _say(f"  hessian {prec}: {e:.3e} <= {tol:.1e}")
    assert e <= tol
    for b in range(nrhs):
        assert _rel(hx[b], ref[b]) <= tol
    lhs, rhs = float(np.vdot(hx, Z)), float(np.vdot(X, hz))
    assert abs(lhs - rhs) <= 4 * tol * (abs(lhs) + abs(rhs))
    from paper_2508_10202_amd import FtmError
    with pytest.raises(FtmError):                # a workspace one byte short
        from paper_2508_10202_amd import _lib
        out = torch.empty_like(Xt)
        _lib.check(_lib.lib().ftm_hessian_apply(op.handle, Xt.data_ptr(), out.data_ptr(), nrhs, ws.data_ptr(),
                                                op.hessian_workspace_size(nrhs) - 1, None), "ftm_hessian_apply")
    op.close()


# --- HIP graphs and the autotuner ------------------------------------------------------

def test_graph_replays_match_eager(gpu):
    """A captured matvec replayed several times, with eager work and
    synchronisations in between: every replay equals the eager result."""
    import torch
    from paper_2508_10202_amd import Operator
    s = Shape(64, 16, 256)
    F, m, d = make_F(s, 101), make_m(s, 102)[0], make_d(s, 103)[0]
    op = Operator(torch.from_numpy(F).cuda(), spectra=("s",))
    mt, dt = torch.from_numpy(m).cuda(), torch.from_numpy(d).cuda()
    for prec in ("ddddd", "dssdd"):
        op.set_precision(fwd=prec, adj=prec)
        ef, ea = op.matvec(mt).clone(), op.rmatvec(dt).clone()
        gf, ga = op.graph(mt), op.graph(dt, adjoint=True)
        for rep in range(4):
            gf.y.zero_()
            ga.y.zero_()
            torch.cuda.synchronize()
            gf.launch()
            ga.launch()
            op.matvec(mt)                       # eager work between replays
            torch.cuda.synchronize()
            assert torch.equal(gf.y[0], ef) and torch.equal(ga.y[0], ea), (prec, rep)
        gf.close()
        ga.close()
    op.close()
    assert _rel(ef.cpu().numpy(), oracle.forward(F, m)) <= 1e-6


def test_autotune_keeps_results_and_caches(gpu, tmp_path):
    """The autotuner picks among kernels that all compute the same product:
    every product tile variant and every transform kernel (fixed-plan large
    and small tile, runtime-plan) against the oracle, in float64 and float32."""
    import torch
    from paper_2508_10202_amd import Operator
    from paper_2508_10202_amd._lib import FFT_GENERIC
    for s in (Shape(200, 37, 1000), Shape(90, 11, 333, decay=30.0)):   # L = 400 (fixed plan), 180 (runtime plan)
        _say("case autotune", s)
        F, m, d = make_F(s, 111), make_m(s, 112)[0], make_d(s, 113)[0]
        op = Operator(torch.from_numpy(F).cuda(), spectra=("s",))
        cache = str(tmp_path / f"tune{s.Nt}.json")
        rec = op.autotune(reps=3, cache=cache)
        assert not rec["cached"] and all(0 <= v < 4 for v in rec["gemv_variant"])
        assert all(0 <= v <= FFT_GENERIC for r in rec["fft_shape"] for v in r)
        assert all(t > 0 for t in rec["ms"])
        assert all(2 <= c <= 33 for c in rec["gemm_min_rhs"])
        assert all(k in (0, 1, 2) for k in rec["gemm_kind"])
        assert op.autotune(cache=cache)["cached"]
        mt, dt = torch.from_numpy(m).cuda(), torch.from_numpy(d).cuda()
        ref_d, ref_m = oracle.forward(F, m), oracle.adjoint(F, d)
        for prec, tol in (("ddddd", FP64_TOL), ("sssss", mp_bounds("sssss", s.L, s.Nm)[1])):
            op.set_precision(fwd=prec, adj=prec)
            outs = []
            for v in range(4):                      # every product variant computes the same product
                for sh in range(FFT_GENERIC + 1):   # and every transform kernel
                    op.set_tuning(gemv_variant=(v, v), fft_shape=((sh, sh), (sh, sh)))
                    yd, ym = op.matvec(mt).cpu().numpy(), op.rmatvec(dt).cpu().numpy()
                    assert _rel(yd, ref_d) <= tol and _rel(ym, ref_m) <= tol, (prec, v, sh)
                    outs.append((yd, ym))
            if prec == "ddddd":
                for yd, ym in outs[1:]:
                    assert _rel(yd, outs[0][0]) <= 1e-14 and _rel(ym, outs[0][1]) <= 1e-14
        from paper_2508_10202_amd import FtmError
        with pytest.raises(FtmError):
            op.set_tuning(gemv_variant=(4, 0))
        with pytest.raises(FtmError):
            op.set_tuning(fft_shape=((4, 0), (0, 0)))
        with pytest.raises(FtmError):
            op.set_tuning(gemm_kind=(3, 0))
        op.close()


# --- rounding into the storage formats ---------------------------------------------------

def _rne_ref(x, fmt):
    """Round to nearest, ties to even, by the definition: scale by the format's
    quantum at x's binade (exact powers of two), numpy.rint (ties to even) and
    scale back; beyond the largest finite value, infinity."""
    x = np.asarray(x, dtype=np.float64)
    if fmt == "d":
        return x.copy()
    if fmt == "s":
        with np.errstate(over="ignore"):
            return x.astype(np.float32).astype(np.float64)
    p, emin, vmax = (11, -14, 65504.0) if fmt == "h" else (8, -126, float.fromhex("0x1.fep127"))
    out = x.copy()
    fin = np.isfinite(x) & (x != 0)
    _, e = np.frexp(x[fin])
    E = np.maximum(e - 1, emin)
    q = np.ldexp(1.0, E - (p - 1))
    r = np.rint(x[fin] / q) * q
    r = np.where(np.abs(r) > vmax, np.copysign(np.inf, x[fin]), r)
    out[fin] = r
    return out


def _rounding_cases():
    rng = np.random.default_rng(131)
    v = [rng.standard_normal(20000) * 10.0 ** rng.uniform(-44, 38, 20000)]
    # exact bfloat16 ties (low 16 bits 0x8000) and just off them in float64
    bits = (rng.integers(0x00800000, 0x7f000000, 4000, dtype=np.int64) & ~0xffff) | 0x8000
    ties_b = bits.astype(np.uint32).view(np.float32).astype(np.float64)
    v += [ties_b, -ties_b, ties_b * (1 + 2.0 ** -40), ties_b * (1 - 2.0 ** -40)]
    # exact FP16 ties (midpoints of neighbours, subnormal range included) and just off them
    with np.errstate(over="ignore"):
        h = np.sort(np.abs(rng.standard_normal(4000) * 10.0 ** rng.uniform(-7, 4.8, 4000))).astype(np.float16)
    hn = np.nextafter(h, np.float16(np.inf))
    mid = (h.astype(np.float64) + hn.astype(np.float64)) / 2
    mid = mid[np.isfinite(mid)]
    v += [mid, -mid, mid * (1 + 2.0 ** -40), mid * (1 - 2.0 ** -40)]
    v.append(np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 65504.0, 65519.99, 65520.0, 65536.0, 1e-8, 5.96e-8,
                       2.98e-8, 2.99e-8, float.fromhex("0x1.fep127"), float.fromhex("0x1.ffp127"),
                       float.fromhex("0x1.fefffffffffffp127"), 3.4e38, 1e-45, 1e-40, 1e300, -1e300]))
    return np.concatenate(v)


@pytest.mark.parametrize("fmt", ["s", "h", "b"])
@pytest.mark.parametrize("from_f32", [False, True])
def test_rounding_matches_round_to_nearest_even(gpu, fmt, from_f32):
    """The kernels' rounding into FP32/FP16/BF16 (ftm_round, the same device
    functions every phase uses) equals round-to-nearest-even by its
    definition, bitwise: ties, values just off ties in float64, subnormals,
    overflow to infinity, infinities and NaN; from float64 directly, and from
    float32 (the float32-compute phases)."""
    import torch
    from paper_2508_10202_amd import round_values
    x = _rounding_cases()
    got = round_values(torch.from_numpy(x).cuda(), fmt, from_f32=from_f32).cpu().numpy()
    src = _rne_ref(x, "s") if from_f32 else x
    want = _rne_ref(src, fmt)
    same = (got == want) | (np.isnan(got) & np.isnan(want))
    assert same.all(), (x[~same][:5], got[~same][:5], want[~same][:5])
    assert np.array_equal(np.signbit(got[~np.isnan(got)]), np.signbit(want[~np.isnan(want)]))


# --- first block column in other memory layouts --------------------------------------------

@pytest.mark.parametrize("s", [Shape(64, 7, 45, decay=None), Shape(45, 13, 31, decay=30.0), Shape(200, 5, 130)],
                         ids=lambda s: f"Nt{s.Nt}_Nd{s.Nd}_Nm{s.Nm}")
def test_setup_layouts(gpu, s):
    """F given as [Nd][Nm][Nt], [Nm][Nd][Nt], [Nt][Nm][Nd] and a padded
    [Nt][Nd][Nm] view: the setup transform reads the strides directly; the
    stored spectrum equals the plain layout's bitwise, and the matvecs match
    the oracle."""
    import torch
    from paper_2508_10202_amd import Operator
    F, m, d = make_F(s, 141), make_m(s, 142)[0], make_d(s, 143)[0]
    Ft = torch.from_numpy(F).cuda()
    base = Operator(Ft)
    ref_spec = base.spectrum("d").cpu().numpy()
    base.close()
    pad = torch.full((s.Nt, s.Nd + 3, s.Nm + 5), float("nan"), dtype=torch.float64, device="cuda")
    pad[:, : s.Nd, : s.Nm] = Ft
    views = {
        "dmt": Ft.permute(1, 2, 0).contiguous().permute(2, 0, 1),
        "mdt": Ft.permute(2, 1, 0).contiguous().permute(2, 1, 0),
        "tmd": Ft.permute(0, 2, 1).contiguous().permute(0, 2, 1),
        "padded": pad[:, : s.Nd, : s.Nm],
    }
    mt, dt = torch.from_numpy(m).cuda(), torch.from_numpy(d).cuda()
    ref_d, ref_m = oracle.forward(F, m), oracle.adjoint(F, d)
    for name, V in views.items():
        _say("case layout", name, tuple(V.stride()))
        assert not V.is_contiguous()
        op = Operator(V)
        assert np.array_equal(op.spectrum("d").cpu().numpy(), ref_spec), name
        assert _rel(op.matvec(mt).cpu().numpy(), ref_d) <= FP64_TOL
        assert _rel(op.rmatvec(dt).cpu().numpy(), ref_m) <= FP64_TOL
        op.close()


def test_setup_rejects_overlapping_strides(gpu):
    import ctypes
    import torch
    from paper_2508_10202_amd import _lib
    L = _lib.lib()
    F = torch.zeros(64, dtype=torch.float64, device="cuda")
    h = ctypes.c_void_p()
    # (t, r, c) strides (4, 2, 1) with Nd = 3: rows overlap
    assert L.ftm_setup_operator_strided(ctypes.byref(h), F.data_ptr(), 4, 3, 2, 4, 2, 1, None, None, 0, 1,
                                        None) == _lib.ERR_INVALID
    assert b"overlap" in L.ftm_last_error()



# --- tolerance-driven precision --------------------------------------------------------

@pytest.mark.parametrize("tol", [1e-12, 1e-6, 1e-3])
def test_select_precision_meets_tolerance(gpu, tol):
    """The library picks, per direction, the fastest configuration whose
    measured error on the probe is within the tolerance: the chosen
    configuration, run on another input, stays within it against the oracle
    (with a factor 4 for the input change); at 1e-12 only float64 qualifies."""
    import torch
    from paper_2508_10202_amd import Operator
    s = Shape(200, 24, 1000)
    F, m, d = make_F(s, 151), make_m(s, 152)[0], make_d(s, 153)[0]
    op = Operator(torch.from_numpy(F).cuda(), spectra=("s", "h", "b"))
    rf = op.select_precision(tol, adjoint=False, reps=2)
    ra = op.select_precision(tol, adjoint=True, reps=2)
    _say(f"case select {tol:g}: fwd {rf} adj {ra}")
    assert rf["err"] <= tol and ra["err"] <= tol and rf["ms"] > 0 and ra["ms"] > 0
    assert str(op.fwd) == rf["prec"] and str(op.adj) == ra["prec"]
    if tol < 1e-9:
        assert rf["prec"] == "ddddd" and ra["prec"] == "ddddd"
    e_f = _rel(op.matvec(torch.from_numpy(m).cuda()).cpu().numpy(), oracle.forward(F, m))
    e_a = _rel(op.rmatvec(torch.from_numpy(d).cuda()).cpu().numpy(), oracle.adjoint(F, d))
    assert e_f <= 4 * tol and e_a <= 4 * tol
    op.close()
