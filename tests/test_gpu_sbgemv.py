"""Parity of the strided-batched matrix-vector product (``ftm_sbgemv``, via
the C ABI) against the CPU oracle: every type (s, d, c, z) and op (N, T, C),
ragged shapes, padded leading dimensions (which switch off the 16-byte loads),
alpha / beta, and the short-wide shape of the paper's kernel benchmark
(batch 100, m = 128, n = 4096)."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

DTYPES = {"s": ("float32", 2e-6), "d": ("float64", 1e-14), "c": ("complex64", 2e-6), "z": ("complex128", 1e-14)}


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _inputs(t, batch, m, n, lda, op, seed):
    import torch
    rng = np.random.default_rng(seed)
    cplx = t in "cz"
    nx, ny = (n, m) if op == "N" else (m, n)

    def draw(shape):
        v = rng.standard_normal(shape)
        return v + 1j * rng.standard_normal(shape) if cplx else v
    dt = getattr(torch, DTYPES[t][0])
    A = torch.from_numpy(draw((batch, n, lda))).to(dt)
    x = torch.from_numpy(draw((batch, nx))).to(dt)
    y = torch.from_numpy(draw((batch, ny))).to(dt)
    return A, x, y


def _tol(t, length):
    # relative L2 error of a dot product of `length` terms, generously: the
    # unit roundoff times sqrt(length) (random signs) times 8
    u = DTYPES[t][1]
    return u * max(1.0, np.sqrt(length)) * 8


SHAPES = [(1, 1, 1, 1), (3, 5, 5, 2), (3, 5, 8, 3), (7, 300, 7, 2), (33, 1000, 36, 3),
          (200, 130, 201, 2), (65, 65, 65, 1), (128, 4096, 128, 3)]


@pytest.mark.parametrize("t", list("sdcz"))
@pytest.mark.parametrize("op", ["N", "T", "C"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "m%d_n%d_lda%d_b%d" % s)
def test_sbgemv_vs_oracle(gpu, t, op, shape):
    from paper_2508_10202_amd import sbgemv
    m, n, lda, batch = shape
    _say("case sbgemv", t, op, shape)
    A, x, y0 = _inputs(t, batch, m, n, lda, op, 7 + m + n)
    ref = oracle.sbgemv(op, A.numpy(), m, x.numpy())
    got = sbgemv(A.cuda(), x.cuda(), m=m, op=op).cpu().numpy()
    assert got.shape == ref.shape
    assert oracle.relative_l2(got, ref) <= _tol(t, n if op == "N" else m)
    # alpha / beta, y read and updated in place
    alpha, beta = (0.75 - 0.5j, 1.25 + 0.25j) if t in "cz" else (0.75, -1.25)
    yd = y0.cuda()
    sbgemv(A.cuda(), x.cuda(), m=m, op=op, alpha=alpha, beta=beta, y=yd)
    ref2 = oracle.sbgemv(op, A.numpy(), m, x.numpy(), alpha=alpha, beta=beta, y=y0.numpy())
    assert oracle.relative_l2(yd.cpu().numpy(), ref2) <= _tol(t, n if op == "N" else m) * 2


@pytest.mark.parametrize("t", list("sz"))
def test_beta_zero_does_not_read_y(gpu, t):
    import torch
    from paper_2508_10202_amd import sbgemv
    A, x, _ = _inputs(t, 2, 40, 300, 40, "C", 5)
    for op in ("N", "C"):
        xs = x if op == "C" else _inputs(t, 2, 40, 300, 40, "N", 6)[1]
        ny = 300 if op == "C" else 40
        y = torch.full((2, ny), float("nan"), dtype=A.dtype, device="cuda")
        sbgemv(A.cuda(), xs.cuda(), op=op, alpha=2.0, beta=0.0, y=y)
        assert torch.isfinite(torch.view_as_real(y) if y.is_complex() else y).all()
        ref = oracle.sbgemv(op, A.numpy(), 40, xs.numpy(), alpha=2.0)
        assert oracle.relative_l2(y.cpu().numpy(), ref) <= _tol(t, 300)


def test_paper_kernel_shape_all_types(gpu):
    """batch 100, m = 128, n = 4096 (short-wide), transposed ops as in the
    paper's kernel benchmark: sampled batch entries against the oracle."""
    import torch
    from paper_2508_10202_amd import sbgemv
    m, n, batch = 128, 4096, 100
    for t, op in (("s", "T"), ("d", "T"), ("c", "C"), ("z", "C")):
        _say("case sbgemv paper shape", t, op)
        A, x, _ = _inputs(t, batch, m, n, m, op, 99)
        got = sbgemv(A.cuda(), x.cuda(), op=op).cpu().numpy()
        pick = [0, 37, 99]
        ref = oracle.sbgemv(op, A.numpy()[pick], m, x.numpy()[pick])
        assert oracle.relative_l2(got[pick], ref) <= _tol(t, m)
        torch.cuda.synchronize()


@pytest.mark.parametrize("t", list("sdcz"))
@pytest.mark.parametrize("m,batch", [(256, 300), (512, 600)])
def test_op_n_load_widths(gpu, t, m, batch):
    """op N picks 16-, 8- or 4-byte loads from the grid size: batches large
    enough for the full and the halved width, against the oracle."""
    from paper_2508_10202_amd import sbgemv
    n = 40
    _say("case sbgemv op N widths", t, m, batch)
    A, x, _ = _inputs(t, batch, m, n, m, "N", 31 + m)
    got = sbgemv(A.cuda(), x.cuda(), op="N").cpu().numpy()
    ref = oracle.sbgemv("N", A.numpy(), m, x.numpy())
    assert oracle.relative_l2(got, ref) <= _tol(t, n)
