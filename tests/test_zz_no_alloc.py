"""ftm_apply_scratch: the matvec on the library's static per-GPU scratch
(no device allocation) against ftm_apply on a caller workspace, through the
C ABI.  Two calls in a row, the second with a smaller input, in float64 and
with float32 intermediates (the matrix-core path for several right-hand
sides); both also against the oracle."""
import sys

import numpy as np
import pytest

import oracle
from workloads import Shape, make_d, make_F, make_m

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _op(s, seed, **kw):
    import torch
    from paper_2508_10202_amd import Operator
    F = make_F(s, seed)
    return F, Operator(torch.from_numpy(F).cuda(), **kw)


def _nan_workspace(op, nrhs, adjoint):
    import torch
    n = op.workspace_size(nrhs, adjoint)
    return torch.full(((n + 7) // 8,), float("nan"), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("prec", ["ddddd", "dssdd"])
def test_scratch_matches_caller_workspace(gpu, prec):
    import torch
    big, small = Shape(100, 37, 1000), Shape(45, 13, 301, decay=30.0)
    F1, op1 = _op(big, 301, fwd=prec, adj=prec, max_rhs=3)
    F2, op2 = _op(small, 302, fwd=prec, adj=prec)
    tol = 1e-12 if prec == "ddddd" else 1e-5
    for F, op, s, nrhs, seed in ((F1, op1, big, 3, 303), (F2, op2, small, 1, 304)):
        m, d = make_m(s, seed, nrhs), make_d(s, seed + 1, nrhs)
        mt, dt = torch.from_numpy(m).cuda(), torch.from_numpy(d).cuda()
        for adjoint, x, ref in ((False, mt, oracle.forward(F, m)), (True, dt, oracle.adjoint(F, d))):
            _say(f"case scratch {prec} shape {s.Nt}x{s.Nd}x{s.Nm} nrhs {nrhs} adjoint {adjoint}")
            got = op.apply_scratch(x, adjoint=adjoint)
            want = op.apply(x, _nan_workspace(op, nrhs, adjoint), adjoint=adjoint)
            torch.cuda.synchronize()
            g, w = got.cpu().numpy(), want.cpu().numpy()
            assert np.array_equal(g, w), f"max diff {np.max(np.abs(g - w))}"
            assert oracle.relative_l2(g, ref) <= tol
    op1.close()
    op2.close()


def test_scratch_rejects_calls_beyond_its_size(gpu):
    import torch
    from paper_2508_10202_amd import _lib
    s = Shape(1000, 1, 5000)
    _, op = _op(s, 305)
    assert op.workspace_size(1) <= _lib.SCRATCH_BYTES < op.workspace_size(2)
    m = torch.from_numpy(make_m(s, 306, 2)).cuda()
    with pytest.raises(_lib.FtmError) as ei:
        op.apply_scratch(m)
    assert ei.value.status == _lib.ERR_UNSUPPORTED
    one = op.apply_scratch(m[0])
    torch.cuda.synchronize()
    assert oracle.relative_l2(one.cpu().numpy(), oracle.forward(make_F(s, 305), m[0].cpu().numpy())) <= 1e-12
    op.close()
