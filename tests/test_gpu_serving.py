"""Serving loop on the GPU: continuous batching, budget admission, and that
every result is the same alone and in the mix."""
import sys

import numpy as np
import pytest

import oracle
from workloads import Shape, make_F, normal

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ops():
    import torch
    from paper_2508_10202_amd import Operator
    shapes = [Shape(40, 12, 300, decay=30.0), Shape(64, 20, 500), Shape(25, 7, 130, decay=None)]
    Fs = [make_F(s, 500 + i) for i, s in enumerate(shapes)]
    out = []
    for s, F in zip(shapes, Fs):
        out.append((s, F, Operator(torch.from_numpy(F).cuda(), spectra=("s",), max_rhs=8)))
    yield out
    for _, _, op in out:
        op.close()


def _requests(ops, n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        k = int(rng.integers(len(ops)))
        adj = bool(rng.integers(2))
        nrhs = int(rng.integers(1, 9))
        s = ops[k][0]
        x = normal((nrhs, s.Nt, s.Nd if adj else s.Nm), 10_000 * seed + i)
        reqs.append((k, adj, x))
    return reqs


def _alone(op, adj, x):
    import torch
    xt = torch.from_numpy(x).cuda()
    return (op.rmatvec(xt) if adj else op.matvec(xt)).cpu().numpy()


@pytest.mark.parametrize("prec", ["ddddd", "sssss"])
def test_mix_equals_alone(gpu, ops, prec):
    """A burst of mixed requests (3 operators, both directions, 1-8 vectors)
    through the server: each output equals the oracle and the request run
    alone within the configuration's tolerance, and bitwise whenever the lone
    run takes the same product (the matrix-core GEMM is batch invariant, so a
    request of several vectors gives the same bits alone and in any batch; a
    lone single vector runs the matrix-vector kernel)."""
    import torch
    from paper_2508_10202_amd import Server
    for _, _, op in ops:
        op.set_precision(fwd=prec, adj=prec)
    try:
        _mix_equals_alone(ops, prec, Server, torch)
    finally:
        for _, _, op in ops:
            op.set_precision(fwd="ddddd", adj="ddddd")


def _mix_equals_alone(ops, prec, Server, torch):
    reqs = _requests(ops, 60, seed=1 if prec == "ddddd" else 2)
    xs = [torch.from_numpy(x).cuda() for _, _, x in reqs]
    torch.cuda.synchronize()
    with Server(workspace_budget=1 << 30, n_slots=3, max_batch_rhs=32) as srv:
        tickets = [srv.submit(ops[k][2], xs[i], adjoint=adj) for i, (k, adj, _) in enumerate(reqs)]
        lat = [srv.wait(t, timeout=60) for t, _ in tickets]
        st = srv.stats()
    _say(f"  serving {prec}: {st}")
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["coalesced_requests"] > 0            # requests did share batches
    assert all(l > 0 for l in lat)
    tol = 1e-12 if prec == "ddddd" else 2e-5
    n_bitwise = 0
    for (k, adj, x), (t, y) in zip(reqs, tickets):
        s, F, op = ops[k]
        got = y.cpu().numpy()
        ref = oracle.adjoint(F, x) if adj else oracle.forward(F, x)
        assert oracle.relative_l2(got, ref) <= tol
        alone = _alone(op, adj, x)
        assert oracle.relative_l2(got, alone) <= tol
        if x.shape[0] >= 2:                    # the lone run takes the GEMM too
            assert np.array_equal(got, alone)
        n_bitwise += int(np.array_equal(got, alone))
    _say(f"  {n_bitwise}/{len(reqs)} bitwise equal to the lone run")


def test_tiny_budget_queues_instead_of_failing(gpu, ops):
    """A budget that holds only one of the largest requests at a time: requests
    wait for workspace (budget_waits > 0), never fail, never exceed it."""
    import torch
    from paper_2508_10202_amd import Server
    for _, _, op in ops:
        op.set_precision(fwd="ddddd", adj="ddddd")
    need = max(op.workspace_size(8, adjoint=a) for _, _, op in ops for a in (False, True))
    reqs = _requests(ops, 40, seed=3)
    xs = [torch.from_numpy(x).cuda() for _, _, x in reqs]
    torch.cuda.synchronize()
    with Server(workspace_budget=need, n_slots=4, max_batch_rhs=8) as srv:
        tickets = [srv.submit(ops[k][2], xs[i], adjoint=adj) for i, (k, adj, _) in enumerate(reqs)]
        for t, _ in tickets:
            srv.wait(t, timeout=60)
        st = srv.stats()
    _say(f"  tiny budget: {st}")
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["budget_waits"] > 0
    assert st["peak_workspace_bytes"] <= need
    for (k, adj, x), (t, y) in zip(reqs, tickets):
        s, F, op = ops[k]
        ref = oracle.adjoint(F, x) if adj else oracle.forward(F, x)
        assert oracle.relative_l2(y.cpu().numpy(), ref) <= 1e-12


def _ws(op, nrhs):
    """Workspace bytes of one float64 batch (both directions' maximum), as the
    library sizes it."""
    keep = (op.fwd, op.adj)
    op.set_precision(fwd="ddddd", adj="ddddd")
    n = max(op.workspace_size(nrhs, adjoint=a) for a in (False, True))
    op.set_precision(fwd=keep[0], adj=keep[1])
    return n


def test_float32_batches_take_float32_workspace(gpu, ops):
    """With float32 intermediates a batch needs half the float64 workspace:
    a budget that holds exactly one float32 batch of 8 vectors admits it (the
    float64 sizing would reject it) and never exceeds the budget."""
    import torch
    from paper_2508_10202_amd import FtmError, Server
    s, F, op = ops[1]
    op.set_precision(fwd="sssss", adj="sssss")
    budget = op.workspace_size(8)
    op.set_precision(fwd="ddddd", adj="ddddd")
    assert budget < op.workspace_size(8)
    budget += 255                       # not a multiple of the arena's 256-byte granule
    x = normal((8, s.Nt, s.Nm), 4242)
    xt = torch.from_numpy(x).cuda()
    try:
        op.set_precision(fwd="sssss", adj="sssss")
        with Server(workspace_budget=budget, n_slots=2, max_batch_rhs=8) as srv:
            tickets = [srv.submit(op, xt) for _ in range(3)]
            for t, _ in tickets:
                srv.wait(t, timeout=60)
            st = srv.stats()
            op.set_precision(fwd="ddddd", adj="ddddd")
            with pytest.raises(FtmError) as ei:            # the float64 batch does not fit
                srv.submit(op, xt)
            assert ei.value.status == 4
    finally:
        op.set_precision(fwd="ddddd", adj="ddddd")
    _say(f"  float32 workspace: budget {budget}, {st}")
    assert st["completed"] == 3 and st["failed"] == 0
    assert st["peak_workspace_bytes"] <= budget
    ref = oracle.forward(F, x)
    tol = 2e-5
    for t, y in tickets:
        assert oracle.relative_l2(y.cpu().numpy(), ref) <= tol


def test_request_beyond_budget_is_rejected(gpu, ops):
    import torch
    from paper_2508_10202_amd import FtmError, Server
    s, F, op = ops[1]
    x = torch.zeros((8, s.Nt, s.Nm), dtype=torch.float64, device="cuda")
    with Server(workspace_budget=_ws(op, 2), n_slots=1, max_batch_rhs=8) as srv:
        with pytest.raises(FtmError) as ei:
            srv.submit(op, x)
        assert ei.value.status == 4            # FTM_ERR_BUDGET
        t, y = srv.submit(op, x[:1])           # one vector fits
        srv.wait(t, timeout=60)


def test_budget_not_a_multiple_of_the_granule(gpu, ops):
    """The budget is used in 256-byte granules: a budget a little above one
    request's workspace admits it, one byte below rejects it at submit."""
    import torch
    from paper_2508_10202_amd import FtmError, Server
    s, F, op = ops[0]
    op.set_precision(fwd="sssss", adj="sssss")
    try:
        need = op.workspace_size(1)
        assert need % 256 == 0
        x = torch.from_numpy(normal((1, s.Nt, s.Nm), 777)).cuda()
        with Server(workspace_budget=need + 100, n_slots=1, max_batch_rhs=1) as srv:
            t, y = srv.submit(op, x)
            srv.wait(t, timeout=60)
            assert oracle.relative_l2(y.cpu().numpy(), oracle.forward(F, x.cpu().numpy())) <= 2e-5
        with Server(workspace_budget=need - 1, n_slots=1, max_batch_rhs=1) as srv:
            with pytest.raises(FtmError) as ei:
                srv.submit(op, x)
            assert ei.value.status == 4
    finally:
        op.set_precision(fwd="ddddd", adj="ddddd")


def test_precision_change_while_queued(gpu, ops):
    """Switching an operator between float32 and float64 intermediates while
    its requests queue: each batch is sized and run with the configuration it
    was admitted with, so every request completes and is correct."""
    import torch
    from paper_2508_10202_amd import Server
    s, F, op = ops[1]
    x = normal((4, s.Nt, s.Nm), 888)
    xt = torch.from_numpy(x).cuda()
    ref = oracle.forward(F, x)
    budget = 3 * op.workspace_size(8)            # float64 sizing (the larger)
    tickets = []
    try:
        with Server(workspace_budget=budget, n_slots=2, max_batch_rhs=8) as srv:
            for i in range(40):
                op.set_precision(fwd="sssss" if i % 2 else "ddddd")
                tickets.append(srv.submit(op, xt))
            for t, _ in tickets:
                srv.wait(t, timeout=60)
            st = srv.stats()
    finally:
        op.set_precision(fwd="ddddd", adj="ddddd")
    _say(f"  precision switching: {st}")
    assert st["completed"] == 40 and st["failed"] == 0
    assert st["peak_workspace_bytes"] <= budget
    for t, y in tickets:
        assert oracle.relative_l2(y.cpu().numpy(), ref) <= 2e-5
