"""Pins of the CPU oracle against things other than itself.

Each pin checks the oracle against the paper's printed structure, a closed
form, a textbook special case solved by a library routine, an invariant, or
brute force on tiny inputs.  ``test_planted_mistakes_are_caught`` plants
plausible mistakes in copies of the oracle and shows that some pin fails for
each of them.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from workloads import Shape, make_F, make_m, make_d, normal

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_case(Nt, Nd, Nm, seed=7):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((Nt, Nd, Nm)), rng.standard_normal((Nt, Nm)),
            rng.standard_normal((Nt, Nd)))


def _dense(F):
    """The block matrix of eq. (ShiftInvariance), assembled block by block."""
    Nt, Nd, Nm = F.shape
    A = np.zeros((Nt * Nd, Nt * Nm))
    for i in range(Nt):
        for j in range(i + 1):
            A[i * Nd:(i + 1) * Nd, j * Nm:(j + 1) * Nm] = F[i - j]
    return A


# --- pins, written as functions of (forward, adjoint) so mutants can be fed in

def pin_dense(fwd, adj):
    F, m, d = _rand_case(5, 3, 4)
    A = _dense(F)
    ok_f = np.allclose(fwd(F, m).ravel(), A @ m.ravel(), rtol=1e-13, atol=1e-13)
    ok_a = np.allclose(adj(F, d).ravel(), A.T @ d.ravel(), rtol=1e-13, atol=1e-13)
    return ok_f and ok_a


def pin_adjoint_identity(fwd, adj):
    F, m, d = _rand_case(9, 4, 6, seed=3)
    lhs = float(np.dot(fwd(F, m).ravel(), d.ravel()))
    rhs = float(np.dot(m.ravel(), adj(F, d).ravel()))
    return abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def pin_identity_block(fwd, adj):
    Nt, n = 6, 4
    F = np.zeros((Nt, n, n))
    F[0] = np.eye(n)
    _, m, _ = _rand_case(Nt, n, n, seed=5)
    return np.array_equal(fwd(F, m), m) and np.array_equal(adj(F, m), m)


def pin_delay_block(fwd, adj):
    Nt, n, s = 7, 3, 2
    F = np.zeros((Nt, n, n))
    F[s] = np.eye(n)
    _, m, _ = _rand_case(Nt, n, n, seed=6)
    want_f = np.zeros_like(m)
    want_f[s:] = m[:Nt - s]          # d_i = m_{i-s}
    want_a = np.zeros_like(m)
    want_a[:Nt - s] = m[s:]          # adjoint advances by s
    return np.array_equal(fwd(F, m), want_f) and np.array_equal(adj(F, m), want_a)


def pin_scalar_convolution(fwd, adj):
    """Nd = Nm = 1: the product is the causal convolution truncated to Nt."""
    rng = np.random.default_rng(11)
    Nt = 13
    f, x, y = rng.standard_normal(Nt), rng.standard_normal(Nt), rng.standard_normal(Nt)
    want_f = np.convolve(f, x)[:Nt]
    want_a = np.correlate(y, f, mode="full")[Nt - 1:]  # sum_{i>=j} f_{i-j} y_i
    got_f = fwd(f[:, None, None], x[:, None])[:, 0]
    got_a = adj(f[:, None, None], y[:, None])[:, 0]
    return np.allclose(got_f, want_f, rtol=1e-13, atol=1e-13) and \
        np.allclose(got_a, want_a, rtol=1e-13, atol=1e-13)


def pin_geometric_recursion(fwd, adj):
    """F_t = a^t I gives the first-order recursion d_i = a d_{i-1} + m_i."""
    a, Nt, n = 0.75, 20, 3
    F = np.stack([a ** t * np.eye(n) for t in range(Nt)])
    _, m, _ = _rand_case(Nt, n, n, seed=9)
    want = np.zeros_like(m)
    want[0] = m[0]
    for i in range(1, Nt):
        want[i] = a * want[i - 1] + m[i]
    back = np.zeros_like(m)                 # adjoint: x_j = a x_{j+1} + y_j
    back[-1] = m[-1]
    for j in range(Nt - 2, -1, -1):
        back[j] = a * back[j + 1] + m[j]
    return np.allclose(fwd(F, m), want, rtol=1e-12, atol=1e-12) and \
        np.allclose(adj(F, m), back, rtol=1e-12, atol=1e-12)


def pin_single_block(fwd, adj):
    F, m, d = _rand_case(1, 5, 8, seed=12)
    return np.allclose(fwd(F, m)[0], F[0] @ m[0], rtol=1e-14, atol=1e-14) and \
        np.allclose(adj(F, d)[0], F[0].T @ d[0], rtol=1e-14, atol=1e-14)


def pin_time_shift(fwd, adj):
    """Time invariance (Section 2.1): delaying m by one block delays d by one block."""
    F, m, _ = _rand_case(8, 3, 5, seed=13)
    ms = np.zeros_like(m)
    ms[1:] = m[:-1]
    d, ds = fwd(F, m), fwd(F, ms)
    return np.allclose(ds[1:], d[:-1], rtol=1e-13, atol=1e-13) and np.all(ds[0] == 0)


def pin_hand_example(fwd, adj):
    g = _golden("hand_worked_example.txt")
    F = np.stack([g["F0"], g["F1"], g["F2"]])[:, None, :]
    m = np.stack([g["m0"], g["m1"], g["m2"]])
    y = np.stack([g["y0"], g["y1"], g["y2"]])
    return np.array_equal(fwd(F, m).ravel(), g["d_expected"]) and \
        np.array_equal(adj(F, y).ravel(), g["x_expected"])


PINS = [pin_dense, pin_adjoint_identity, pin_identity_block, pin_delay_block,
        pin_scalar_convolution, pin_geometric_recursion, pin_single_block,
        pin_time_shift, pin_hand_example]


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out[key] = np.array([float(v) for v in vals])
    return out


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_oracle_pin(pin):
    assert pin(oracle.forward, oracle.adjoint)


def test_batched_rhs_matches_single():
    F, m, d = _rand_case(6, 3, 4, seed=21)
    M = np.stack([m, 2 * m + 1])
    got = oracle.forward(F, M)
    assert np.allclose(got[0], oracle.forward(F, m), rtol=0, atol=0)
    assert np.allclose(got[1], oracle.forward(F, 2 * m + 1), rtol=0, atol=0)


# --- mutation check: a plausible mistake anywhere must trip a pin ------------

def _mut_lag_off_by_one(F, m):
    Nt = F.shape[0]
    d = np.zeros(m.shape[:-2] + (Nt, F.shape[1]))
    for t in range(Nt):
        d[..., t:, :] += m[..., : Nt - t, :] @ F[min(t + 1, Nt - 1)].T
    return d


def _mut_anticausal(F, m):
    Nt = F.shape[0]
    d = np.zeros(m.shape[:-2] + (Nt, F.shape[1]))
    for t in range(Nt):
        d[..., : Nt - t, :] += m[..., t:, :] @ F[t].T
    return d


def _mut_drop_last_lag(F, m):
    Nt = F.shape[0]
    d = np.zeros(m.shape[:-2] + (Nt, F.shape[1]))
    for t in range(Nt - 1):
        d[..., t:, :] += m[..., : Nt - t, :] @ F[t].T
    return d


def _mut_transposed_block(F, m):
    """Uses F_t where F_t^T belongs (only shape-compatible for square blocks)."""
    Nt = F.shape[0]
    d = np.zeros(m.shape[:-2] + (Nt, F.shape[1]))
    for t in range(Nt):
        d[..., t:, :] += m[..., : Nt - t, :] @ F[t]
    return d


def _mut_adj_sign(F, d):
    return -oracle.adjoint(F, d) if F.shape[0] > 1 else oracle.adjoint(F, d)


def _mut_adj_forward_lags(F, d):
    Nt = F.shape[0]
    m = np.zeros(d.shape[:-2] + (Nt, F.shape[2]))
    for t in range(Nt):
        m[..., t:, :] += d[..., : Nt - t, :] @ F[t]
    return m


@pytest.mark.parametrize("fwd,adj", [
    (_mut_lag_off_by_one, oracle.adjoint),
    (_mut_anticausal, oracle.adjoint),
    (_mut_drop_last_lag, oracle.adjoint),
    (_mut_transposed_block, oracle.adjoint),
    (oracle.forward, _mut_adj_sign),
    (oracle.forward, _mut_adj_forward_lags),
], ids=["lag+1", "anticausal", "drop-last-lag", "transposed-block", "adj-sign", "adj-causal"])
def test_planted_mistakes_are_caught(fwd, adj):
    failed = [p.__name__ for p in PINS if not _safe(p, fwd, adj)]
    assert failed, "no pin caught the planted mistake"


def _safe(pin, fwd, adj):
    try:
        return pin(fwd, adj)
    except Exception:
        return False


# --- exact single entries ------------------------------------------------------

def test_exact_dot_is_correctly_rounded():
    rng = np.random.default_rng(5)
    for _ in range(20):
        a = rng.standard_normal(50) * 10.0 ** rng.integers(-8, 8, 50)
        b = rng.standard_normal(50)
        exact = sum(Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b))
        assert oracle.exact_dot(a, b) == float(exact)


def test_entries_match_full_product():
    s = Shape(40, 5, 33, decay=20.0)
    F, m, d = make_F(s, 1), make_m(s, 2)[0], make_d(s, 3)[0]
    rng = np.random.default_rng(0)
    ii, rr = rng.integers(0, s.Nt, 25), rng.integers(0, s.Nd, 25)
    jj, cc = rng.integers(0, s.Nt, 25), rng.integers(0, s.Nm, 25)
    full_f, full_a = oracle.forward(F, m), oracle.adjoint(F, d)
    ef = oracle.forward_entries(F, m, ii, rr)
    ea = oracle.adjoint_entries(F, d, jj, cc)
    assert np.allclose(ef, full_f[ii, rr], rtol=1e-13, atol=1e-13)
    assert np.allclose(ea, full_a[jj, cc], rtol=1e-13, atol=1e-13)


def test_entries_exact_on_integers():
    rng = np.random.default_rng(8)
    F = rng.integers(-5, 6, (6, 2, 3)).astype(float)
    m = rng.integers(-5, 6, (6, 3)).astype(float)
    A = _dense(F).astype(np.int64)
    want = A @ m.ravel().astype(np.int64)
    got = oracle.forward_entries(F, m, [i for i in range(6) for _ in range(2)], [0, 1] * 6)
    assert np.array_equal(got, want.astype(float))


# --- spectrum ------------------------------------------------------------------

def test_spectrum_hand_example():
    g = _golden("hand_worked_example.txt")
    F = np.stack([g["F0"], g["F1"], g["F2"]])[:, None, :]
    S = oracle.spectrum(F, ks=[0, 3])
    assert np.allclose(S[0, 0], g["Fhat0"], atol=1e-15)
    assert np.allclose(S[1, 0], g["Fhat3"], atol=1e-14)


def test_spectrum_matches_library_rfft():
    rng = np.random.default_rng(1)
    F = rng.standard_normal((25, 3, 4))
    ref = np.fft.rfft(F, n=50, axis=0)
    assert np.allclose(oracle.spectrum(F), ref, rtol=1e-12, atol=1e-12)


def test_spectrum_closed_forms():
    Nt, L = 16, 32
    imp = np.zeros((Nt, 1, 1))
    imp[0] = 1.0
    assert np.allclose(oracle.spectrum(imp)[:, 0, 0], 1.0, atol=1e-15)
    s = 5
    dl = np.zeros((Nt, 1, 1))
    dl[s] = 1.0
    k = np.arange(L // 2 + 1)
    assert np.allclose(oracle.spectrum(dl)[:, 0, 0], np.exp(-2j * np.pi * k * s / L), atol=1e-14)
    a = 0.9
    geo = (a ** np.arange(Nt))[:, None, None]
    z = a * np.exp(-2j * np.pi * k / L)
    closed = (1 - z ** Nt) / (1 - z)
    assert np.allclose(oracle.spectrum(geo)[:, 0, 0], closed, rtol=1e-13, atol=1e-13)


def test_spectrum_parseval():
    rng = np.random.default_rng(2)
    Nt = 30
    x = rng.standard_normal((Nt, 1, 1))
    X = oracle.spectrum(x)[:, 0, 0]
    L = 2 * Nt
    energy = abs(X[0]) ** 2 + abs(X[-1]) ** 2 + 2 * np.sum(abs(X[1:-1]) ** 2)
    assert math.isclose(energy, L * float(np.sum(x ** 2)), rel_tol=1e-13)


@pytest.mark.parametrize("L,exact", [(None, True), ("2Nt-1", True), ("2Nt-2", False)])
def test_fourier_route_reaches_the_definition(L, exact):
    """Zero padding to L >= 2Nt-1 makes the circulant product equal the Toeplitz one."""
    F, m, d = _rand_case(12, 3, 5, seed=30)
    Nt = 12
    Lv = {None: 2 * Nt, "2Nt-1": 2 * Nt - 1, "2Nt-2": 2 * Nt - 2}[L]
    Fh = np.fft.fft(F, n=Lv, axis=0)
    mh = np.fft.fft(m, n=Lv, axis=0)
    dh = np.einsum("krc,kc->kr", Fh, mh)
    via_fft = np.real(np.fft.ifft(dh, axis=0))[:Nt]
    close = np.allclose(via_fft, oracle.forward(F, m), rtol=1e-12, atol=1e-12)
    assert close == exact


def test_inputs_are_not_float32_representable():
    x = normal((1000,), 4)
    assert not np.any(x.astype(np.float32).astype(np.float64) == x)
    s = Shape(10, 3, 7)
    F = make_F(s, 5)
    assert not np.any(F.astype(np.float32).astype(np.float64) == F)


def test_relative_l2():
    ref = np.array([3.0, 4.0])
    assert oracle.relative_l2(ref + np.array([0.0, 0.5]), ref) == pytest.approx(0.1)


# --- the data-space Hessian F Gamma F^T (Gamma = I) ---------------------------------

def test_hessian_matches_dense_product():
    """Against the dense A A^T of the block matrix of eq. (ShiftInvariance)."""
    for Nt, Nd, Nm in ((5, 3, 4), (4, 6, 2), (1, 3, 5)):
        F, _, _ = _rand_case(Nt, Nd, Nm, seed=21)
        x = np.random.default_rng(22).standard_normal((2, Nt, Nd))
        A = _dense(F)
        H = A @ A.T
        got = oracle.hessian_data_space(F, x)
        for b in range(2):
            assert np.allclose(got[b].ravel(), H @ x[b].ravel(), rtol=1e-13, atol=1e-13)


def test_hessian_symmetric_and_semidefinite():
    F, _, _ = _rand_case(9, 4, 6, seed=23)
    rng = np.random.default_rng(24)
    x, y = rng.standard_normal((9, 4)), rng.standard_normal((9, 4))
    Hx, Hy = oracle.hessian_data_space(F, x), oracle.hessian_data_space(F, y)
    assert abs(np.vdot(Hx, y) - np.vdot(x, Hy)) <= 1e-12 * abs(np.vdot(Hx, y))
    # <Hx, x> = ||F^T x||^2 >= 0, with F^T x as the dense transpose computes it
    ft_x = _dense(F).T @ x.ravel()
    assert abs(np.vdot(Hx, x) - ft_x @ ft_x) <= 1e-12 * (ft_x @ ft_x)


def test_hessian_single_block_is_gram_matrix():
    """Nt = 1: H = F_0 F_0^T, a plain Gram matrix."""
    F, _, _ = _rand_case(1, 5, 7, seed=25)
    x = np.random.default_rng(26).standard_normal((1, 5))
    assert np.allclose(oracle.hessian_data_space(F, x)[0], F[0] @ (F[0].T @ x[0]), rtol=1e-14, atol=1e-14)
