"""Pins of the batched matrix-vector oracle (``oracle.sbgemv``) against closed
forms and identities, not against its own formula (CPU only)."""
import numpy as np
import pytest

import oracle


def _cols(M):
    """column-major storage (batch, n, lda=m) of a batch of m x n matrices"""
    return np.ascontiguousarray(np.swapaxes(M, 1, 2))


def _rng(seed):
    return np.random.default_rng(seed)


def _randc(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_identity_diagonal_permutation_ones():
    rng = _rng(1)
    n = 6
    x = rng.standard_normal((1, n))
    I = np.eye(n)[None]
    for op in "NTC":
        assert np.array_equal(oracle.sbgemv(op, _cols(I), n, x), x)
    d = rng.standard_normal(n)
    D = np.diag(d)[None]
    for op in "NTC":
        assert np.allclose(oracle.sbgemv(op, _cols(D), n, x), d * x, rtol=0, atol=1e-15)
    perm = rng.permutation(n)
    P = np.eye(n)[perm][None]                      # (P x)_i = x_{perm[i]}
    assert np.array_equal(oracle.sbgemv("N", _cols(P), n, x), x[:, perm])
    inv = np.argsort(perm)                         # P^T undoes P
    assert np.array_equal(oracle.sbgemv("T", _cols(P), n, x), x[:, inv])
    m, n2 = 3, 5
    ones = np.ones((1, m, n2))
    xn, xm = rng.standard_normal((1, n2)), rng.standard_normal((1, m))
    assert np.allclose(oracle.sbgemv("N", _cols(ones), m, xn), np.full((1, m), xn.sum()), atol=1e-14)
    assert np.allclose(oracle.sbgemv("T", _cols(ones), m, xm), np.full((1, n2), xm.sum()), atol=1e-14)


@pytest.mark.parametrize("cplx", [False, True])
def test_adjoint_identity_links_n_and_c(cplx):
    rng = _rng(2)
    b, m, n = 3, 7, 11
    M = _randc(rng, (b, m, n)) if cplx else rng.standard_normal((b, m, n))
    x = _randc(rng, (b, n)) if cplx else rng.standard_normal((b, n))
    w = _randc(rng, (b, m)) if cplx else rng.standard_normal((b, m))
    Ax = oracle.sbgemv("N", _cols(M), m, x)
    AHw = oracle.sbgemv("C", _cols(M), m, w)
    for k in range(b):
        lhs = np.vdot(w[k], Ax[k])                 # <A x, w>
        rhs = np.vdot(AHw[k], x[k])                # <x, A^H w>
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_conjugate_transpose_vs_transpose():
    rng = _rng(3)
    b, m, n = 2, 5, 9
    Mr = rng.standard_normal((b, m, n))
    xr = rng.standard_normal((b, m))
    assert np.array_equal(oracle.sbgemv("C", _cols(Mr), m, xr), oracle.sbgemv("T", _cols(Mr), m, xr))
    Mc, xc = _randc(rng, (b, m, n)), _randc(rng, (b, m))
    got = oracle.sbgemv("C", _cols(Mc), m, xc)
    via_t = np.conj(oracle.sbgemv("T", _cols(Mc), m, np.conj(xc)))
    assert np.allclose(got, via_t, rtol=0, atol=1e-13)
    assert not np.allclose(got, oracle.sbgemv("T", _cols(Mc), m, xc))   # a dropped conjugation shows


def test_lda_padding_ignored_and_alpha_beta_linear():
    rng = _rng(4)
    b, m, n, lda = 2, 4, 6, 7
    cols = rng.standard_normal((b, n, lda))
    cols_junk = cols.copy()
    cols_junk[:, :, m:] = np.nan                   # rows m .. lda-1 are never used
    x = rng.standard_normal((b, n))
    y0 = rng.standard_normal((b, m))
    base = oracle.sbgemv("N", cols, m, x)
    assert np.array_equal(oracle.sbgemv("N", cols_junk, m, x), base)
    got = oracle.sbgemv("N", cols, m, x, alpha=2.5, beta=-0.5, y=y0)
    assert np.allclose(got, 2.5 * base - 0.5 * y0, rtol=0, atol=1e-14)
    y_nan = np.full((b, m), np.nan)
    assert np.all(np.isfinite(oracle.sbgemv("N", cols, m, x, alpha=1.0, beta=0.0, y=y_nan)))


def test_single_entry_matrix():
    # A = e_i e_j^T: op N moves x_j to row i, op T moves x_i to column j
    m, n, i, j = 4, 5, 2, 3
    M = np.zeros((1, m, n))
    M[0, i, j] = 1.0
    xn, xm = np.arange(1.0, n + 1)[None], np.arange(1.0, m + 1)[None]
    yn, yt = oracle.sbgemv("N", _cols(M), m, xn), oracle.sbgemv("T", _cols(M), m, xm)
    assert yn[0, i] == xn[0, j] and np.count_nonzero(yn) == 1
    assert yt[0, j] == xm[0, i] and np.count_nonzero(yt) == 1


def test_relative_l2_counts_imaginary_parts():
    # ||(1+i) - 1|| / ||1|| = 1: an error only in the imaginary part is seen
    assert oracle.relative_l2(np.array([1 + 1j]), np.array([1 + 0j])) == 1.0
    assert oracle.relative_l2(np.array([3.0, 4.0]), np.array([0.0, 4.0])) == 0.75
