"""The near-identity factorization used by the second CholeskyQR pass.

For G = I + E (E symmetric, every |E_ij| <= 2^-30) the GPU kernel forms
X0 = Phi(E), X1 = Phi(E - X0^T X0), R = I + X1 and R^{-1} = I - X1 + X1^2,
Phi(M) = strict upper part of M plus half its diagonal, instead of pivoting.
These CPU checks pin that arithmetic to LAPACK's Cholesky factor: R^T R = G
exactly in the second-order terms, the factor differs from the pivoted one
by at most 2 ||E||_F^3 (plus rounding), and the inverse series by ||X1||^3.
They also show why the bound is needed: at |E| ~ 1e-3 one correction step
is no longer exact to rounding.
"""
import numpy as np
import pytest

TAU = 2.0 ** -30
U = np.finfo(np.float64).eps / 2


def phi(m):
    return np.triu(m, 1) + 0.5 * np.diag(np.diag(m))


def series(g):
    n = g.shape[0]
    e = g - np.eye(n)
    x0 = phi(e)
    x1 = phi(e - x0.T @ x0)
    return np.eye(n) + x1, np.eye(n) - x1 + x1 @ x1, x1


def near_identity_gram(n, scale, seed):
    """Gram matrix of a slightly non-orthonormal basis: Q^T Q with Q = orth + noise."""
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((4 * n, n)))
    q = q + scale * rng.standard_normal(q.shape)
    return q.T @ q


@pytest.mark.parametrize("scale", [1e-16, 1e-14, 1e-12])
def test_series_matches_cholesky_within_bound(scale):
    g = near_identity_gram(64, scale, seed=7)
    e = g - np.eye(64)
    assert np.abs(e).max() <= TAU
    r, rinv, x1 = series(g)
    rref = np.linalg.cholesky(g).T
    eps = np.linalg.norm(e)
    # both factors are upper triangular with positive diagonal
    assert np.allclose(np.tril(r, -1), 0.0) and (np.diag(r) > 0).all()
    # same factor up to the series error and the rounding of entries near 1
    assert np.abs(r - rref).max() <= 2 * eps ** 3 + 8 * U
    # residual of the factorization as small as the pivoted one's (to rounding)
    res = np.abs(r.T @ r - g).max()
    res_ref = np.abs(rref.T @ rref - g).max()
    assert res <= max(4 * res_ref, 16 * U)
    # inverse series
    assert np.abs(r @ rinv - np.eye(64)).max() <= np.linalg.norm(x1) ** 3 + 16 * U


def test_second_order_term_is_needed():
    """With X0 alone the residual is X0^T X0 (of size ||E||^2): visible once
    ||E|| is above sqrt(u); the correction step removes it."""
    g = near_identity_gram(64, 1e-6, seed=3)
    e = g - np.eye(64)
    x0 = phi(e)
    r0 = np.eye(64) + x0
    r, _, _ = series(g)
    res0 = np.abs(r0.T @ r0 - g).max()
    res1 = np.abs(r.T @ r - g).max()
    assert res0 > 1e3 * res1


def test_bound_is_what_keeps_one_step_exact():
    """At |E| ~ 1e-3 (far beyond 2^-30) one correction step leaves an error
    of order ||E||^3, well above rounding: the kernel then pivots instead."""
    g = near_identity_gram(64, 1e-4, seed=5)
    e = g - np.eye(64)
    assert np.abs(e).max() > TAU
    r, _, _ = series(g)
    rref = np.linalg.cholesky(g).T
    assert np.abs(r - rref).max() > 1e3 * U
