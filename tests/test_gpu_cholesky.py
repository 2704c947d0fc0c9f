"""GPU parity of the Cholesky factorization (hqr_cholesky) and the rank-one
factor update (hqr_chol_update) against the oracle's, with the identities
that fix them: S = R^T R and R'^T R' = R^T R + v v^T to rounding."""
import numpy as np
import pytest

from tests.gpu_util import U, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hqr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2506_09463_amd as h
    h.load()
    return h


@pytest.mark.parametrize("n,seed", [(1, 1), (5, 2), (64, 3), (65, 4), (200, 5), (700, 6), (1500, 7)])
def test_cholesky_matches_oracle(hqr, oracle_mod, n, seed):
    import torch
    rng = np.random.default_rng(400 + seed)
    G = rng.standard_normal((n + 10, n))
    S = G.T @ G + n * np.eye(n) * 0.01
    L = np.tril(rng.standard_normal((n, n)), -1)      # the strict lower part must stay as it is
    Sin = np.triu(S) + L
    print("[case] hqr_cholesky", n, flush=True)
    dS = to_dev(Sin)
    _, info = hqr.cholesky(dS)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    F = to_host(dS)
    R = np.triu(F)
    assert np.array_equal(np.tril(F, -1), L)
    Ro, info_o = oracle_mod.cholesky(S)
    assert info_o == 0
    kappa = np.linalg.cond(S)
    assert np.abs(R - Ro).max() <= 50 * n * U * kappa * np.abs(Ro).max()
    assert np.linalg.norm(S - R.T @ R) <= 50 * n * U * np.linalg.norm(S)


def test_cholesky_not_positive_definite(hqr, oracle_mod):
    import torch
    rng = np.random.default_rng(9)
    n = 150
    G = rng.standard_normal((n + 10, n))
    S = G.T @ G
    S[100, 100] = -1.0               # pivot 100 becomes negative
    dS = to_dev(S)
    _, info = hqr.cholesky(dS)
    torch.cuda.synchronize()
    _, info_o = oracle_mod.cholesky(S)
    assert int(info.item()) == info_o == 101


@pytest.mark.parametrize("n,seed", [(1, 1), (7, 2), (300, 3), (1025, 4), (3000, 5)])
def test_chol_update_matches_oracle(hqr, oracle_mod, n, seed):
    import torch
    rng = np.random.default_rng(500 + seed)
    G = rng.standard_normal((n + 10, n))
    signs = np.where(rng.standard_normal(n) >= 0, 1.0, -1.0)
    R = signs[:, None] * np.linalg.cholesky(G.T @ G / n + np.eye(n)).T   # well conditioned, mixed signs
    v = rng.standard_normal(n)
    print("[case] hqr_chol_update", n, flush=True)
    dR, dv = to_dev(R), to_dev(v.reshape(-1, 1))[:, 0]
    hqr.chol_update(dR, dv)
    torch.cuda.synchronize()
    R2 = to_host(dR)
    assert np.array_equal(np.tril(R2, -1), np.zeros((n, n)))
    Ro = oracle_mod.chol_update(R, v)
    S2 = R.T @ R + np.outer(v, v)
    assert np.linalg.norm(S2 - R2.T @ R2) <= 50 * n * U * np.linalg.norm(S2)
    assert np.array_equal(np.sign(np.diag(R2)), np.sign(np.diag(R)))
    kappa = np.linalg.cond(S2) ** 0.5
    assert np.abs(R2 - Ro).max() <= 100 * n * U * kappa * np.abs(Ro).max()
