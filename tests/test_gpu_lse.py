"""GPU parity of the equality-constrained least-squares solve
(qr_lse_solve, null-space method on the library's QR) against the oracle's
own null-space solve of the same problem, plus the optimality invariants
(C x = d, gradient orthogonal to the null space of C) on the GPU result.

x is compared with the oracle's within the perturbation bound of the
problem: 50 n u kappa (1 + kappa ||r|| / (||A|| ||x||)) with kappa the
condition number of the stacked [A; C] (an upper estimate for the
constrained problem's)."""
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


SHAPES = [
    # (m, n, p, seed): one-workgroup sizes, blocked sizes, ragged panels,
    # p = 0 (plain least squares), p = n (fully constrained), m = n - p
    (20, 8, 3, 1), (128, 64, 16, 2), (300, 150, 40, 3), (700, 400, 100, 4), (1200, 600, 300, 5),
    (90, 40, 0, 6), (50, 30, 30, 7), (40, 70, 30, 8), (2000, 1100, 70, 9),
]


@pytest.mark.parametrize("m,n,p,seed", SHAPES)
def test_lse_matches_oracle(hqr, oracle_mod, m, n, p, seed):
    import torch
    rng = np.random.default_rng(1000 + seed)
    A = rng.standard_normal((m, n))
    C = rng.standard_normal((p, n))
    b = rng.standard_normal(m)
    d = rng.standard_normal(p)
    print("[case] qr_lse_solve", (m, n, p), flush=True)
    dA, dC = to_dev(A), to_dev(C) if p > 0 else to_dev(np.zeros((1, n)))[:0]
    db = to_dev(b.reshape(-1, 1))[:, 0]
    dd = to_dev(d.reshape(-1, 1))[:, 0] if p > 0 else None
    x, info = hqr.qr_lse_solve(dA, dC, db, dd)
    torch.cuda.synchronize()
    xg = to_host(x)[:n]
    assert int(info.item()) == 0
    xo, infoo = oracle_mod.lse_solve(A, C, b, d)
    assert infoo == 0
    S = np.vstack([A, C]) if p > 0 else A
    sv = np.linalg.svd(S, compute_uv=False)
    kappa, nA = sv[0] / sv[-1], sv[0]
    r = b - A @ xo
    bound = 50 * n * U * kappa * (1 + kappa * np.linalg.norm(r) / (nA * np.linalg.norm(xo)))
    err = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    print("[case] |x - x_oracle|/|x_oracle| %.2e (bound %.2e)" % (err, bound), flush=True)
    assert err <= bound
    if p > 0:
        assert np.linalg.norm(C @ xg - d) <= 100 * n * U * np.linalg.norm(C, 2) * np.linalg.norm(xg)
    if p < n:
        from scipy.linalg import null_space
        Z = null_space(C) if p > 0 else np.eye(n)
        g = A.T @ (A @ xg - b)
        assert np.linalg.norm(Z.T @ g) <= 100 * n * U * nA * (nA * np.linalg.norm(xg) + np.linalg.norm(b))


def test_lse_rank_deficient_constraints(hqr):
    import torch
    rng = np.random.default_rng(77)
    A = rng.standard_normal((30, 12))
    C = rng.standard_normal((4, 12))
    C[1] = 0.0
    print("[case] qr_lse_solve singular C", flush=True)
    x, info = hqr.qr_lse_solve(to_dev(A), to_dev(C), to_dev(rng.standard_normal((30, 1)))[:, 0],
                               to_dev(rng.standard_normal((4, 1)))[:, 0])
    torch.cuda.synchronize()
    assert int(info.item()) == 2


def test_lse_argument_errors(hqr):
    A = to_dev(np.ones((3, 5)))
    C = to_dev(np.ones((1, 5)))
    b = to_dev(np.ones((3, 1)))[:, 0]
    d = to_dev(np.ones((1, 1)))[:, 0]
    with pytest.raises(hqr.HQRError) as e:
        hqr.qr_lse_solve(A, C, b, d)       # m = 3 < n - p = 4
    assert e.value.status == -3
