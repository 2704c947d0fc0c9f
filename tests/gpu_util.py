"""Helpers shared by the GPU parity tests (host-side checking only)."""
import numpy as np

U = 2.0 ** -53


def to_dev(a, ld=None):
    from paper_2506_09463_amd import colmajor
    return colmajor(np.asarray(a, dtype=np.float64), ld=ld)


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def kappa(A):
    s = np.linalg.svd(A, compute_uv=False)
    return s[0] / s[-1] if s[-1] > 0 else np.inf


def factor_tol(A):
    """Element-wise bound on the difference of two backward-stable Householder
    factorizations with the same sign convention: 50 n u kappa ||A||_2."""
    n = A.shape[1]
    return 50 * max(n, 1) * U * kappa(A) * np.linalg.norm(A, 2)


def lsq_forward_bound(A, x, r):
    """50 n u kappa (1 + kappa ||r|| / (||A|| ||x||)) (standard LSQ perturbation bound)."""
    n = A.shape[1]
    k = kappa(A)
    nA = np.linalg.norm(A, 2)
    return 50 * n * U * k * (1 + k * np.linalg.norm(r) / (nA * max(np.linalg.norm(x), 1e-300)))


def lsq_orthogonality(A, x, b):
    r = b - A @ x
    nA = np.linalg.norm(A, 2)
    return np.linalg.norm(A.T @ r) / (nA * (nA * np.linalg.norm(x) + np.linalg.norm(b)))


def check_reflector_invariants(A0, F, up):
    """Sign rule, ||v||^2 = -2 b, and column-norm preservation on GPU output."""
    m, n = A0.shape
    for k in range(n):
        if up[k] == 0.0:
            continue
        x0 = up[k] + F[k, k]
        assert F[k, k] * x0 <= 0.0, ("sign rule", k)
        v2 = up[k] ** 2 + np.sum(F[k + 1:, k] ** 2)
        assert abs(v2 + 2 * up[k] * F[k, k]) <= 100 * m * U * v2, ("|v|^2 = -2b", k)
    cn = np.linalg.norm(A0, axis=0)
    rn = np.array([np.linalg.norm(F[: j + 1, j]) for j in range(n)])
    assert np.all(np.abs(cn - rn) <= 100 * m * U * np.maximum(cn, 1e-300)), "column norms"


def check_backward_orthogonality(oracle, A0, F, up, ncols=None, seed=0, factor=50.0):
    """Spec invariants on a GPU factorization: with Q applied from the
    GPU's own stored reflectors (F, up) by the oracle's apply_q,
      ||A - Q R||_F / ||A||_F <= 50 n u  and  ||Q^T Q - I||_F <= 50 n u
    (thin Q, n columns).  With ncols < n both are taken over a seeded sample
    of ncols columns (of A and R, and of Q); by default all columns up to
    n = 256 and a sample of 256 beyond.  Returns the two measured values."""
    m, n = A0.shape
    if n == 0:
        return 0.0, 0.0
    if ncols is None:
        ncols = 256
    if ncols >= n:
        cols = np.arange(n)
    else:
        cols = np.sort(np.random.default_rng(seed).choice(n, ncols, replace=False))
    E = np.zeros((m, cols.size))
    E[:n] = np.triu(F[:n, :n])[:, cols]
    QR = oracle.apply_q(F, up, E)
    berr = np.linalg.norm(A0[:, cols] - QR) / max(np.linalg.norm(A0[:, cols]), 1e-300)
    I = np.zeros((m, cols.size))
    I[cols, np.arange(cols.size)] = 1.0
    Qc = oracle.apply_q(F, up, I)
    orth = np.linalg.norm(Qc.T @ Qc - np.eye(cols.size))
    bound = factor * n * U
    assert berr <= bound, ("||A - QR|| / ||A||", berr, bound)
    assert orth <= bound, ("||Q^T Q - I||", orth, bound)
    return berr, orth
