"""Seeded synthetic inputs for the QR least-squares workloads.

This module holds no arithmetic of the factorization or the solve: it only
draws random numbers (numpy PCG64, ``default_rng(seed)``) and shapes them.
The tests, the benchmark and the oracle comparisons all take their inputs
from here, so both sides of every parity check see the same arrays.

Every matrix is float64 in column-major (Fortran) order.  Recipes:

* ``gaussian(m, n, seed)``: entries iid N(0, 1), drawn row-major then
  reordered to column-major storage.
* ``conditioned(m, n, kappa, seed)``: A = U diag(sigma) V^T with U, V the
  orthogonal factors of seeded Gaussian matrices (numpy's LAPACK QR, used as
  a random-orthogonal generator only), sigma = geomspace(1, 1/kappa, n);
  x_true ~ N(0, 1); b = A x_true + 1e-8 N(0, 1).
* ``batch_shapes(count, seed)``: n ~ U{16..512}, m = n + U{0..n}.
* ``served_shapes(count, seed)``: n = round(exp(U[ln 16, ln 2048])),
  m = n + U{0..floor(n/2)}, precision FP64 or mixed with p = 1/2,
  nrhs ~ U{1..4}.
"""
from __future__ import annotations

import numpy as np

SEED_SMALL = 1          # 128 x 64 FP64
SEED_LARGE = 2          # 8192 x 4096, kappa = 1e6
SEED_MIXED = (3, 4)     # 128 x 64 at kappa 1e2 and 1e6
SEED_BATCH = 5          # 2000 uneven instances
SEED_SERVED = 6         # request stream


def gaussian(m: int, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((m, n)))


def small_problem(seed: int = SEED_SMALL, m: int = 128, n: int = 64):
    """A ~ N(0,1) (m x n) and one N(0,1) right-hand side, same generator."""
    rng = np.random.default_rng(seed)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    b = rng.standard_normal(m)
    return A, b


def random_orthogonal(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    """m x n matrix with orthonormal columns: Q factor of a Gaussian matrix."""
    G = rng.standard_normal((m, n))
    Q, _ = np.linalg.qr(G)
    return Q


def conditioned(m: int, n: int, kappa: float, seed: int, noise: float = 1e-8):
    """A = U diag(sigma) V^T with sigma geometric from 1 to 1/kappa.

    Returns (A, b, x_true) with b = A x_true + noise * N(0, 1).
    """
    rng = np.random.default_rng(seed)
    U = random_orthogonal(rng, m, n)
    V = random_orthogonal(rng, n, n)
    sigma = np.geomspace(1.0, 1.0 / kappa, n)
    A = np.asfortranarray((U * sigma) @ V.T)
    x_true = rng.standard_normal(n)
    b = A @ x_true + noise * rng.standard_normal(m)
    return A, b, x_true


def large_problem(seed: int = SEED_LARGE, m: int = 8192, n: int = 4096,
                  kappa: float = 1e6):
    return conditioned(m, n, kappa, seed)


def batch_shapes(count: int = 2000, seed: int = SEED_BATCH,
                 nmin: int = 16, nmax: int = 512):
    rng = np.random.default_rng(seed)
    n = rng.integers(nmin, nmax + 1, size=count)
    m = n + rng.integers(0, n + 1)
    return m.astype(np.int64), n.astype(np.int64), rng


def batch_problem(count: int = 2000, seed: int = SEED_BATCH, nrhs: int = 8,
                  nmin: int = 16, nmax: int = 512):
    """List of (A_i, B_i) with A_i ~ N(0,1) (m_i x n_i), B_i ~ N(0,1) (m_i x nrhs)."""
    m, n, rng = batch_shapes(count, seed, nmin, nmax)
    out = []
    for i in range(count):
        A = np.asfortranarray(rng.standard_normal((int(m[i]), int(n[i]))))
        B = np.asfortranarray(rng.standard_normal((int(m[i]), nrhs)))
        out.append((A, B))
    return out


def served_shapes(count: int = 5000, seed: int = SEED_SERVED,
                  nmin: int = 16, nmax: int = 2048):
    rng = np.random.default_rng(seed)
    n = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=count)))
    n = n.astype(np.int64)
    m = n + rng.integers(0, n // 2 + 1)
    mixed = rng.random(count) < 0.5
    nrhs = rng.integers(1, 5, size=count)
    return m.astype(np.int64), n, mixed, nrhs.astype(np.int64), rng
