"""Pins of the oracle's equality-constrained least squares
(min ||A x - b|| subject to C x = d, the form of SLSQP's least-squares
subproblem with its linearized equality constraints).

The oracle solves it by the null-space method on its own Householder
routines.  It is pinned here against what fixes the answer independently:
  * the exact solution of the KKT system [[A^T A, C^T], [C, 0]] [x; l] =
    [A^T b; d] in rational arithmetic on small integer inputs (brute force);
  * special cases: p = 0 is bitwise the oracle's plain least-squares solve,
    p = n is x = C^{-1} d;
  * invariants at larger sizes: C x = d to rounding, and the residual's
    gradient A^T (A x - b) has no component in the null space of C;
  * planted mistakes in the method's steps fail the exact check.
"""
import ctypes
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

U = 2.0 ** -53
HERE = os.path.dirname(os.path.abspath(__file__))


def _exact_kkt(A, C, b, d):
    """x of the KKT system solved exactly (Gauss-Jordan over Fractions)."""
    A = [[Fraction(int(v)) for v in r] for r in A]
    C = [[Fraction(int(v)) for v in r] for r in C]
    b = [Fraction(int(v)) for v in b]
    d = [Fraction(int(v)) for v in d]
    m, n, p = len(A), len(A[0]), len(C)
    N = n + p
    K = [[Fraction(0)] * (N + 1) for _ in range(N)]
    for i in range(n):
        for j in range(n):
            K[i][j] = sum(A[k][i] * A[k][j] for k in range(m))
        for j in range(p):
            K[i][n + j] = C[j][i]
        K[i][N] = sum(A[k][i] * b[k] for k in range(m))
    for i in range(p):
        for j in range(n):
            K[n + i][j] = C[i][j]
        K[n + i][N] = d[i]
    for col in range(N):
        piv = next(r for r in range(col, N) if K[r][col] != 0)
        K[col], K[piv] = K[piv], K[col]
        pv = K[col][col]
        K[col] = [v / pv for v in K[col]]
        for r in range(N):
            if r != col and K[r][col] != 0:
                f = K[r][col]
                K[r] = [a - f * c for a, c in zip(K[r], K[col])]
    return [K[i][N] for i in range(n)]


CASES = [
    # (m, n, p, seed): small integer problems, full rank with probability ~1
    (4, 3, 1, 1), (5, 3, 2, 2), (6, 4, 2, 3), (3, 3, 1, 4), (2, 3, 2, 5), (7, 5, 3, 6),
]


def _int_case(m, n, p, seed):
    rng = np.random.default_rng(seed)
    A = rng.integers(-4, 5, size=(m, n)).astype(float)
    C = rng.integers(-4, 5, size=(p, n)).astype(float)
    b = rng.integers(-4, 5, size=m).astype(float)
    d = rng.integers(-4, 5, size=p).astype(float)
    return A, C, b, d


def _check_exact(lse, m, n, p, seed):
    A, C, b, d = _int_case(m, n, p, seed)
    xe = [float(v) for v in _exact_kkt(A, C, b, d)]
    x, info = lse(A, C, b, d)
    if info != 0:
        return False
    kappa = np.linalg.cond(np.vstack([A, C]))
    return all(abs(x[j] - xe[j]) <= 200 * n * U * kappa * max(1.0, max(abs(v) for v in xe)) for j in range(n))


@pytest.mark.parametrize("m,n,p,seed", CASES)
def test_lse_matches_exact_kkt(oracle_mod, m, n, p, seed):
    assert _check_exact(oracle_mod.lse_solve, m, n, p, seed)


def test_lse_without_constraints_is_plain_lsq(oracle_mod):
    rng = np.random.default_rng(7)
    A = rng.standard_normal((30, 12))
    b = rng.standard_normal(30)
    x, info = oracle_mod.lse_solve(A, np.zeros((0, 12)), b, np.zeros(0))
    xo = oracle_mod.lsq_solve(A, b)[0][:, 0]
    assert info == 0 and np.array_equal(x, xo)


def test_lse_square_constraints_fix_x(oracle_mod):
    rng = np.random.default_rng(8)
    n = 9
    A = rng.standard_normal((15, n))
    C = rng.standard_normal((n, n))
    d = rng.standard_normal(n)
    x, info = oracle_mod.lse_solve(A, C, rng.standard_normal(15), d)
    assert info == 0
    assert np.linalg.norm(x - np.linalg.solve(C, d)) <= 1e3 * n * U * np.linalg.cond(C) * np.linalg.norm(x)


@pytest.mark.parametrize("m,n,p", [(60, 40, 10), (200, 120, 60), (50, 50, 5)])
def test_lse_invariants(oracle_mod, m, n, p):
    """C x = d to rounding, and the gradient of the objective is orthogonal
    to the null space of C (first-order optimality on the feasible set)."""
    from scipy.linalg import null_space
    rng = np.random.default_rng(m + p)
    A = rng.standard_normal((m, n))
    C = rng.standard_normal((p, n))
    b = rng.standard_normal(m)
    d = rng.standard_normal(p)
    x, info = oracle_mod.lse_solve(A, C, b, d)
    assert info == 0
    assert np.linalg.norm(C @ x - d) <= 100 * n * U * np.linalg.norm(C, 2) * np.linalg.norm(x)
    Z = null_space(C)
    g = A.T @ (A @ x - b)
    nA = np.linalg.norm(A, 2)
    assert np.linalg.norm(Z.T @ g) <= 100 * n * U * nA * (nA * np.linalg.norm(x) + np.linalg.norm(b))


def test_lse_rank_deficient_constraints_info(oracle_mod):
    rng = np.random.default_rng(9)
    A = rng.standard_normal((10, 5))
    C = rng.standard_normal((3, 5))
    C[2] = 0.0          # C^T's third column is zero: R_22 == 0
    x, info = oracle_mod.lse_solve(A, C, rng.standard_normal(10), rng.standard_normal(3))
    assert info == 3


LSE_MUTATIONS = {
    "b1_sign": ("for (int64_t j = 0; j < p; ++j) t -= AT(At, j, i, n) * x[j];",
                "for (int64_t j = 0; j < p; ++j) t += AT(At, j, i, n) * x[j];"),
    "q_instead_of_qt_on_A": ("if (p > 0) oracle_apply_qt(n, p, m, Ct, n, upc, At, n);",
                             "if (p > 0) oracle_apply_q(n, p, m, Ct, n, upc, At, n);"),
    "qt_instead_of_q_on_x": ("if (p > 0) oracle_apply_q(n, p, 1, Ct, n, upc, x, n);",
                             "if (p > 0) oracle_apply_qt(n, p, 1, Ct, n, upc, x, n);"),
    "r_instead_of_rt": ("oracle_backsolve_t(p, 1, Ct, n, x, p > 1 ? p : 1, &inf);",
                        "oracle_backsolve(p, 1, Ct, n, x, p > 1 ? p : 1, &inf);"),
    "reduced_columns_off_by_one": ("AT(Ar, i, j, m) = AT(At, p + j, i, n);",
                                   "AT(Ar, i, j, m) = AT(At, p + j - (j > 0), i, n);"),
}


@pytest.mark.parametrize("name", sorted(LSE_MUTATIONS))
def test_lse_planted_mistakes(tmp_path, name):
    src = os.path.join(HERE, "..", "oracle", "hqr_oracle.c")
    text = open(src).read()
    old, new = LSE_MUTATIONS[name]
    assert old in text, name
    d = tmp_path / name
    d.mkdir()
    shutil.copy(os.path.join(HERE, "..", "oracle", "hqr_oracle.h"), d)
    (d / "m.c").write_text(text.replace(old, new, 1))
    so = d / "libm.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC",
                           "-shared", "-o", str(so), str(d / "m.c"), "-lm"])
    lib = ctypes.CDLL(str(so))
    i64, dp = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_lse_solve.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, dp, dp, dp]

    def lse(A, C, b, d_):
        A = np.asfortranarray(A)
        Cm = np.asfortranarray(C)
        m, n = A.shape
        p = Cm.shape[0]
        b = np.ascontiguousarray(b)
        d_ = np.ascontiguousarray(d_)
        x = np.zeros(n)
        info = ctypes.c_int(0)
        lib.oracle_lse_solve(m, n, p, A.ctypes.data, m, Cm.ctypes.data, max(p, 1), b.ctypes.data, d_.ctypes.data,
                             x.ctypes.data, ctypes.addressof(info))
        return x, info.value

    assert not all(_check_exact(lse, *c) for c in CASES), name


def test_unmutated_lse_passes_exact_pins(oracle_mod):
    assert all(_check_exact(oracle_mod.lse_solve, *c) for c in CASES)
