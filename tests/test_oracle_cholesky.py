"""Pins of the oracle's Cholesky factorization and rank-one factor update.

Cholesky: an integer upper-triangular R with positive diagonal gives an
integer S = R^T R whose factorization the textbook recurrence computes
exactly (every square root and quotient is an integer); LAPACK's factor
(numpy) for random SPD matrices; the backward error ||S - R^T R||; the info
code of a matrix that is not positive definite; planted mistakes.

Update: R'^T R' = R^T R + v v^T to rounding; R' matches LAPACK's Cholesky
factor of R^T R + v v^T after the rows' signs are matched; the sign of each
diagonal entry is kept; the 3-4-5 case is exact; appending a row to a
matrix gives the R of the QR of the extended matrix (up to row signs).
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

U = 2.0 ** -53
HERE = os.path.dirname(os.path.abspath(__file__))

EXACT_R = [
    np.array([[2.0]]),
    np.array([[2.0, 1.0, 3.0], [0.0, 3.0, 1.0], [0.0, 0.0, 1.0]]),
    np.array([[1.0, -2.0, 0.0, 4.0], [0.0, 2.0, 1.0, -1.0], [0.0, 0.0, 5.0, 2.0], [0.0, 0.0, 0.0, 3.0]]),
]


@pytest.mark.parametrize("k", range(len(EXACT_R)))
def test_cholesky_exact_integer_factor(oracle_mod, k):
    R = EXACT_R[k]
    R2, info = oracle_mod.cholesky(R.T @ R)
    assert info == 0 and np.array_equal(R2, R)


@pytest.mark.parametrize("n,seed", [(5, 1), (40, 2), (130, 3)])
def test_cholesky_matches_lapack(oracle_mod, n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n + 5, n))
    S = G.T @ G
    R, info = oracle_mod.cholesky(S)
    assert info == 0
    L = np.linalg.cholesky(S)
    kappa = np.linalg.cond(S)
    assert np.abs(R - L.T).max() <= 50 * n * U * np.sqrt(kappa) * np.sqrt(np.abs(S).max()) * 10
    assert np.linalg.norm(S - R.T @ R) <= 50 * n * U * np.linalg.norm(S)


def test_cholesky_not_positive_definite(oracle_mod):
    S = np.array([[4.0, 2.0, 0.0], [2.0, 1.0, 3.0], [0.0, 3.0, 5.0]])   # second pivot 1 - 1 = 0
    R, info = oracle_mod.cholesky(S)
    assert info == 2


def test_update_three_four_five(oracle_mod):
    assert np.array_equal(oracle_mod.chol_update(np.array([[3.0]]), [4.0]), np.array([[5.0]]))
    assert np.array_equal(oracle_mod.chol_update(np.array([[-3.0]]), [4.0]), np.array([[-5.0]]))


@pytest.mark.parametrize("n,seed", [(1, 4), (7, 5), (64, 6), (200, 7)])
def test_update_identity_and_lapack(oracle_mod, n, seed):
    rng = np.random.default_rng(seed)
    R = np.triu(rng.standard_normal((n, n))) + np.diag(np.sign(rng.standard_normal(n)) * 3.0)
    v = rng.standard_normal(n)
    R2 = oracle_mod.chol_update(R, v)
    assert np.array_equal(np.tril(R2, -1), np.zeros((n, n)))
    assert np.array_equal(np.sign(np.diag(R2)), np.sign(np.diag(R)))
    S2 = R.T @ R + np.outer(v, v)
    assert np.linalg.norm(S2 - R2.T @ R2) <= 50 * n * U * np.linalg.norm(S2)
    L = np.linalg.cholesky(S2)
    D = np.sign(np.diag(R2))
    assert np.abs(D[:, None] * R2 - L.T).max() <= 1e3 * n * U * np.linalg.cond(S2) ** 0.5 * np.abs(L).max()


def test_update_is_qr_row_append(oracle_mod):
    """R of the QR of [A; v^T] equals the update of A's R by v (row signs
    matched), the QR use of the same operation."""
    rng = np.random.default_rng(8)
    A = rng.standard_normal((30, 10))
    v = rng.standard_normal(10)
    F, up = oracle_mod.qr_factor(A)
    R2 = oracle_mod.chol_update(np.triu(F[:10]), v)
    F3, _ = oracle_mod.qr_factor(np.vstack([A, v]))
    R3 = np.triu(F3[:10])
    D = np.sign(np.diag(R2)) * np.sign(np.diag(R3))
    assert np.abs(D[:, None] * R2 - R3).max() <= 1e-12 * np.abs(R3).max()


MUTATIONS = {
    "chol_dropped_square": ("for (int64_t k = 0; k < j; ++k) t -= AT(S, k, j, lds) * AT(S, k, j, lds);",
                            "for (int64_t k = 1; k < j; ++k) t -= AT(S, k, j, lds) * AT(S, k, j, lds);"),
    "chol_transposed_index": ("for (int64_t k = 0; k < j; ++k) u -= AT(S, k, j, lds) * AT(S, k, i, lds);",
                              "for (int64_t k = 0; k < j; ++k) u -= AT(S, k, j, lds) * AT(S, i, k, lds);"),
    "update_rotation_sign": ("v[j] = -s * a + c * b;", "v[j] = s * a + c * b;"),
    "update_swapped_cs": ("AT(R, k, j, ldr) = c * a + s * b;", "AT(R, k, j, ldr) = s * a + c * b;"),
}


def _passes(lib):
    i64, dp = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_cholesky.argtypes = [i64, dp, i64, dp]
    lib.oracle_chol_update.argtypes = [i64, dp, i64, dp]
    for R in EXACT_R:
        S = np.asfortranarray(R.T @ R)
        n = S.shape[0]
        info = ctypes.c_int(0)
        lib.oracle_cholesky(n, S.ctypes.data, n, ctypes.addressof(info))
        if info.value != 0 or not np.array_equal(np.triu(S), R):
            return False
    rng = np.random.default_rng(9)
    for n in (3, 12):
        R = np.asfortranarray(np.triu(rng.standard_normal((n, n))) + 3 * np.eye(n))
        v = rng.standard_normal(n)
        R0, v0 = R.copy(), v.copy()
        lib.oracle_chol_update(n, R.ctypes.data, n, v.ctypes.data)
        S2 = R0.T @ R0 + np.outer(v0, v0)
        if np.linalg.norm(S2 - R.T @ R) > 1e-12 * np.linalg.norm(S2):
            return False
    return True


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistakes(tmp_path, name):
    src = os.path.join(HERE, "..", "oracle", "hqr_oracle.c")
    text = open(src).read()
    old, new = MUTATIONS[name]
    assert old in text, name
    d = tmp_path / name
    d.mkdir()
    shutil.copy(os.path.join(HERE, "..", "oracle", "hqr_oracle.h"), d)
    (d / "m.c").write_text(text.replace(old, new, 1))
    so = d / "libm.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so),
                           str(d / "m.c"), "-lm"])
    assert not _passes(ctypes.CDLL(str(so))), name


def test_unmutated_oracle_passes(oracle_mod):
    assert _passes(ctypes.CDLL(oracle_mod.build(force=False)))
