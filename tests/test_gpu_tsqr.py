"""GPU parity of the TSQR panel (HQR_OPT_TSQR_PANEL / HQR_PANEL=tsqr): a
reduction tree of row-block Householder QRs, the explicit orthonormal
factor, then Householder reconstruction of the one-reflector-per-column form.

Against the oracle: the factored matrix element-wise within
50 n u kappa ||A||_2, up, x within the LSQ perturbation bound, and the
backward error / orthogonality of Q applied from the GPU's own reflectors
(<= 50 n u).  Panels whose CholeskyQR pivots flag them (near-dependent
columns) must go through the tree instead of the exact one-workgroup loop,
which the per-class kernel times show; panels with an exactly zero column
tail keep the exact loop (identity reflector, up == 0 bit-exact)."""
import numpy as np
import pytest

from tests.gpu_util import (U, check_backward_orthogonality, factor_tol, lsq_forward_bound, to_dev,
                            to_host)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hqr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2506_09463_amd as h
    h.load()
    return h


def _say(*a):
    print("[case]", *a, flush=True)


def _solve(hqr, A, B, tsqr, profile=False):
    import torch
    n = A.shape[1]
    dA, dB = to_dev(A), to_dev(B)
    if profile:
        torch.cuda.synchronize()
        hqr.profile_begin()
    up, res, info, it = hqr.qr_lsq_solve(dA, dB, tsqr=tsqr)
    torch.cuda.synchronize()
    prof = hqr.profile_end() if profile else None
    return to_host(dA), to_host(up)[:n], to_host(dB), int(info.item()), prof


@pytest.mark.parametrize("m,n,nrhs", [(1100, 129, 1), (2500, 200, 2), (17000, 130, 1)])
def test_tsqr_matches_oracle(hqr, oracle_mod, m, n, nrhs):
    """One leaf, several leaves, and a two-level tree (17000 rows: 17 leaves,
    their 1088 stacked rows in two blocks, then one block of 128 rows)."""
    rng = np.random.default_rng(400 + m)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    B = np.asfortranarray(rng.standard_normal((m, nrhs)))
    _say("qr_lsq_solve tsqr", (m, n, nrhs))
    F, up, X, info, _ = _solve(hqr, A, B, True)
    Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, B)
    assert info == 0
    tol = factor_tol(A)
    assert np.abs(F - Fo).max() <= tol
    assert np.abs(up - upo).max() <= tol
    berr, orth = check_backward_orthogonality(oracle_mod, A, F, up)
    _say("backward error %.2e, orthogonality %.2e" % (berr, orth))
    for c in range(nrhs):
        r = B[:, c] - A @ Xo[:, c]
        assert np.linalg.norm(X[:n, c] - Xo[:, c]) / np.linalg.norm(Xo[:, c]) <= 2 * lsq_forward_bound(A, Xo[:, c], r)


def _near_dependent(m, n, j, k, delta, seed):
    """Gaussian A with column j replaced by column k + delta * noise: the
    panel holding both has conditioning about 1/delta."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    A[:, j] = A[:, k] + delta * rng.standard_normal(m)
    return np.asfortranarray(A)


@pytest.mark.parametrize("delta", [1e-9, 1e-12, 1e-15])
def test_tsqr_takes_flagged_panels(hqr, oracle_mod, delta):
    """Columns 66 and 70 nearly equal: panel 1 fails the CholeskyQR pivot test.
    The default path factors it with the exact one-workgroup loop; the TSQR
    panel must factor it through the tree (the Cholesky kernel's time stays
    that of two ordinary passes per panel) with the same quality: backward
    error and orthogonality within 50 n u, x within the perturbation bound of
    the oracle's x."""
    m, n = 3000, 200
    A = _near_dependent(m, n, 70, 66, delta, seed=410)
    b = np.asfortranarray(np.random.default_rng(411).standard_normal((m, 1)))
    _say("flagged panel, delta", delta)
    Fd, upd, Xd, infod, profd = _solve(hqr, A, b, False, profile=True)
    Ft, upt, Xt, infot, proft = _solve(hqr, A, b, True, profile=True)
    chol_d, chol_t = profd["cqr_chol"][0], proft["cqr_chol"][0]
    _say("cqr_chol ms: default %.3f, tsqr %.3f; tsqr class %s" % (chol_d, chol_t, proft.get("tsqr")))
    assert "tsqr" in proft and "tsqr" not in profd
    assert chol_t < 0.25 * chol_d
    for F, up in ((Fd, upd), (Ft, upt)):
        berr, orth = check_backward_orthogonality(oracle_mod, A, F, up)
        _say("backward error %.2e, orthogonality %.2e" % (berr, orth))
    Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, b)
    r = b[:, 0] - A @ Xo[:, 0]
    bound = 2 * lsq_forward_bound(A, Xo[:, 0], r)
    if bound < 1.0:
        assert np.linalg.norm(Xt[:n, 0] - Xo[:, 0]) / np.linalg.norm(Xo[:, 0]) <= bound
        assert infot == 0


def test_tsqr_keeps_exact_zero_tails(hqr, oracle_mod):
    """A column whose part below the diagonal is exactly zero keeps the
    identity reflector (up == 0) in the TSQR mode too: its panel is left to
    the exact loop, the other panels go through the tree.  Column 0's tail is
    zero from the start; column 64 is 5 e_64 with row 64 of panel 0 zero, so
    panel 0's reflectors vanish in row 64 and leave it exactly e_64 (its tail
    is still exactly zero when panel 1 is factored)."""
    m, n = 1500, 192
    rng = np.random.default_rng(420)
    A = rng.standard_normal((m, n))
    A[1:, 0] = 0.0
    A[64, :64] = 0.0
    A[:, 64] = 0.0
    A[64, 64] = 5.0
    A = np.asfortranarray(A)
    b = np.asfortranarray(rng.standard_normal((m, 1)))
    _say("exact zero tail in tsqr mode", (m, n))
    F, up, X, info, _ = _solve(hqr, A, b, True)
    Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, b)
    assert info == 0
    assert up[0] == 0.0 and upo[0] == 0.0
    assert up[64] == 0.0 and upo[64] == 0.0
    assert ((up == 0.0) == (upo == 0.0)).all()
    tol = factor_tol(A)
    assert np.abs(F - Fo).max() <= tol
    check_backward_orthogonality(oracle_mod, A, F, up)


def test_tsqr_deterministic_and_workspace(hqr):
    """Two TSQR solves of the same input are bitwise equal, also with a
    caller-provided work area of hqr_workspace_size_opts bytes."""
    import torch
    m, n = 5000, 192
    rng = np.random.default_rng(430)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    b = np.asfortranarray(rng.standard_normal((m, 1)))
    _say("tsqr determinism", (m, n))
    F1, up1, X1, i1, _ = _solve(hqr, A, b, True)
    nbytes = hqr.workspace_size_opts(m, n, 1, tsqr=True)
    assert nbytes > hqr.workspace_size(m, n, 1)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dA, dB = to_dev(A), to_dev(b)
    up, res, info, it = hqr.qr_lsq_solve(dA, dB, tsqr=True, work=work)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(dA), F1)
    assert np.array_equal(to_host(up)[:n], up1)
    assert np.array_equal(to_host(dB), X1)
