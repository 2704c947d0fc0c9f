"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Every case prints the entry point, shape and seed before its GPU work so a
failing run names its case.  Tolerances:
  * factored matrix: element-wise 50 n u kappa ||A||_2 (two backward-stable
    Householder factorizations with the same sign convention);
  * x: the LSQ perturbation bound 50 n u kappa (1 + kappa ||r||/(||A|| ||x||))
    against the oracle's x;
  * LSQ orthogonality ||A^T r|| / (||A|| (||A|| ||x|| + ||b||)) <= 50 n u;
  * integers (info) and identity reflectors (up == 0) bit-exact.
"""
import numpy as np
import pytest

from paper_2506_09463_amd import workloads
from tests.gpu_util import (U, check_backward_orthogonality, check_reflector_invariants, factor_tol,
                            lsq_forward_bound, lsq_orthogonality, to_dev, to_host)
from tests.test_oracle_pins import CASES, _col

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


def _run_lsq(hqr, A, B, ld_pad=0):
    import torch
    m, n = A.shape
    dA = to_dev(A, ld=m + ld_pad)
    dB = to_dev(B, ld=m + ld_pad)
    up, res, info, it = hqr.qr_lsq_solve(dA, dB)
    torch.cuda.synchronize()
    return to_host(dA), to_host(up)[:n], to_host(dB), to_host(res), int(info.item())


# --------------------------------------------------- closed-form examples
@pytest.mark.parametrize("name", sorted(CASES))
def test_worked_examples_on_gpu(hqr, name):
    c = CASES[name]
    A = np.array([[float(v) for v in r] for r in c["A"]])
    b = np.array([float(v) for v in _col(c["b"])]).reshape(-1, 1)
    _say("qr_lsq_solve worked example", name, A.shape)
    F, up, X, res, info = _run_lsq(hqr, A, b)
    m, n = A.shape
    assert info == 0
    for i in range(m):
        for j in range(n):
            assert abs(F[i, j] - float(c["F"][i][j])) <= 32 * U * 20
    for k in range(n):
        assert abs(up[k] - float(c["up"][0][k])) <= 32 * U * 20
        assert (up[k] == 0.0) == (c["up"][0][k] == 0)
    for j in range(n):
        assert abs(X[j, 0] - float(_col(c["x"])[j])) <= 32 * U * 4
    assert abs(res[0] - float(c["resnorm"][0][0])) <= 32 * U * 4


# ------------------------------------------- element-wise parity vs oracle
SHAPES = [
    # (m, n, nrhs, seed) -- single-workgroup path
    (1, 1, 1, 31), (2, 1, 1, 32), (7, 7, 2, 33), (64, 64, 1, 34), (128, 64, 1, 1),
    (128, 127, 1, 35), (200, 100, 3, 36), (256, 64, 8, 37),
    # blocked path: several panels, ragged panel and tile tails, TRSV groups
    (300, 70, 1, 41), (513, 200, 9, 42), (1000, 333, 2, 43), (1536, 700, 1, 44),
    (640, 640, 1, 45),
]


@pytest.mark.parametrize("m,n,nrhs,seed", SHAPES)
def test_lsq_parity(hqr, oracle_mod, m, n, nrhs, seed):
    rng = np.random.default_rng(seed)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    B = np.asfortranarray(rng.standard_normal((m, nrhs)))
    _say("qr_lsq_solve", (m, n, nrhs), "seed", seed)
    F, up, X, res, info = _run_lsq(hqr, A, B, ld_pad=3)
    Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, B)
    assert info == infoo == 0
    tol = factor_tol(A)
    assert np.abs(F - Fo).max() <= tol
    assert np.array_equal(up == 0.0, upo == 0.0)
    assert np.abs(up - upo).max() <= tol
    check_reflector_invariants(A, F, up)
    check_backward_orthogonality(oracle_mod, A, F, up)
    for c in range(nrhs):
        x, xo = X[:n, c], Xo[:, c]
        r = B[:, c] - A @ xo
        bound = lsq_forward_bound(A, xo, r)
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 2 * bound
        assert lsq_orthogonality(A, x, B[:, c]) <= 50 * n * U
        assert abs(res[c] - reso[c]) <= 50 * m * U * max(reso[c], 1e-300) + tol
        assert abs(res[c] - np.linalg.norm(B[:, c] - A @ x)) <= 1e-9 * max(1.0, res[c])


@pytest.mark.parametrize("m,n,nrhs,seed", [(128, 64, 1, 51), (300, 70, 2, 52), (1000, 333, 3, 53)])
def test_factor_apply_backsolve_split(hqr, oracle_mod, m, n, nrhs, seed):
    """qr_factor, qr_apply_qt, qr_backsolve called one by one."""
    import torch
    rng = np.random.default_rng(seed)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    B = np.asfortranarray(rng.standard_normal((m, nrhs)))
    _say("qr_factor/qr_apply_qt/qr_backsolve", (m, n, nrhs))
    dA, dB = to_dev(A), to_dev(B)
    up, info = hqr.qr_factor(dA)
    hqr.qr_apply_qt(dA, up, dB)
    qtb = to_host(dB).copy()
    _, info2 = hqr.qr_backsolve(dA[:n, :n], dB)
    torch.cuda.synchronize()
    F, upn = to_host(dA), to_host(up)[:n]
    Fo, upo = oracle_mod.qr_factor(A)
    tol = factor_tol(A)
    assert int(info.item()) == 0 and int(info2.item()) == 0
    assert np.abs(F - Fo).max() <= tol
    check_backward_orthogonality(oracle_mod, A, F, upn)
    qtbo = oracle_mod.apply_qt(Fo, upo, B)
    assert np.abs(qtb - qtbo).max() <= tol * max(1.0, np.abs(B).max())
    Xo, _ = oracle_mod.backsolve(Fo, qtbo)
    X = to_host(dB)[:n]
    for c in range(nrhs):
        r = B[:, c] - A @ Xo[:, c]
        assert np.linalg.norm(X[:, c] - Xo[:, c]) / np.linalg.norm(Xo[:, c]) <= 2 * lsq_forward_bound(A, Xo[:, c], r)


def _dominant_upper(rng, n):
    """Upper triangle with |R_ii| = n + U(0,1) against N(0,1) entries above:
    strictly diagonally dominant by rows, so kappa(R) stays near 1 at any n."""
    R = np.triu(rng.standard_normal((n, n)))
    np.fill_diagonal(R, (n + rng.random(n)) * np.where(rng.random(n) < 0.5, -1.0, 1.0))
    return np.asfortranarray(R)


@pytest.mark.parametrize("n,nrhs,seed", [(1, 1, 61), (64, 3, 62), (65, 8, 63), (1000, 11, 64), (4133, 1, 65),
                                         (4133, 9, 66)])
def test_backsolve_blocks_and_chunks(hqr, oracle_mod, n, nrhs, seed):
    """qr_backsolve (the multi-workgroup TRSV: 64-row blocks that wait on the
    values their predecessors publish; more than 8 right-hand sides take two
    launches over the same published-value buffer) against the oracle's
    substitution: max |x - x_o| <= 50 n u max |x_o| per column (kappa ~ 1)."""
    import torch
    rng = np.random.default_rng(seed)
    R = _dominant_upper(rng, n)
    B = np.asfortranarray(rng.standard_normal((n + 5, nrhs)))
    _say("qr_backsolve", (n, nrhs, seed))
    dR, dB = to_dev(R), to_dev(B)
    _, info = hqr.qr_backsolve(dR, dB)
    torch.cuda.synchronize()
    X = to_host(dB)
    Xo, info_o = oracle_mod.backsolve(R, B)
    assert int(info.item()) == 0 and info_o == 0
    for c in range(nrhs):
        assert np.abs(X[:n, c] - Xo[:, c]).max() <= 50 * n * U * np.abs(Xo[:, c]).max()
    assert np.array_equal(X[n:], B[n:])   # rows below n untouched


def test_backsolve_nonfinite_rhs(hqr, oracle_mod):
    """NaN, +Inf and the signalling-NaN pattern the TRSV's published-value
    slots hold before they are written, each in one right-hand side: the wait
    ends (info 0, no timeout), the non-finite rows are those of the oracle's
    substitution, and the finite rows agree with it."""
    import torch
    rng = np.random.default_rng(67)
    n = 1000
    R = _dominant_upper(rng, n)
    B = np.asfortranarray(rng.standard_normal((n, 4)))
    B[700, 0] = np.nan
    B[999, 1] = np.inf
    B[300, 2] = np.array([0x7FF47FF47FF47FF4], dtype=np.uint64).view(np.float64)[0]
    _say("qr_backsolve nonfinite", (n, 4))
    dR, dB = to_dev(R), to_dev(B)
    _, info = hqr.qr_backsolve(dR, dB)
    torch.cuda.synchronize()
    X = to_host(dB)
    Xo, _ = oracle_mod.backsolve(R, B)
    assert int(info.item()) == 0
    fin = np.isfinite(Xo)
    assert np.array_equal(np.isfinite(X), fin)
    assert not fin[:701, 0].any() and fin[701:, 0].all()
    assert not fin[:, 1].any()
    assert not fin[:301, 2].any() and fin[301:, 2].all()
    assert fin[:, 3].all()
    assert np.abs(X[fin] - Xo[fin]).max() <= 50 * n * U * np.abs(Xo[fin]).max()


@pytest.mark.parametrize("m,n", [(128, 64), (700, 300)])
def test_deterministic(hqr, m, n):
    """Same input, same launch configuration: bitwise identical results."""
    rng = np.random.default_rng(61)
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((m, 2))
    _say("determinism", (m, n))
    r1 = _run_lsq(hqr, A, B)
    r2 = _run_lsq(hqr, A, B)
    for a, b in zip(r1[:4], r2[:4]):
        assert np.array_equal(a, b)


# ------------------------------------------------------------ edge cases
@pytest.mark.parametrize("m,n", [(9, 5), (400, 150)])
def test_zero_column_identity(hqr, oracle_mod, m, n):
    rng = np.random.default_rng(71)
    A = rng.standard_normal((m, n))
    A[:, 1] = 0.0
    B = rng.standard_normal((m, 1))
    _say("zero column", (m, n))
    dA = to_dev(A)
    up, info = hqr.qr_factor(dA)
    F, upn = to_host(dA), to_host(up)[:n]
    Fo, upo = oracle_mod.qr_factor(A)
    assert upn[1] == 0.0 and upo[1] == 0.0
    assert np.array_equal(upn == 0.0, upo == 0.0)
    assert np.abs(F - Fo).max() <= 1e-10 * np.abs(A).max() * m


@pytest.mark.parametrize("m,n", [(6, 4), (300, 130)])
def test_singular_info(hqr, oracle_mod, m, n):
    rng = np.random.default_rng(72)
    A = rng.standard_normal((m, n))
    A[:, 2] = 0.0                      # R[2][2] == 0 exactly
    B = rng.standard_normal((m, 1))
    _say("singular", (m, n))
    F, up, X, res, info = _run_lsq(hqr, A, B)
    Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, B)
    assert info == infoo == 3
    qtbo = oracle_mod.apply_qt(Fo, upo, B)
    assert np.abs(X[:, 0] - qtbo[:, 0]).max() <= 1e-10 * m   # B left as Q^T B


@pytest.mark.parametrize("m,n", [(10, 4), (300, 80)])
def test_tiny_column_scaled_norm(hqr, oracle_mod, m, n):
    """A column of magnitude 1e-145 takes the scaled-norm branch (largest
    entry below 2^-460) on both paths."""
    rng = np.random.default_rng(73)
    A = rng.standard_normal((m, n))
    A[:, 0] *= 1e-145
    _say("tiny column", (m, n))
    dA = to_dev(A)
    up, info = hqr.qr_factor(dA)
    F = to_host(dA)
    Fo, upo = oracle_mod.qr_factor(A)
    assert np.isfinite(F).all() and np.isfinite(Fo).all()
    assert abs(F[0, 0] - Fo[0, 0]) <= 1e-13 * abs(Fo[0, 0])
    R, Ro = np.triu(F[:n]), np.triu(Fo[:n])
    assert np.abs(R[:, 1:] - Ro[:, 1:]).max() <= 1e-10 * np.abs(A[:, 1:]).max() * m


def test_underflowing_b_matches_oracle(hqr, oracle_mod):
    """Below ~1e-154 the product b = up * R_kk underflows; both paths then
    produce the same pattern of non-finite values."""
    rng = np.random.default_rng(75)
    A = rng.standard_normal((10, 4))
    A[:, 0] *= 1e-165
    _say("underflowing b", A.shape)
    dA = to_dev(A)
    hqr.qr_factor(dA)
    F = to_host(dA)
    Fo, _ = oracle_mod.qr_factor(A)
    assert np.array_equal(np.isfinite(F), np.isfinite(Fo))


def test_nan_propagates(hqr, oracle_mod):
    """Single-workgroup path: exactly the oracle's pattern of NaN entries."""
    rng = np.random.default_rng(74)
    A = rng.standard_normal((20, 6))
    A[5, 2] = np.nan
    _say("nan", A.shape)
    dA = to_dev(A)
    hqr.qr_factor(dA)
    F = to_host(dA)
    Fo, _ = oracle_mod.qr_factor(A)
    assert np.array_equal(np.isnan(F), np.isnan(Fo))


def test_nan_propagates_blocked(hqr):
    """Blocked path: NaN reaches the solution.  The compact-WY contraction
    multiplies the structural zeros of V by NaN, so more entries of R may turn
    NaN than in the one-reflector-at-a-time order."""
    rng = np.random.default_rng(76)
    A = rng.standard_normal((300, 80))
    A[150, 70] = np.nan
    B = rng.standard_normal((300, 1))
    _say("nan blocked", A.shape)
    F, up, X, res, info = _run_lsq(hqr, A, B)
    assert np.isfinite(F[:, :64]).all()
    assert np.isnan(F[:, 70:]).any() and np.isnan(X[:80]).any()


def test_argument_errors(hqr):
    import torch
    dA = to_dev(np.ones((3, 4)))
    with pytest.raises(hqr.HQRError) as e:
        hqr.qr_factor(dA)
    assert e.value.status == -2
    dA = to_dev(np.ones((4, 3)))
    dB = to_dev(np.ones((4, 1)))
    up, info = hqr.qr_factor(dA)
    torch.cuda.synchronize()
    with pytest.raises(ValueError):
        hqr.qr_apply_qt(dA, up, to_dev(np.ones((5, 1))))
    hqr.qr_apply_qt(dA, up, dB)


# -------------------------------------------------- panel algorithms
@pytest.mark.parametrize("mode", ["cqr", "exact", "percol", "tsqr"])
@pytest.mark.parametrize("m,n,nrhs", [(700, 300, 2), (1100, 129, 1)])
def test_panel_modes(hqr, oracle_mod, monkeypatch, mode, m, n, nrhs):
    """CholeskyQR2 + reconstruction (default), the exact one-workgroup panel
    and the one-launch-per-pivot panel all match the oracle."""
    monkeypatch.setenv("HQR_PANEL", mode)
    rng = np.random.default_rng(81)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    B = np.asfortranarray(rng.standard_normal((m, nrhs)))
    _say("panel mode", mode, (m, n, nrhs))
    F, up, X, res, info = _run_lsq(hqr, A, B)
    Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, B)
    assert info == 0
    tol = factor_tol(A)
    assert np.abs(F - Fo).max() <= tol
    assert np.abs(up - upo).max() <= tol
    check_backward_orthogonality(oracle_mod, A, F, up)
    for c in range(nrhs):
        r = B[:, c] - A @ Xo[:, c]
        assert np.linalg.norm(X[:n, c] - Xo[:, c]) / np.linalg.norm(Xo[:, c]) <= 2 * lsq_forward_bound(A, Xo[:, c], r)


@pytest.mark.parametrize("kappa", [1e3, 3e4, 1e6, 1e9, 1e12])
def test_ill_conditioned(hqr, oracle_mod, kappa):
    """kappa 1e3 keeps every second CholeskyQR pass on the near-identity
    series (Gram entries within 2^-30 of I), 3e4 puts panels on both sides of
    that bound, 1e9 and 1e12 send panels to the exact path.  The backward
    error ||A - QR|| / ||A|| and the orthogonality of Q (from the GPU's own
    reflectors) must stay within 50 n u at every conditioning -- the checks
    that catch a loss of orthogonality in a CholeskyQR panel.  Where the
    element-wise perturbation bound 50 n u kappa ||A|| is below 1e-4 it is
    checked as well (at kappa >= 1e9 it says nothing)."""
    A, b, _ = workloads.conditioned(900, 320, kappa, seed=82)
    _say("ill conditioned", kappa)
    F, up, X, res, info = _run_lsq(hqr, A, b.reshape(-1, 1))
    Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, b)
    assert info == 0
    berr, orth = check_backward_orthogonality(oracle_mod, A, F, up)
    _say("backward error %.2e, orthogonality %.2e, |F - F_oracle| %.2e" % (berr, orth, np.abs(F - Fo).max()))
    if factor_tol(A) < 1e-4:
        assert np.abs(F - Fo).max() <= factor_tol(A)
    r = b - A @ Xo[:, 0]
    assert np.linalg.norm(X[:320, 0] - Xo[:, 0]) / np.linalg.norm(Xo[:, 0]) <= 2 * lsq_forward_bound(A, Xo[:, 0], r)
    assert lsq_orthogonality(A, X[:320, 0], b) <= 50 * 320 * U


def test_upper_triangular_input_keeps_identity(hqr, oracle_mod):
    """Columns already reduced (zero below the diagonal): every reflector is
    the identity, exactly as in the one-reflector loop."""
    rng = np.random.default_rng(83)
    A = np.zeros((500, 200))
    A[:200] = np.triu(rng.standard_normal((200, 200))) + 3 * np.eye(200)
    _say("upper triangular input")
    dA = to_dev(A)
    up, info = hqr.qr_factor(dA)
    F, upn = to_host(dA), to_host(up)[:200]
    Fo, upo = oracle_mod.qr_factor(A)
    assert np.all(upn == 0.0) and np.all(upo == 0.0)
    assert np.array_equal(F, A)


def test_square_blocked(hqr, oracle_mod):
    """m == n on the blocked path: the last panel (empty last tail) is exact."""
    rng = np.random.default_rng(84)
    A = rng.standard_normal((384, 384))
    b = rng.standard_normal((384, 1))
    _say("square blocked")
    F, up, X, res, info = _run_lsq(hqr, A, b)
    Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, b)
    assert up[-1] == 0.0 and upo[-1] == 0.0
    assert np.abs(F - Fo).max() <= factor_tol(A)
    check_backward_orthogonality(oracle_mod, A, F, up)
    r = b[:, 0] - A @ Xo[:, 0]
    assert np.linalg.norm(X[:, 0] - Xo[:, 0]) / np.linalg.norm(Xo[:, 0]) <= 2 * lsq_forward_bound(A, Xo[:, 0], r)


@pytest.mark.parametrize("lookahead", ["0", "1"])
def test_lookahead_on_off(hqr, oracle_mod, monkeypatch, lookahead):
    """The side-stream look-ahead changes only the grouping of partial sums."""
    monkeypatch.setenv("HQR_LOOKAHEAD", lookahead)
    rng = np.random.default_rng(85)
    A = np.asfortranarray(rng.standard_normal((1200, 450)))
    B = np.asfortranarray(rng.standard_normal((1200, 3)))
    _say("lookahead", lookahead)
    F, up, X, res, info = _run_lsq(hqr, A, B)
    Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, B)
    assert info == 0
    assert np.abs(F - Fo).max() <= factor_tol(A)
    check_backward_orthogonality(oracle_mod, A, F, up)
    for c in range(3):
        r = B[:, c] - A @ Xo[:, c]
        assert np.linalg.norm(X[:450, c] - Xo[:, c]) / np.linalg.norm(Xo[:, c]) <= 2 * lsq_forward_bound(A, Xo[:, c], r)


# ------------------------------------------------- Q B and explicit Q
QSHAPES = [(9, 5, 3), (128, 64, 2), (256, 100, 17), (300, 70, 4), (1000, 333, 70), (700, 300, 700)]


@pytest.mark.parametrize("m,n,nrhs", QSHAPES)
def test_apply_q_matches_oracle(hqr, oracle_mod, m, n, nrhs):
    """qr_apply_q (Q B = H_0 .. H_{n-1} B) on the GPU's own factor against the
    oracle's apply_q of the same stored reflectors, and Q^T (Q B) = B."""
    import torch
    rng = np.random.default_rng(200 + m)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    B = np.asfortranarray(rng.standard_normal((m, nrhs)))
    _say("qr_apply_q", (m, n, nrhs))
    dA = to_dev(A)
    up, info = hqr.qr_factor(dA)
    dB = to_dev(B)
    hqr.qr_apply_q(dA, up, dB)
    torch.cuda.synchronize()
    QB = to_host(dB).copy()
    F, upn = to_host(dA), to_host(up)[:n]
    QBo = oracle_mod.apply_q(F, upn, B)
    assert np.abs(QB - QBo).max() <= 50 * m * U * max(1.0, np.abs(B).max())
    hqr.qr_apply_qt(dA, up, dB)
    torch.cuda.synchronize()
    assert np.abs(to_host(dB) - B).max() <= 100 * m * U * max(1.0, np.abs(B).max())


@pytest.mark.parametrize("m,n,nrhs,zero_first", [(2600, 1100, 3, False), (1500, 700, 2, True)])
def test_stored_factor_t_blocks(hqr, oracle_mod, m, n, nrhs, zero_first):
    """Q^T B and Q B with a stored blocked factor, where every panel's T is
    rebuilt from V^T V as the inverse of diag(1/tau) + the strict upper
    triangle of V^T V (16 x 16 diagonal blocks, then the blocks above them):
    18 and 11 panels with a ragged last one; with zero_first column 0's tail
    is exactly zero, so its reflector is the identity (up_0 == 0, tau_0 == 0).
    Against the oracle's application of the same stored reflectors."""
    import torch
    rng = np.random.default_rng(300 + m)
    A = rng.standard_normal((m, n))
    if zero_first:
        A[1:, 0] = 0.0
    A = np.asfortranarray(A)
    B = np.asfortranarray(rng.standard_normal((m, nrhs)))
    _say("stored-factor T blocks", (m, n, nrhs, zero_first))
    dA = to_dev(A)
    up, info = hqr.qr_factor(dA)
    torch.cuda.synchronize()
    F, upn = to_host(dA), to_host(up)[:n]
    if zero_first:
        assert upn[0] == 0.0
    dB = to_dev(B)
    hqr.qr_apply_qt(dA, up, dB)
    torch.cuda.synchronize()
    QtB = to_host(dB).copy()
    QtBo = oracle_mod.apply_qt(F, upn, B)
    assert np.abs(QtB - QtBo).max() <= 50 * m * U * max(1.0, np.abs(B).max())
    hqr.qr_apply_q(dA, up, dB)
    torch.cuda.synchronize()
    assert np.abs(to_host(dB) - B).max() <= 100 * m * U * max(1.0, np.abs(B).max())
    dB = to_dev(B)
    hqr.qr_apply_q(dA, up, dB)
    torch.cuda.synchronize()
    QBo = oracle_mod.apply_q(F, upn, B)
    assert np.abs(to_host(dB) - QBo).max() <= 50 * m * U * max(1.0, np.abs(B).max())


@pytest.mark.parametrize("m,n,k", [(7, 7, 7), (128, 64, 64), (128, 64, 128), (200, 150, 90), (1000, 333, 333),
                                   (900, 500, 900), (513, 200, 1)])
def test_form_q_matches_oracle(hqr, oracle_mod, m, n, k):
    """qr_form_q: the leading k columns of Q, against the oracle's Q formed
    from the same stored reflectors; orthonormal columns; A = Q[:, :n] R."""
    import torch
    rng = np.random.default_rng(300 + m + k)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    _say("qr_form_q", (m, n, k))
    dA = to_dev(A)
    up, info = hqr.qr_factor(dA)
    Q = hqr.qr_form_q(dA, up, k)
    torch.cuda.synchronize()
    Qg = to_host(Q)
    F, upn = to_host(dA), to_host(up)[:n]
    Qo = oracle_mod.apply_q(F, upn, np.eye(m)[:, :k])
    assert np.abs(Qg - Qo).max() <= 50 * m * U
    assert np.linalg.norm(Qg.T @ Qg - np.eye(k)) <= 50 * max(n, 1) * U * max(1.0, np.sqrt(k / max(n, 1)))
    if k >= n:
        assert np.linalg.norm(A - Qg[:, :n] @ np.triu(F[:n])) / np.linalg.norm(A) <= 50 * n * U
