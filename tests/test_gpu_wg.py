"""GPU parity of the one-workgroup blocked kernel in each variant.

Every variant is forced through the tuning rules and compared with the FP64
oracle: single problems (factor + Q^T B + residual norms + solve), factor
only, apply only on a stored factorization, and batches.  Shapes cover
several 16-column panels with a ragged last panel, the variant's maximum row
count, square matrices (identity last reflector), a zero column (identity
reflector mid-panel), a single column, and n * nrhs near the staging limit.
"""
import numpy as np
import pytest

from tests.gpu_util import U, factor_tol, lsq_forward_bound, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hqr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2506_09463_amd as h
    h.load()
    yield h
    h.tune_clear()
    if __import__("os").path.exists(h.hqr.TUNE_DB_PATH):
        h.load_tune_db()


def _variants(hqr):
    out = []
    for i, nm in enumerate(hqr.tune_variants()):
        nt, qm, _ = hqr.variant_shape(nm)
        out.append((i, nm, nt * qm))
    return out


def _force_single(hqr, idx):
    hqr.tune_clear()
    hqr.tune_set(hqr.HQR_TUNE_SINGLE, 0, 1 << 40, 0, 1 << 40, idx)


def _check_solve(oracle_mod, A, B, F, up, X, res, info):
    m, n = A.shape
    Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, B)
    assert info == infoo
    assert np.array_equal(up[:n] == 0.0, upo == 0.0)
    tol = factor_tol(A)
    assert np.abs(F - Fo).max() <= tol
    for c in range(B.shape[1]):
        r = B[:, c] - A @ Xo[:, c]
        assert np.linalg.norm(X[:n, c] - Xo[:, c]) / np.linalg.norm(Xo[:, c]) <= 2 * lsq_forward_bound(A, Xo[:, c], r)
        assert abs(res[c] - reso[c]) <= 50 * m * U * max(reso[c], 1e-300) + tol


def _shapes(maxrows):
    return [(min(128, maxrows), 64, 1), (maxrows, 40, 2), (maxrows, 70, 1), (60, 60, 3), (maxrows, 1, 2),
            (97, 33, 5)]


@pytest.mark.parametrize("vi", list(range(13)))
def test_single_each_variant(hqr, oracle_mod, vi):
    import torch
    vs = _variants(hqr)
    if vi >= len(vs):
        pytest.skip("variant not built")
    idx, name, maxrows = vs[vi]
    _force_single(hqr, idx)
    rng = np.random.default_rng(200 + vi)
    for (m, n, r) in _shapes(maxrows):
        print("[case] single", name, (m, n, r), flush=True)
        A = rng.standard_normal((m, n))
        if n > 20:
            A[:, 18] = 0.0
        B = rng.standard_normal((m, r))
        dA, dB = to_dev(A), to_dev(B)
        up, res, info, _ = hqr.qr_lsq_solve(dA, dB)
        torch.cuda.synchronize()
        _check_solve(oracle_mod, A, B, to_host(dA), to_host(up), to_host(dB), to_host(res), int(info.item()))


@pytest.mark.parametrize("vi", [0, 6])
def test_factor_and_apply_each_variant(hqr, oracle_mod, vi):
    import torch
    vs = _variants(hqr)
    idx, name, maxrows = vs[vi]
    _force_single(hqr, idx)
    rng = np.random.default_rng(300 + vi)
    for (m, n, r) in [(maxrows, 48, 3), (77, 77, 2), (min(150, maxrows), 20, 1)]:
        print("[case] factor/apply", name, (m, n, r), flush=True)
        A = rng.standard_normal((m, n))
        B = rng.standard_normal((m, r))
        dA = to_dev(A)
        up, info = hqr.qr_factor(dA)
        torch.cuda.synchronize()
        Fo, upo = oracle_mod.qr_factor(A)
        assert int(info.item()) == 0
        assert np.abs(to_host(dA) - Fo).max() <= factor_tol(A)
        # apply the oracle's stored factorization with the GPU
        dF, dU, dB = to_dev(Fo), to_dev(upo.reshape(-1, 1))[:, 0].contiguous(), to_dev(B)
        hqr.qr_apply_qt(dF, dU, dB)
        torch.cuda.synchronize()
        qtb = oracle_mod.apply_qt(Fo, upo, B)
        assert np.abs(to_host(dB) - qtb).max() <= 50 * m * U * np.abs(B).max() * 10


def test_staging_limit_and_blocked_choice(hqr, oracle_mod):
    """n * nrhs at the staging limit of the smallest variant stays on it; a
    blocked-path rule sends a small problem to the multi-kernel path."""
    import torch
    vs = _variants(hqr)
    idx, name, maxrows = vs[0]
    _force_single(hqr, idx)
    rng = np.random.default_rng(400)
    m, n = maxrows, 128
    r = (maxrows * 17) // n
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((m, r))
    print("[case] staging limit", name, (m, n, r), flush=True)
    dA, dB = to_dev(A), to_dev(B)
    up, res, info, _ = hqr.qr_lsq_solve(dA, dB)
    torch.cuda.synchronize()
    _check_solve(oracle_mod, A, B, to_host(dA), to_host(up), to_host(dB), to_host(res), int(info.item()))
    hqr.tune_clear()
    hqr.tune_set(hqr.HQR_TUNE_SINGLE, 0, 1 << 40, 0, 1 << 40, -1)
    A = rng.standard_normal((100, 30))
    B = rng.standard_normal((100, 1))
    dA, dB = to_dev(A), to_dev(B)
    up, res, info, _ = hqr.qr_lsq_solve(dA, dB)
    torch.cuda.synchronize()
    _check_solve(oracle_mod, A, B, to_host(dA), to_host(up), to_host(dB), to_host(res), int(info.item()))


@pytest.mark.parametrize("qm", [1, 2, 4])
def test_batched_each_variant(hqr, oracle_mod, qm):
    import torch
    vs = [v for v in _variants(hqr) if v[1] == "wg256x%d" % qm]
    if not vs:
        pytest.skip("variant not built")
    idx, name, maxrows = vs[0]
    hqr.tune_clear()
    hqr.tune_set(hqr.HQR_TUNE_BATCHED, 0, 1 << 40, 0, 1 << 40, idx)
    rng = np.random.default_rng(500 + qm)
    probs = []
    for i in range(24):
        n = int(rng.integers(1, 100))
        m = min(maxrows, n + int(rng.integers(0, n + 1)))
        probs.append((rng.standard_normal((m, n)), rng.standard_normal((m, 4))))
    # one instance beyond the one-workgroup kernel's rows goes to the streaming kernel
    probs.append((rng.standard_normal((1100, 20)), rng.standard_normal((1100, 2))))
    print("[case] batched", name, len(probs), flush=True)
    As = [to_dev(A) for A, _ in probs]
    Bs = [to_dev(B) for _, B in probs]
    ups, res, info = hqr.qr_lsq_solve_batched(As, Bs)
    torch.cuda.synchronize()
    info = to_host(info).astype(int)
    for i, (A, B) in enumerate(probs):
        _check_solve(oracle_mod, A, B, to_host(As[i]), to_host(ups[i]), to_host(Bs[i]),
                     to_host(res[i])[:B.shape[1]], int(info[i]))


def test_batched_schedules_are_bitwise_equal(hqr):
    """The 256-thread variants (rows per thread, load depth) and the
    workgroups per CU change only how the batch is scheduled, never an
    instance's arithmetic: every candidate the autotuner may pick gives
    bitwise the same results."""
    import torch
    rng = np.random.default_rng(777)
    probs = []
    for i in range(40):
        n = int(rng.integers(1, 200))
        m = min(256, n + int(rng.integers(0, n + 1)))
        probs.append((rng.standard_normal((m, n)), rng.standard_normal((m, 3))))
    ref = None
    names = hqr.tune_variants()
    cands = [(i, nm) for i, nm in enumerate(names) if nm.startswith("wg256x")]
    print("[case] batched schedules", [nm for _, nm in cands], flush=True)
    for idx, nm in cands:
        for occ in (1, 2, 4):
            hqr.tune_clear()
            hqr.tune_set(hqr.HQR_TUNE_BATCHED, 0, 1 << 40, 0, 1 << 40, idx)
            hqr.tune_set(hqr.HQR_TUNE_OCCUPANCY, 0, 1 << 40, 0, 1 << 40, occ)
            As = [to_dev(A) for A, _ in probs]
            Bs = [to_dev(B) for _, B in probs]
            ups, res, info = hqr.qr_lsq_solve_batched(As, Bs)
            torch.cuda.synchronize()
            out = [(to_host(a), to_host(u), to_host(b)) for a, u, b in zip(As, ups, Bs)]
            if ref is None:
                ref = out
                continue
            for i, (x, y) in enumerate(zip(out, ref)):
                for p, q in zip(x, y):
                    assert np.array_equal(p, q), (nm, occ, i)
    hqr.tune_clear()
    hqr.load_tune_db()
