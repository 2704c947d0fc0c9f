"""qr_lsq_solve_static -- the entry point that allocates nothing -- against
qr_lsq_solve, through the C ABI.

Two calls in a row on one stream, the second smaller (the scratch array
keeps the first call's contents), each compared with qr_lsq_solve on the
same input: bitwise with the look-ahead off (the static entry runs the
same kernels on one stream), and against the oracle within the same
tolerances as every parity test.  A problem whose workspace exceeds the
array is refused with HQR_ENOMEM before anything runs.
"""
import ctypes
import os

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
    return h


def _static(hqr, A, B):
    import torch
    lib = hqr.load()
    m, n = A.shape
    nrhs = B.shape[1]
    dA, dB = to_dev(A), to_dev(B)
    up = torch.empty(n, dtype=torch.float64, device="cuda")
    res = torch.empty(nrhs, dtype=torch.float64, device="cuda")
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    rc = lib.qr_lsq_solve_static(m, n, nrhs, ctypes.c_void_p(dA.data_ptr()), dA.stride(1), ctypes.c_void_p(up.data_ptr()),
                                 ctypes.c_void_p(dB.data_ptr()), dB.stride(1), ctypes.c_void_p(res.data_ptr()),
                                 ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    assert rc == 0, rc
    torch.cuda.synchronize()
    return to_host(dA), to_host(up), to_host(dB), to_host(res), int(info.item())


def _regular(hqr, A, B):
    import torch
    dA, dB = to_dev(A), to_dev(B)
    up, res, info, _ = hqr.qr_lsq_solve(dA, dB)
    torch.cuda.synchronize()
    return to_host(dA), to_host(up)[:A.shape[1]], to_host(dB), to_host(res)[:B.shape[1]], int(info.item())


@pytest.mark.parametrize("shapes", [[(1000, 333, 2, 1), (600, 200, 1, 2)], [(2100, 900, 3, 3), (128, 64, 1, 4)]])
def test_static_matches_qr_lsq_solve(hqr, oracle_mod, monkeypatch, shapes):
    for (m, n, nrhs, seed) in shapes:
        rng = np.random.default_rng(900 + seed)
        A = np.asfortranarray(rng.standard_normal((m, n)))
        B = np.asfortranarray(rng.standard_normal((m, nrhs)))
        print("[case] qr_lsq_solve_static", (m, n, nrhs), flush=True)
        got = _static(hqr, A, B)
        monkeypatch.setenv("HQR_LOOKAHEAD", "0")
        ref = _regular(hqr, A, B)
        monkeypatch.delenv("HQR_LOOKAHEAD")
        for a, b in zip(got[:4], ref[:4]):
            assert np.array_equal(a, b)
        assert got[4] == ref[4] == 0
        la = _regular(hqr, A, B)          # default (look-ahead) entry point
        assert np.abs(got[0] - la[0]).max() <= factor_tol(A)
        Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, B)
        assert np.abs(got[0] - Fo).max() <= factor_tol(A)
        for c in range(nrhs):
            r = B[:, c] - A @ Xo[:, c]
            rel = np.linalg.norm(got[2][:n, c] - Xo[:, c]) / np.linalg.norm(Xo[:, c])
            assert rel <= 2 * lsq_forward_bound(A, Xo[:, c], r)


def test_static_refuses_oversized(hqr):
    import torch
    lib = hqr.load()
    m, n = 16384, 8192
    assert lib.hqr_workspace_size(m, n, 1, 0) > (80 << 20)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    fake = ctypes.c_void_p(info.data_ptr())     # never touched: refused first
    rc = lib.qr_lsq_solve_static(m, n, 1, fake, m, fake, fake, m, None, fake, None)
    assert rc == hqr.HQR_ENOMEM
