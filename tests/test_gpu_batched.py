"""GPU parity of the batched persistent launch (qr_lsq_solve_batched).

Each instance is checked against the FP64 oracle with the same tolerances as
the single-problem tests; info is exact; a result computed alone and inside
a batch is bitwise identical (the batch composition never changes an
instance's arithmetic).
"""
import numpy as np
import pytest

from paper_2506_09463_amd import workloads
from tests.gpu_util import U, factor_tol, lsq_forward_bound, lsq_orthogonality, to_dev, to_host

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


def _solve_batch(hqr, problems):
    import torch
    As = [to_dev(A) for A, _ in problems]
    Bs = [to_dev(B) for _, B in problems]
    ups, res, info = hqr.qr_lsq_solve_batched(As, Bs)
    torch.cuda.synchronize()
    out = []
    for i, (A, B) in enumerate(problems):
        n = A.shape[1]
        out.append((to_host(As[i]), to_host(ups[i])[:n], to_host(Bs[i]), to_host(res[i])[:B.shape[1]]))
    return out, to_host(info).astype(int)


def _mixed_problems(seed, count, nmax, nrhs):
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(count):
        n = int(rng.integers(1, nmax + 1))
        m = n + int(rng.integers(0, n + 1))
        probs.append((np.asfortranarray(rng.standard_normal((m, n))),
                      np.asfortranarray(rng.standard_normal((m, nrhs)))))
    return probs


def test_batched_parity(hqr, oracle_mod):
    probs = _mixed_problems(91, 40, 200, 8)
    # edge instances: square, single column, zero column, singular
    rng = np.random.default_rng(92)
    probs.append((np.asfortranarray(rng.standard_normal((50, 50))), np.asfortranarray(rng.standard_normal((50, 2)))))
    probs.append((np.asfortranarray(rng.standard_normal((7, 1))), np.asfortranarray(rng.standard_normal((7, 3)))))
    Z = rng.standard_normal((30, 10))
    Z[:, 4] = 0.0
    probs.append((np.asfortranarray(Z), np.asfortranarray(rng.standard_normal((30, 1)))))
    _say("batched parity", len(probs))
    out, info = _solve_batch(hqr, probs)
    for i, ((A, B), (F, up, X, res)) in enumerate(zip(probs, out)):
        m, n = A.shape
        Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, B)
        assert info[i] == infoo, i
        assert np.array_equal(up == 0.0, upo == 0.0), i
        if infoo:
            qtbo = oracle_mod.apply_qt(Fo, upo, B)
            assert np.abs(X - qtbo).max() <= 1e-10 * m, i
            continue
        tol = factor_tol(A)
        assert np.abs(F - Fo).max() <= tol, i
        for c in range(B.shape[1]):
            r = B[:, c] - A @ Xo[:, c]
            assert np.linalg.norm(X[:n, c] - Xo[:, c]) / np.linalg.norm(Xo[:, c]) <= 2 * lsq_forward_bound(A, Xo[:, c], r), i
            assert abs(res[c] - reso[c]) <= 50 * m * U * max(reso[c], 1e-300) + tol, i


def test_batched_alone_equals_in_batch(hqr):
    probs = _mixed_problems(93, 25, 300, 4)
    _say("alone vs in batch")
    out, info = _solve_batch(hqr, probs)
    for i in (0, 7, 24):
        alone, info1 = _solve_batch(hqr, [probs[i]])
        for a, b in zip(alone[0], out[i]):
            assert np.array_equal(a, b), i
        assert info1[0] == info[i]


def test_batched_workload_sample(hqr, oracle_mod):
    """A slice of the 2000-instance workload (n ~ U{16..512}, m = n + U{0..n},
    8 right-hand sides): every instance passes the orthogonality check and a
    sample matches the oracle."""
    probs = workloads.batch_problem(count=120, seed=workloads.SEED_BATCH)
    _say("workload sample", len(probs))
    out, info = _solve_batch(hqr, probs)
    assert np.all(info == 0)
    for i, ((A, B), (F, up, X, res)) in enumerate(zip(probs, out)):
        n = A.shape[1]
        for c in range(B.shape[1]):
            assert lsq_orthogonality(A, X[:n, c], B[:, c]) <= 50 * n * U, i
    for i in (0, 5, 60, 119):
        A, B = probs[i]
        n = A.shape[1]
        Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, B)
        F, up, X, res = out[i]
        assert np.abs(F - Fo).max() <= factor_tol(A)
        for c in range(B.shape[1]):
            r = B[:, c] - A @ Xo[:, c]
            assert np.linalg.norm(X[:n, c] - Xo[:, c]) / np.linalg.norm(Xo[:, c]) <= 2 * lsq_forward_bound(A, Xo[:, c], r)


def test_batched_argument_errors(hqr):
    A = to_dev(np.ones((3, 4)))
    B = to_dev(np.ones((3, 1)))
    with pytest.raises(hqr.HQRError) as e:
        hqr.qr_lsq_solve_batched([A], [B])
    assert e.value.status == -3


@pytest.mark.timeout(900)
def test_batched_full_workload_vs_oracle(hqr, oracle_mod):
    """All 2000 instances of the batched workload (n ~ U{16..512},
    m = n + U{0..n}, 8 right-hand sides) in one launch, the launch the
    benchmark times, each compared with the oracle: the factored matrix
    element-wise within 50 n u kappa ||A||, every x within the LSQ forward
    bound, info exact.  kappa is taken from the oracle's R (same singular
    values as A)."""
    import time
    probs = workloads.batch_problem(count=2000, seed=workloads.SEED_BATCH)
    _say("full batched workload", len(probs))
    out, info = _solve_batch(hqr, probs)
    assert np.all(info == 0)
    t0 = time.time()
    worst_f, worst_x = 0.0, 0.0
    for i, ((A, B), (F, up, X, res)) in enumerate(zip(probs, out)):
        m, n = A.shape
        Xo, Fo, upo, reso, infoo = oracle_mod.lsq_solve(A, B)
        assert infoo == 0, i
        sv = np.linalg.svd(np.triu(Fo[:n]), compute_uv=False)
        k, nA = sv[0] / sv[-1], sv[0]
        ftol = 50 * n * U * k * nA
        df = np.abs(F - Fo).max()
        assert df <= ftol, (i, df, ftol)
        assert np.array_equal(up == 0.0, upo == 0.0), i
        worst_f = max(worst_f, df / ftol)
        for c in range(B.shape[1]):
            xo = Xo[:, c]
            r = B[:, c] - A @ xo
            bound = 50 * n * U * k * (1 + k * np.linalg.norm(r) / (nA * np.linalg.norm(xo)))
            e = np.linalg.norm(X[:n, c] - xo) / np.linalg.norm(xo)
            assert e <= 2 * bound, (i, c, e, bound)
            worst_x = max(worst_x, e / bound)
        if i % 250 == 0:
            _say("checked %d instances (%.0f s)" % (i + 1, time.time() - t0))
    _say("worst |F - F_o| / tol %.2e, worst x error / bound %.2e" % (worst_f, worst_x))


def test_batch_plan_reuse_is_bitwise(hqr):
    """A BatchPlan marshals the pointers once; running it again on restored
    inputs gives bitwise the results of a fresh qr_lsq_solve_batched call."""
    import torch
    probs = _mixed_problems(95, 60, 300, 4)
    _say("BatchPlan reuse", len(probs))
    ref, ref_info = _solve_batch(hqr, probs)
    A0 = [to_dev(A) for A, _ in probs]
    B0 = [to_dev(B) for _, B in probs]
    As = [a.clone() for a in A0]
    Bs = [b.clone() for b in B0]
    plan = hqr.BatchPlan(As, Bs)
    for rep in range(2):
        for a, a0 in zip(As, A0):
            a.copy_(a0)
        for b, b0 in zip(Bs, B0):
            b.copy_(b0)
        ups, res, info = plan.run()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(info).astype(int), ref_info)
        for i, (A, B) in enumerate(probs):
            n = A.shape[1]
            assert np.array_equal(to_host(As[i]), ref[i][0])
            assert np.array_equal(to_host(ups[i])[:n], ref[i][1])
            assert np.array_equal(to_host(Bs[i]), ref[i][2])
