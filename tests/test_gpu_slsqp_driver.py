"""The synthetic SLSQP-style driver on the GPU: its Gauss-Newton/chord
request stream through the continuous-batching server (factor reuse for the
chord solves), and the constrained mode through qr_lse_solve.  Both reach
the same stationary point of the constrained fit, and the served iterates
equal those of the same driver run against the oracle (within the solves'
rounding)."""
import time

import numpy as np
import pytest

from paper_2506_09463_amd import slsqp_driver
from paper_2506_09463_amd.server import GpuExecutor, Server
from tests.test_slsqp_driver_cpu import OracleNow

pytestmark = pytest.mark.gpu


def test_served_driver_converges_like_the_oracle_run(oracle_mod):
    import torch
    assert torch.cuda.is_available()
    probs = slsqp_driver.make_problems(24, seed=5, nmin=32, nmax=700)
    print("[case] slsqp driver served", [p.n for p in probs], flush=True)
    srv = Server(GpuExecutor(nstreams=2), budget_bytes=8 << 30)
    stats, us = slsqp_driver.run_served(probs, srv, max_outer=15, tol=1e-11)
    print("[case] outer %d requests %d wall %.2f s" % (stats.outer_iterations, stats.requests, stats.wall_s),
          flush=True)
    assert stats.converged == len(probs)
    ref_probs = slsqp_driver.make_problems(24, seed=5, nmin=32, nmax=700)
    srv2 = Server(OracleNow(oracle_mod), budget_bytes=8 << 30, clock=time.perf_counter)
    _, uo = slsqp_driver.run_served(ref_probs, srv2, max_outer=15, tol=1e-11)
    for p, u, v in zip(probs, us, uo):
        assert np.linalg.norm(u - v) <= 1e-8 * np.linalg.norm(v), p.n
        J = p.jacobian(u)[:, 1:-1]
        r = p.residual(u)
        assert np.linalg.norm(J.T @ r) <= 1e-8 * np.linalg.norm(J, 2) * np.linalg.norm(r)


def test_lse_driver_reaches_the_same_point():
    probs = slsqp_driver.make_problems(3, seed=6, nmin=40, nmax=300)
    print("[case] slsqp driver lse", [p.n for p in probs], flush=True)
    res, us = slsqp_driver.run_lse(probs, max_outer=20, tol=1e-11)
    srv = Server(GpuExecutor(nstreams=1), budget_bytes=8 << 30)
    _, ue = slsqp_driver.run_served(slsqp_driver.make_problems(3, seed=6, nmin=40, nmax=300), srv,
                                    max_outer=15, tol=1e-11)
    for p, u, v in zip(probs, us, ue):
        C, c = p.constraints()
        assert np.abs(C @ u - c).max() <= 1e-12
        assert np.linalg.norm(u - v) <= 1e-8 * np.linalg.norm(v), p.n
