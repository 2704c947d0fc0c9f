"""The synthetic SLSQP-style driver on the CPU: its request stream goes
through the server's policy with an executor that solves each request with
the oracle at once.  The iterates converge to a stationary point of the
constrained fit (the interior gradient J^T r vanishes, the boundary values
hold exactly), and every outer iteration sends one factor+solve and two
solve-only requests per active instance."""
import time

import numpy as np

from paper_2506_09463_amd import slsqp_driver
from paper_2506_09463_amd.server import Server


class OracleNow:
    """Executor that completes every batch at once with the oracle."""

    def __init__(self, oracle):
        self.oracle = oracle
        self.busy = False
        self.batches = []

    def idle_stream(self):
        return True

    def free_factor(self, handle):
        pass

    def launch(self, batch, entries):
        self.batches.append([(r.kind, r.instance) for r in batch])
        for r, e in zip(batch, entries):
            if r.kind == "factor_solve":
                e.handle = self.oracle.qr_factor(r.A)
        return (batch, entries)

    def poll(self, h):
        return True

    def collect(self, h, batch):
        for r, e in zip(*h):
            F, up = e.handle
            qtb = self.oracle.apply_qt(F, up, r.B)
            x, info = self.oracle.backsolve(F, qtb)
            r.x, r.info = x, info


def test_driver_converges_and_request_pattern(oracle_mod):
    probs = slsqp_driver.make_problems(4, seed=3, nmin=32, nmax=80)
    ex = OracleNow(oracle_mod)
    srv = Server(ex, budget_bytes=1 << 30, clock=time.perf_counter)
    stats, us = slsqp_driver.run_served(probs, srv, max_outer=20, tol=1e-11)
    assert stats.converged == len(probs)
    kinds = [k for b in ex.batches for k, _ in b]
    assert kinds.count("solve") == 2 * kinds.count("factor_solve")
    assert stats.requests == len(kinds)
    for p, u in zip(probs, us):
        assert u[0] == p.a and u[-1] == p.b
        J = p.jacobian(u)[:, 1:-1]
        r = p.residual(u)
        g = J.T @ r
        assert np.linalg.norm(g) <= 1e-8 * np.linalg.norm(J, 2) * np.linalg.norm(r)
