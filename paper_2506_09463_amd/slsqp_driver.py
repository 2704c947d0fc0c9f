"""Synthetic SLSQP-style driver: real iteration sequences turned into request
streams for the least-squares server.

The paper's end-to-end experiment (Section 4.4, Exp. 4) runs SLSQP on a
finite-element boundary-value problem whose data are not available.  This
driver stands in for it with a synthetic nonlinear least-squares problem of
the same structure -- a discretized 1-D nonlinear boundary-value problem fit
to observations, n degrees of freedom:

    r(u) = [ K u + g u^3 - f ; w (u - y) ]          (2n residuals)
    u_0 = a, u_{n-1} = b                            (equality constraints)

with K = (n+1)^2 tridiag(-1, 2, -1), g > 0 and f, y, a, b from a seed.
Each outer iteration of the sequential-quadratic (Gauss-Newton) method
linearizes r and the constraints and solves the least-squares subproblem

    min ||J d + r||  subject to  C d = c - C u,

the subproblem SLSQP solves with the in-place Householder QR (Section 1).
Two modes:

  * ``served``: the two constraints fix u_0 and u_{n-1}, so the subproblem
    becomes an ordinary least-squares problem in the n-2 interior unknowns.
    Per outer iteration each instance sends one factor+solve request (the
    Gauss-Newton step) and then two solve-only requests on the cached factor
    (two chord corrections: d_k = argmin ||J d + r(u + d_1 + .. + d_{k-1})||
    with the same J) -- the three successive solves on one factor of the
    served workload.  Instances run in lock step, so every phase is one
    burst of requests, continuously batched by the server.
  * ``lse``: the constraints stay in the subproblem, solved by qr_lse_solve
    (equality-constrained least squares on the GPU), one call per instance
    and iteration.

All the driver's own arithmetic (residuals, Jacobians, step updates) runs on
the host in NumPy: it is the optimizer's outer loop, not the solver's path.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np

from paper_2506_09463_amd.server import Request


@dataclasses.dataclass
class BvpFit:
    n: int
    g: float
    w: float
    f: np.ndarray
    y: np.ndarray
    a: float
    b: float

    @staticmethod
    def make(n: int, seed: int) -> "BvpFit":
        rng = np.random.default_rng(seed)
        t = np.linspace(0.0, 1.0, n)
        y = np.sin(np.pi * t) + 0.1 * rng.standard_normal(n)
        f = 40.0 * np.cos(3.0 * t) + 5.0 * rng.standard_normal(n)
        return BvpFit(n, g=float(5.0 + 5.0 * rng.random()), w=2.0 * (n + 1), f=f, y=y,
                      a=float(rng.standard_normal() * 0.1), b=float(rng.standard_normal() * 0.1))

    def K(self) -> np.ndarray:
        n = self.n
        h2 = (n + 1) ** 2
        return h2 * (2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1))

    def residual(self, u: np.ndarray) -> np.ndarray:
        Ku = self.K() @ u
        return np.concatenate([Ku + self.g * u ** 3 - self.f, self.w * (u - self.y)])

    def jacobian(self, u: np.ndarray) -> np.ndarray:
        return np.vstack([self.K() + np.diag(3.0 * self.g * u ** 2), self.w * np.eye(self.n)])

    def constraints(self):
        C = np.zeros((2, self.n))
        C[0, 0] = 1.0
        C[1, -1] = 1.0
        return C, np.array([self.a, self.b])

    def start(self) -> np.ndarray:
        u = np.linspace(self.a, self.b, self.n)
        return u

    def objective(self, u: np.ndarray) -> float:
        r = self.residual(u)
        return 0.5 * float(r @ r)


def _interior(M: np.ndarray) -> np.ndarray:
    return np.asfortranarray(M[:, 1:-1])


@dataclasses.dataclass
class DriverStats:
    outer_iterations: int
    requests: int
    wall_s: float
    converged: int
    instances: int
    final_objectives: List[float]
    latencies_ms: List[float]


def run_served(problems: List[BvpFit], server, max_outer: int = 20, tol: float = 1e-10,
               chord_steps: int = 2):
    """Gauss-Newton with chord corrections, every subproblem a request to
    `server` (a paper_2506_09463_amd.server.Server).  Constraints are
    eliminated (boundary values fixed), so each request is an ordinary
    least-squares problem in the interior unknowns.  Returns (DriverStats,
    final iterates)."""
    us = []
    for p in problems:
        u = p.start()
        u[0], u[-1] = p.a, p.b
        us.append(u)
    active = list(range(len(problems)))
    rid = 0
    t0 = time.perf_counter()
    outer = 0
    latencies = []

    def serve(reqs):
        for r in reqs:
            server.submit(r)
        server.drain()
        for r in reqs:
            latencies.append((r.t_done - r.t_arrival) * 1e3)
            if r.status != "done" or r.info != 0:
                raise RuntimeError("request %d failed: status %s info %d" % (r.rid, r.status, r.info))

    for outer in range(1, max_outer + 1):
        if not active:
            outer -= 1
            break
        # Gauss-Newton step: factor J, solve J d = -r
        reqs = []
        for i in active:
            p, u = problems[i], us[i]
            J = _interior(p.jacobian(u))
            r = p.residual(u)
            reqs.append(Request(rid, instance=i, kind="factor_solve", m=J.shape[0], n=J.shape[1],
                                B=np.asfortranarray(-r.reshape(-1, 1)), A=J))
            rid += 1
        serve(reqs)
        steps = {}
        for i, rq in zip(active, reqs):
            d = rq.x[:, 0]
            us[i][1:-1] += d
            steps[i] = np.linalg.norm(d)
        # chord corrections on the same factor
        for _ in range(chord_steps):
            reqs = []
            for i in active:
                p, u = problems[i], us[i]
                r = p.residual(u)
                reqs.append(Request(rid, instance=i, kind="solve", m=2 * p.n, n=p.n - 2,
                                    B=np.asfortranarray(-r.reshape(-1, 1))))
                rid += 1
            serve(reqs)
            for i, rq in zip(active, reqs):
                d = rq.x[:, 0]
                us[i][1:-1] += d
                steps[i] = max(steps[i], np.linalg.norm(d))
        active = [i for i in active if steps[i] > tol * max(1.0, np.linalg.norm(us[i]))]
    wall = time.perf_counter() - t0
    return DriverStats(outer_iterations=outer, requests=rid, wall_s=wall,
                       converged=len(problems) - len(active), instances=len(problems),
                       final_objectives=[p.objective(u) for p, u in zip(problems, us)], latencies_ms=latencies), us


def run_lse(problems: List[BvpFit], max_outer: int = 20, tol: float = 1e-10):
    """Sequential-quadratic iterations with the linearized constraints kept in
    each subproblem, solved on the GPU by qr_lse_solve."""
    import torch
    import paper_2506_09463_amd as hqr
    us = [p.start() for p in problems]
    iters = [0] * len(problems)
    t0 = time.perf_counter()
    calls = 0
    for i, p in enumerate(problems):
        C, c = p.constraints()
        for it in range(1, max_outer + 1):
            u = us[i]
            J = p.jacobian(u)
            r = p.residual(u)
            dA, dC = hqr.colmajor(J), hqr.colmajor(C)
            db = hqr.colmajor(-r.reshape(-1, 1))[:, 0]
            dd = hqr.colmajor((c - C @ u).reshape(-1, 1))[:, 0]
            x, info = hqr.qr_lse_solve(dA, dC, db, dd)
            d = x[: p.n].cpu().numpy()
            calls += 1
            if int(info.item()) != 0:
                raise RuntimeError("qr_lse_solve info %d" % int(info.item()))
            us[i] = u + d
            iters[i] = it
            if np.linalg.norm(d) <= tol * max(1.0, np.linalg.norm(us[i])):
                break
    torch.cuda.synchronize()
    return {"calls": calls, "wall_s": time.perf_counter() - t0, "iterations": iters,
            "final_objectives": [p.objective(u) for p, u in zip(problems, us)]}, us


def make_problems(count: int, seed: int, nmin: int = 32, nmax: int = 1024) -> List[BvpFit]:
    """`count` instances, n log-uniform in [nmin, nmax]."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=count))).astype(int)
    return [BvpFit.make(int(n), seed * 100003 + i) for i, n in enumerate(ns)]
