"""Served workload on the GPU: every result computed in the continuous-batching
mix is bitwise the result of the same requests served alone (batched and
whole-GPU paths alike: every kernel's reduction order depends on the
problem's shape only, and solves on different server streams share no
library state), and matches the oracle."""
import numpy as np
import pytest

from paper_2506_09463_amd.server import GpuExecutor, Server, make_stream
from tests.gpu_util import lsq_forward_bound

pytestmark = pytest.mark.gpu


def _serve(reqs, nstreams=2):
    ex = GpuExecutor(nstreams=nstreams)
    srv = Server(ex, budget_bytes=8 << 30)
    for r in reqs:
        srv.submit(r)
        srv.step()
    srv.drain(timeout=300)
    return srv


def _clone(r):
    import copy
    c = copy.copy(r)
    c.t_arrival, c.t_done, c.x, c.status = 0.0, -1.0, None, "new"
    return c


def test_served_mix_equals_alone(oracle_mod):
    import torch
    assert torch.cuda.is_available()
    reqs = make_stream(24, seed=6, solves_per_instance=3, nmax=700)
    keep = {r.rid: _clone(r) for r in reqs}
    mats = {r.instance: r.A.copy() for r in reqs if r.kind == "factor_solve"}
    print("[case] served mix", len(reqs), flush=True)
    srv = _serve(reqs)
    assert len(srv.done) == len(reqs) and not srv.rejected
    by_inst = {}
    for r in reqs:
        by_inst.setdefault(r.instance, []).append(keep[r.rid])
    # every instance above the batched range, and the first ten below it
    large = [i for i, g in by_inst.items() if g[0].n > 512]
    small = [i for i, g in by_inst.items() if g[0].n <= 512][:10]
    assert large, "the seeded stream has whole-GPU instances"
    for inst in large + small:
        group = by_inst[inst]
        print("[case] alone instance", inst, flush=True)
        alone = _serve(group, nstreams=1)
        for a in alone.done:
            mix = next(r for r in reqs if r.rid == a.rid)
            assert np.array_equal(a.x, mix.x), (inst, a.rid, a.n)
            assert np.array_equal(a.resnorm, mix.resnorm), (inst, a.rid, a.n)
            assert a.info == mix.info
    for r in reqs[:12]:
        A = mats[r.instance]
        xo, *_ = oracle_mod.lsq_solve(A, r.B)
        for c in range(r.nrhs):
            rr = r.B[:, c] - A @ xo[:, c]
            assert np.linalg.norm(r.x[:, c] - xo[:, c]) / np.linalg.norm(xo[:, c]) <= 2 * lsq_forward_bound(A, xo[:, c], rr)


def test_served_mixed_precision_requests(oracle_mod):
    """Mixed-flagged instances above the batched range are served by the
    mixed-precision path (their factor and the FP64 copy of A cached for the
    later solve-only requests); every such result is within 1e-10 of the
    extended-precision reference, and FP64 ones within the FP64 bound."""
    import torch
    from paper_2506_09463_amd.server import MIXED_MIN_N
    reqs = make_stream(40, seed=8, solves_per_instance=3, nmax=900)
    mats = {r.instance: r.A.copy() for r in reqs if r.kind == "factor_solve"}
    mixed = [r for r in reqs if r.mixed_path]
    assert mixed, "the seeded stream has mixed-path instances"
    assert all(r.n >= MIXED_MIN_N for r in mixed)
    print("[case] served mixed", len(reqs), len(mixed), flush=True)
    srv = _serve(reqs)
    assert len(srv.done) == len(reqs) and not srv.rejected
    for r in mixed:
        assert r.info == 0, r.rid
        A = mats[r.instance]
        for c in range(r.nrhs):
            xref, _ = oracle_mod.lsq_reference(A, r.B[:, c])
            assert np.linalg.norm(r.x[:, c] - xref) / np.linalg.norm(xref) <= 1e-10, (r.rid, c)
