"""Server policy on the CPU: a fake executor runs the oracle and completes
batches on a scripted clock.  Covers admission by HBM budget, rejection of
requests larger than the budget, wait-list release when a factorization
completes, LRU eviction, continuous batching, and the p50/p99 arithmetic."""
import numpy as np
import pytest

from paper_2506_09463_amd.server import Request, Server, percentile


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Completes a batch `dur` seconds (scripted clock) after launch."""

    def __init__(self, clock, nstreams=1, dur=1.0, oracle=None):
        self.clock, self.dur, self.oracle = clock, dur, oracle
        self.busy = [False] * nstreams
        self.batches = []
        self.freed = []

    def idle_stream(self):
        return not all(self.busy)

    def free_factor(self, handle):
        self.freed.append(handle)

    def launch(self, batch, entries):
        si = self.busy.index(False)
        self.busy[si] = True
        self.batches.append([r.rid for r in batch])
        for r, e in zip(batch, entries):
            if r.kind == "factor_solve":
                F, up = self.oracle.qr_factor(r.A)
                e.handle = (F, up, r.instance)
        return {"si": si, "t": self.clock() + self.dur, "batch": batch, "entries": entries}

    def poll(self, h):
        return self.clock() >= h["t"]

    def collect(self, h, batch):
        self.busy[h["si"]] = False
        for r, e in zip(h["batch"], h["entries"]):
            F, up, _ = e.handle
            qtb = self.oracle.apply_qt(F, up, r.B)
            x, info = self.oracle.backsolve(F, qtb)
            r.x, r.info = x, info


def _req(rid, inst, kind, m=8, n=4, nrhs=1, seed=0):
    rng = np.random.default_rng(seed + rid)
    A = rng.standard_normal((m, n)) if kind == "factor_solve" else None
    return Request(rid, inst, kind, m, n, rng.standard_normal((m, nrhs)), A=A)


@pytest.fixture
def env(oracle_mod):
    clk = Clock()
    ex = FakeExecutor(clk, nstreams=1, dur=1.0, oracle=oracle_mod)
    return clk, ex


def test_results_match_oracle_and_wait_list(env, oracle_mod):
    clk, ex = env
    srv = Server(ex, budget_bytes=1 << 20, clock=clk)
    a = srv.submit(_req(0, 7, "factor_solve"))
    b = srv.submit(_req(1, 7, "solve"))        # factor still in flight -> wait list
    srv.step()
    assert a.status == "running" and b.status == "waiting"
    clk.t = 1.0
    srv.step()                                  # a completes, b released and launched
    assert a.status == "done" and b.status == "running"
    clk.t = 2.0
    srv.step()
    assert b.status == "done"
    for r in (a, b):
        A = a.A if a.A is not None else None
    # x of both requests equals the oracle's least-squares solution
    A0 = np.random.default_rng(0).standard_normal((8, 4))
    for r in (a, b):
        xo, *_ = oracle_mod.lsq_solve(A0, r.B)
        assert np.allclose(r.x, xo, rtol=1e-12, atol=1e-12)
    st = srv.stats()
    assert st["completed"] == 2 and st["p50_ms"] == pytest.approx(1000.0) and st["p99_ms"] == pytest.approx(2000.0)


def test_admission_by_budget_and_rejection(env):
    clk, ex = env
    one = _req(0, 0, "factor_solve").bytes_needed(False)
    srv = Server(ex, budget_bytes=2 * one, clock=clk)
    big = srv.submit(_req(9, 9, "factor_solve", m=64, n=32))
    assert big.status == "rejected"             # larger than the whole budget
    reqs = [srv.submit(_req(i, i, "factor_solve")) for i in range(3)]
    srv.step()
    # two fit the budget and launch as one batch; the third waits for bytes
    assert [r.status for r in reqs] == ["running", "running", "new"]
    assert ex.batches == [[0, 1]]
    clk.t = 1.0
    srv.step()
    # the request buffers came back, but the two cached factors still hold
    # bytes; the third is admitted by evicting the least recently used
    assert reqs[2].status == "running" and len(ex.freed) >= 1
    assert srv.in_use <= srv.budget


def test_continuous_batching_joins_next_launch(env):
    clk, ex = env
    srv = Server(ex, budget_bytes=1 << 20, clock=clk)
    srv.submit(_req(0, 0, "factor_solve"))
    srv.step()                                  # launched alone
    clk.t = 0.5
    srv.submit(_req(1, 1, "factor_solve"))      # arrive while the GPU is busy
    srv.submit(_req(2, 2, "factor_solve"))
    srv.step()
    assert ex.batches == [[0]]
    clk.t = 1.0
    srv.step()
    assert ex.batches == [[0], [1, 2]]          # both join the next launch


def test_lru_eviction_skips_factors_in_use(env):
    clk, ex = env
    one = _req(0, 0, "factor_solve").bytes_needed(False)
    srv = Server(ex, budget_bytes=2 * one + 100, clock=clk)
    srv.submit(_req(0, 0, "factor_solve"))
    srv.submit(_req(1, 1, "factor_solve"))
    srv.step()
    clk.t = 1.0
    srv.step()
    srv.submit(_req(2, 0, "solve"))             # touches instance 0 (most recent)
    srv.step()
    clk.t = 2.0
    srv.step()
    srv.submit(_req(3, 2, "factor_solve"))      # needs an eviction: instance 1 is LRU
    srv.step()
    assert 1 not in srv.cache and 0 in srv.cache


def test_solve_without_factor_rejected(env):
    clk, ex = env
    srv = Server(ex, clock=clk)
    r = srv.submit(_req(0, 5, "solve"))
    assert r.status == "rejected"


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50 and percentile(v, 99) == 99 and percentile(v, 100) == 100
    assert percentile([3.0], 99) == 3.0


class NoConvExecutor(FakeExecutor):
    """Reports an unconverged refinement for every mixed request until it is
    re-run as a fallback."""

    def collect(self, h, batch):
        super().collect(h, batch)
        for r in batch:
            if r.mixed_path and not r.fallback:
                r.info |= (1 << 29)


def test_unconverged_mixed_request_is_requeued_as_fp64(oracle_mod, monkeypatch):
    from paper_2506_09463_amd import server
    monkeypatch.setattr(server, "MIXED_MIN_N", 1)
    clk = Clock()
    ex = NoConvExecutor(clk, nstreams=1, dur=1.0, oracle=oracle_mod)
    srv = Server(ex, budget_bytes=1 << 20, clock=clk)
    a = _req(0, 3, "factor_solve")
    a.precision = "mixed"
    b = _req(1, 4, "factor_solve")
    srv.submit(a)
    srv.submit(b)
    srv.step()
    assert ex.batches == [[0, 1]]
    clk.t = 1.0
    srv.step()
    # b is done; a came back unconverged and runs again as a fallback, keeping
    # its slot; its solve-only followers still wait for its factor
    assert b.status == "done" and a.status == "running" and a.fallback
    assert ex.batches == [[0, 1], [0]] and srv.slots == 1
    clk.t = 2.0
    srv.step()
    assert a.status == "done" and a.t_done == 2.0 and not srv.busy()
    A0 = np.random.default_rng(0).standard_normal((8, 4))
    xo, *_ = oracle_mod.lsq_solve(A0, a.B)
    assert np.allclose(a.x, xo, rtol=1e-12, atol=1e-12)


class ClassExecutor(FakeExecutor):
    """Sorts requests into launch classes like the GPU executor: n <= 4 into
    one batched launch, larger ones one per launch; large launches take 3 s,
    batched ones 1 s."""

    def launch_class(self, r):
        return ("batched", 1 << 30) if r.n <= 4 else ("single", 1)

    def launch(self, batch, entries):
        h = super().launch(batch, entries)
        if batch[0].n > 4:
            h["t"] = self.clock() + 3.0
        return h


def test_launch_classes_keep_small_requests_off_large_launches(oracle_mod):
    """The class of the oldest ready request goes first; small requests join
    one batched launch and never ride on a large one, so they complete after
    1 s while the large ones (one launch each) take 3 s."""
    clk = Clock()
    ex = ClassExecutor(clk, nstreams=3, dur=1.0, oracle=oracle_mod)
    srv = Server(ex, budget_bytes=1 << 24, clock=clk)
    reqs = [srv.submit(_req(0, 0, "factor_solve", m=16, n=8)),
            srv.submit(_req(1, 1, "factor_solve")),
            srv.submit(_req(2, 2, "factor_solve", m=16, n=8)),
            srv.submit(_req(3, 3, "factor_solve"))]
    srv.step()
    assert ex.batches == [[0], [1, 3], [2]]
    clk.t = 1.0
    srv.step()
    assert [r.status for r in reqs] == ["running", "done", "running", "done"]
    clk.t = 3.0
    srv.step()
    assert all(r.status == "done" for r in reqs)
    st = srv.stats()
    assert st["p50_ms"] == pytest.approx(1000.0) and st["p99_ms"] == pytest.approx(3000.0)
    A0 = np.random.default_rng(1).standard_normal((8, 4))
    xo, *_ = oracle_mod.lsq_solve(A0, reqs[1].B)
    assert np.allclose(reqs[1].x, xo, rtol=1e-12, atol=1e-12)
