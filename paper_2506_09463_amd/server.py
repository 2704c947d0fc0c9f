"""Continuous-batching server for least-squares solves with on-device factor reuse.

Requests arrive over time (the client decides when).  Each carries either a
new matrix to factor and solve (``kind="factor_solve"``) or only new
right-hand sides for an instance whose factorization the server still holds
(``kind="solve"``, the successive solves of one SLSQP-like iteration).

Scheduling policy (host side; the GPU work is libhqr's):
  * admission: a request is admitted when its device bytes (matrix, reflector
    scalars, right-hand sides) fit the HBM budget next to everything the
    server holds, and a slot is free; a request larger than the whole budget
    is rejected at submit time;
  * a solve-only request whose factorization is still in flight goes to a
    wait list and is released when that factorization completes (the
    main/wait queue pattern of the paper's Alg. 5, applied to request
    dependencies);
  * continuous batching: whenever one of the executor's streams is idle,
    admitted requests that are ready are launched on it, so requests that
    arrived while others ran join the next launch and launches on different
    streams overlap on the device.  An executor may sort requests into
    launch classes (``launch_class(r) -> (key, group limit)``): the class of
    the oldest ready request is launched next, as one group of at most its
    limit in arrival order.  The GPU executor's classes are "batched" (all
    small requests in one persistent launch) and "single" (one large request
    per launch), so a small request never waits for a large one launched
    beside it, and large ones complete one by one; without classes all
    ready requests go into one batch;
  * factor cache: completed factorizations stay on the device (LRU) for
    later solve-only requests and are evicted least-recently-used when the
    budget needs the bytes;
  * mixed precision without host waits: a mixed request whose refinement
    does not converge comes back flagged (HQR_INFO_NOCONV) and is queued
    again as an FP64 solve of its instance (``fallback``), keeping its slot;
    the dispatcher never blocks on a convergence read;
  * latency = completion observed by the dispatcher minus arrival.

The executor is pluggable: ``GpuExecutor`` drives libhqr on torch streams;
the tests drive the same policy with a CPU executor on a scripted clock.
"""
from __future__ import annotations

import collections
import dataclasses
import heapq
import itertools
import time
from typing import Callable, Dict, List, Optional

import numpy as np

GiB = 1 << 30
MIXED_MIN_N = 513   # smallest n served by the mixed-precision path
INFO_NOCONV = 1 << 29  # HQR_INFO_NOCONV


@dataclasses.dataclass
class Request:
    rid: int
    instance: int
    kind: str                      # "factor_solve" | "solve"
    m: int
    n: int
    B: np.ndarray                  # m x nrhs host right-hand sides
    A: Optional[np.ndarray] = None # m x n host matrix (factor_solve only)
    precision: str = "fp64"
    t_arrival: float = 0.0
    # filled by the server
    t_done: float = -1.0
    x: Optional[np.ndarray] = None
    resnorm: Optional[np.ndarray] = None
    info: int = 0
    status: str = "new"            # new|waiting|pending|running|done|rejected
    fallback: bool = False         # re-run in FP64 after an unconverged refinement

    @property
    def nrhs(self) -> int:
        return self.B.shape[1]

    @property
    def mixed_path(self) -> bool:
        """Served in mixed precision (FP32 trailing updates + FP64
        refinement): mixed-flagged instances above the batched kernel's
        range.  Smaller mixed-flagged instances are solved in FP64 by the
        batched launch, which already meets the accuracy target and gains
        nothing from FP32 at those sizes."""
        return self.precision == "mixed" and self.n >= MIXED_MIN_N

    def factor_bytes(self) -> int:
        """Device bytes of the cached factorization: A's factor and up, plus
        the FP64 copy of A that mixed-precision refinement reads."""
        return 8 * (self.m * self.n + self.n) + (8 * self.m * self.n if self.mixed_path else 0)

    def bytes_needed(self, have_factor: bool) -> int:
        b = 8 * self.m * self.nrhs
        if not have_factor:
            b += self.factor_bytes()
        return b


@dataclasses.dataclass
class FactorEntry:
    instance: int
    m: int
    n: int
    bytes: int
    handle: object = None          # executor-owned device storage
    ready: bool = False
    users: int = 0                 # requests in flight that use it
    last_use: float = 0.0


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100]) of a non-empty list."""
    if not values:
        return float("nan")
    v = sorted(values)
    k = max(0, min(len(v) - 1, int(np.ceil(q / 100.0 * len(v))) - 1))
    return v[k]


class Server:
    def __init__(self, executor, budget_bytes: int = 64 * GiB, max_slots: int = 4096,
                 max_batch: int = 512, clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        self.max_batch = max_batch
        self.clock = clock
        self.cache: "collections.OrderedDict[int, FactorEntry]" = collections.OrderedDict()
        self.in_use = 0                     # bytes held (cache + request buffers)
        self.high_water = 0
        self.pending: List[Request] = []    # admitted, ready to launch
        self.queued: "collections.deque[Request]" = collections.deque()  # not yet admitted
        self.waiting: Dict[int, List[Request]] = collections.defaultdict(list)
        self.running: List[tuple] = []      # (handle, [requests])
        self.done: List[Request] = []
        self.rejected: List[Request] = []
        self.slots = 0
        self.launches = 0
        self.announced = set()              # instances with a factor_solve submitted
        self.fs_queued = collections.Counter()  # factor_solve requests not yet admitted

    # ------------------------------------------------------------ client side
    def submit(self, req: Request) -> Request:
        req.t_arrival = self.clock() if req.t_arrival <= 0 else req.t_arrival
        have = req.instance in self.cache or req.instance in self.announced
        if req.kind == "solve" and not have:
            req.status = "rejected"
            self.rejected.append(req)
            return req
        if req.bytes_needed(req.kind == "solve") > self.budget:
            req.status = "rejected"
            self.rejected.append(req)
            return req
        if req.kind == "factor_solve":
            self.announced.add(req.instance)
            self.fs_queued[req.instance] += 1
        req.status = "new"
        self.queued.append(req)
        return req

    # ------------------------------------------------------------ accounting
    def _take(self, nbytes: int) -> bool:
        if self.in_use + nbytes > self.budget:
            self._evict(self.in_use + nbytes - self.budget)
        if self.in_use + nbytes > self.budget:
            return False
        self.in_use += nbytes
        self.high_water = max(self.high_water, self.in_use)
        return True

    def _give(self, nbytes: int):
        self.in_use -= nbytes

    def _evict(self, need: int):
        freed = 0
        for inst in list(self.cache.keys()):
            if freed >= need:
                break
            e = self.cache[inst]
            if e.users or not e.ready or self.waiting.get(inst):
                continue
            self.ex.free_factor(e.handle)
            del self.cache[inst]
            self._give(e.bytes)
            freed += e.bytes

    # ------------------------------------------------------------ dispatcher
    def _admit(self):
        keep = collections.deque()
        while self.queued:
            if self.slots >= self.max_slots:
                break                      # the rest stays queued, in order
            req = self.queued.popleft()
            entry = self.cache.get(req.instance)
            if req.kind == "solve":
                if entry is None:
                    if self.fs_queued[req.instance]:
                        # its factor_solve is still queued: keep the arrival order
                        keep.append(req)
                    else:
                        # the factorization was evicted: the client must resubmit it
                        req.status = "rejected"
                        self.rejected.append(req)
                    continue
                if not self._take(req.bytes_needed(True)):
                    keep.append(req)
                    continue
                entry.users += 1
                self.slots += 1
                if entry.ready:
                    req.status = "pending"
                    self.pending.append(req)
                else:
                    req.status = "waiting"
                    self.waiting[req.instance].append(req)
            else:
                if entry is not None:
                    # a new matrix for an instance: the old factor is dropped
                    if entry.users:
                        keep.append(req)
                        continue
                    self.ex.free_factor(entry.handle)
                    self._give(entry.bytes)
                    del self.cache[req.instance]
                fbytes = req.factor_bytes()
                if not self._take(req.bytes_needed(False)):
                    keep.append(req)
                    continue
                self.cache[req.instance] = FactorEntry(req.instance, req.m, req.n, fbytes, users=1)
                self.fs_queued[req.instance] -= 1
                self.slots += 1
                req.status = "pending"
                self.pending.append(req)
        keep.extend(self.queued)
        self.queued = keep

    def _launch(self):
        klass = getattr(self.ex, "launch_class", None)
        while self.pending and self.ex.idle_stream():
            if klass is None:
                batch = self.pending[: self.max_batch]
                self.pending = self.pending[self.max_batch:]
            else:
                key, limit = klass(self.pending[0])
                limit = min(limit, self.max_batch)
                batch, rest = [], []
                for r in self.pending:
                    if len(batch) < limit and klass(r)[0] == key:
                        batch.append(r)
                    else:
                        rest.append(r)
                self.pending = rest
            entries = [self.cache[r.instance] for r in batch]
            for r in batch:
                r.status = "running"
            handle = self.ex.launch(batch, entries)
            self.running.append((handle, batch))
            self.launches += 1

    def _complete(self):
        still = []
        now = None
        for handle, batch in self.running:
            if not self.ex.poll(handle):
                still.append((handle, batch))
                continue
            now = self.clock() if now is None else now
            self.ex.collect(handle, batch)
            for r in batch:
                if r.mixed_path and (r.info & INFO_NOCONV) and not r.fallback:
                    # refinement did not converge: solve the instance again in
                    # FP64 (the request keeps its slot and bytes)
                    r.fallback = True
                    r.status = "pending"
                    self.pending.append(r)
                    continue
                r.t_done = now
                r.status = "done"
                self.done.append(r)
                e = self.cache[r.instance]
                e.users -= 1
                e.last_use = now
                self.cache.move_to_end(r.instance)
                self.slots -= 1
                # request buffers are returned; the factor stays cached
                self._give(8 * r.m * r.nrhs)
                if r.kind == "factor_solve":
                    e.ready = True
                    for w in self.waiting.pop(r.instance, []):
                        w.status = "pending"
                        self.pending.append(w)
        self.running = still

    def step(self):
        self._complete()
        self._admit()
        self._launch()

    def busy(self) -> bool:
        return bool(self.queued or self.pending or self.running or any(self.waiting.values()))

    def drain(self, timeout: float = 600.0):
        t0 = time.perf_counter()
        while self.busy():
            self.step()
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError("server did not drain")

    # ------------------------------------------------------------ statistics
    def stats(self) -> dict:
        lat = [r.t_done - r.t_arrival for r in self.done]
        span = (max(r.t_done for r in self.done) - min(r.t_arrival for r in self.done)) if self.done else 0.0
        return {"completed": len(self.done), "rejected": len(self.rejected),
                "p50_ms": percentile(lat, 50) * 1e3, "p99_ms": percentile(lat, 99) * 1e3,
                "mean_ms": float(np.mean(lat)) * 1e3 if lat else float("nan"),
                "throughput_per_s": len(self.done) / span if span > 0 else float("nan"),
                "hbm_high_water_bytes": self.high_water, "launches": self.launches}


# ------------------------------------------------------------------ executors
class GpuExecutor:
    """Runs batches through libhqr on `nstreams` torch streams.

    Instances with n <= ``batch_n_max`` go to one persistent batched launch
    per batch (FP64); larger ones are solved one by one with the whole-GPU
    path on the same stream, after the batched launch: FP64 requests by
    qr_lsq_solve (cached factors: qr_apply_qt + qr_backsolve), mixed ones by
    the mixed-precision qr_lsq_solve, keeping an FP64 copy of A beside the
    factor, and for cached factors qr_lsq_refine against that copy -- both
    with HQR_OPT_NO_FALLBACK, so no call waits on the host.  A request
    marked ``fallback`` solves its instance again in FP64 from that copy, in
    buffers of its own (the cached factor is left as it is).

    ``plain=True`` is the reference executor: one plain FP64 library call
    per request (qr_lsq_solve, or qr_apply_qt + qr_backsolve on a cached
    factor), whatever the size and precision flag, no batched launch.

    Launch classes (see Server): requests for the batched launch form one
    class, every other request is launched on its own (``single_group`` per
    launch), so it completes on its own event; the plain executor keeps one
    class."""

    def __init__(self, nstreams: int = 2, batch_n_max: int = 512, device="cuda", plain: bool = False,
                 single_group: int = 1):
        import torch
        import paper_2506_09463_amd as hqr
        self.torch = torch
        self.hqr = hqr
        hqr.load()
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(nstreams)]
        self.busy = [False] * nstreams
        self.batch_n_max = batch_n_max
        self.plain = plain
        self.single_group = single_group

    def launch_class(self, r):
        if self.plain:
            return "plain", 1 << 30
        if r.n <= self.batch_n_max and not r.fallback:
            return "batched", 1 << 30
        return "single", self.single_group

    def idle_stream(self) -> bool:
        return not all(self.busy)

    def _host(self, a):
        """Pinned host tensor for an asynchronous upload (pre-pinned tensors pass through)."""
        if isinstance(a, self.torch.Tensor):
            return a
        return self.torch.from_numpy(np.asfortranarray(a)).pin_memory()

    def free_factor(self, handle):
        pass  # tensors are released when the cache entry drops them

    def launch(self, batch, entries):
        torch, hqr = self.torch, self.hqr
        si = self.busy.index(False)
        self.busy[si] = True
        s = self.streams[si]
        with torch.cuda.stream(s):
            small_A, small_B, small_up, small_res, small_fact, small_req = [], [], [], [], [], []
            large = []
            keep = []
            for r, e in zip(batch, entries):
                mixed = r.mixed_path and r.n > self.batch_n_max and not self.plain
                if r.kind == "factor_solve" and not r.fallback:
                    A = hqr.empty_colmajor(r.m, r.n, device=self.device)
                    A.copy_(self._host(r.A), non_blocking=True)
                    up = torch.empty(max(r.n, 1), dtype=torch.float64, device=self.device)
                    A0 = A.clone() if mixed else None
                    e.handle = [A, up, A0, mixed]
                A, up, A0, mixed_factor = e.handle
                B = hqr.empty_colmajor(r.m, r.nrhs, device=self.device)
                B.copy_(self._host(r.B), non_blocking=True)
                res = torch.empty(max(r.nrhs, 1), dtype=torch.float64, device=self.device)
                if r.fallback:
                    # FP64 solve of the instance from its unmodified copy, in
                    # buffers of its own (other requests may be reading the
                    # cached factor on another stream); the cache is unchanged
                    Afb = A0.clone()
                    upfb = torch.empty_like(up)
                    keep += [Afb, upfb]
                    large.append((r, Afb, upfb, None, B, res, "fp64"))
                elif r.n <= self.batch_n_max and not self.plain:
                    small_A.append(A)
                    small_B.append(B)
                    small_up.append(up)
                    small_res.append(res)
                    small_fact.append(r.kind == "solve")
                    small_req.append(r)
                else:
                    kind = "mixed" if mixed_factor else "fp64"
                    large.append((r, A, up, A0, B, res, kind))
            info = torch.zeros(max(len(small_req), 1), dtype=torch.int32, device=self.device)
            if small_req:
                hqr.qr_lsq_solve_batched(small_A, small_B, ups=small_up, resnorms=small_res, info=info,
                                         stream=s, factored=small_fact)
            linfo = []
            for r, A, up, A0, B, res, kind in large:
                li = torch.zeros(1, dtype=torch.int32, device=self.device)
                if kind == "mixed":
                    if r.kind == "factor_solve":
                        hqr.qr_lsq_solve(A, B, up=up, resnorm=res, info=li, precision=hqr.HQR_PREC_MIXED,
                                         A_orig=A0, stream=s, no_fallback=True)
                    else:
                        hqr.qr_lsq_refine(A, up, B, A0, resnorm=res, info=li, stream=s, no_fallback=True)
                elif r.kind == "factor_solve" or r.fallback:
                    hqr.qr_lsq_solve(A, B, up=up, resnorm=res, info=li, stream=s)
                else:
                    hqr.qr_apply_qt(A, up, B, stream=s)
                    hqr.qr_backsolve(A[: r.n, : r.n], B, info=li, stream=s)
                linfo.append(li)
            ev = torch.cuda.Event()
            ev.record(s)
        outs = {id(r): (B, res) for r, B, res in zip(small_req, small_B, small_res)}
        for r, A, up, A0, B, res, kind in large:
            outs[id(r)] = (B, res)
        return {"stream": si, "event": ev, "outs": outs, "small": small_req, "info": info,
                "large": [(r, li) for (r, *_), li in zip(large, linfo)], "keep": keep}

    def poll(self, h) -> bool:
        return h["event"].query()

    def collect(self, h, batch):
        self.busy[h["stream"]] = False
        info = h["info"].cpu().numpy()
        for i, r in enumerate(h["small"]):
            r.info = int(info[i])
        for r, li in h["large"]:
            r.info = int(li.item()) | (INFO_NOCONV if r.fallback else 0)
        for r in batch:
            B, res = h["outs"][id(r)]
            r.x = B[: r.n].cpu().numpy()
            r.resnorm = res[: r.nrhs].cpu().numpy()
            # the request's right-hand sides are done with; drop host copies
            r.A = None


def poisson_arrivals(rate_per_s: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def make_stream(count_instances: int, seed: int, solves_per_instance: int = 3, nmax: int = 2048):
    """Requests for the served workload: per instance one factor_solve and
    (solves_per_instance - 1) solve-only requests, interleaved in arrival
    order; shapes and precision flags from workloads.served_shapes."""
    from paper_2506_09463_amd import workloads
    m, n, mixed, nrhs, rng = workloads.served_shapes(count_instances, seed, nmax=nmax)
    reqs = []
    rid = itertools.count()
    order = []
    for i in range(count_instances):
        for s in range(solves_per_instance):
            order.append((i, s))
    # a solve of instance i follows its factor_solve: sort by (i + jitter) keeping s order
    jitter = rng.random(len(order)) * 8.0
    keyed = sorted(range(len(order)), key=lambda t: (order[t][0] + jitter[t] + 4.0 * order[t][1], order[t][1]))
    seen = set()
    for t in keyed:
        i, s = order[t]
        mi, ni, ri = int(m[i]), int(n[i]), int(nrhs[i])
        B = np.asfortranarray(rng.standard_normal((mi, ri)))
        if i not in seen:
            A = np.asfortranarray(rng.standard_normal((mi, ni)))
            reqs.append(Request(next(rid), i, "factor_solve", mi, ni, B, A=A,
                                precision="mixed" if mixed[i] else "fp64"))
            seen.add(i)
        else:
            reqs.append(Request(next(rid), i, "solve", mi, ni, B, precision="mixed" if mixed[i] else "fp64"))
    return reqs
