"""Autotuner: measures libhqr's kernel choices on the GPU and writes the rule
database that ``hqr.load()`` installs (``tune_db.json`` next to the library).

Three decisions are tuned, each per shape bucket:
  * single problems (qr_lsq_solve, qr_factor, qr_apply_qt): the blocked
    multi-kernel path or one of the one-workgroup kernel variants (threads,
    rows per thread, trailing-update load depth), bucketed by (m, n); timed
    on one seeded N(0,1) problem at the bucket's upper corner with one
    right-hand side;
  * batched launches: the one-workgroup variant (256-thread variants only:
    rows per thread and load depth) together with the workgroups per CU of
    the persistent launch, bucketed by the batch's largest m; timed on a
    seeded batch of uneven instances (n ~ U{16..min(512, m_hi/2)},
    m = n + U{0..n}, 8 RHS).
Every candidate that can hold the bucket's shape is run (exhaustive search,
as in the paper's parameter sweep of Section 4.1, here over kernel tile and
schedule parameters instead of thread counts and chunk sizes); the fastest
median wins.

    python -m paper_2506_09463_amd.autotune --out tune_db.json

The library's built-in choice (no rule) is timed beside the candidates and
recorded for reference.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

M_BUCKETS = [(1, 64), (65, 128), (129, 256), (257, 512), (513, 1024)]
N_BUCKETS = [(1, 16), (17, 32), (33, 64), (65, 128), (129, 256), (257, 512), (513, 1024)]
BATCH_M_BUCKETS = [(1, 256), (257, 512), (513, 1024)]
OCCUPANCIES = (1, 2, 3, 4)
LDS_BYTES = 160 * 1024


def _median_ms(fn, reps, stream, setup=None):
    """Median event time of fn() on `stream`; setup() (restoring the inputs)
    runs before each repetition, outside the timed region."""
    import torch
    ts = []
    for _ in range(reps):
        if setup is not None:
            setup()
            torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def _variant_rows(name):
    from paper_2506_09463_amd.hqr import variant_shape
    nt, qm, _ = variant_shape(name)
    return nt, nt * qm, nt * qm * 17


def _max_per_cu(name):
    """Workgroups per CU the variant's LDS (V area, T, reductions) allows."""
    from paper_2506_09463_amd.hqr import variant_shape
    nt, qm, _ = variant_shape(name)
    lds = 8 * (nt * qm * 17 + 16 * 17 + 2 * (nt // 64) * 17 + 32 + nt // 64) + 16
    return max(1, LDS_BYTES // lds)


def tune_single(hqr, seed=11, reps=7, log=print):
    import torch
    names = hqr.tune_variants()
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(seed)
    rules, meas = [], []
    for (mlo, mhi) in M_BUCKETS:
        for (nlo, nhi) in N_BUCKETS:
            if nlo > mhi:
                continue
            m, n = mhi, min(nhi, mhi)
            A_h = rng.standard_normal((m, n))
            b_h = rng.standard_normal((m, 1))
            A0, B0 = hqr.colmajor(A_h), hqr.colmajor(b_h)
            A, B = A0.clone(), B0.clone()
            up = torch.empty(n, dtype=torch.float64, device="cuda")
            res = torch.empty(1, dtype=torch.float64, device="cuda")
            info = torch.zeros(1, dtype=torch.int32, device="cuda")

            def restore():
                A.copy_(A0)
                B.copy_(B0)

            def run():
                hqr.qr_lsq_solve(A, B, up=up, resnorm=res, info=info, stream=stream)

            cands = ["blocked"] + [nm for nm in names if _variant_rows(nm)[1] >= m and _variant_rows(nm)[2] >= n]
            times = {}
            for c in cands:
                hqr.tune_clear()
                hqr.tune_set(hqr.HQR_TUNE_SINGLE, 0, 1 << 40, 0, 1 << 40, -1 if c == "blocked" else names.index(c))
                restore()
                run()
                torch.cuda.synchronize()
                times[c] = _median_ms(run, reps, stream, restore)
            hqr.tune_clear()
            base = _median_ms(run, reps, stream, restore)  # built-in default
            best = min(times, key=times.get)
            meas.append({"op": "single", "m": [mlo, mhi], "n": [nlo, nhi], "shape": [m, n], "ms": times,
                         "default_ms": base})
            rules.append({"op": "single", "m": [mlo, mhi], "n": [nlo, nhi], "choice": best})
            log("[tune] single m<=%d n<=%d: %s -> %s" % (mhi, nhi, {k: round(v, 4) for k, v in times.items()}, best))
    return rules, meas


def tune_batched(hqr, seed=12, count=512, reps=5, log=print):
    import torch
    names = hqr.tune_variants()
    stream = torch.cuda.current_stream()
    rules, meas = [], []
    for (mlo, mhi) in BATCH_M_BUCKETS:
        rng = np.random.default_rng(seed)
        probs = []
        nmax = max(16, min(512, mhi // 2))
        for _ in range(count):
            n = int(rng.integers(16, nmax + 1))
            m = min(mhi, n + int(rng.integers(0, n + 1)))
            probs.append((rng.standard_normal((m, n)), rng.standard_normal((m, 8))))
        A0 = [hqr.colmajor(A) for A, _ in probs]
        B0 = [hqr.colmajor(B) for _, B in probs]
        As = [a.clone() for a in A0]
        Bs = [b.clone() for b in B0]
        ups = [torch.empty(A.shape[1], dtype=torch.float64, device="cuda") for A, _ in probs]
        res = [torch.empty(8, dtype=torch.float64, device="cuda") for _ in probs]
        info = torch.zeros(len(probs), dtype=torch.int32, device="cuda")
        work = torch.empty(hqr.batched_workspace_size(len(probs)), dtype=torch.uint8, device="cuda")

        def restore():
            for a, a0 in zip(As, A0):
                a.copy_(a0)
            for b, b0 in zip(Bs, B0):
                b.copy_(b0)

        plan = hqr.BatchPlan(As, Bs, ups=ups, resnorms=res, info=info, work=work)

        def run():
            plan.run(stream)

        mmax = max(A.shape[0] for A, _ in probs)
        cands = [(nm, occ) for nm in names if nm.startswith("wg256x") and _variant_rows(nm)[1] >= mmax
                 for occ in OCCUPANCIES if occ <= _max_per_cu(nm)]
        times = {}
        for nm, occ in cands:
            hqr.tune_clear()
            hqr.tune_set(hqr.HQR_TUNE_BATCHED, 0, 1 << 40, 0, 1 << 40, names.index(nm))
            hqr.tune_set(hqr.HQR_TUNE_OCCUPANCY, 0, 1 << 40, 0, 1 << 40, occ)
            restore()
            run()
            torch.cuda.synchronize()
            times["%s/%d" % (nm, occ)] = _median_ms(run, reps, stream, restore)
        hqr.tune_clear()
        best = min(times, key=times.get)
        bname, bocc = best.split("/")
        meas.append({"op": "batched", "m": [mlo, mhi], "count": count, "ms": times})
        rules.append({"op": "batched", "m": [mlo, mhi], "n": [0, 1 << 40], "choice": bname})
        rules.append({"op": "occupancy", "m": [mlo, mhi], "n": [0, 1 << 40], "choice": int(bocc)})
        log("[tune] batched m<=%d: %s -> %s" % (mhi, {k: round(v, 3) for k, v in times.items()}, best))
    return rules, meas


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="database path (default: next to libhqr.so)")
    args = ap.parse_args(argv)
    import torch
    import paper_2506_09463_amd as hqr
    if not torch.cuda.is_available():
        print("autotune: no GPU", file=sys.stderr)
        return 1
    hqr.load()
    t0 = time.time()
    r1, m1 = tune_single(hqr, log=lambda s: print(s, flush=True))
    r2, m2 = tune_batched(hqr, log=lambda s: print(s, flush=True))
    db = {"device": torch.cuda.get_device_name(0), "library": hqr.version(), "variants": hqr.tune_variants(),
          "rules": r1 + r2, "measurements": m1 + m2, "seconds": time.time() - t0}
    out = args.out or hqr.hqr.TUNE_DB_PATH
    with open(out, "w") as f:
        json.dump(db, f, indent=1)
    print("[tune] wrote %s (%d rules, %.1f s)" % (out, len(db["rules"]), db["seconds"]), flush=True)
    hqr.load_tune_db(out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
