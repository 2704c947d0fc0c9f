#!/usr/bin/env python3
"""Benchmark: FP64 in-place Householder QR + least-squares solve on one MI355X.

Workload (the large single-GPU configuration): A = U diag(sigma) V^T,
8192 x 4096, sigma geometric from 1 to 1e-6, one right-hand side
b = A x_true + 1e-8 N(0,1); inputs from paper_2506_09463_amd.workloads.

A step is one qr_lsq_solve: factor A in place (R + reflectors), apply Q^T
to b (fused into the trailing updates), residual norm, back-substitution.
Inputs are resident in HBM; before every step A and b are restored from
device copies outside the timed region, and each step is bracketed by a
device synchronization with HIP events recorded around the call on the
stream it runs on.  value = (2 m n^2 - 2/3 n^3) / (time per step).

Prints ONE JSON line.  Extra fields: `roofline` for the kernel class that
takes the most time (timed live with libhqr's event profiler), and
`cpu_baseline` (the FP64 CPU oracle on a bounded sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QR GFLOP/s (2mn²−⅔n³) vs plain FP64; batched LSQ solves/s; p99 latency"
PEAK_F64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch (read, write) of each kernel class on the default
# workload, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs scaled by the
# same counters on a 1 GiB device copy (x2.0 and x1.0).  Valid only for the
# kernel sources they were taken on (SHA-256 over the files that define the
# blocked path's kernels and their arguments, C2_KERNEL_SOURCES); otherwise
# the roofline's traffic is null.  A class's figure averages over all its
# launches (update: the 64-column launch for panel p+2 and the bulk launch;
# gram_reduce: the two Gram reductions and the X/W reduction).
HBM_TRAFFIC = {
    "csrc_sha256": "f54c4f5036ab3d3bfd8fc23efb83dd58192a88f2b74df80f766175199e9fccc4",
    "per_launch_bytes": {"update": [73637700, 55161771], "vtx": [130921559, 15503360],
                         "wsolve": [15226391, 1001984], "trsv": [68917337, 65536],
                         "cqr_gram1": [6731192, 6294032], "cqr_gram2": [3524511, 3194880],
                         "cqr_chol": [198140, 82176], "cqr_finish": [2447281, 2097152],
                         "narrow_vtx": [6770741, 6324224], "gram_reduce": [3307072, 32779]},
}


C2_KERNEL_SOURCES = ("hqr_args.hpp", "hqr_device.hpp", "hqr_blocked.hpp", "hqr_cqr.hpp", "k_blocked.hip",
                     "k_cqr.hip")

# HBM bytes of the batched workload's one launch (read, write), from the same
# two counters and scaling; valid for the one-workgroup kernel's sources, the
# tuning database (which picks the variant) and the batch recipe hashed here.
BATCHED_TRAFFIC = {
    "sha256": "28e71dc2dff17136784fa7f16f4cd614d23f174b3782add429ad80007ba199ad",
    "bytes": [41010364032, 22412739968],
}
BATCHED_SOURCES = ("csrc/hqr_args.hpp", "csrc/hqr_device.hpp", "csrc/hqr_wg.hpp", "csrc/k_wg.hip", "tune_db.json",
                   "workloads.py")


def csrc_sha256(names=None, prefix="csrc"):
    import hashlib
    h = hashlib.sha256()
    for nm in (names if names is not None else C2_KERNEL_SOURCES):
        h.update(nm.encode())
        path = os.path.join(ROOT, "paper_2506_09463_amd", prefix, nm) if prefix else \
            os.path.join(ROOT, "paper_2506_09463_amd", nm)
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def wg_design_bytes(shapes, nrhs):
    """HBM bytes the one-workgroup kernel moves by design for instances of
    the given (m, n): per 16-column panel at c0 (m_p = m - c0 rows) the panel
    is read and written once and the later columns and the right-hand sides
    are read twice and written once (W = V^T C, then C - V W'); then the
    triangle of R and B are read for the back-substitution."""
    tot = 0.0
    for m, n in shapes:
        m, n = int(m), int(n)
        for c0 in range(0, n, 16):
            pw = min(16, n - c0)
            mp = m - c0
            tot += 16.0 * mp * pw + 24.0 * mp * ((n - c0 - pw) + nrhs)
        tot += 4.0 * n * n + 16.0 * m * nrhs
    return tot


def qr_flops(m, n):
    return 2.0 * m * n * n - 2.0 / 3.0 * n ** 3


def class_work(m, n, nrhs, nb=64):
    """Algorithmic work of each kernel class over one solve with look-ahead,
    per panel of width bw at row offset c0 (m_p = m - c0 rows; the next
    panel has bw1 columns; ncR = later columns plus right-hand sides, the
    side stream's share).  Returns {class: (bound, amount, peak, unit)}:

      vtx         X = V^T [C | B] over the ncR columns:
                  2 m_p bw ncR flops                                   (FP64 MFMA)
      update      C <- C - V W' over the ncR columns: reads and writes C,
                  reads V and W': 16 m_p ncR + 8 m_p bw + 8 bw ncR bytes (HBM)
      wsolve      sum of the split-K partials of X and W' = T^T X: reads
                  nsplit bw ncR doubles, writes bw ncR                 (HBM)
      narrow_vtx  V_bot = A_bot W^-1 and X = V^T C for the next panel:
                  2 (m_p - bw) bw^2 + 2 m_p bw bw1 flops               (FP64 MFMA)
      cqr_gram1   next panel: C -= V W and the pass-1 Gram partials:
                  2 m_p bw bw1 + 2 (m_p - bw) bw1^2 flops              (FP64 MFMA)
      cqr_gram2   Q1 = A_p R1^-1 and its Gram: 4 m_p bw^2 flops        (FP64 MFMA)
      gram_reduce sums of the per-tile 64 x 64 partials (X, followed by
                  W = T^T X in the same kernel; G1; G2): reads ceil(m_p/64)
                  bw^2 doubles, writes bw^2, three per panel            (HBM)
      cqr_chol    64 x 64 Cholesky/inverse/LU work of one workgroup:
                  2/3 bw^3 flops (pass 1) + 14/3 bw^3 (pass 2)          (one CU)
      trsv        reads the n x n triangle once: 4 n^2 bytes            (HBM)
    """
    out = {}

    def add(k, bound, amount):
        b, a = out.get(k, (bound, 0.0))
        out[k] = (bound, a + amount)

    for c0 in range(0, n, nb):
        bw = min(nb, n - c0)
        bw1 = min(nb, max(0, n - c0 - bw))
        mp = m - c0
        ncR = max(0, n - c0 - bw - bw1) + nrhs
        tiles = -(-mp // 64)
        ntiles = -(-ncR // 128)
        nsplit = max(1, min(-(-512 // max(ntiles, 1)), max(1, mp // 256), 16))
        add("vtx", "mfma", 2.0 * mp * bw * ncR)
        add("update", "hbm", 16.0 * mp * ncR + 8.0 * mp * bw + 8.0 * bw * ncR)
        add("wsolve", "hbm", 8.0 * (nsplit + 1) * bw * ncR)
        if bw1 > 0:
            add("narrow_vtx", "mfma", 2.0 * max(mp - bw, 0) * bw * bw + 2.0 * mp * bw * bw1)
            add("cqr_gram1", "mfma", 2.0 * mp * bw * bw1 + 2.0 * max(mp - bw, 0) * bw1 * bw1)
        else:
            add("cqr_finish", "mfma", 2.0 * max(mp - bw, 0) * bw * bw)
        if c0 == 0:
            add("cqr_gram1", "mfma", 2.0 * mp * bw * bw)
        add("cqr_gram2", "mfma", 4.0 * mp * bw * bw)
        add("gram_reduce", "hbm", 3 * 8.0 * (tiles + 1) * bw * bw)
        add("cqr_chol", "cu", (2.0 / 3.0 + 14.0 / 3.0) * bw ** 3)
    add("trsv", "hbm", 4.0 * n * n)
    peaks = {"mfma": (PEAK_F64_TFLOPS, "TFLOP/s", 1e12), "hbm": (PEAK_HBM_GBS, "GB/s", 1e9),
             "cu": (PEAK_F64_TFLOPS / 256.0, "TFLOP/s", 1e12)}
    return {k: (b, a) + peaks[b] for k, (b, a) in out.items()}


def roofline_entry(name, work, prof):
    """Roofline of one kernel class from its summed event time and launch count."""
    bound, amount, peak, unit, scale = work
    t_ms, cnt = prof[name]
    avg_ms = t_ms / cnt
    achieved = amount / cnt / (avg_ms * 1e-3) / scale
    return {"kernel": name, "bound": "alu" if bound == "cu" else bound, "achieved": achieved, "peak": peak,
            "unit": unit, "frac": achieved / peak, "traffic": None, "launches_per_step": None,
            "avg_launch_ms": avg_ms, "algorithmic_per_launch": amount / cnt}


def host_cpu():
    """(usable cores, CPU model name) of this host."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def cpu_baseline_full_start(A_host, b_host):
    """Start the oracle's whole least-squares solve of the workload in a
    thread (single-threaded C); returns the handle for the join."""
    import threading
    import oracle
    oracle.build(force=False)
    out = {}

    def run():
        t = time.perf_counter()
        xo, _, _, reso, infoo = oracle.lsq_solve(A_host, b_host)
        out.update(x=xo[:, 0], res=float(reso[0]), info=int(infoo), seconds=time.perf_counter() - t)

    th = threading.Thread(target=run, daemon=True)
    th.start()
    return th, out


def cpu_baseline_full_join(handle):
    th, out = handle
    th.join()
    return out


def cpu_baseline(A_host, ncols):
    """The oracle's QR on the leading ncols columns of the workload matrix:
    single-threaded, and under the paper's barrier schedule on every usable
    host core (bitwise the same factorization)."""
    import oracle
    oracle.build(force=False)
    sample = np.asfortranarray(A_host[:, :ncols])
    m, n = sample.shape
    t0 = time.perf_counter()
    oracle.qr_factor(sample)
    dt = time.perf_counter() - t0
    cores, model = host_cpu()
    threads = max(1, min(cores, 64))
    t0 = time.perf_counter()
    oracle.qr_factor_barrier(sample, threads)
    dtb = time.perf_counter() - t0
    return {"value": qr_flops(m, n) / dt / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": "oracle qr_factor of the leading %dx%d block of the workload matrix "
                      "(single thread, %.1f s)" % (m, n, dt),
            "barrier": {"value": qr_flops(m, n) / dtb / 1e9, "unit": "GFLOP/s", "cores": threads,
                        "seconds": dtb,
                        "sample": "the same block under the paper's barrier schedule (one barrier after each "
                                  "reflector's generation and application), %d threads" % threads},
            "host_nproc": cores, "host_cpu_model": model}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=8192)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--kappa", type=float, default=1e6)
    ap.add_argument("--ld-pad", type=int, default=0)
    ap.add_argument("--cpu-cols", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--workload", default="large", choices=["large", "small", "batched", "mixed", "served", "slsqp"],
                    help="large (default, the headline line), or one of the other configurations")
    ap.add_argument("--count", type=int, default=2000, help="batched: number of instances")
    ap.add_argument("--streams", type=int, default=2, help="served, slsqp: the executor's streams")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 3 device-to-device copies of MIB MiB (scale for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the path has no multi-GPU "
              "form); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2506_09463_amd as hqr
    from paper_2506_09463_amd import workloads

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        nel = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": nel * 8, "copies": 3}), flush=True)
        return
    hqr.load()
    if args.workload != "large":
        return OTHER[args.workload](args)
    dev = torch.device("cuda:0")
    m, n = args.m, args.n
    t0 = time.time()
    A_h, b_h, x_true = workloads.conditioned(m, n, args.kappa, seed=workloads.SEED_LARGE)
    print("[bench] inputs generated in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)

    # CPU baseline leg, part 1: the FP64 oracle's whole solve of the same
    # input, in a thread of its own while the GPU is timed (the C call
    # releases the interpreter lock); its x also gives the GPU result's error
    # against the oracle
    full_oracle = None if args.no_cpu_baseline else cpu_baseline_full_start(A_h, b_h)

    lda = m + args.ld_pad
    A0 = hqr.colmajor(A_h, ld=lda)
    B0 = hqr.colmajor(b_h.reshape(-1, 1), ld=lda)
    A = hqr.empty_colmajor(m, n, ld=lda)
    B = hqr.empty_colmajor(m, 1, ld=lda)
    up = torch.empty(n, dtype=torch.float64, device=dev)
    res = torch.empty(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    iters = torch.zeros(1, dtype=torch.int32, device=dev)
    work = torch.empty(hqr.workspace_size(m, n, 1), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def restore():
        A.copy_(A0)
        B.copy_(B0)

    def solve():
        hqr.qr_lsq_solve(A, B, up=up, resnorm=res, info=info, iters=iters, work=work, stream=stream)

    for _ in range(args.warmup):
        restore()
        solve()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    # The timed region: K steps.  Then K more steps of the same workload with
    # every library launch bracketed by HIP events on its own stream (the
    # per-kernel durations of the roofline; the events slow a step down, so
    # these steps are not the ones `value` comes from).
    def run_steps(k):
        ts = []
        for _ in range(k):
            restore()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            solve()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return ts

    wall0 = time.perf_counter()
    times = run_steps(args.steps)
    wall = time.perf_counter() - wall0
    prof = {}
    prof_ms = None
    if not args.no_profile:
        hqr.profile_begin()
        prof_ms = float(np.mean(run_steps(args.steps)))
        prof = hqr.profile_end()
    ms = float(np.mean(times))
    if int(info.item()) != 0:
        print("bench.py: solve reported info=%d" % int(info.item()), file=sys.stderr)
        sys.exit(1)
    print("[bench] timed %d steps: %.3f ms/step (min %.3f); with kernel events %s ms/step"
          % (args.steps, ms, min(times), prof_ms), file=sys.stderr, flush=True)

    # accuracy of the last step: LSQ orthogonality and distance to x_true
    x = B[:n, 0].double().cpu().numpy()
    r = b_h - A_h @ x
    nA = 1.0  # sigma_max = 1 by construction
    ortho = float(np.linalg.norm(A_h.T @ r) / (nA * (nA * np.linalg.norm(x) + np.linalg.norm(b_h))))

    roof = None
    classes = {}
    if prof:
        work_by = class_work(m, n, 1)
        # per step: divide the summed time and launches by the step count
        prof1 = {k: (v[0] / args.steps, v[1] / args.steps) for k, v in prof.items()}
        for k in prof1:
            if k in work_by:
                classes[k] = roofline_entry(k, work_by[k], prof1)
        dom = max(classes, key=lambda k: prof1[k][0])
        roof = dict(classes[dom])
        roof["launches_per_step"] = prof1[dom][1]
        if csrc_sha256() == HBM_TRAFFIC["csrc_sha256"] and dom in HBM_TRAFFIC["per_launch_bytes"]:
            rd, wr = HBM_TRAFFIC["per_launch_bytes"][dom]
            roof["traffic"] = rd + wr
            roof["traffic_read_write"] = [rd, wr]
        print("[bench] profile per step: " + ", ".join("%s %.3f ms/%d" % (k, v[0], v[1]) for k, v in
                                                     sorted(prof1.items(), key=lambda kv: -kv[1][0])),
              file=sys.stderr, flush=True)

    cpu = None
    oracle_err = None
    if full_oracle is not None:
        # CPU baseline leg, part 2: join the whole solve, then the bounded samples
        fo = cpu_baseline_full_join(full_oracle)
        xo = fo["x"]
        oracle_err = {"x_rel_err_vs_oracle": float(np.linalg.norm(x - xo) / np.linalg.norm(xo)),
                      "resnorm_rel_diff_vs_oracle": abs(float(res.item()) - fo["res"]) / fo["res"],
                      "oracle_info": fo["info"]}
        print("[bench] vs oracle: %s (oracle solve %.1f s)" % (oracle_err, fo["seconds"]), file=sys.stderr,
              flush=True)
        cpu = cpu_baseline(A_h, min(args.cpu_cols, n))
        cpu["full_solve_seconds_single_thread"] = fo["seconds"]

    gflops = qr_flops(m, n) / (ms * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": gflops,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 QR + LSQ solve, 8192x4096, kappa 1e6, 1 RHS (seeded synthetic)",
                   "m": m, "n": n, "nrhs": 1, "lda": lda, "kappa": args.kappa,
                   "frac_of_fp64_peak": gflops / 1e3 / PEAK_F64_TFLOPS,
                   "lsq_orthogonality": ortho,
                   "error_vs_oracle": oracle_err,
                   "x_true_rel_err": float(np.linalg.norm(x - x_true) / np.linalg.norm(x_true)),
                   "wall_s_timed_loop": wall,
                   "ms_per_step_with_kernel_events": prof_ms,
                   "profile_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in prof.items()},
                   "kernel_rooflines": {k: {"bound": v["bound"], "frac": round(v["frac"], 4),
                                            "avg_launch_ms": round(v["avg_launch_ms"], 5)}
                                        for k, v in classes.items()}},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def _line(metric_unit, value, ms, args, config, roofline=None, cpu=None, hib=True, dtype="f64"):
    metric, unit = metric_unit
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": hib, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config,
            "roofline": roofline, "cpu_baseline": cpu}


def run_batched(args):
    """2000 uneven instances (n ~ U{16..512}, m = n + U{0..n}, 8 RHS) in one launch."""
    import torch
    import paper_2506_09463_amd as hqr
    from paper_2506_09463_amd import workloads
    t0 = time.time()
    probs = workloads.batch_problem(count=args.count, seed=workloads.SEED_BATCH)
    print("[bench] %d instances generated in %.1f s" % (len(probs), time.time() - t0), file=sys.stderr, flush=True)
    A0 = [hqr.colmajor(A) for A, _ in probs]
    B0 = [hqr.colmajor(B) for _, B in probs]
    As = [a.clone() for a in A0]
    Bs = [b.clone() for b in B0]
    # clone() keeps strides, so the copies stay column-major
    ups = [torch.empty(A.shape[1], dtype=torch.float64, device="cuda") for A, _ in probs]
    res = [torch.empty(B.shape[1], dtype=torch.float64, device="cuda") for _, B in probs]
    info = torch.zeros(len(probs), dtype=torch.int32, device="cuda")
    work = torch.empty(hqr.batched_workspace_size(len(probs)), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    fl = sum(qr_flops(A.shape[0], A.shape[1]) for A, _ in probs)
    fl_all = fl + sum(4.0 * A.shape[0] * A.shape[1] * B.shape[1] + A.shape[1] ** 2 * B.shape[1] for A, B in probs)

    def restore():
        for a, a0 in zip(As, A0):
            a.copy_(a0)
        for b, b0 in zip(Bs, B0):
            b.copy_(b0)

    # the pointer arrays are marshalled once (the buffers are reused); a step
    # is the library call: LPT order, descriptors, upload, persistent launch
    plan = hqr.BatchPlan(As, Bs, ups=ups, resnorms=res, info=info, work=work)
    for _ in range(args.warmup):
        restore()
        plan.run(stream)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        restore()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.run(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    assert int(info.abs().sum().item()) == 0
    # same GPU, same instances, one plain qr_lsq_solve call each
    restore()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(len(probs)):
        hqr.qr_lsq_solve(As[i], Bs[i], up=ups[i], resnorm=res[i], info=info[i:i + 1], stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1)
    print("[bench] batched %.3f ms, loop of single solves %.3f ms" % (ms, loop_ms), file=sys.stderr, flush=True)
    # the kernel moves about 2.5 flops per HBM byte, below the FP64 ridge
    # (78.6 TFLOP/s / 8 TB/s = 9.8): its roofline is HBM
    tflops = fl_all / (ms * 1e-3) / 1e12
    dbytes = wg_design_bytes([A.shape for A, _ in probs], probs[0][1].shape[1])
    achieved = dbytes / (ms * 1e-3) / 1e9
    valid = csrc_sha256(BATCHED_SOURCES, prefix="") == BATCHED_TRAFFIC["sha256"] and len(probs) == 2000
    roof = {"kernel": "batched_lsq", "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": sum(BATCHED_TRAFFIC["bytes"]) if valid else None,
            "launches": 1, "avg_launch_ms": ms, "algorithmic_per_launch": dbytes,
            "fp64_tflops": tflops, "fp64_frac": tflops / PEAK_F64_TFLOPS}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        t0 = time.perf_counter()
        k = 0
        while k < len(probs) and time.perf_counter() - t0 < 10.0:
            A, B = probs[k]
            oracle.lsq_solve(A, B)
            k += 1
        dt = time.perf_counter() - t0
        cpu = {"value": k / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": "oracle lsq_solve of the first %d instances of the batch (caller order), %.1f s" % (k, dt)}
    cfg = {"workload": "batched FP64 LSQ: %d instances, n ~ U{16..512}, m = n + U{0..n}, 8 RHS, one persistent launch"
           % len(probs), "count": len(probs), "factor_gflop": fl / 1e9, "total_gflop": fl_all / 1e9,
           "loop_of_single_solves_ms": loop_ms, "speedup_vs_loop": loop_ms / ms}
    print(json.dumps(_line(("batched LSQ solves/s", "solves/s"), len(probs) / (ms * 1e-3), ms, args, cfg, roof, cpu)),
          flush=True)


def run_small(args):
    """One 128 x 64 FP64 least-squares solve: median of back-to-back calls and single-call latency."""
    import torch
    import paper_2506_09463_amd as hqr
    from paper_2506_09463_amd import workloads
    A_h, b_h = workloads.small_problem(seed=workloads.SEED_SMALL)
    m, n = A_h.shape
    A0 = hqr.colmajor(A_h)
    B0 = hqr.colmajor(b_h.reshape(-1, 1))
    A, B = A0.clone(), B0.clone()
    up = torch.empty(n, dtype=torch.float64, device="cuda")
    res = torch.empty(1, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    reps = 1000
    for _ in range(20):
        hqr.qr_lsq_solve(A, B, up=up, resnorm=res, info=info, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        hqr.qr_lsq_solve(A, B, up=up, resnorm=res, info=info, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    per_call = e0.elapsed_time(e1) / reps
    lat = []
    for _ in range(50):
        A.copy_(A0)
        B.copy_(B0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hqr.qr_lsq_solve(A, B, up=up, resnorm=res, info=info, stream=stream)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    hqr.profile_begin()
    hqr.qr_lsq_solve(A, B, up=up, resnorm=res, info=info, stream=stream)
    prof = hqr.profile_end()
    kms = prof.get("small_lsq", (float("nan"), 1))[0]
    fl = qr_flops(m, n)
    one_cu_peak = PEAK_F64_TFLOPS / 256.0
    achieved = fl / (kms * 1e-3) / 1e12
    roof = {"kernel": "small_lsq", "bound": "alu", "achieved": achieved, "peak": one_cu_peak, "unit": "TFLOP/s",
            "frac": achieved / one_cu_peak, "traffic": None, "launches": 1, "avg_launch_ms": kms,
            "note": "one workgroup: peak is one CU's FP64 rate (78.6/256 TFLOP/s)"}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        ts = []
        for _ in range(100):
            t0 = time.perf_counter()
            oracle.lsq_solve(A_h, b_h)
            ts.append(time.perf_counter() - t0)
        cpu = {"value": fl / np.median(ts) / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
               "sample": "oracle lsq_solve of the same 128x64 problem, median of 100 (%.1f us)" % (np.median(ts) * 1e6)}
    cfg = {"workload": "FP64 QR + LSQ solve, 128x64, 1 RHS", "m": m, "n": n, "us_per_call_back_to_back": per_call * 1e3,
           "single_call_latency_us_median": float(np.median(lat)) * 1e3, "kernel_us": kms * 1e3}
    print(json.dumps(_line((METRIC, "GFLOP/s"), fl / (per_call * 1e-3) / 1e9, per_call, args, cfg, roof, cpu)),
          flush=True)


def run_served(args):
    """Poisson stream of LSQ requests: n log-uniform in [16, 2048], m = n + U{0..n/2},
    1-4 RHS, FP64 or mixed precision per request (p = 1/2), 3 successive solves
    per instance on its cached factor, 64 GB admission budget, 2 streams.
    Saturation throughput first (everything submitted at t = 0), then Poisson
    arrivals at 0.5/0.8/0.95 x saturation: p50/p99 latency and throughput.
    The same stream is then served with one plain FP64 library call per
    request on one stream (no batched launch, no mixed precision): the
    speedup is the ratio of the two saturation throughputs."""
    import copy
    import torch
    from paper_2506_09463_amd.server import GpuExecutor, Server, make_stream, poisson_arrivals, GiB

    ninst = args.count if args.count != 2000 else 5000
    t0 = time.time()
    base = make_stream(ninst, seed=6, solves_per_instance=3)
    host_bytes = 0
    # pre-pin host data so uploads are asynchronous
    for r in base:
        r.B = torch.from_numpy(np.asfortranarray(r.B)).pin_memory()
        host_bytes += r.B.numel() * 8
        if r.A is not None:
            r.A = torch.from_numpy(np.asfortranarray(r.A)).pin_memory()
            host_bytes += r.A.numel() * 8
    print("[bench] %d requests (%d instances, %.1f GB pinned) in %.1f s"
          % (len(base), ninst, host_bytes / 1e9, time.time() - t0), file=sys.stderr, flush=True)

    def fresh(reqs):
        out = []
        for r in reqs:
            c = copy.copy(r)
            c.t_arrival, c.t_done, c.x, c.status, c.fallback, c.info = 0.0, -1.0, None, "new", False, 0
            out.append(c)
        return out

    def run(rate, plain=False, reqs_in=None, keep=False):
        reqs = fresh(base if reqs_in is None else reqs_in)
        ex = GpuExecutor(nstreams=1 if plain else args.streams, plain=plain)
        srv = Server(ex, budget_bytes=64 * GiB)
        start = time.perf_counter()
        if rate is None:
            for r in reqs:
                r.t_arrival = start
                srv.submit(r)
            srv.drain(timeout=900)
        else:
            arr = poisson_arrivals(rate, len(reqs), seed=7)
            i = 0
            while i < len(reqs) or srv.busy():
                now = time.perf_counter() - start
                while i < len(reqs) and arr[i] <= now:
                    reqs[i].t_arrival = start + arr[i]
                    srv.submit(reqs[i])
                    i += 1
                srv.step()
                if time.perf_counter() - start > 900:
                    raise TimeoutError("served run did not finish")
        torch.cuda.synchronize()
        st = srv.stats()
        st["fallbacks"] = sum(1 for r in srv.done if r.fallback)
        st["nonzero_info"] = sum(1 for r in srv.done if r.info & ~(1 << 29))
        return (st, reqs) if keep else st

    run(None, reqs_in=base[:600])                 # warm-up (kernels, allocator)
    run(None, plain=True, reqs_in=base[:600])
    sat, done = run(None, keep=True)
    print("[bench] saturation: %s" % sat, file=sys.stderr, flush=True)
    plain = run(None, plain=True)
    print("[bench] plain FP64, one call per request: %s" % plain, file=sys.stderr, flush=True)
    rate_sat = sat["throughput_per_s"]
    loads = {}
    for f in (0.5, 0.8, 0.95):
        st = run(f * rate_sat)
        loads["%.2f" % f] = st
        print("[bench] load %.2f: %s" % (f, st), file=sys.stderr, flush=True)
    cpu = None
    err = None
    if not args.no_cpu_baseline:
        cpu, err = served_cpu_baseline(done, base)
    cfg = {"workload": "served LSQ stream: %d instances x 3 solves, n log-uniform [16,2048], m = n + U{0..n/2}, "
                       "1-4 RHS, FP64 or mixed per request, factor reuse, 64 GB budget, %d streams" % (ninst, args.streams),
           "requests": len(base), "saturation": sat, "poisson_loads": loads,
           "plain_fp64_one_call_per_request": plain,
           "speedup_vs_plain_fp64": sat["throughput_per_s"] / plain["throughput_per_s"],
           "error_vs_oracle_sample": err}
    p99 = loads["0.80"]["p99_ms"]
    print(json.dumps(_line(("p99 latency at 0.8 x saturation", "ms"), p99, sat["mean_ms"], args, cfg,
                           None, cpu, hib=False)), flush=True)


def served_cpu_baseline(done, base, nsample=40):
    """CPU baseline leg of the served workload: the oracle's solves of a
    seeded sample of the stream's requests, timed (solves/s on one core), and
    the served results' relative errors against them."""
    import oracle
    oracle.build(force=False)
    mats = {}
    for r in base:
        if r.kind == "factor_solve":
            mats[r.instance] = r.A
    rng = np.random.default_rng(17)
    pick = rng.choice(len(done), size=min(nsample, len(done)), replace=False)
    worst, t_total, nmixed = 0.0, 0.0, 0
    for i in pick:
        r = done[i]
        A = mats[r.instance].numpy()
        B = r.B.numpy()
        t = time.perf_counter()
        xo, *_ = oracle.lsq_solve(A, B)
        t_total += time.perf_counter() - t
        e = float(np.linalg.norm(r.x - xo) / np.linalg.norm(xo))
        worst = max(worst, e)
        nmixed += int(r.mixed_path)
    cpu = {"value": len(pick) / t_total, "unit": "solves/s", "cores": 1, "kind": "oracle",
           "sample": "oracle lsq_solve of %d requests drawn from the stream (seed 17), %.1f s" % (len(pick), t_total)}
    return cpu, {"requests": int(len(pick)), "mixed_path_requests": nmixed, "max_x_rel_err_vs_oracle": worst}


def run_mixed(args):
    """Mixed precision (FP32-MFMA trailing updates, FP64 refinement) against
    plain FP64 on the same GPU: 128x64 at kappa 1e2 and 1e6 (seeds 3, 4), and
    the 8192x4096 kappa-1e6 matrix where the FP32 contraction can pay off.
    Each step restores A and b (untimed) and times one call, which includes
    the refinement and its convergence read-back."""
    import torch
    import paper_2506_09463_amd as hqr
    from paper_2506_09463_amd import workloads
    import oracle
    oracle.build(force=False)
    stream = torch.cuda.current_stream()

    def timed(A0, B0, prec, steps):
        m, n = A0.shape
        A, B = A0.clone(), B0.clone()
        up = torch.empty(n, dtype=torch.float64, device="cuda")
        res = torch.empty(B0.shape[1], dtype=torch.float64, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        iters = torch.zeros(1, dtype=torch.int32, device="cuda")
        kw = dict(precision=prec, A_orig=A0) if prec == hqr.HQR_PREC_MIXED else {}
        ts = []
        for i in range(args.warmup + steps):
            A.copy_(A0)
            B.copy_(B0)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            hqr.qr_lsq_solve(A, B, up=up, resnorm=res, info=info, iters=iters, stream=stream, **kw)
            e1.record(stream)
            torch.cuda.synchronize()
            if i >= args.warmup:
                ts.append(e0.elapsed_time(e1))
        return float(np.median(ts)), B[:n, 0].double().cpu().numpy(), int(info.item()), int(iters.item())

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    cases = []
    for kappa, seed in ((1e2, workloads.SEED_MIXED[0]), (1e6, workloads.SEED_MIXED[1])):
        A_h, b_h, _ = workloads.conditioned(128, 64, kappa, seed=seed)
        A0, B0 = hqr.colmajor(A_h), hqr.colmajor(b_h.reshape(-1, 1))
        ms64, x64, _, _ = timed(A0, B0, hqr.HQR_PREC_FP64, max(args.steps, 20))
        msmx, xmx, info, it = timed(A0, B0, hqr.HQR_PREC_MIXED, max(args.steps, 20))
        xref, _ = oracle.lsq_reference(A_h, b_h)
        xo = oracle.lsq_solve(A_h, b_h)[0][:, 0]
        cases.append({"shape": "128x64", "kappa": kappa, "ms_fp64": ms64, "ms_mixed": msmx,
                      "speedup_vs_fp64": ms64 / msmx, "refine_steps": it, "info": info,
                      "err_vs_xref": rel(xmx, xref), "err_vs_oracle": rel(xmx, xo),
                      "fp64_err_vs_xref": rel(x64, xref)})
        print("[bench] mixed %s" % cases[-1], file=sys.stderr, flush=True)
    m, n = 8192, 4096
    A_h, b_h, _ = workloads.conditioned(m, n, 1e6, seed=workloads.SEED_LARGE)
    A0, B0 = hqr.colmajor(A_h), hqr.colmajor(b_h.reshape(-1, 1))
    ms64, x64, _, _ = timed(A0, B0, hqr.HQR_PREC_FP64, args.steps)
    msmx, xmx, info, it = timed(A0, B0, hqr.HQR_PREC_MIXED, args.steps)
    big = {"shape": "8192x4096", "kappa": 1e6, "ms_fp64": ms64, "ms_mixed": msmx, "speedup_vs_fp64": ms64 / msmx,
           "refine_steps": it, "info": info, "err_vs_fp64_gpu": rel(xmx, x64),
           "gflops_mixed": qr_flops(m, n) / (msmx * 1e-3) / 1e9}
    print("[bench] mixed %s" % big, file=sys.stderr, flush=True)
    cfg = {"workload": "mixed-precision QR + LSQ with refinement: 128x64 at kappa 1e2/1e6 and 8192x4096 at kappa 1e6",
           "cases": cases + [big],
           "note": "value = 8192x4096 rate in (2mn^2-2/3n^3)/s; errors are relative 2-norm errors of x; x_ref = "
                   "oracle solution refined with 80-bit residuals"}
    print(json.dumps(_line((METRIC, "GFLOP/s"), big["gflops_mixed"], msmx, args, cfg, None, None, dtype="f32+f64")),
          flush=True)


def run_slsqp(args):
    """The synthetic SLSQP-style driver (Gauss-Newton with two chord
    corrections per factorization on a discretized nonlinear boundary-value
    fit, n log-uniform in [32, 1024]): every subproblem is a request to the
    continuous-batching server; reports the request rate, latency and the
    outer iterations to convergence."""
    from paper_2506_09463_amd import slsqp_driver
    from paper_2506_09463_amd.server import GpuExecutor, Server, percentile, GiB
    count = args.count if args.count != 2000 else 200
    probs = slsqp_driver.make_problems(count, seed=11, nmin=32, nmax=1024)
    warm = slsqp_driver.make_problems(8, seed=12, nmin=32, nmax=1024)
    slsqp_driver.run_served(warm, Server(GpuExecutor(nstreams=args.streams), budget_bytes=64 * GiB), max_outer=3)
    srv = Server(GpuExecutor(nstreams=args.streams), budget_bytes=64 * GiB)
    stats, us = slsqp_driver.run_served(probs, srv, max_outer=15, tol=1e-11)
    lat = stats.latencies_ms
    print("[bench] slsqp driver: %d instances, %d outer iterations, %d requests in %.2f s, %d converged"
          % (count, stats.outer_iterations, stats.requests, stats.wall_s, stats.converged), file=sys.stderr,
          flush=True)
    cfg = {"workload": "synthetic SLSQP-style driver: %d nonlinear BVP fits, n log-uniform [32, 1024], "
                       "Gauss-Newton step + 2 chord solves per factor, served" % count,
           "instances": count, "outer_iterations": stats.outer_iterations, "requests": stats.requests,
           "converged": stats.converged, "wall_s": stats.wall_s,
           "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99)}
    print(json.dumps(_line(("LSQ requests/s (synthetic SLSQP driver)", "requests/s"), stats.requests / stats.wall_s,
                           stats.wall_s * 1e3, args, cfg)), flush=True)


OTHER = {"batched": run_batched, "small": run_small, "mixed": run_mixed, "served": run_served, "slsqp": run_slsqp}


if __name__ == "__main__":
    main()
