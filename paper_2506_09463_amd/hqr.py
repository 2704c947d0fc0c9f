"""Thin ctypes binding of libhqr (include/hqr.h).

Argument marshalling only: every step of the factorization, Q^T B and the
back-substitution runs in libhqr's HIP kernels.  PyTorch supplies device
memory and the current stream.  Matrices are float64 CUDA tensors in
column-major layout (stride (1, ld)); ``colmajor`` and ``empty_colmajor``
build such tensors.  There is no fallback: if libhqr.so is missing or no GPU
is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhqr.so")

HQR_ENOMEM = -1001
HQR_EDEVICE = -1002
HQR_ENOTSUP = -1003
HQR_INFO_TIMEOUT = -2001
HQR_INFO_NOCONV = 1 << 29
HQR_PREC_FP64 = 0
HQR_PREC_MIXED = 1
HQR_TUNE_SINGLE = 0
HQR_TUNE_BATCHED = 1
HQR_TUNE_OCCUPANCY = 2
TUNE_DB_PATH = os.path.join(PKG, "tune_db.json")

HQR_OPT_NO_FALLBACK = 1
HQR_OPT_TSQR_PANEL = 2
EXPORTS = ("hqr_workspace_size", "hqr_workspace_size_opts", "qr_factor", "qr_apply_qt", "qr_apply_q", "qr_form_q", "qr_backsolve",
           "qr_lsq_solve", "qr_lsq_solve_static", "qr_lsq_refine", "hqr_lse_workspace_size", "qr_lse_solve",
           "hqr_cholesky", "hqr_chol_update", "hqr_batched_workspace_size",
           "qr_lsq_solve_batched",
           "qr_lsq_batched_mixed",
           "hqr_tune_set", "hqr_tune_clear", "hqr_tune_variants", "hqr_tune_variant_name",
           "hqr_profile_begin", "hqr_profile_end", "hqr_profile_class",
           "hqr_status_string", "hqr_version")


class HQRError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__("%s failed: status %d (%s)" % (fn, status, status_string(status)))


class hqr_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("flags", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libhqr.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libhqr.so not built: run __graft_entry__.build() (%s)" % path)
    lib = ctypes.CDLL(path)
    i64, vp, ip = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
    lib.hqr_workspace_size.argtypes = [i64, i64, i64, ctypes.c_int]
    lib.hqr_workspace_size.restype = i64
    lib.hqr_workspace_size_opts.argtypes = [i64, i64, i64, ctypes.c_void_p]
    lib.hqr_workspace_size_opts.restype = i64
    lib.qr_factor.argtypes = [i64, i64, vp, i64, vp, vp, i64, ip, vp]
    lib.qr_apply_qt.argtypes = [i64, i64, i64, vp, i64, vp, vp, i64, vp, i64, vp]
    lib.qr_apply_q.argtypes = [i64, i64, i64, vp, i64, vp, vp, i64, vp, i64, vp]
    lib.qr_form_q.argtypes = [i64, i64, i64, vp, i64, vp, vp, i64, vp, i64, vp]
    lib.qr_backsolve.argtypes = [i64, i64, vp, i64, vp, i64, ip, vp]
    lib.qr_lsq_solve.argtypes = [i64, i64, i64, vp, i64, vp, vp, i64, vp,
                                 ctypes.POINTER(hqr_opts), vp, i64, vp, i64, ip, ip, vp]
    lib.qr_lsq_refine.argtypes = [i64, i64, i64, vp, i64, vp, vp, i64, vp,
                                  ctypes.POINTER(hqr_opts), vp, i64, vp, i64, ip, ip, vp]
    lib.qr_lsq_solve_static.argtypes = [i64, i64, i64, vp, i64, vp, vp, i64, vp, ip, vp]
    lib.qr_lsq_solve_static.restype = ctypes.c_int
    lib.hqr_lse_workspace_size.argtypes = [i64, i64, i64]
    lib.hqr_lse_workspace_size.restype = i64
    lib.qr_lse_solve.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, vp, vp, vp, i64, ip, vp]
    lib.qr_lse_solve.restype = ctypes.c_int
    lib.hqr_cholesky.argtypes = [i64, vp, i64, vp, i64, ip, vp]
    lib.hqr_cholesky.restype = ctypes.c_int
    lib.hqr_chol_update.argtypes = [i64, vp, i64, vp, vp]
    lib.hqr_chol_update.restype = ctypes.c_int
    for fn in ("qr_factor", "qr_apply_qt", "qr_apply_q", "qr_form_q", "qr_backsolve", "qr_lsq_solve",
               "qr_lsq_refine"):
        getattr(lib, fn).restype = ctypes.c_int
    lib.hqr_status_string.argtypes = [ctypes.c_int]
    lib.hqr_status_string.restype = ctypes.c_char_p
    lib.hqr_batched_workspace_size.argtypes = [ctypes.c_int]
    lib.hqr_batched_workspace_size.restype = i64
    lib.qr_lsq_solve_batched.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp, ip, vp, i64, vp]
    lib.qr_lsq_solve_batched.restype = ctypes.c_int
    lib.qr_lsq_batched_mixed.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ip, vp, i64, vp]
    lib.qr_lsq_batched_mixed.restype = ctypes.c_int
    lib.hqr_profile_begin.argtypes = []
    lib.hqr_profile_begin.restype = ctypes.c_int
    lib.hqr_profile_end.argtypes = [ctypes.c_int, vp, vp]
    lib.hqr_profile_end.restype = ctypes.c_int
    lib.hqr_profile_class.argtypes = [ctypes.c_int]
    lib.hqr_profile_class.restype = ctypes.c_char_p
    lib.hqr_version.argtypes = []
    lib.hqr_version.restype = ctypes.c_char_p
    lib.hqr_tune_set.argtypes = [ctypes.c_int, i64, i64, i64, i64, ctypes.c_int, ctypes.c_int]
    lib.hqr_tune_set.restype = ctypes.c_int
    lib.hqr_tune_clear.argtypes = []
    lib.hqr_tune_clear.restype = ctypes.c_int
    lib.hqr_tune_variants.argtypes = []
    lib.hqr_tune_variants.restype = ctypes.c_int
    lib.hqr_tune_variant_name.argtypes = [ctypes.c_int]
    lib.hqr_tune_variant_name.restype = ctypes.c_char_p
    _lib = lib
    if os.path.exists(TUNE_DB_PATH):
        load_tune_db(TUNE_DB_PATH)
    return lib


# ------------------------------------------------------------------- tuning
def variant_shape(name):
    """(threads, rows per thread, 16-row blocks loaded together) of a
    one-workgroup variant name "wgNTxQM" or "wgNTxQMpP"."""
    nt, rest = name[2:].split("x")
    qm, _, pipe = rest.partition("p")
    return int(nt), int(qm), int(pipe) if pipe else 4


def tune_variants():
    """Names of the one-workgroup kernel variants, by index."""
    lib = load()
    return [lib.hqr_tune_variant_name(i).decode() for i in range(lib.hqr_tune_variants())]


def tune_clear():
    _check("hqr_tune_clear", load().hqr_tune_clear())


def tune_set(op, m_lo, m_hi, n_lo, n_hi, choice, precision=HQR_PREC_FP64):
    """Add one rule (see hqr.h); `choice` is a variant index, or -1 for the
    blocked path of single problems."""
    _check("hqr_tune_set", load().hqr_tune_set(int(op), int(m_lo), int(m_hi), int(n_lo), int(n_hi),
                                               int(precision), int(choice)))


def load_tune_db(path=TUNE_DB_PATH):
    """Replace the rules with those of an autotuner database (JSON written by
    paper_2506_09463_amd.autotune).  Variants are stored by name."""
    import json
    with open(path) as f:
        db = json.load(f)
    names = tune_variants()
    tune_clear()
    for r in db.get("rules", []):
        choice = r["choice"]
        idx = -1 if choice == "blocked" else (names.index(choice) if isinstance(choice, str) else int(choice))
        op = {"single": HQR_TUNE_SINGLE, "batched": HQR_TUNE_BATCHED, "occupancy": HQR_TUNE_OCCUPANCY}[r["op"]]
        if op == HQR_TUNE_OCCUPANCY:
            idx = int(choice)
        tune_set(op, r["m"][0], r["m"][1], r["n"][0], r["n"][1], idx,
                 HQR_PREC_MIXED if r.get("precision") == "mixed" else HQR_PREC_FP64)


def status_string(status: int) -> str:
    try:
        return load().hqr_status_string(int(status)).decode()
    except ImportError:
        return "libhqr not loaded"


def version() -> str:
    return load().hqr_version().decode()


# ------------------------------------------------------------ tensor helpers
def _torch():
    import torch
    return torch


def empty_colmajor(m: int, n: int, ld: Optional[int] = None, device="cuda", dtype=None):
    """Uninitialised m x n column-major tensor with leading dimension ld >= m."""
    torch = _torch()
    ld = max(1, m) if ld is None else ld
    if ld < max(1, m):
        raise ValueError("ld < m")
    dtype = torch.float64 if dtype is None else dtype
    base = torch.empty((max(n, 1), ld), device=device, dtype=dtype)
    return base.t()[:m, :n]


def colmajor(a, ld: Optional[int] = None, device="cuda"):
    """Copy a 1-D/2-D array or tensor into a column-major float64 tensor."""
    torch = _torch()
    t = torch.as_tensor(a, dtype=torch.float64)
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    m, n = t.shape
    out = empty_colmajor(m, n, ld, device=device)
    out.copy_(t.to(device))
    return out


def _ld(t, name):
    """Leading dimension of a column-major 2-D float64 device tensor."""
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if t.dtype != _torch().float64:
        raise TypeError("%s must be float64" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    m, n = t.shape
    if m > 1 and t.stride(0) != 1:
        raise ValueError("%s must be column-major (stride(0) == 1)" % name)
    ld = t.stride(1) if n > 1 else max(m, 1)
    if ld < max(m, 1):
        raise ValueError("%s: leading dimension smaller than its rows" % name)
    return ld


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _int_dev(t, device):
    torch = _torch()
    return torch.zeros(1, dtype=torch.int32, device=device) if t is None else t


def _check(fn, rc):
    if rc != 0:
        raise HQRError(fn, rc)


# ----------------------------------------------------------- the entry points
def workspace_size(m: int, n: int, nrhs: int = 0, precision: int = HQR_PREC_FP64) -> int:
    r = load().hqr_workspace_size(m, n, nrhs, precision)
    if r < 0:
        raise HQRError("hqr_workspace_size", int(r))
    return int(r)


def workspace_size_opts(m: int, n: int, nrhs: int = 0, precision: int = HQR_PREC_FP64, tsqr: bool = False) -> int:
    opts = hqr_opts(int(precision), 0.0, -1, HQR_OPT_TSQR_PANEL if tsqr else 0)
    r = load().hqr_workspace_size_opts(m, n, nrhs, ctypes.byref(opts))
    if r < 0:
        raise HQRError("hqr_workspace_size_opts", int(r))
    return int(r)


def qr_factor(A, up=None, info=None, work=None, stream=None):
    """Factor A (m x n, column-major float64 device tensor) in place.

    Returns (up, info): up holds the reflectors' leading components, info a
    device int32 tensor (0 or HQR_INFO_TIMEOUT)."""
    torch = _torch()
    lib = load()
    m, n = A.shape
    lda = _ld(A, "A")
    if up is None:
        up = torch.empty(max(n, 1), dtype=torch.float64, device=A.device)
    info = _int_dev(info, A.device)
    lw = 0 if work is None else work.numel() * work.element_size()
    _check("qr_factor", lib.qr_factor(m, n, _ptr(A), lda, _ptr(up), _ptr(work), lw, _ptr(info), _stream(stream)))
    return up, info


def qr_apply_qt(A, up, B, work=None, stream=None):
    """B <- Q^T B in place using the output of qr_factor."""
    lib = load()
    m, n = A.shape
    mb, nrhs = B.shape
    if mb != m:
        raise ValueError("B must have m rows")
    lw = 0 if work is None else work.numel() * work.element_size()
    _check("qr_apply_qt", lib.qr_apply_qt(m, n, nrhs, _ptr(A), _ld(A, "A"), _ptr(up), _ptr(B), _ld(B, "B"),
                                          _ptr(work), lw, _stream(stream)))
    return B


def qr_apply_q(A, up, B, work=None, stream=None):
    """B <- Q B in place using the output of qr_factor."""
    lib = load()
    m, n = A.shape
    mb, nrhs = B.shape
    if mb != m:
        raise ValueError("B must have m rows")
    lw = 0 if work is None else work.numel() * work.element_size()
    _check("qr_apply_q", lib.qr_apply_q(m, n, nrhs, _ptr(A), _ld(A, "A"), _ptr(up), _ptr(B), _ld(B, "B"),
                                        _ptr(work), lw, _stream(stream)))
    return B


def qr_form_q(A, up, k=None, Q=None, work=None, stream=None):
    """Leading k columns (default n) of Q from the output of qr_factor, into
    a new (or the given) m x k column-major device tensor."""
    lib = load()
    m, n = A.shape
    k = n if k is None else int(k)
    if Q is None:
        Q = empty_colmajor(m, k, device=A.device)
    if tuple(Q.shape) != (m, k):
        raise ValueError("Q must be m x k")
    lw = 0 if work is None else work.numel() * work.element_size()
    _check("qr_form_q", lib.qr_form_q(m, n, k, _ptr(A), _ld(A, "A"), _ptr(up), _ptr(Q), _ld(Q, "Q"),
                                      _ptr(work), lw, _stream(stream)))
    return Q


def qr_backsolve(R, B, info=None, stream=None):
    """B[0:n] <- R^{-1} B[0:n] with R the upper triangle of the n x n view R."""
    lib = load()
    n = R.shape[1]
    if R.shape[0] < n or B.shape[0] < n:
        raise ValueError("R must be at least n x n and B at least n rows")
    info = _int_dev(info, B.device)
    _check("qr_backsolve", lib.qr_backsolve(n, B.shape[1], _ptr(R), _ld(R, "R"), _ptr(B), _ld(B, "B"),
                                            _ptr(info), _stream(stream)))
    return B, info


def qr_lsq_solve(A, B, up=None, resnorm=None, info=None, iters=None, precision=HQR_PREC_FP64,
                 tol=0.0, max_iter=-1, A_orig=None, work=None, stream=None, no_fallback=False, tsqr=False):
    """Least squares in place: A factored, B[0:n] <- x, returns (up, resnorm, info, iters).
    tsqr: TSQR panels with Householder reconstruction (HQR_OPT_TSQR_PANEL)."""
    torch = _torch()
    lib = load()
    m, n = A.shape
    mb, nrhs = B.shape
    if mb != m:
        raise ValueError("B must have m rows")
    dev = A.device
    if up is None:
        up = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    if resnorm is None:
        resnorm = torch.empty(max(nrhs, 1), dtype=torch.float64, device=dev)
    info = _int_dev(info, dev)
    iters = _int_dev(iters, dev)
    flags = (HQR_OPT_NO_FALLBACK if no_fallback else 0) | (HQR_OPT_TSQR_PANEL if tsqr else 0)
    opts = hqr_opts(int(precision), float(tol), int(max_iter), flags)
    lda_o = _ld(A_orig, "A_orig") if A_orig is not None else max(1, m)
    lw = 0 if work is None else work.numel() * work.element_size()
    _check("qr_lsq_solve", lib.qr_lsq_solve(m, n, nrhs, _ptr(A), _ld(A, "A"), _ptr(up), _ptr(B), _ld(B, "B"),
                                            _ptr(resnorm), ctypes.byref(opts), _ptr(A_orig), lda_o,
                                            _ptr(work), lw, _ptr(info), _ptr(iters), _stream(stream)))
    return up, resnorm, info, iters


def qr_lsq_refine(A, up, B, A_orig, resnorm=None, info=None, iters=None, tol=0.0, max_iter=-1, work=None,
                  stream=None, no_fallback=False):
    """Solve again with the stored factorization in (A, up) and refine against
    A_orig (FP64 copy of the original matrix); B[0:n] <- x.  A, up are not
    modified.  Returns (resnorm, info, iters)."""
    torch = _torch()
    lib = load()
    m, n = A.shape
    mb, nrhs = B.shape
    if mb != m or tuple(A_orig.shape) != (m, n):
        raise ValueError("B and A_orig must match A's rows (and A_orig A's shape)")
    dev = A.device
    if resnorm is None:
        resnorm = torch.empty(max(nrhs, 1), dtype=torch.float64, device=dev)
    info = _int_dev(info, dev)
    iters = _int_dev(iters, dev)
    opts = hqr_opts(HQR_PREC_MIXED, float(tol), int(max_iter), HQR_OPT_NO_FALLBACK if no_fallback else 0)
    lw = 0 if work is None else work.numel() * work.element_size()
    _check("qr_lsq_refine", lib.qr_lsq_refine(m, n, nrhs, _ptr(A), _ld(A, "A"), _ptr(up), _ptr(B), _ld(B, "B"),
                                              _ptr(resnorm), ctypes.byref(opts), _ptr(A_orig), _ld(A_orig, "A_orig"),
                                              _ptr(work), lw, _ptr(info), _ptr(iters), _stream(stream)))
    return resnorm, info, iters


def qr_lse_solve(A, C, b, d, x=None, info=None, work=None, stream=None):
    """x = argmin ||A x - b|| subject to C x = d (device tensors: A m x n and
    C p x n column-major, b (m) and d (p) vectors).  A and b are overwritten.
    Returns (x, info)."""
    torch = _torch()
    lib = load()
    m, n = A.shape
    p = C.shape[0]
    if C.shape[1] != n and p > 0:
        raise ValueError("C must have n columns")
    if x is None:
        x = torch.empty(max(n, 1), dtype=torch.float64, device=A.device)
    info = _int_dev(info, A.device)
    ldc = _ld(C, "C") if p > 0 else 1
    lw = 0 if work is None else work.numel() * work.element_size()
    _check("qr_lse_solve", lib.qr_lse_solve(m, n, p, _ptr(A), _ld(A, "A"), _ptr(C) if p > 0 else None, ldc,
                                            _ptr(b), _ptr(d) if p > 0 else None, _ptr(x), _ptr(work), lw,
                                            _ptr(info), _stream(stream)))
    return x, info


def cholesky(S, info=None, work=None, stream=None):
    """S (n x n column-major device tensor, upper triangle) <- R with
    S = R^T R in place; returns (S, info)."""
    lib = load()
    n = S.shape[0]
    if S.shape[1] != n:
        raise ValueError("S must be square")
    info = _int_dev(info, S.device)
    lw = 0 if work is None else work.numel() * work.element_size()
    _check("hqr_cholesky", lib.hqr_cholesky(n, _ptr(S), _ld(S, "S"), _ptr(work), lw, _ptr(info), _stream(stream)))
    return S, info


def chol_update(R, v, stream=None):
    """R (n x n upper, column-major device tensor) <- R' with
    R'^T R' = R^T R + v v^T in place; v (device vector) is overwritten."""
    lib = load()
    n = R.shape[1]
    _check("hqr_chol_update", lib.hqr_chol_update(n, _ptr(R), _ld(R, "R"), _ptr(v), _stream(stream)))
    return R


def profile_begin():
    """Start per-kernel-class event timing inside libhqr."""
    load().hqr_profile_begin()


def profile_end(max_classes: int = 64):
    """Stop timing; return {class name: (total ms, launches)} for classes used."""
    lib = load()
    ms = (ctypes.c_double * max_classes)()
    cnt = (ctypes.c_int64 * max_classes)()
    nc = lib.hqr_profile_end(max_classes, ctypes.cast(ms, ctypes.c_void_p), ctypes.cast(cnt, ctypes.c_void_p))
    if nc < 0:
        raise HQRError("hqr_profile_end", nc)
    out = {}
    for c in range(min(nc, max_classes)):
        if cnt[c]:
            out[lib.hqr_profile_class(c).decode()] = (ms[c], int(cnt[c]))
    return out


class BatchPlan:
    """The marshalled arguments of one batched launch: shapes, leading
    dimensions and device pointers of a list of problems, kept so that a
    caller reusing the same buffers (an SLSQP loop, a benchmark) marshals them
    once and then only pays for the library call.  ``run`` enqueues
    qr_lsq_solve_batched (or qr_lsq_batched_mixed when ``factored`` is given)
    on ``stream``; the tensors must stay alive and keep their storage."""

    def __init__(self, As, Bs, ups=None, resnorms=None, info=None, work=None, factored=None):
        torch = _torch()
        self.lib = load()
        count = len(As)
        if len(Bs) != count:
            raise ValueError("As and Bs differ in length")
        self.count = count
        if count == 0:
            self.ups, self.resnorms, self.info = [], [], torch.zeros(0, dtype=torch.int32)
            return
        dev = As[0].device
        if ups is None:
            ups = [torch.empty(max(A.shape[1], 1), dtype=torch.float64, device=dev) for A in As]
        if resnorms is None:
            resnorms = [torch.empty(max(Bm.shape[1], 1), dtype=torch.float64, device=dev) for Bm in Bs]
        for i, (A, Bm) in enumerate(zip(As, Bs)):
            if Bm.shape[0] != A.shape[0]:
                raise ValueError("instance %d: B must have m rows" % i)
        i64, vp = ctypes.c_int64 * count, ctypes.c_void_p * count
        self.ms = i64(*[A.shape[0] for A in As])
        self.ns = i64(*[A.shape[1] for A in As])
        self.rs = i64(*[Bm.shape[1] for Bm in Bs])
        self.ldas = i64(*[_ld(A, "A[%d]" % i) for i, A in enumerate(As)])
        self.ldbs = i64(*[_ld(Bm, "B[%d]" % i) for i, Bm in enumerate(Bs)])
        self.pa = vp(*[A.data_ptr() for A in As])
        self.pb = vp(*[Bm.data_ptr() for Bm in Bs])
        self.pu = vp(*[u.data_ptr() for u in ups])
        self.pr = vp(*[r.data_ptr() for r in resnorms])
        self.fl = None if factored is None else (ctypes.c_int * count)(*[1 if f else 0 for f in factored])
        self.info = torch.zeros(count, dtype=torch.int32, device=dev) if info is None else info
        self.work = work
        self.lw = 0 if work is None else work.numel() * work.element_size()
        self.ups, self.resnorms = ups, resnorms
        self._keep = (As, Bs)

    def run(self, stream=None):
        if self.count == 0:
            return self.ups, self.resnorms, self.info
        cast = lambda a: ctypes.cast(a, ctypes.c_void_p)
        lib = self.lib
        if self.fl is None:
            _check("qr_lsq_solve_batched", lib.qr_lsq_solve_batched(
                self.count, cast(self.ms), cast(self.ns), cast(self.rs), cast(self.pa), cast(self.ldas),
                cast(self.pu), cast(self.pb), cast(self.ldbs), cast(self.pr), _ptr(self.info), _ptr(self.work),
                self.lw, _stream(stream)))
        else:
            _check("qr_lsq_batched_mixed", lib.qr_lsq_batched_mixed(
                self.count, cast(self.ms), cast(self.ns), cast(self.rs), cast(self.pa), cast(self.ldas),
                cast(self.pu), cast(self.pb), cast(self.ldbs), cast(self.pr), cast(self.fl), _ptr(self.info),
                _ptr(self.work), self.lw, _stream(stream)))
        return self.ups, self.resnorms, self.info


def qr_lsq_solve_batched(As, Bs, ups=None, resnorms=None, info=None, work=None, stream=None, factored=None):
    """Solve a list of least-squares problems in one persistent launch.

    As, Bs: lists of column-major float64 device tensors (A_i m_i x n_i,
    B_i m_i x nrhs_i), overwritten in place like qr_lsq_solve.  Returns
    (ups, resnorms, info) with info a device int32 tensor of len(As)."""
    return BatchPlan(As, Bs, ups, resnorms, info, work, factored).run(stream)


def batched_workspace_size(count: int) -> int:
    return int(load().hqr_batched_workspace_size(count))
