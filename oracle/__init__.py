"""Plain FP64 CPU oracle of the in-place Householder QR least-squares path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_2506_09463_amd``) never imports it and shares no code with it.

The arithmetic lives in ``hqr_oracle.c`` (sequential C, ``-ffp-contract=off``);
this module only builds it and marshals numpy arrays (column-major FP64).
See ``hqr_oracle.c`` for the paper passages each routine follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hqr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, dp, ip = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
        lib.oracle_qr_factor.argtypes = [i64, i64, dp, i64, dp]
        lib.oracle_qr_factor_barrier.argtypes = [i64, i64, dp, i64, dp, ctypes.c_int]
        lib.oracle_apply_qt.argtypes = [i64, i64, i64, dp, i64, dp, dp, i64]
        lib.oracle_apply_q.argtypes = [i64, i64, i64, dp, i64, dp, dp, i64]
        lib.oracle_backsolve.argtypes = [i64, i64, dp, i64, dp, i64, ip]
        lib.oracle_backsolve_t.argtypes = [i64, i64, dp, i64, dp, i64, ip]
        lib.oracle_norm2.argtypes = [i64, dp]
        lib.oracle_norm2.restype = ctypes.c_double
        lib.oracle_lsq_solve.argtypes = [i64, i64, i64, dp, i64, dp, dp, i64,
                                         dp, ip]
        lib.oracle_lsq_refine_ext.argtypes = [i64, i64, dp, i64, dp, i64, dp,
                                              dp, dp, dp, ctypes.c_int]
        lib.oracle_lse_solve.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, dp, dp, ip]
        lib.oracle_cholesky.argtypes = [i64, dp, i64, ip]
        lib.oracle_chol_update.argtypes = [i64, dp, i64, dp]
        for name in ("oracle_qr_factor", "oracle_qr_factor_barrier", "oracle_apply_qt", "oracle_apply_q",
                     "oracle_lse_solve", "oracle_cholesky", "oracle_chol_update",
                     "oracle_backsolve", "oracle_backsolve_t",
                     "oracle_lsq_solve", "oracle_lsq_refine_ext"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _fmat(a, rows=None):
    """Return a Fortran-ordered float64 2-D copy of ``a``."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return np.array(a, dtype=np.float64, order="F", copy=True)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, name):
    if rc < 0:
        raise ValueError("%s: argument %d invalid" % (name, -rc))
    return rc


def qr_factor(A):
    """Return (F, up): F holds R above/on the diagonal and reflector tails below."""
    F = _fmat(A)
    m, n = F.shape
    up = np.zeros(n, dtype=np.float64)
    _check(_load().oracle_qr_factor(m, n, _p(F), max(1, m), _p(up)), "qr_factor")
    return F, up


def qr_factor_barrier(A, nthreads):
    """The paper's barrier schedule on `nthreads` threads (timing only; the
    result is bitwise qr_factor's)."""
    F = _fmat(A)
    m, n = F.shape
    up = np.zeros(n, dtype=np.float64)
    _check(_load().oracle_qr_factor_barrier(m, n, _p(F), max(1, m), _p(up), int(nthreads)), "qr_factor_barrier")
    return F, up


def apply_qt(F, up, B):
    F = _fmat(F)
    Bm = _fmat(B)
    m, n = F.shape
    _check(_load().oracle_apply_qt(m, n, Bm.shape[1], _p(F), max(1, m), _p(np.ascontiguousarray(up, dtype=np.float64)),
                                   _p(Bm), max(1, m)), "apply_qt")
    return Bm


def apply_q(F, up, B):
    F = _fmat(F)
    Bm = _fmat(B)
    m, n = F.shape
    _check(_load().oracle_apply_q(m, n, Bm.shape[1], _p(F), max(1, m), _p(np.ascontiguousarray(up, dtype=np.float64)),
                                  _p(Bm), max(1, m)), "apply_q")
    return Bm


def backsolve(F, B, transpose=False):
    """Return (X, info) with X = R^{-1} B[0:n] (or R^{-T} B[0:n])."""
    F = _fmat(F)
    n = F.shape[1]
    Bm = _fmat(B)[:n].copy(order="F")
    info = ctypes.c_int(0)
    fn = _load().oracle_backsolve_t if transpose else _load().oracle_backsolve
    _check(fn(n, Bm.shape[1], _p(F), max(1, F.shape[0]), _p(Bm), max(1, n),
              ctypes.byref(info)), "backsolve")
    return Bm, info.value


def norm2(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return _load().oracle_norm2(x.size, _p(x))


def lsq_solve(A, B):
    """Return (X, F, up, resnorm, info) of min ||B - A X|| column by column."""
    F = _fmat(A)
    m, n = F.shape
    Bm = _fmat(B)
    nrhs = Bm.shape[1]
    up = np.zeros(n, dtype=np.float64)
    res = np.zeros(nrhs, dtype=np.float64)
    info = ctypes.c_int(0)
    _check(_load().oracle_lsq_solve(m, n, nrhs, _p(F), max(1, m), _p(up), _p(Bm),
                                    max(1, m), _p(res), ctypes.byref(info)),
           "lsq_solve")
    return Bm[:n].copy(), F, up, res, info.value


def lse_solve(A, C, b, d):
    """Return (x, info) of min ||A x - b|| subject to C x = d."""
    A = _fmat(A)
    m, n = A.shape
    Cm = np.array(np.asarray(C, dtype=np.float64).reshape(-1, n), order="F", copy=True)
    p = Cm.shape[0]
    bv = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
    dv = np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(-1))
    x = np.zeros(n, dtype=np.float64)
    info = ctypes.c_int(0)
    _check(_load().oracle_lse_solve(m, n, p, _p(A), max(1, m), _p(Cm), max(1, p), _p(bv), _p(dv), _p(x),
                                    ctypes.byref(info)), "lse_solve")
    return x, info.value


def cholesky(S):
    """Return (R, info): R upper with S = R^T R (strict lower part zero)."""
    F = _fmat(S)
    n = F.shape[0]
    info = ctypes.c_int(0)
    _check(_load().oracle_cholesky(n, _p(F), max(1, n), ctypes.byref(info)), "cholesky")
    return np.triu(F), info.value


def chol_update(R, v):
    """R' (upper) with R'^T R' = R^T R + v v^T."""
    F = _fmat(np.triu(R))
    n = F.shape[0]
    vv = np.array(np.asarray(v, dtype=np.float64).reshape(-1), copy=True)
    _check(_load().oracle_chol_update(n, _p(F), max(1, n), _p(vv)), "chol_update")
    return F


def lsq_reference(A, b, steps=10):
    """Extended-precision reference solution x_ref of min ||b - A x||.

    The oracle's FP64 solution refined with long-double residuals
    (augmented-system correction).  Returns (x_ref, r_ref).
    """
    A0 = _fmat(A)
    m, n = A0.shape
    bv = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
    x, F, up, _, info = lsq_solve(A0, bv)
    if info:
        raise np.linalg.LinAlgError("singular R (info=%d)" % info)
    x = np.ascontiguousarray(x[:, 0])
    r = np.zeros(m, dtype=np.float64)
    rc = _load().oracle_lsq_refine_ext(m, n, _p(A0), max(1, m), _p(F), max(1, m),
                                       _p(up), _p(bv), _p(x), _p(r), int(steps))
    _check(rc, "lsq_refine_ext")
    return x, r


def form_q(F, up, full=True):
    """Explicit Q (m x m, or m x n thin) by applying the reflectors to I."""
    m, n = np.asarray(F).shape
    I = np.eye(m, m if full else n)
    return apply_q(F, up, I)
