"""The stopping rule of the mixed-precision refinement (host build of the
same header the refinement kernel includes).

The rule must never accept a run whose corrections stall above the level
that guarantees the 1e-10 relative solution error: a correction that stops
halving is accepted only at or below 3e-11 ||x||; above it, two such steps in
a row end the run as failed (HQR_INFO_NOCONV and the FP64 fallback).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_09463_amd", "csrc")
FLOOR = 3e-11   # REFINE_STALL_FLOOR in hqr_args.hpp

DRIVER = r'''
#include "hqr_refine_rule.hpp"
extern "C" void rule_run(int nsteps, const double *ndx, const double *nx, double tol, double floor, int *out)
{
    hqr::RefineState st{0, 0, 0, 0, 0.0};
    for (int s = 0; s < nsteps; ++s) hqr::refine_rule_step(st, s, ndx[s], nx[s], tol, floor);
    out[0] = st.first;
    out[1] = st.failed;
    out[2] = st.stalls;
    out[3] = st.frozen;
}
'''


@pytest.fixture(scope="module")
def rule(tmp_path_factory):
    d = tmp_path_factory.mktemp("rule")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    lib = d / "librule.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-DHQR_HD=", "-I", CSRC,
                           str(src), "-o", str(lib)])
    L = ctypes.CDLL(str(lib))
    L.rule_run.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                           ctypes.c_void_p]

    def run(ndx, nx=None, tol=1e-13, floor=FLOOR):
        ndx = np.ascontiguousarray(ndx, dtype=np.float64)
        nx = np.ones_like(ndx) if nx is None else np.ascontiguousarray(nx, dtype=np.float64)
        out = np.zeros(4, dtype=np.int32)
        L.rule_run(len(ndx), ndx.ctypes.data, nx.ctypes.data, tol, floor, out.ctypes.data)
        return dict(first=int(out[0]), failed=int(out[1]), stalls=int(out[2]), frozen=int(out[3]))

    return run


def test_floor_matches_library_constant():
    text = open(os.path.join(CSRC, "hqr_args.hpp")).read()
    assert "constexpr double REFINE_STALL_FLOOR = 3e-11;" in text


def test_geometric_convergence(rule):
    # ||dx|| = 1e-3, 1e-6, ..., reaching <= 1e-13 ||x|| at the 5th step
    r = rule([10.0 ** (-3 * (k + 1)) for k in range(8)])
    assert r == dict(first=5, failed=0, stalls=0, frozen=1)


def test_stall_below_floor_is_converged(rule):
    r = rule([1e-4, 1e-8, 5e-12, 4e-12, 4e-12])
    assert r["first"] == 4 and r["failed"] == 0 and r["frozen"] == 1
    # the measured kappa = 1e6 sequence of a 1000 x 400 problem
    r = rule([7.2e-3, 7.7e-4, 8.9e-6, 1.3e-6, 2.0e-8, 3.1e-9, 5.8e-11, 2.5e-11, 2.0e-11, 2.1e-11])
    assert r["first"] == 9 and r["failed"] == 0


@pytest.mark.parametrize("level", [5e-9, 2e-10, 5e-11])
def test_stall_above_floor_fails(rule, level):
    """Corrections that stop shrinking anywhere above 3e-11 ||x|| -- the band
    between 1e-10 and 1e-8 included, which a 1e-8 floor used to accept --
    end the run as failed, never as converged."""
    r = rule([1e-4, level, 0.9 * level, 0.9 * level, 0.9 * level, 0.9 * level])
    assert r["first"] == 0 and r["failed"] == 1 and r["frozen"] == 1


def test_one_stall_then_progress_keeps_going(rule):
    r = rule([1e-4, 8e-5, 1e-8, 1e-12, 1e-14])
    assert r["first"] == 5 and r["failed"] == 0


def test_nan_never_converges(rule):
    r = rule([1e-4, np.nan, np.nan, np.nan])
    assert r["first"] == 0 and r["frozen"] == 0


def test_frozen_state_does_not_change(rule):
    r = rule([1e-14, 1.0, 1.0, 1.0])
    assert r == dict(first=1, failed=0, stalls=0, frozen=1)


def test_relative_to_x(rule):
    # the same corrections against ||x|| = 1e6: converged once ||dx|| <= 1e-7
    r = rule([1e-3, 1e-5, 1e-7, 1e-9], nx=[1e6] * 4)
    assert r["first"] == 3
