"""The C-ABI library loads and exports every entry point include/hqr.h declares.

CPU-only: only calls that return before touching a GPU (argument validation,
workspace sizing, status strings) are made.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hqr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


@pytest.fixture(scope="module")
def lib():
    from paper_2506_09463_amd import hqr
    if not os.path.exists(hqr.LIB_PATH):
        from paper_2506_09463_amd import _build
        _build.build()
    return hqr.load()


def test_header_declares_expected():
    names = declared_functions()
    for n in ("hqr_workspace_size", "qr_factor", "qr_apply_qt", "qr_backsolve", "qr_lsq_solve",
              "hqr_status_string", "hqr_version"):
        assert n in names, n


def test_every_declared_symbol_exported(lib):
    from paper_2506_09463_amd import hqr
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(hqr.EXPORTS)


def test_argument_validation_without_gpu(lib):
    assert lib.hqr_workspace_size(-1, 0, 0, 0) == -1
    assert lib.hqr_workspace_size(3, 4, 0, 0) == -2
    assert lib.hqr_workspace_size(4, 3, -1, 0) == -3
    assert lib.hqr_workspace_size(4, 3, 1, 7) == -4
    assert lib.hqr_workspace_size(8192, 4096, 1, 0) > 0
    info = ctypes.c_int(0)
    assert lib.qr_factor(3, 4, None, 3, None, None, 0, ctypes.byref(info), None) == -2
    assert lib.qr_factor(4, 3, None, 2, None, None, 0, ctypes.byref(info), None) == -4
    assert lib.qr_apply_qt(4, 3, -1, None, 4, None, None, 4, None, 0, None) == -3
    assert lib.qr_backsolve(3, 1, None, 2, None, 3, ctypes.byref(info), None) == -4
    assert lib.hqr_status_string(-1002).decode().startswith("a HIP call")
    assert "gfx950" in lib.hqr_version().decode()
