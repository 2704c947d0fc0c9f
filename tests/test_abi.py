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
    from paper_2506_09463_amd import hqr
    assert hqr.workspace_size_opts(8192, 4096, 1) == lib.hqr_workspace_size(8192, 4096, 1, 0)
    # the TSQR tree's buffers: level 0's Q (m x 64) at least
    assert hqr.workspace_size_opts(8192, 4096, 1, tsqr=True) >= lib.hqr_workspace_size(8192, 4096, 1, 0) + 8192 * 64 * 8
    assert lib.hqr_workspace_size_opts(-1, 0, 0, None) == -1
    info = ctypes.c_int(0)
    assert lib.qr_factor(3, 4, None, 3, None, None, 0, ctypes.byref(info), None) == -2
    assert lib.qr_factor(4, 3, None, 2, None, None, 0, ctypes.byref(info), None) == -4
    assert lib.qr_apply_qt(4, 3, -1, None, 4, None, None, 4, None, 0, None) == -3
    assert lib.qr_backsolve(3, 1, None, 2, None, 3, ctypes.byref(info), None) == -4
    assert lib.qr_lsq_refine(3, 4, 1, None, 3, None, None, 3, None, None, None, 3, None, 0,
                             ctypes.byref(info), None, None) == -2
    assert lib.qr_lsq_refine(4, 3, 1, None, 2, None, None, 4, None, None, None, 4, None, 0,
                             ctypes.byref(info), None, None) == -5
    assert lib.qr_lsq_refine(4, 3, 1, None, 4, None, None, 4, None, None, None, 4, None, 0,
                             None, None, None) == -15
    assert lib.hqr_status_string(-1002).decode().startswith("a HIP call")
    assert "gfx950" in lib.hqr_version().decode()


def test_tuning_rules_without_gpu(lib):
    """Tuning rules are host state: variant names, argument checks, clearing."""
    from paper_2506_09463_amd import hqr
    names = hqr.tune_variants()
    assert len(names) >= 2 and all(n.startswith("wg") for n in names)
    for nm in names:
        nt, qm, pipe = hqr.variant_shape(nm)
        assert nt % 64 == 0 and (nt * qm) % 16 == 0 and pipe in (2, 4, 8)
    assert lib.hqr_tune_variant_name(len(names)) is None
    assert lib.hqr_tune_set(7, 0, 1, 0, 1, 0, 0) == -1          # op
    assert lib.hqr_tune_set(0, 5, 4, 0, 1, 0, 0) == -3          # m range
    assert lib.hqr_tune_set(0, 0, 1, 0, 1, 9, 0) == -6          # precision
    assert lib.hqr_tune_set(0, 0, 1, 0, 1, 0, len(names)) == -7  # choice
    assert lib.hqr_tune_set(1, 0, 1, 0, 1, 0, -1) == -7          # batched has no blocked choice
    for i, nm in enumerate(names):                              # batched: 256-thread variants only
        assert (lib.hqr_tune_set(1, 0, 1, 0, 1, 0, i) == 0) == nm.startswith("wg256x")
    assert lib.hqr_tune_set(0, 0, 1, 0, 1, 0, -1) == 0
    assert lib.hqr_tune_set(2, 0, 1, 0, 1, 0, 0) == -7          # occupancy 1..8
    assert lib.hqr_tune_set(2, 0, 1, 0, 1, 0, 9) == -7
    assert lib.hqr_tune_set(2, 0, 1, 0, 1, 0, 3) == 0
    assert lib.hqr_tune_clear() == 0


def test_tune_db_roundtrip(lib, tmp_path):
    import json
    from paper_2506_09463_amd import hqr
    names = hqr.tune_variants()
    db = {"rules": [{"op": "single", "m": [0, 100], "n": [0, 50], "choice": names[0]},
                    {"op": "single", "m": [0, 100], "n": [51, 100], "choice": "blocked"},
                    {"op": "batched", "m": [0, 1024], "n": [0, 1024], "choice": names[-1]}]}
    p = tmp_path / "db.json"
    p.write_text(json.dumps(db))
    hqr.load_tune_db(str(p))
    hqr.tune_clear()
