"""Host-side checks of the back-substitution's published-value pattern.

The multi-workgroup back-substitution marks its published-value slots with
one 64-bit pattern until a block stores its solved values there, and the
successors wait while a slot still holds it.  That is sound only if the
pattern is what the integer fill writes (the same 32-bit word twice) and if
no solved value can carry it: the pattern must be a signalling NaN, which
IEEE-754 arithmetic never returns (operations on a signalling NaN deliver a
quiet NaN).  These tests read the constants from the kernel header.
"""
import os
import re

import numpy as np

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2506_09463_amd", "csrc", "hqr_args.hpp")


def _constants():
    text = open(HDR).read()
    full = int(re.search(r"TRSV_EMPTY\s*=\s*(0x[0-9A-Fa-f]+)ull", text).group(1), 16)
    word = int(re.search(r"TRSV_EMPTY_WORD\s*=\s*(0x[0-9A-Fa-f]+)", text).group(1), 16)
    return full, word


def test_pattern_is_the_fill_word_twice():
    full, word = _constants()
    assert full == (word << 32) | word


def test_pattern_is_a_signalling_nan():
    full, _ = _constants()
    exponent = (full >> 52) & 0x7FF
    mantissa = full & ((1 << 52) - 1)
    assert exponent == 0x7FF and mantissa != 0       # a NaN
    assert not (mantissa >> 51) & 1                  # quiet bit clear: signalling


def test_arithmetic_never_returns_the_pattern():
    """Multiplying or fusing the pattern itself (as the solve's multiply by
    1/R_ll and its FMAs would) returns a quiet NaN with other bits."""
    full, _ = _constants()
    v = np.array([full], dtype=np.uint64).view(np.float64)
    with np.errstate(invalid="ignore"):
        outs = [v * 1.0, v * 0.5, v - 0.0, 2.0 * v + 1.0, -v]
    for o in outs[:-1]:
        bits = int(o.view(np.uint64)[0])
        assert np.isnan(o[0]) and bits != full and (bits >> 51) & 1
    # negation only flips the sign bit: still not the pattern
    assert int(outs[-1].view(np.uint64)[0]) != full
