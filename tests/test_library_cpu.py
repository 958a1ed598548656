"""CPU-side checks of the C-ABI library: it loads and exports every entry point
that include/r1.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2211_14318_amd", "libr1.so")
HDR = os.path.join(ROOT, "include", "r1.h")


def declared():
    src = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:r1_status|const char\*)\s+(r1_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("r1_create", "r1_destroy", "r1_envelope", "r1_envelope_stress",
                 "r1_envelope_batched"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libr1.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libr1.so not built")
def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.r1_status_string.restype = ctypes.c_char_p
    assert lib.r1_status_string(0) == b"ok"
    assert lib.r1_status_string(-1) == b"invalid argument"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libr1.so not built")
def test_argument_checks_need_no_gpu():
    """Null handle / null outputs are rejected before any device call."""
    from paper_2211_14318_amd import r1
    L = r1.lib()
    assert L.r1_envelope(None, None, None, 1, 0, None, None, None, None, None) == -1
    assert L.r1_create(None, 0) == -1


def test_grid_reduced_directions_match_oracle():
    """r1_grid_r11 is host code: the library's reduced direction set (eq. 5.1) equals the
    oracle's, in the same order (16 steps in 2D, 169 in 3D)."""
    from oracle import oracle as O
    from paper_2211_14318_amd import r1
    for dim in (2, 3):
        assert np.array_equal(r1.grid_r11(dim), O.grid_r11(dim))
