"""The C ABI loads, exports every declared symbol and rejects bad arguments
without touching a GPU (argument checks run before any HIP call)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "perks.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(perks_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2204_02064_amd as pk
    return pk.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "perks_stencil_run" in names and "perks_cg_solve" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_strerror(L):
    assert L.perks_strerror(0) == b"success"
    assert L.perks_strerror(-1) == b"invalid argument"


def test_invalid_arguments_are_rejected(L):
    import paper_2204_02064_amd as pk
    w = np.zeros(9)
    wp = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    fake = ctypes.c_void_p(0x1000)
    assert L.perks_stencil_run(None, wp, pk.Shape(2, 0, 8, 8, 1), 1, 1, None, None) == -1
    assert L.perks_stencil_run(fake, wp, pk.Shape(4, 0, 8, 8, 1), 1, 1, None, None) == -1
    assert L.perks_stencil_run(fake, wp, pk.Shape(2, 0, 2, 8, 1), 1, 1, None, None) == -1
    assert L.perks_stencil_run(fake, wp, pk.Shape(2, 0, 8, 8, 1), -1, 1, None, None) == -1
    assert L.perks_stencil_run(fake, wp, pk.Shape(2, 0, 8, 8, 1), 1, 7, None, None) == -1
    w27 = np.zeros(27)
    w27[0] = 1.0          # a 3D corner weight: outside the 7-point star
    assert L.perks_stencil_run(fake, w27.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               pk.Shape(3, 0, 8, 8, 8), 1, 1, None, None) == -5
    wn = np.full(9, np.nan)
    assert L.perks_stencil_run(fake, wn.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               pk.Shape(2, 0, 8, 8, 1), 1, 1, None, None) == -1
    assert b"finite" in L.perks_last_error()
