"""CPU checks of the C ABI: the library loads, exports every function include/dmrgtst.h
declares, and rejects malformed problems before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1103_5391_amd import inputs as I
from paper_1103_5391_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "dmrgtst.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dmrg_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert _declared() == sorted(L.SYMBOLS)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libdmrgtst.so not built")
    return L.load()


def test_library_exports_every_symbol(lib):
    for s in _declared():
        assert hasattr(lib, s), s


def test_strerror(lib):
    assert lib.dmrg_strerror(0) == b"success"
    assert lib.dmrg_strerror(-1) == b"invalid argument"


def _create_status(pb, extra_terms=()):
    lib = L.load()
    cpb, keep = L.problem_to_c(pb, extra_terms)
    h = C.c_void_p()
    rc = lib.dmrg_create(C.byref(cpb), None, C.byref(h))
    return rc, lib.dmrg_last_error(None).decode(), h


def test_create_rejects_bad_problems(lib):
    pb = I.exact_problem(4, 4.0, (2, 2))
    # empty target sector
    bad = I.exact_problem(4, 4.0, (9, 9))
    rc, msg, h = _create_status(bad)
    assert rc == -1 and "empty" in msg and not h.value
    # term whose quantum-number changes do not cancel (c+ on both sides)
    rc, msg, h = _create_status(pb, extra_terms=[(1.0, 0, 0, 0, 0, 1)])
    assert rc == -1 and "cancel" in msg
    # operator index out of range
    rc, msg, h = _create_status(pb, extra_terms=[(1.0, 7, 0, 0, 1, 1)])
    assert rc == -1 and "range" in msg
    # unsorted sectors
    import copy
    pb2 = copy.deepcopy(pb)
    pb2.S.space.qn = pb2.S.space.qn[::-1].copy()
    rc, msg, h = _create_status(pb2)
    assert rc == -1 and "increasing" in msg
