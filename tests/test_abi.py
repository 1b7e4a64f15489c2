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


# workloads of the GPU product parity tests (kept in step with tests/test_gpu_parity.py)
_FLOP_CASES = ["chain4_exact", "chain8_exact", "ladder2x4_U10", "chain12_m30", "ladder2x6_m40",
               "chain8_m17_odd", "chain14_m25_off", "chain20_m150", "chain32_m400",
               "ladder16_m800", "ladder16_m1000", "ladder32_m2000"]


@pytest.mark.parametrize("name", _FLOP_CASES)
def test_plan_flops_equal_oracle(lib, name):
    """The library's algorithmic flop count (the numerator of every throughput figure) is
    exactly the oracle's, which test_oracle_matvec pins by a brute-force tally; the executed
    count is never below it, and the host-only plan agrees with the vector length."""
    from oracle import matvec as M
    from tests.test_gpu_parity import problem
    pb = problem(name)
    st = L.plan_stats(pb)
    assert st["flops"] == float(M.flop_count(pb))
    assert st["flops_executed"] >= st["flops"]
    assert st["n"] == M.layout(pb)[1]
    assert st["create_bytes"] > 0 and st["krylov_bytes"] > 16 * st["n"] * 16


def test_plan_stats_rejects_bad_problems(lib):
    pb = I.exact_problem(4, 4.0, (9, 9))
    with pytest.raises(L.DmrgError) as e:
        L.plan_stats(pb)
    assert e.value.status == -1 and "empty" in str(e.value)
    with pytest.raises(L.DmrgError) as e:
        L.plan_stats(I.exact_problem(4, 4.0, (2, 2)), kdim=65)
    assert e.value.status == -1


def test_workspace_cap_refuses_handle_before_any_device_call(lib):
    """DMRG_MAX_WORKSPACE smaller than the handle's first buffer (one stage-1 block descriptor,
    more than 64 bytes): DMRG_ENOMEM after the plan is built and before any memory is requested
    (so this runs without a GPU); a value that is not a byte count: DMRG_EINVAL."""
    pb = I.exact_problem(6, 4.0, (3, 3))
    need = L.plan_stats(pb)["create_bytes"]
    assert need > 64
    for cap, code, text in [("1", -2, "DMRG_MAX_WORKSPACE"), ("64", -2, "DMRG_MAX_WORKSPACE"),
                            ("12kB", -1, "byte count")]:
        os.environ["DMRG_MAX_WORKSPACE"] = cap
        try:
            rc, msg, h = _create_status(pb)
        finally:
            del os.environ["DMRG_MAX_WORKSPACE"]
        assert rc == code and text in msg and not h.value, (cap, rc, msg)
