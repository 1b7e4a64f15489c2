"""GPU checks of the C ABI's accounting and failure paths, and parity at the two largest
configurations (needs an MI355X):

  * the algorithmic flop count of the library equals the oracle's on every product workload;
  * the ladder 2 x 32 at m = 2000 (kdim 20, tau 0.05) from the holon-doublon-like state
    (c+_{s1,up} P_S) (x) c_{s2,dn} psi0 in the sector (33, 31): Krylov steps and
    time-step-targeting vectors against the oracle (1e-10), with the Lanczos vectors of every
    step recorded;
  * the ladder 2 x 16 at m = 800 with BF16x3 block products against the FP64 oracle;
  * non-finite inputs, a device-memory cap, and a ground state that runs out of restarts are
    reported by status codes, and leave the handle usable.
"""
import os
import sys

import numpy as np
import pytest

from oracle import krylov as K
from oracle import matvec as M
from oracle import observables as O
from paper_1103_5391_amd import inputs as I

pytestmark = pytest.mark.gpu

KR_TOL = 1e-10
BF3_TOL = 3e-5      # the BF16x3 error model of the mixed-precision tests


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1103_5391_amd import lib as L
    L.load()
    return torch, L


def _dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _problem(name):
    from tests.test_gpu_parity import problem
    return problem(name)


FLOP_CASES = ["chain4_exact", "chain8_exact", "ladder2x4_U10", "chain12_m30", "ladder2x6_m40",
              "chain8_m17_odd", "chain14_m25_off", "chain20_m150", "chain32_m400",
              "ladder16_m800", "ladder16_m1000", "ladder32_m2000"]


@pytest.mark.parametrize("name", FLOP_CASES)
def test_flops_match_oracle(env, name):
    """dmrg_flops (the numerator of every throughput figure) equals oracle.flop_count, which the
    CPU tests pin by a brute-force tally; the executed count is never below it."""
    torch, L = env
    say("flops", name)
    pb = _problem(name)
    h = L.dmrg_create(pb)
    f, fx = h.flops(), h.flops_executed()
    ref = M.flop_count(pb)
    say("  algorithmic", f, "oracle", ref, "executed", fx)
    assert f == float(ref)
    assert fx >= f
    h.destroy()


# ---------------------------------------------------------------------------------------------
# config 5: ladder 2 x 32, U = 8, m = 2000, kdim 20, tau 0.05, holon-doublon-like start
# ---------------------------------------------------------------------------------------------
def _config5(env):
    """(problem of the (33, 31) sector, the normalised start vector prepared by the oracle,
    the GPU's unnormalised preparation, its oracle counterpart)."""
    torch, L = env
    pb = _problem("ladder32_m2000")
    s1, s2 = pb.Sblk.sites[-1], pb.Eblk.sites[0]
    ops_s, ops_e = I.site_ops(pb.Sblk, s1), I.site_ops(pb.Eblk, s2)
    extra_S, extra_E = [ops_s["cdag_0"]], [ops_e["c_1"]]
    psrc, iS, iE = I.with_ops(pb, extra_S, extra_E)
    tgt = (pb.target[0] + 1, pb.target[1] - 1)
    pdst = I.with_ops(pb, extra_S, extra_E, target=tgt)[0]
    psi0 = I.random_psi(M.layout(psrc)[1], np.random.default_rng(I.SEED_BASE + 5 + 1000))
    # (c+_{s1 up} P_S) (x) c_{s2 dn}: the environment factor is odd, so the term is fermionic
    ref = O.apply_terms(psrc, pdst, [(1.0, extra_S[0], extra_E[0], True)], psi0)
    hs, hd = L.dmrg_create(psrc), L.dmrg_create(pdst)
    yd = torch.empty(2 * hd.n, dtype=torch.float64, device="cuda")
    hs.apply_local(hd, [(1.0, iS[0], 0, iE[0], 0, 1)], _dev(torch, psi0), yd)
    torch.cuda.synchronize()
    gpu_prep = _host(yd)
    hs.destroy()
    return pdst, hd, ref / np.linalg.norm(ref), gpu_prep, ref


def test_config5_holon_doublon_krylov_and_tst(env):
    torch, L = env
    say("config 5: holon-doublon-like start in (33, 31), ladder 2x32, m = 2000")
    pb, h, psi, prep, prep_ref = _config5(env)
    assert tuple(pb.target) == (33, 31)
    err = rel(prep, prep_ref)
    say("  preparation rel err", err)
    assert err <= 1e-13
    n = h.n
    assert n > 524288          # above the vector passes' 1024-block cap: grid-stride loops
    xd = _dev(torch, psi)
    # two steps: the chained start of the second step runs at this size too
    yd = torch.empty_like(xd)
    info = h.krylov_expm(xd, yd, 0.05, 20, 2)
    yref, oinfo = K.krylov_expm(lambda v: M.matvec_sector(pb, v), psi, 0.05, 20, 2)
    err = rel(_host(yd), yref)
    say("  krylov 2 steps rel err", err, info)
    assert err <= KR_TOL
    assert info["k_eff_steps"] == list(oinfo.k_eff) == [20, 20]
    assert abs(np.linalg.norm(_host(yd)) - 1.0) < 1e-12
    # time-step targeting from the same start: one basis at 0, tau/3, 2 tau/3, tau
    td = torch.empty(8 * n, dtype=torch.float64, device="cuda")
    w, tinfo = h.tst_targets(xd, 0.05, 20, td)
    ys, wref, _ = K.tst_targets(lambda v: M.matvec_sector(pb, v), psi, 0.05, 20)
    t = _host(td)
    assert np.array_equal(w, wref)
    for i in range(4):
        e = rel(t[2 * n * i:2 * n * (i + 1)], ys[i])
        say("  target", i, e)
        assert e <= KR_TOL
    h.destroy()


# ---------------------------------------------------------------------------------------------
# config 3: ladder 2 x 16, U = 8, m = 800, BF16x3 block products, FP64 Lanczos
# ---------------------------------------------------------------------------------------------
def test_config3_bf16x3_matvec_krylov_tst(env):
    torch, L = env
    say("config 3: ladder 2x16, m = 800, bf16x3")
    pb = _problem("ladder16_m800")
    h = L.dmrg_create(pb)
    h.set_precision(L.DMRG_BF16X3)
    n = h.n
    x = I.random_psi(n, np.random.default_rng(I.SEED_BASE + 3))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    h.matvec(xd, yd)
    torch.cuda.synchronize()
    err = rel(_host(yd), M.matvec_sector(pb, x))
    say("  matvec rel err", err)
    assert err <= BF3_TOL
    f = lambda v: M.matvec_sector(pb, v)
    h.krylov_expm(xd, yd, 0.05, 15, 1)
    y = _host(yd)
    yref, _ = K.krylov_expm(f, x, 0.05, 15, 1)
    err = rel(y, yref)
    say("  krylov rel err", err, "norm drift", abs(np.linalg.norm(y) - 1.0))
    assert err <= BF3_TOL
    assert abs(np.linalg.norm(y) - 1.0) <= 1e-8
    td = torch.empty(8 * n, dtype=torch.float64, device="cuda")
    h.tst_targets(xd, 0.05, 15, td)
    ys, _, _ = K.tst_targets(f, x, 0.05, 15)
    t = _host(td)
    for i in range(4):
        e = rel(t[2 * n * i:2 * n * (i + 1)], ys[i])
        say("  target", i, e)
        assert e <= BF3_TOL
        assert abs(np.linalg.norm(t[2 * n * i:2 * n * (i + 1)]) - 1.0) <= 1e-8
    h.destroy()


# ---------------------------------------------------------------------------------------------
# per-step Lanczos vectors, non-finite inputs, memory cap, ground-state status
# ---------------------------------------------------------------------------------------------
def test_keff_per_step_with_breakdown(env):
    """An eigenvector stays an eigenvector: every step breaks down after one vector; a random
    vector of a 36-state sector exhausts the space within kdim 40 in every step."""
    torch, L = env
    say("k_eff per step")
    pb = _problem("chain6_exact")
    h = L.dmrg_create(pb)
    n = h.n
    Hd = M.superblock_matrix(pb)
    wv, vv = np.linalg.eigh(Hd)
    ed = _dev(torch, np.concatenate([vv[:, 5], np.zeros(n)]))
    yd = torch.empty_like(ed)
    info = h.krylov_expm(ed, yd, 0.3, 12, 3)
    assert info["k_eff_steps"] == [1, 1, 1] and info["breakdown"] == 1
    pb4 = _problem("chain4_exact")
    h4 = L.dmrg_create(pb4)
    x = I.random_psi(h4.n, np.random.default_rng(11))
    xd = _dev(torch, x)
    yd4 = torch.empty_like(xd)
    info = h4.krylov_expm(xd, yd4, 0.5, 40, 2)
    _, oinfo = K.krylov_expm(lambda v: M.matvec_sector(pb4, v), x, 0.5, 40, 2)
    assert info["k_eff_steps"] == list(oinfo.k_eff)
    assert all(k <= h4.n for k in info["k_eff_steps"])
    h.destroy()
    h4.destroy()


def test_nonfinite_inputs(env):
    """A NaN or an infinity in the input: with checking on, every Krylov call and the product
    return DMRG_ENONFINITE before computing; with checking off, a Krylov call with info
    returns DMRG_ENONFINITE from the non-finite starting norm; finite inputs are unaffected."""
    torch, L = env
    say("non-finite inputs")
    pb = _problem("chain12_m30")
    h = L.dmrg_create(pb)
    n = h.n
    x = I.random_psi(n, np.random.default_rng(21))
    bad = x.copy()
    bad[n + 17] = np.nan
    inf = x.copy()
    inf[3] = np.inf
    yd = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    td = torch.empty(8 * n, dtype=torch.float64, device="cuda")
    for v in (bad, inf):
        vd = _dev(torch, v)
        with pytest.raises(L.DmrgError) as e:
            h.krylov_expm(vd, yd, 0.1, 10, 1)
        assert e.value.status == -4
    h.set_check_finite(True)
    for v in (bad, inf):
        vd = _dev(torch, v)
        for call in (lambda: h.matvec(vd, yd), lambda: h.krylov_expm(vd, yd, 0.1, 10, 2),
                     lambda: h.tst_targets(vd, 0.1, 10, td),
                     lambda: h.ground_state(vd, yd, 10, 2, 0.0)):
            with pytest.raises(L.DmrgError) as e:
                call()
            assert e.value.status == -4 and "non-finite" in str(e.value)
    # finite input with checking on: the same result as without
    xd = _dev(torch, x)
    h.krylov_expm(xd, yd, 0.1, 10, 2)
    y1 = _host(yd).copy()
    h.set_check_finite(False)
    h.krylov_expm(xd, yd, 0.1, 10, 2)
    assert np.array_equal(y1, _host(yd))
    yref, _ = K.krylov_expm(lambda v: M.matvec_sector(pb, v), x, 0.1, 10, 2)
    assert rel(y1, yref) <= KR_TOL
    h.destroy()


def test_workspace_cap(env):
    """DMRG_MAX_WORKSPACE against the byte counts of dmrg_plan_stats: a cap of exactly the
    handle's creation bytes plus a kdim-8 Krylov workspace admits both; a 64-vector basis is
    then refused with DMRG_ENOMEM and the handle stays usable at kdim 8; one byte less than the
    creation bytes refuses the handle."""
    torch, L = env
    say("workspace cap")
    pb = _problem("chain32_m400")
    st8 = L.plan_stats(pb, kdim=8)
    cap = st8["create_bytes"] + st8["krylov_bytes"]
    os.environ["DMRG_MAX_WORKSPACE"] = str(cap)
    try:
        h = L.dmrg_create(pb)
    finally:
        del os.environ["DMRG_MAX_WORKSPACE"]
    n = h.n
    x = I.random_psi(n, np.random.default_rng(31))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    h.krylov_expm(xd, yd, 0.1, 8, 2, info=False)
    torch.cuda.synchronize()
    with pytest.raises(L.DmrgError) as e:
        h.krylov_expm(xd, yd, 0.1, 64, 1, info=False)
    assert e.value.status == -2 and "DMRG_MAX_WORKSPACE" in str(e.value)
    h.krylov_expm(xd, yd, 0.1, 8, 2, info=False)
    torch.cuda.synchronize()
    yref, _ = K.krylov_expm(lambda v: M.matvec_sector(pb, v), x, 0.1, 8, 2)
    assert rel(_host(yd), yref) <= KR_TOL
    h.destroy()
    os.environ["DMRG_MAX_WORKSPACE"] = str(st8["create_bytes"] - 1)
    try:
        with pytest.raises(L.DmrgError) as e:
            L.dmrg_create(pb)
        assert e.value.status == -2
    finally:
        del os.environ["DMRG_MAX_WORKSPACE"]


def test_ground_state_not_converged_status(env):
    """Too few restarts for the tolerance: DMRG_WNOTCONV is reported (info converged = 0) and
    the last Ritz pair is returned; with enough restarts the same call converges."""
    torch, L = env
    say("ground state status")
    pb = _problem("chain8_exact")
    h = L.dmrg_create(pb)
    x = I.random_psi(h.n, np.random.default_rng(41))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    lib = L.load()
    import ctypes as C
    e = C.c_double()
    used = C.c_int32()
    info = L._info(2)
    n2 = 2 * h.n
    rc = lib.dmrg_ground_state(h.h, L._tensor_ptr(xd, n2), L._tensor_ptr(yd, n2), 8, 2, 1e-12,
                               C.byref(e), C.byref(used), C.byref(info))
    assert rc == L.DMRG_WNOTCONV and info.converged == 0 and used.value == 2
    assert info.as_dict(2)["k_eff_steps"] == [8, 8]
    assert abs(np.linalg.norm(_host(yd)) - 1.0) < 1e-12
    energy, used2, d = h.ground_state(xd, yd, 30, 40, 1e-9)
    assert d["converged"] == 1 and used2 < 40
    h.destroy()


def test_ground_state_headline_converges(env):
    """The ladder 2 x 16 at m = 1000 from a random start: restarted Lanczos with kdim 64 reaches
    the relative residual 1e-6 within 20 bases.  The residual ||H y - E y|| and the Rayleigh
    quotient y^H H y are formed with the oracle's product on the host, so neither rests on the
    HIP path."""
    torch, L = env
    say("ground state at the headline, kdim 64")
    pb = _problem("ladder16_m1000")
    h = L.dmrg_create(pb)
    x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 5))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    e, used, info = h.ground_state(xd, yd, 64, 20, 1e-6)
    y = _host(yd)
    hy = M.matvec_sector(pb, y)
    yc = y[:h.n] + 1j * y[h.n:]
    hyc = hy[:h.n] + 1j * hy[h.n:]
    rq = float(np.vdot(yc, hyc).real)
    resid = float(np.linalg.norm(hyc - e * yc))
    say("  E", e, "bases", used, "estimate", info["err_est"], "residual", resid, "y^H H y", rq)
    assert info["converged"] == 1 and used <= 20
    assert abs(np.linalg.norm(yc) - 1.0) < 1e-12
    assert resid <= 1e-6 * abs(e)
    assert abs(rq - e) <= 1e-10 * abs(e)
    h.destroy()
