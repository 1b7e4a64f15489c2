"""GPU parity of the HIP library against the FP64 oracle (needs an MI355X).

Every case is compared element by element on the same seeded inputs.  Tolerances:
H_sb.psi <= 1e-12 relative (FP64 block products, sums of at most a few thousand terms), Krylov
steps and time-step-targeting vectors <= 1e-10 relative (the FP64 target), as
||gpu - oracle||_2 / ||oracle||_2 over the whole 2n-vector.
"""
import sys

import numpy as np
import pytest

from oracle import krylov as K
from oracle import matvec as M
from paper_1103_5391_amd import inputs as I

pytestmark = pytest.mark.gpu

MV_TOL = 1e-12
KR_TOL = 1e-10


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


_PROBLEMS = {}


def problem(name):
    if name not in _PROBLEMS:
        if name in I.WORKLOADS:
            _PROBLEMS[name] = I.make_workload(name)
        elif name == "chain12_m30":
            _PROBLEMS[name] = I.synthetic_problem(12, 30, 4.0, I.chain_bonds(12), 7, name=name)
        elif name == "ladder2x6_m40":
            _PROBLEMS[name] = I.synthetic_problem(12, 40, 8.0, I.ladder_bonds(6), 8, name=name)
        elif name == "chain14_m25_off":
            _PROBLEMS[name] = I.synthetic_problem(14, 25, 2.0, I.chain_bonds(14), 9, name=name,
                                                  target=(6, 8))
        elif name == "chain8_m17_odd":   # odd vector length: the scalar path of the vector passes
            _PROBLEMS[name] = I.synthetic_problem(8, 17, 4.0, I.chain_bonds(8), 47, name=name)
        elif name == "chain20_m150":
            _PROBLEMS[name] = I.synthetic_problem(20, 150, 4.0, I.chain_bonds(20), 12, name=name)
        elif name == "ladder2x8_m700_big":   # concentrated sectors: one of 624 states, four of 330
            _PROBLEMS[name] = I.synthetic_problem(16, 700, 8.0, I.ladder_bonds(8), 90, name=name,
                                                  width=0.7)
        elif name == "ladder2x8_m340_edge":  # sectors of 160 and 161 states (the two eigensolver
            # kernels' boundary) and up to 304 (back-transformation blocks of four)
            _PROBLEMS[name] = I.synthetic_problem(16, 340, 8.0, I.ladder_bonds(8), 90, name=name,
                                                  width=0.7)
        elif name == "ladder2x8_m620_257":   # a sector of 257 states: the first with blocks of four
            _PROBLEMS[name] = I.synthetic_problem(16, 620, 8.0, I.ladder_bonds(8), 90, name=name,
                                                  width=1.2)
        elif name == "ladder2x4_U10":
            _PROBLEMS[name] = I.exact_problem(8, 10.0, (4, 4), bonds=I.ladder_bonds(4, 1.0, 0.5))
        elif name == "chain4_exact":
            _PROBLEMS[name] = I.exact_problem(4, 4.0, (2, 2))
        elif name == "chain6_exact":
            _PROBLEMS[name] = I.exact_problem(6, 4.0, (3, 3))
        else:
            raise KeyError(name)
    return _PROBLEMS[name]


MATVEC_CASES = ["chain4_exact", "chain8_exact", "ladder2x4_U10", "chain12_m30", "ladder2x6_m40",
                "chain8_m17_odd",
                "chain14_m25_off", "chain20_m150", "chain32_m400", "ladder16_m800",
                "ladder16_m1000", "ladder32_m2000"]


def test_layout_matches_oracle(env):
    torch, L = env
    for name in ["chain8_exact", "ladder2x6_m40", "chain14_m25_off"]:
        say("layout", name)
        pb = problem(name)
        h = L.dmrg_create(pb)
        lay = h.psi_layout()
        ol, n = M.layout(pb)
        assert h.n == n
        assert [int(v) for v in lay["off"]] == [o[4] for o in ol]
        assert [int(v) for v in lay["rows"]] == [o[2] for o in ol]
        assert [int(v) for v in lay["cols"]] == [o[3] for o in ol]
        assert [int(v) for v in lay["secS"]] == [o[0] for o in ol]
        assert [int(v) for v in lay["secE"]] == [o[1] for o in ol]
        h.destroy()


GEMM_VARIANTS = pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 6, 8, 9, 12, 16, 32],
                                        ids=["reg-reg", "lds-reg", "reg-lds", "lds-lds",
                                             "narrow-reg", "narrow-lds", "reg-narrow",
                                             "lds-narrow", "narrow-narrow", "x", "k"])


@GEMM_VARIANTS
@pytest.mark.parametrize("name", MATVEC_CASES)
def test_matvec_parity(env, name, variant):
    """Both kernel families of each stage (register-tiled, LDS-tiled with K slices)."""
    torch, L = env
    say("matvec", name, "variant", variant)
    pb = problem(name)
    h = L.dmrg_create(pb)
    h.set_gemm(variant)
    n = h.n
    x = I.random_psi(n, np.random.default_rng(I.SEED_BASE + 77))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    h.matvec(xd, yd)
    torch.cuda.synchronize()
    y = _host(yd)
    yref = M.matvec_sector(pb, x)
    err = rel(y, yref)
    say("  rel err", err)
    assert err <= MV_TOL
    # bitwise reproducible
    yd2 = torch.empty_like(xd)
    h.matvec(xd, yd2)
    torch.cuda.synchronize()
    assert torch.equal(yd, yd2)
    h.destroy()


def test_matvec_multi_vector_and_hermitian(env):
    torch, L = env
    say("matvec nvec=2 + hermiticity")
    pb = problem("ladder2x6_m40")
    h = L.dmrg_create(pb)
    n = h.n
    rng = np.random.default_rng(5)
    xs = np.concatenate([I.random_psi(n, rng), I.random_psi(n, rng)])
    xd = _dev(torch, xs)
    yd = torch.empty_like(xd)
    h.matvec(xd, yd, nvec=2)
    torch.cuda.synchronize()
    ys = _host(yd)
    for v in range(2):
        sl = slice(2 * n * v, 2 * n * (v + 1))
        assert rel(ys[sl], M.matvec_sector(pb, xs[sl])) <= MV_TOL
    z = [xs[2 * n * v:2 * n * v + n] + 1j * xs[2 * n * v + n:2 * n * (v + 1)] for v in range(2)]
    hz = [ys[2 * n * v:2 * n * v + n] + 1j * ys[2 * n * v + n:2 * n * (v + 1)] for v in range(2)]
    assert abs(np.vdot(z[0], hz[1]) - np.vdot(hz[0], z[1])) < 1e-12 * np.linalg.norm(hz[0])
    h.destroy()


def test_matvec_generic_terms(env):
    """Generic connection terms (non-fermionic and transposed forms) next to the bonds."""
    torch, L = env
    say("matvec generic terms")
    pb = problem("chain12_m30")
    extra = [(0.37, 0, 0, 0, 1, 0), (-0.21, 1, 1, 1, 0, 1), (0.5, 0, 1, 0, 0, 0)]
    h = L.dmrg_create(pb, extra_terms=extra)
    x = I.random_psi(h.n, np.random.default_rng(6))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    h.matvec(xd, yd)
    torch.cuda.synchronize()
    assert rel(_host(yd), M.matvec_sector(pb, x, extra_terms=extra)) <= MV_TOL
    h.destroy()


KRYLOV_CASES = [
    # name, kdim, tau, nsteps
    ("chain8_exact", 12, 0.1, 10),
    ("chain12_m30", 15, 0.1, 3),
    ("chain8_m17_odd", 12, 0.1, 3),     # odd n
    ("chain20_m150", 20, 0.05, 2),
    ("chain32_m400", 15, 0.1, 2),
    ("ladder16_m1000", 15, 0.05, 1),
    ("ladder2x6_m40", 40, 0.3, 1),      # kdim > 32: unfused reorthogonalisation path
]


@pytest.mark.parametrize("variant", [0, 16, 32], ids=["register", "x", "k"])
@pytest.mark.parametrize("name,kdim,tau,nsteps", KRYLOV_CASES)
def test_krylov_parity(env, name, kdim, tau, nsteps, variant):
    torch, L = env
    say("krylov", name, kdim, tau, nsteps, "variant", variant)
    pb = problem(name)
    h = L.dmrg_create(pb)
    h.set_gemm(variant)
    x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 3))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    info = h.krylov_expm(xd, yd, tau, kdim, nsteps)
    y = _host(yd)
    yref, oinfo = K.krylov_expm(lambda v: M.matvec_sector(pb, v), x, tau, kdim, nsteps)
    err = rel(y, yref)
    say("  rel err", err, info)
    assert err <= KR_TOL
    assert info["k_eff"] == oinfo.k_eff[-1]
    assert abs(info["beta0"] - 1.0) < 1e-14
    assert abs(np.linalg.norm(y) - 1.0) < 1e-10
    h.destroy()


@pytest.mark.parametrize("name,kdim,tau", [("chain8_exact", 12, 0.1), ("ladder16_m1000", 15, 0.05),
                                           ("chain14_m25_off", 10, 0.2)])
def test_tst_parity(env, name, kdim, tau):
    torch, L = env
    say("tst", name)
    pb = problem(name)
    h = L.dmrg_create(pb)
    n = h.n
    phi = I.random_psi(n, np.random.default_rng(I.SEED_BASE + 4))
    pd = _dev(torch, phi)
    td = torch.empty(8 * n, dtype=torch.float64, device="cuda")
    w, info = h.tst_targets(pd, tau, kdim, td)
    t = _host(td)
    ys, wref, b = K.tst_targets(lambda v: M.matvec_sector(pb, v), phi, tau, kdim)
    assert np.array_equal(w, wref)
    for i in range(4):
        err = rel(t[2 * n * i:2 * n * (i + 1)], ys[i])
        say("  target", i, err)
        assert err <= KR_TOL
    h.destroy()


def test_krylov_edge_cases(env):
    torch, L = env
    pb = problem("chain6_exact")
    h = L.dmrg_create(pb)
    n = h.n
    # zero vector: zero result, k_eff 0, no error
    say("edge zero vector")
    zd = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
    yd = torch.full_like(zd, 7.0)
    info = h.krylov_expm(zd, yd, 0.3, 10, 2)
    assert torch.count_nonzero(yd).item() == 0 and info["k_eff"] == 0
    # tau = 0: identity (to rounding)
    say("edge tau 0")
    x = I.random_psi(n, np.random.default_rng(8))
    xd = _dev(torch, x)
    info = h.krylov_expm(xd, yd, 0.0, 10, 1)
    assert rel(_host(yd), x) < 1e-13
    # kdim = 1
    say("edge kdim 1")
    info = h.krylov_expm(xd, yd, 0.05, 1, 3)
    yref, _ = K.krylov_expm(lambda v: M.matvec_sector(pb, v), x, 0.05, 1, 3)
    assert rel(_host(yd), yref) <= KR_TOL
    # eigenvector input: breakdown after one vector, exact phase
    say("edge eigenvector")
    Hd = M.superblock_matrix(pb)
    wv, vv = np.linalg.eigh(Hd)
    ev = np.concatenate([vv[:, 3], np.zeros(n)])
    ed = _dev(torch, ev)
    info = h.krylov_expm(ed, yd, 0.7, 12, 1)
    assert info["k_eff"] == 1 and info["breakdown"] == 1
    z = np.exp(-0.7j * wv[3]) * vv[:, 3]
    assert rel(_host(yd), np.concatenate([z.real, z.imag])) < 1e-12
    # y aliases x
    say("edge aliasing")
    xd2 = xd.clone()
    h.krylov_expm(xd2, xd2, 0.1, 8, 2)
    yref, _ = K.krylov_expm(lambda v: M.matvec_sector(pb, v), x, 0.1, 8, 2)
    assert rel(_host(xd2), yref) <= KR_TOL
    h.destroy()


def test_krylov_exhausts_small_space(env):
    """kdim = 64 on a 36-dimensional sector: breakdown at the space dimension, exact result."""
    torch, L = env
    say("edge exhaust")
    pb = problem("chain4_exact")
    h = L.dmrg_create(pb)
    n = h.n
    x = I.random_psi(n, np.random.default_rng(10))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    info = h.krylov_expm(xd, yd, 2.0, 64, 1)
    import scipy.linalg as sla
    Hd = M.superblock_matrix(pb)
    z = sla.expm(-2.0j * Hd) @ (x[:n] + 1j * x[n:])
    assert info["breakdown"] == 1 and info["k_eff"] <= n
    assert rel(_host(yd), np.concatenate([z.real, z.imag])) < 1e-10
    h.destroy()


def test_chain8_against_dense_exponential(env):
    """Config chain L=8, U=4, exact blocks: GPU Krylov (kdim 12, tau 0.1, 10 steps) against the
    exponential of the ED Hamiltonian (scipy expm_multiply)."""
    torch, L = env
    say("chain8 vs ED")
    from tests.helpers import exact_case, expm_flat
    pb, sec, Hsp, perm = exact_case(8, 4.0, (4, 4))
    h = L.dmrg_create(pb)
    x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 1))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    h.krylov_expm(xd, yd, 0.1, 12, 10)
    assert rel(_host(yd), expm_flat(Hsp, x, 1.0)) < 1e-9
    h.destroy()


# ---------------------------------------------------------------------------------------------
# mixed precision: FP32 and split-bf16 block products, FP64 Lanczos / reorthogonalisation / expm
# ---------------------------------------------------------------------------------------------
# FP32: products rounded at 2^-24 and accumulated in FP32 over K <= ~2500 terms: the 1e-6
# relative bound of the mixed path.  BF16x3: a = a0 + a1 with bf16 pieces leaves a residual of
# about 2^-16 of each operand, and the dropped a1*b1 term is of the same order: per-element
# errors of a few 1e-5 averaging down to a few 1e-6 over a vector; the bound 3e-5 is that model.
# BF16x6: three pieces, the dropped terms of order 3 and the residual are about 2^-24: FP32-like,
# the 1e-6 bound.  Measured values are printed.
MIXED_TOL = {1: 1e-6, 2: 3e-5, 3: 1e-6}
MIXED = pytest.mark.parametrize("prec", [1, 2, 3], ids=["fp32", "bf16x3", "bf16x6"])


@MIXED
@pytest.mark.parametrize("name", ["chain8_exact", "chain14_m25_off", "chain32_m400",
                                  "ladder16_m1000", "ladder32_m2000"])
def test_matvec_mixed_precision(env, name, prec):
    torch, L = env
    say("matvec mixed", name, prec)
    pb = problem(name)
    h = L.dmrg_create(pb)
    h.set_precision(prec)
    x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 78))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    h.matvec(xd, yd)
    torch.cuda.synchronize()
    err = rel(_host(yd), M.matvec_sector(pb, x))
    say("  rel err", err)
    assert err <= MIXED_TOL[prec]
    # switching back gives the FP64 product again
    h.set_precision(0)
    h.matvec(xd, yd)
    torch.cuda.synchronize()
    assert rel(_host(yd), M.matvec_sector(pb, x)) <= MV_TOL
    h.destroy()


@MIXED
def test_krylov_mixed_precision_norm_and_error(env, prec):
    """Mixed block products inside an FP64 Lanczos: the norm is kept to 1e-8 (the basis and the
    combination are FP64) and the result stays within the matvec error scale of the oracle."""
    torch, L = env
    say("krylov mixed", prec)
    pb = problem("ladder16_m1000")
    h = L.dmrg_create(pb)
    h.set_precision(prec)
    x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 5))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    info = h.krylov_expm(xd, yd, 0.05, 15, 2)
    y = _host(yd)
    yref, _ = K.krylov_expm(lambda v: M.matvec_sector(pb, v), x, 0.05, 15, 2)
    err = rel(y, yref)
    say("  rel err", err, "norm drift", abs(np.linalg.norm(y) - 1.0))
    assert abs(np.linalg.norm(y) - 1.0) <= 1e-8
    assert err <= MIXED_TOL[prec]
    h.destroy()


# ---------------------------------------------------------------------------------------------
# batching and graphs: one launch per pass for many superblocks, captured Lanczos iterations.
# Both run the same kernels on the same per-problem data as the single-handle eager path, so
# the results must agree bit for bit; the small batch is also checked against the oracle.
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("name,kdim,tau", [("chain12_m30", 15, 0.1), ("chain8_m17_odd", 12, 0.1),
                                           ("ladder16_m1000", 15, 0.05)])
def test_tst_chains_parity(env, name, kdim, tau):
    """4-RHS mode: four different vectors, each advanced by tau with its own basis, against the
    oracle's per-target chains; in place (targets = inputs) gives the same vectors; graph mode
    gives the same bits."""
    torch, L = env
    say("tst chains", name)
    pb = problem(name)
    h = L.dmrg_create(pb)
    n = h.n
    xs = [I.random_psi(n, np.random.default_rng(I.SEED_BASE + 40 + k)) for k in range(4)]
    xds = [_dev(torch, x) for x in xs]
    yds = [torch.full((2 * n,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(4)]
    w, infos = h.tst_chains(xds, tau, kdim, yds)
    ys, wref, oinfos = K.tst_chains(lambda v: M.matvec_sector(pb, v), xs, tau, kdim)
    assert np.array_equal(w, wref)
    for k in range(4):
        err = rel(_host(yds[k]), ys[k])
        say("  chain", k, "rel err", err, infos[k])
        assert err <= KR_TOL
        assert infos[k]["k_eff"] == oinfos[k].k_eff[-1]
    h.set_graph(True)
    zds = [torch.full_like(xds[0], float("nan")) for _ in range(4)]
    h.tst_chains(xds, tau, kdim, zds)
    assert all(torch.equal(z, y) for z, y in zip(zds, yds))
    inplace = [x.clone() for x in xds]
    h.tst_chains(inplace, tau, kdim, inplace)
    assert all(torch.equal(a, y) for a, y in zip(inplace, yds))
    h.destroy()


@pytest.mark.parametrize("name", ["chain12_m30", "chain8_m17_odd", "chain14_m25_off",
                                  "ladder16_m1000"])
def test_tst_chains_shared_operator_stage2_bitwise(env, name):
    """With narrow tiles in both stages (FP64), stage 2 of the 4-RHS mode runs all four chains
    of a tile in one work group, loading the left factors once: each chain equals, bit for bit,
    one step of its own vector through the single-vector path, in graph mode too."""
    torch, L = env
    say("shared-operator chains", name)
    h = L.dmrg_create(problem(name))
    h.set_gemm(L.DMRG_GEMM_STAGE1_NARROW | L.DMRG_GEMM_STAGE2_NARROW)
    n = h.n
    tau, kdim = 0.05, 15
    xds = [_dev(torch, I.random_psi(n, np.random.default_rng(I.SEED_BASE + 700 + k)))
           for k in range(4)]
    for graph in (False, True):
        h.set_graph(graph)
        yds = [torch.full_like(xds[0], float("nan")) for _ in range(4)]
        h.tst_chains(xds, tau, kdim, yds)
        for k in range(4):
            one = torch.empty_like(xds[k])
            h.krylov_expm(xds[k], one, tau, kdim, 1, info=False)
            torch.cuda.synchronize()
            assert torch.equal(one, yds[k]), (graph, k)
    h.destroy()


def test_tst_chains_shared_operator_stage2_with_breakdown(env):
    """One chain starts from an eigenvector and breaks down after one vector while the other
    three go on: the shared-operator stage 2 leaves the broken chain's buffers alone, and every
    chain still equals its single-vector step bit for bit."""
    torch, L = env
    say("shared-operator chains with a breakdown")
    pb = problem("chain6_exact")
    h = L.dmrg_create(pb)
    h.set_gemm(L.DMRG_GEMM_STAGE1_NARROW | L.DMRG_GEMM_STAGE2_NARROW)
    n = h.n
    wv, vv = np.linalg.eigh(M.superblock_matrix(pb))
    xs = [np.concatenate([vv[:, 5], np.zeros(n)])] + \
         [I.random_psi(n, np.random.default_rng(I.SEED_BASE + 710 + k)) for k in range(3)]
    xds = [_dev(torch, x) for x in xs]
    yds = [torch.full_like(xds[0], float("nan")) for _ in range(4)]
    _, infos = h.tst_chains(xds, 0.3, 12, yds)
    assert infos[0]["k_eff"] == 1 and all(i["k_eff"] > 1 for i in infos[1:])
    for k in range(4):
        one = torch.empty_like(xds[k])
        h.krylov_expm(xds[k], one, 0.3, 12, 1, info=False)
        torch.cuda.synchronize()
        assert torch.equal(one, yds[k]), k
    h.destroy()


def test_batch_tst_chains_matches_per_handle(env):
    """4-RHS mode of a batch (odd and even lengths, 12 chains in common launches): bit for bit
    the per-handle chains, and the oracle to 1e-10."""
    torch, L = env
    say("batch chains")
    pbs = [problem("chain12_m30"), problem("chain8_m17_odd"), problem("chain14_m25_off")]
    hs = [L.dmrg_create(pb) for pb in pbs]
    tau, kdim = 0.1, 12
    xs, xds, yds = [], [], []
    for i, h in enumerate(hs):
        for k in range(4):
            x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 600 + 4 * i + k))
            xs.append(x)
            xds.append(_dev(torch, x))
            yds.append(torch.full((2 * h.n,), float("nan"), dtype=torch.float64, device="cuda"))
    b = L.Batch(hs)
    w, infos = b.batch_tst_chains(xds, tau, kdim, yds)
    for i, (pb, h) in enumerate(zip(pbs, hs)):
        own = [torch.empty_like(xds[4 * i + k]) for k in range(4)]
        _, inf1 = h.tst_chains(xds[4 * i:4 * i + 4], tau, kdim, own)
        ys, _, _ = K.tst_chains(lambda v: M.matvec_sector(pb, v), xs[4 * i:4 * i + 4], tau, kdim)
        for k in range(4):
            assert torch.equal(own[k], yds[4 * i + k])
            assert inf1[k] == infos[4 * i + k]
            assert rel(_host(yds[4 * i + k]), ys[k]) <= KR_TOL
    # narrow tiles in both stages: the shared-operator stage 2 over the three owners
    narrow = L.DMRG_GEMM_STAGE1_NARROW | L.DMRG_GEMM_STAGE2_NARROW
    b.set_gemm(narrow)
    zds = [torch.full_like(y, float("nan")) for y in yds]
    b.batch_tst_chains(xds, tau, kdim, zds)
    for i, h in enumerate(hs):
        h.set_gemm(narrow)
        for k in range(4):
            one = torch.empty_like(xds[4 * i + k])
            h.krylov_expm(xds[4 * i + k], one, tau, kdim, 1, info=False)
            torch.cuda.synchronize()
            assert torch.equal(one, zds[4 * i + k]), (i, k)
            assert rel(_host(zds[4 * i + k]), _host(yds[4 * i + k])) <= 1e-13
    b.destroy()
    for h in hs:
        h.destroy()


@pytest.mark.parametrize("name,kdim,restarts", [("chain8_exact", 20, 6), ("chain8_m17_odd", 12, 5),
                                               ("chain12_m30", 16, 4), ("ladder16_m1000", 15, 3)])
def test_ground_state_parity(env, name, kdim, restarts):
    """Restarted Lanczos ground state with a fixed number of bases (tol 0): energy and Ritz
    vector against the oracle's restarted Lanczos."""
    torch, L = env
    say("ground state", name)
    pb = problem(name)
    h = L.dmrg_create(pb)
    x0 = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 70))
    xd = _dev(torch, x0)
    yd = torch.full_like(xd, float("nan"))
    e, used, info = h.ground_state(xd, yd, kdim, restarts, 0.0)
    yref, oinfo = K.ground_state(lambda v: M.matvec_sector(pb, v), x0, kdim, restarts, 0.0)
    err = rel(_host(yd), yref)
    say("  E", e, "oracle", oinfo.energy, "vector rel err", err, "bases", used, info)
    assert used == oinfo.restarts
    assert abs(e - oinfo.energy) <= 1e-10 * max(1.0, abs(oinfo.energy))
    assert err <= 1e-8
    assert abs(info["err_est"] - oinfo.residual_est) <= 1e-8 * max(1.0, oinfo.residual_est)
    h.destroy()


def test_ground_state_converges_to_exact(env):
    """Exact-block chain (L = 8, U = 4): converged to tol 1e-11 in place (y = x0); the energy
    against the lowest eigenvalue of the ED matrix (ARPACK) and the residual ||H y - E y||
    through the library's own product."""
    import scipy.sparse.linalg as spla
    from tests.helpers import exact_case
    torch, L = env
    say("ground state converged")
    pb, sec, H, perm = exact_case(8, 4.0, (4, 4))
    h = L.dmrg_create(pb)
    x0 = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 71))
    xd = _dev(torch, x0)
    e, used, info = h.ground_state(xd, xd, 30, 80, 1e-11)
    e0 = float(np.sort(spla.eigsh(H, k=2, which="SA", tol=1e-14)[0])[0])
    hy = torch.empty_like(xd)
    h.matvec(xd, hy)
    resid = float(torch.linalg.vector_norm(hy - e * xd))
    say("  E", e, "exact", e0, "bases", used, "residual", resid)
    assert used < 80
    assert abs(e - e0) <= 1e-10 * abs(e0)
    assert resid <= 1e-9 * max(1.0, abs(e0))
    assert abs(float(torch.linalg.vector_norm(xd)) - 1.0) < 1e-12
    h.destroy()


def _decaying(pb, x, decades):
    """x with the rows of every block scaled by 10^(-decades i / d): a density matrix whose
    spectrum decays over `decades` decades (clusters of small eigenvalues)."""
    blocks = M.unpack(pb, x)
    out = {p: b * np.logspace(0, -decades, b.shape[0])[:, None] for p, b in blocks.items()}
    y = M.pack(pb, out)
    return y / np.linalg.norm(y)


@pytest.mark.parametrize("name,decades", [("chain12_m30", 0), ("chain8_exact", 0), ("chain8_m17_odd", 0),
                                          ("ladder16_m1000", 0), ("chain12_m30", 12),
                                          ("ladder16_m1000", 14), ("ladder32_m2000", 0),
                                          ("ladder2x8_m700_big", 0), ("ladder2x8_m340_edge", 0),
                                          ("ladder2x8_m340_edge", 12), ("ladder2x8_m620_257", 0)])
def test_density_truncate_parity(env, name, decades):
    """Density matrix of five weighted targets and its truncation against the oracle: every
    eigenvalue, the kept count of every sector and the truncation error; eigen-pairs (residual
    against the oracle's rho, orthonormality); the kept subspace of every sector (its
    projector), which is unique where the kept and discarded eigenvalues are apart.  Decaying
    spectra (clusters of small eigenvalues) take the kernel's other tridiagonal solver.  The
    sectors of ladder32_m2000 (up to 300 states) and ladder2x8_m700_big (330 and 624) take the
    back-transformation's blocks of four and two reflectors; ladder2x8_m340_edge has sectors of
    160 and 161 states, the last of the register-resident eigensolver and the first of the
    general one, and ladder2x8_m620_257 one of 257 states, the first with blocks of four."""
    from oracle import density as Dn
    torch, L = env
    say("density", name, "decades", decades)
    pb = problem(name)
    h = L.dmrg_create(pb)
    n = h.n
    rng = np.random.default_rng(I.SEED_BASE + 80)
    vecs = [I.random_psi(n, rng) for _ in range(5)]
    if decades:
        vecs = [_decaying(pb, v, decades) for v in vecs]
    w = K.tst_weights()
    rows = [int(r) for r in h.psi_layout()["rows"]]
    total = sum(rows)
    # a cut with a clear gap, near a quarter of the states
    ref_all = Dn.truncate(pb, vecs, w, keep=total)
    allv = np.sort(np.concatenate([ref_all.evals[p] for p in ref_all.sectors]))[::-1]
    lo, hi = (1 if decades else max(1, total // 8)), max(2, total // 3)
    gaps = (allv[lo - 1:hi - 1] - allv[lo:hi]) / allv[0]
    keep = lo + int(np.argmax(gaps))
    assert gaps.max() > 1e-6
    ref = Dn.truncate(pb, vecs, w, keep=keep)
    rho = Dn.density_blocks(pb, vecs, w)
    evd = torch.full((total,), float("nan"), dtype=torch.float64, device="cuda")
    vcd = torch.full((sum(2 * r * r for r in rows),), float("nan"), dtype=torch.float64, device="cuda")
    xds = [_dev(torch, v) for v in vecs]
    kept, err = h.density_truncate(xds, w, keep, evd, vcd)
    ev, vc = _host(evd), _host(vcd)
    scale = allv[0]
    eo = vo = 0
    worst = 0.0
    for b, p in enumerate(ref.sectors):
        d = rows[b]
        lam = ev[eo:eo + d]
        U = vc[vo:vo + d * d].reshape(d, d).T + 1j * vc[vo + d * d:vo + 2 * d * d].reshape(d, d).T
        assert np.max(np.abs(lam - ref.evals[p])) <= 1e-12 * scale, (p, lam, ref.evals[p])
        assert kept[b] == ref.kept[p]
        assert np.linalg.norm(U.conj().T @ U - np.eye(d)) <= 1e-11 * d
        assert np.linalg.norm(rho[p] @ U - U * lam[None, :]) <= 1e-11 * scale * d
        k = int(kept[b])
        if 0 < k < d and (lam[k - 1] - lam[k]) > 1e-6 * scale:
            Pg = U[:, :k] @ U[:, :k].conj().T
            Pr = ref.evecs[p][:, :k] @ ref.evecs[p][:, :k].conj().T
            worst = max(worst, np.linalg.norm(Pg - Pr))
        eo += d
        vo += 2 * d * d
    say("  keep", keep, "trunc err", err, ref.trunc_err, "worst projector diff", worst)
    assert abs(err - ref.trunc_err) <= 1e-12
    assert worst <= 1e-8
    # the two ends of the truncation: nothing kept (the error is the trace) and everything kept
    k0, err0 = h.density_truncate(xds, w, 0, torch.empty_like(evd), torch.empty_like(vcd))
    assert sum(int(k) for k in k0) == 0 and abs(err0 - ref.trace) <= 1e-12 * max(1.0, ref.trace)
    kall, errall = h.density_truncate(xds, w, total + 5, torch.empty_like(evd), torch.empty_like(vcd))
    assert [int(k) for k in kall] == rows and abs(errall) <= 1e-12 * max(1.0, ref.trace)
    # a second call gives the same bits (fixed-order arithmetic throughout)
    ev2 = torch.full_like(evd, float("nan"))
    vc2 = torch.full_like(vcd, float("nan"))
    kept2, err2 = h.density_truncate(xds, w, keep, ev2, vc2)
    assert np.array_equal(_host(ev2), ev) and np.array_equal(_host(vc2), vc)
    assert np.array_equal(kept2, kept) and err2 == err
    h.destroy()


def _evecs_layout(rows, evecs_by_block):
    """Eigenvector matrices (complex d x d per psi block) in the layout of density_truncate."""
    parts = []
    for d, U in zip(rows, evecs_by_block):
        parts.append(np.asarray(U.real).T.reshape(-1))
        parts.append(np.asarray(U.imag).T.reshape(-1))
    return np.concatenate(parts)


def _w_device(torch, mv):
    return [_dev(torch, np.concatenate([w.real.T.reshape(-1), w.imag.T.reshape(-1)])) for w in mv.W]


@pytest.mark.parametrize("name,frac", [("chain8_exact", 1.0), ("chain8_exact", 0.3),
                                       ("chain12_m30", 0.5), ("chain8_m17_odd", 0.4),
                                       ("ladder16_m1000", 0.25)])
def test_wft_parity(env, name, frac):
    """Wave-function transformation of five targets against the oracle, with the oracle's
    eigenvectors and kept counts (a global cut at frac of the states) as the input U."""
    from oracle import density as Dn
    from oracle import wft as Wo
    torch, L = env
    say("wft", name, frac)
    pb = problem(name)
    h = L.dmrg_create(pb)
    n = h.n
    rng = np.random.default_rng(I.SEED_BASE + 90)
    vecs = [I.random_psi(n, rng) for _ in range(5)]
    rows = [int(r) for r in h.psi_layout()["rows"]]
    keep = max(1, int(frac * sum(rows)))
    tr = Dn.truncate(pb, vecs, K.tst_weights(), keep)
    kept = [int(tr.kept[p]) for p in tr.sectors]
    mv = I.wft_move(pb, kept, seed=5)
    w = h.wft_create(mv, _w_device(torch, mv))
    assert w.n_new == I.psi_size(mv.layout)
    Ud = _dev(torch, _evecs_layout(rows, [tr.evecs[p] for p in tr.sectors]))
    xs = [_dev(torch, v) for v in vecs]
    ys = [torch.full((2 * w.n_new,), float("nan"), dtype=torch.float64, device="cuda") for _ in vecs]
    fl = w.apply(Ud, xs, ys)
    assert fl > 0
    worst = 0.0
    for v, y in zip(vecs, ys):
        ref = Wo.wft_right(pb, mv, tr.evecs, v)
        got = _host(y)
        assert np.all(np.isfinite(got))
        worst = max(worst, float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)))
    say("  n", n, "n_new", w.n_new, "kept", sum(kept), "max rel err", worst)
    assert worst <= 1e-12
    # one vector at a time gives the same bits as the five together
    y1 = torch.full_like(ys[0], float("nan"))
    w.apply(Ud, xs[2:3], [y1])
    assert torch.equal(y1, ys[2])
    w.destroy()
    h.destroy()


def test_wft_after_gpu_density(env):
    """The GPU's own density eigenvectors feed the GPU transformation: the result depends on
    the basis of the kept states only through its norm, which must equal the weight of each
    target on the kept subspace (the oracle's projector; the cut sits at a clear gap)."""
    from oracle import density as Dn
    torch, L = env
    name = "chain12_m30"
    say("wft after density", name)
    pb = problem(name)
    h = L.dmrg_create(pb)
    n = h.n
    rng = np.random.default_rng(I.SEED_BASE + 91)
    vecs = [I.random_psi(n, rng) for _ in range(5)]
    w8 = K.tst_weights()
    rows = [int(r) for r in h.psi_layout()["rows"]]
    total = sum(rows)
    allv = np.sort(np.concatenate(list(Dn.truncate(pb, vecs, w8, total).evals.values())))[::-1]
    gaps = allv[total // 4:total // 2] - allv[total // 4 + 1:total // 2 + 1]
    keep = total // 4 + 1 + int(np.argmax(gaps))
    tr = Dn.truncate(pb, vecs, w8, keep)
    xs = [_dev(torch, v) for v in vecs]
    evd = torch.empty(total, dtype=torch.float64, device="cuda")
    vcd = torch.empty(sum(2 * r * r for r in rows), dtype=torch.float64, device="cuda")
    kept, _ = h.density_truncate(xs, w8, keep, evd, vcd)
    assert [int(k) for k in kept] == [int(tr.kept[p]) for p in tr.sectors]
    mv = I.wft_move(pb, [int(k) for k in kept], seed=6)
    w = h.wft_create(mv, _w_device(torch, mv))
    ys = [torch.empty(2 * w.n_new, dtype=torch.float64, device="cuda") for _ in vecs]
    w.apply(vcd, xs, ys)
    for v, y in zip(vecs, ys):
        blocks = M.unpack(pb, v)
        want = sum(np.linalg.norm(tr.evecs[p][:, :tr.kept[p]].conj().T @ blocks[p]) ** 2
                   for p in tr.sectors)
        got = float(torch.linalg.vector_norm(y)) ** 2
        assert abs(got - want) <= 1e-12, (got, want)
    w.destroy()
    h.destroy()


def test_wft_rejects_inconsistent_moves(env):
    torch, L = env
    pb = problem("chain12_m30")
    h = L.dmrg_create(pb)
    rows = [int(r) for r in h.psi_layout()["rows"]]
    kept = [max(1, r // 2) for r in rows]
    mv = I.wft_move(pb, kept, seed=7)
    Wd = _w_device(torch, mv)
    bad = I.wft_move(pb, kept, seed=7)
    bad.kept = [r + 1 for r in rows]                      # more than the sector holds
    with pytest.raises(L.DmrgError):
        h.wft_create(bad, Wd)
    bad = I.wft_move(pb, kept, seed=7)
    (b, a), (pp, off) = next(iter(bad.ssub.items()))
    bad.ssub[(b, a)] = (pp, int(bad.layout.S.space.dim[pp]))   # rows outside the sector
    with pytest.raises(L.DmrgError):
        h.wft_create(bad, Wd)
    w = h.wft_create(mv, Wd)
    w.destroy()
    # density matrix: vector counts outside [1, 16] and a negative keep are rejected
    x = _dev(torch, I.random_psi(h.n, np.random.default_rng(3)))
    evd = torch.empty(sum(rows), dtype=torch.float64, device="cuda")
    vcd = torch.empty(sum(2 * r * r for r in rows), dtype=torch.float64, device="cuda")
    for vecs, wts, keep in (([x] * 17, [0.05] * 17, 10), ([x], [1.0], -1)):
        with pytest.raises(L.DmrgError):
            h.density_truncate(vecs, wts, keep, evd, vcd)
    with pytest.raises(L.DmrgError):
        h.density_truncate([x], [float("nan")], 10, evd, vcd)
    h.destroy()


def _local_setup(pb, site_kinds):
    """pb with the requested site operators appended to its halves: returns (problem, {(site,
    kind): (side, op index, BlockOp)})."""
    extra = {"S": [], "E": []}
    keys = []
    for (site, kind) in site_kinds:
        side = "S" if site in pb.Sblk.sites else "E"
        blk = pb.Sblk if side == "S" else pb.Eblk
        extra[side].append(I.site_ops(blk, site)[kind])
        keys.append((site, kind, side, len(extra[side]) - 1))
    pbx, iS, iE = I.with_ops(pb, extra["S"], extra["E"])
    ops = {}
    for (site, kind, side, k) in keys:
        ops[(site, kind)] = (side, (iS if side == "S" else iE)[k], extra[side][k])
    return pbx, extra, ops


_ODD = ("cdag", "c_", "holon", "doublon")


def _gpu_and_oracle_term(pbx, ops, site, kind, trans=0, coef=1.0):
    side, idx, op = ops[(site, kind)]
    sp = pbx.S.space if side == "S" else pbx.E.space
    o = I._transpose(op, sp) if trans else op
    if side == "S":
        return (coef, idx, trans, -1, 0, 0), (coef, o, None, 0)
    f = 1 if kind.startswith(_ODD) else 0
    return (coef, -1, 0, idx, trans, f), (coef, None, o, f)


@pytest.mark.parametrize("name", ["ladder2x4_U10", "chain8_exact", "chain12_m30"])
def test_local_operators_parity(env, name):
    """Single-site operators (also transposed), a holon-doublon pair across the halves and a
    sum of terms, applied through the C ABI into the destination sector's layout, and the
    expectations of n_p and n_p,up n_p,dn: against the oracle."""
    from oracle import observables as Ob
    torch, L = env
    say("local", name)
    pb = problem(name)
    sites = list(range(pb.L)) if pb.Sblk.space.occ is not None else [pb.Sblk.sites[-1], pb.Eblk.sites[0]]
    kinds = ["cdag_0", "cdag_1", "n", "nn", "holon_1", "doublon_0"]
    pbx, extra, ops = _local_setup(pb, [(st, k) for st in sites for k in kinds])
    h = L.dmrg_create(pbx)
    n = h.n
    x = I.random_psi(n, np.random.default_rng(I.SEED_BASE + 95))
    xd = _dev(torch, x)
    dq_of = {"cdag_0": (1, 0), "cdag_1": (0, 1), "n": (0, 0), "nn": (0, 0), "holon_1": (0, -1),
             "doublon_0": (1, 0)}
    handles = {}

    def dst(dq):
        tgt = (pb.target[0] + dq[0], pb.target[1] + dq[1])
        if tgt not in handles:
            pd = I.with_ops(pb, extra["S"], extra["E"], target=tgt)[0]
            handles[tgt] = (pd, L.dmrg_create(pd))
        return handles[tgt]

    worst = 0.0

    def check(gterms, oterms, dq):
        nonlocal worst
        pd, hd = dst(dq)
        y = torch.full((2 * hd.n,), float("nan"), dtype=torch.float64, device="cuda")
        h.apply_local(hd, gterms, xd, y)
        ref = Ob.apply_terms(pbx, pd, oterms, x)
        got = _host(y)
        assert np.all(np.isfinite(got))
        worst = max(worst, float(np.max(np.abs(got - ref))) / max(1.0, float(np.max(np.abs(ref)))))

    for st in sites:
        for k in kinds:
            g, o = _gpu_and_oracle_term(pbx, ops, st, k)
            check([g], [o], dq_of[k])
        g, o = _gpu_and_oracle_term(pbx, ops, st, "cdag_0", trans=1)     # c_up as cdag_up^T
        check([g], [o], (-1, 0))
    # holon at the last system site, doublon at the first environment site (parity of S)
    i, j = pb.Sblk.sites[-1], pb.Eblk.sites[0]
    _, hi, hop = ops[(i, "holon_1")]
    _, dj, dop = ops[(j, "doublon_0")]
    check([(0.7, hi, 0, dj, 0, 1)], [(0.7, hop, dop, 1)], (1, -1))
    # a sum of terms into one sector
    g1, o1 = _gpu_and_oracle_term(pbx, ops, i, "n", coef=0.5)
    g2, o2 = _gpu_and_oracle_term(pbx, ops, j, "nn", coef=-2.0)
    check([g1, g2], [o1, o2], (0, 0))
    # a repeated call reuses its planned lists; a new destination handle plans again
    g1, o1 = _gpu_and_oracle_term(pbx, ops, i, "doublon_0")
    check([g1], [o1], (1, 0))
    check([g1], [o1], (1, 0))
    tgt = (pb.target[0] + 1, pb.target[1])
    handles[tgt][1].destroy()
    pd2 = I.with_ops(pb, extra["S"], extra["E"], target=tgt)[0]
    handles[tgt] = (pd2, L.dmrg_create(pd2))
    check([g1], [o1], (1, 0))
    say("  max rel err (monomial factors)", worst)
    assert worst <= 1e-12
    # dense operators (every element of a block nonzero): the product path
    rng = np.random.default_rng(I.SEED_BASE + 97)
    dS = I.BlockOp((0, 0), {p: rng.standard_normal((int(dd), int(dd))) for p, dd in enumerate(pb.S.space.dim)})
    dE = I.BlockOp((1, 0))
    for q in range(pb.E.space.nsec):
        q2 = pb.E.space.shift(q, (1, 0))
        if q2 is not None:
            dE.blocks[q] = rng.standard_normal((int(pb.E.space.dim[q2]), int(pb.E.space.dim[q])))
    pbd, iS2, iE2 = I.with_ops(pb, [dS], [dE])
    hdn = L.dmrg_create(pbd)
    worst = 0.0
    for (gterms, oterms, dq) in (([(0.3, iS2[0], 0, -1, 0, 0)], [(0.3, dS, None, 0)], (0, 0)),
                                 ([(1.0, -1, 0, iE2[0], 0, 1)], [(1.0, None, dE, 1)], (1, 0)),
                                 ([(-0.7, iS2[0], 1, iE2[0], 0, 1)],
                                  [(-0.7, I._transpose(dS, pb.S.space), dE, 1)], (1, 0))):
        tgt = (pb.target[0] + dq[0], pb.target[1] + dq[1])
        pdd = I.with_ops(pb, [dS], [dE], target=tgt)[0]
        hdd = L.dmrg_create(pdd)
        y = torch.full((2 * hdd.n,), float("nan"), dtype=torch.float64, device="cuda")
        hdn.apply_local(hdd, gterms, xd, y)
        ref = Ob.apply_terms(pbd, pdd, oterms, x)
        got = _host(y)
        assert np.all(np.isfinite(got))
        worst = max(worst, float(np.max(np.abs(got - ref))) / max(1.0, float(np.max(np.abs(ref)))))
        hdd.destroy()
    hdn.destroy()
    say("  max rel err (dense factors)", worst)
    assert worst <= 1e-12
    for st in sites:
        for k in ("n", "nn"):
            g, o = _gpu_and_oracle_term(pbx, ops, st, k)
            e_gpu = h.expect_local([g], xd)
            e_ref = Ob.expect(pbx, [o], x)
            assert abs(e_gpu - e_ref) <= 1e-12 * max(1.0, abs(e_ref)), (st, k, e_gpu, e_ref)
    for (_, hd) in handles.values():
        hd.destroy()
    h.destroy()


@pytest.mark.parametrize("U", [0.0, 10.0])
def test_holon_doublon_workflow(env, U):
    """Fig. 3 and Fig. 5 on the GPU: ground state of the 2x4 ladder (t_x = 1, t_y = 0.5, 4 up +
    4 down) by restarted Lanczos, the holon-doublon operator (i = 2, j = 4) applied into its
    three sectors, densities and double occupations at t = 0 against the paper's values, then
    Krylov evolution to t = 0.5 against the exact evolution of the exact diagonalisation."""
    import itertools
    import json
    import os
    from scipy.sparse.linalg import expm_multiply
    from oracle import ed
    torch, L = env
    say("holon-doublon workflow U =", U)
    Lsites, i, j = 8, 2, 4
    bonds = I.ladder_bonds(4, 1.0, 0.5)
    pb = I.exact_problem(Lsites, U, (4, 4), bonds=bonds)
    kinds = [(i, f"holon_{s}") for s in (0, 1)] + [(j, f"doublon_{s}") for s in (0, 1)] + \
        [(p, k) for p in range(Lsites) for k in ("n", "nn")]
    pbx, extra, ops = _local_setup(pb, kinds)
    h0 = L.dmrg_create(pbx)
    x0 = _dev(torch, I.random_psi(h0.n, np.random.default_rng(I.SEED_BASE + 96), complex_=False))
    gd = torch.empty_like(x0)
    e0, used, info = h0.ground_state(x0, gd, 40, 60, 1e-12)
    assert info["err_est"] <= 1e-10
    hs, phis = {}, {}
    for tgt in [(3, 5), (4, 4), (5, 3)]:
        pd = I.with_ops(pb, extra["S"], extra["E"], target=tgt)[0]
        hs[tgt] = L.dmrg_create(pd)
        terms = []
        for s, s2 in itertools.product((0, 1), (0, 1)):
            if (4 - (s == 0) + (s2 == 0), 4 - (s == 1) + (s2 == 1)) != tgt:
                continue
            _, hi, _ = ops[(i, f"holon_{s}")]
            _, dj, _ = ops[(j, f"doublon_{s2}")]
            terms.append((1.0, hi, 0, dj, 0, 1))
        y = torch.empty(2 * hs[tgt].n, dtype=torch.float64, device="cuda")
        h0.apply_local(hs[tgt], terms, gd, y)
        phis[tgt] = y

    def measure(vecs):
        norm = sum(float(torch.dot(v, v)) for v in vecs.values())
        dens, docc = np.zeros(Lsites), np.zeros(Lsites)
        for tgt, v in vecs.items():
            for p in range(Lsites):
                for k, arr in (("n", dens), ("nn", docc)):
                    side, idx, _ = ops[(p, k)]
                    term = (1.0, idx, 0, -1, 0, 0) if side == "S" else (1.0, -1, 0, idx, 0, 0)
                    arr[p] += hs[tgt].expect_local([term], v).real
        return dens / norm, docc / norm

    dens, docc = measure(phis)
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    g, gdd = golden["holon_doublon_density_t0"], golden["double_occupation_t0"]
    want = np.full(Lsites, g["other_site_value"])
    want[i], want[j] = g["holon_site_value"], g["doublon_site_value"]
    say("  t = 0 density", np.round(dens, 12), "N_d(j), N_d(i)", docc[j], docc[i])
    assert np.allclose(dens, want, atol=1e-9)
    assert abs(docc[j] - gdd["doublon_site_value"]) < 1e-9 and abs(docc[i] - gdd["holon_site_value"]) < 1e-9
    # evolution: 5 Krylov steps of tau = 0.1 per sector, against expm on the ED sectors
    tau, nsteps = 0.1, 5
    evolved = {}
    for tgt, v in phis.items():
        yv = torch.empty_like(v)
        hs[tgt].krylov_expm(v, yv, tau, 16, nsteps)
        evolved[tgt] = yv
    dens_t, docc_t = measure(evolved)
    sec0, H0 = ed.hamiltonian(Lsites, bonds, U, 4, 4)
    _, gs = ed.ground_state(H0)
    ref_n, ref_d, norm = np.zeros(Lsites), np.zeros(Lsites), 0.0
    parts = {}
    for s, s2 in itertools.product((0, 1), (0, 1)):
        v = gs * ed.number(sec0, j, 1 - s2)
        d1 = [4, 4]
        d1[s2] += 1
        sec1 = ed.Sector(Lsites, *d1)
        v = ed.create(sec0, sec1, 2 * j + s2) @ v
        v = v * (1.0 - ed.number(sec1, i, 1 - s))
        d2 = list(d1)
        d2[s] -= 1
        sec2 = ed.Sector(Lsites, *d2)
        v = ed.annihilate(sec1, sec2, 2 * i + s) @ v
        parts[tuple(d2)] = (sec2, parts[tuple(d2)][1] + v) if tuple(d2) in parts else (sec2, v)
    for key, (sec, v) in parts.items():
        _, Hs = ed.hamiltonian(Lsites, bonds, U, *key)
        vt = expm_multiply(-1j * tau * nsteps * Hs, v.astype(complex))
        w = np.abs(vt) ** 2
        norm += float(np.sum(w))
        for p in range(Lsites):
            ref_n[p] += np.sum(w * (ed.number(sec, p, 0) + ed.number(sec, p, 1)))
            ref_d[p] += np.sum(w * ed.number(sec, p, 0) * ed.number(sec, p, 1))
    ref_n /= norm
    ref_d /= norm
    say("  t = 0.5 density", np.round(dens_t, 6), "max err", np.max(np.abs(dens_t - ref_n)))
    assert np.max(np.abs(dens_t - ref_n)) < 1e-8
    assert np.max(np.abs(docc_t - ref_d)) < 1e-8
    assert np.max(np.abs(dens_t - dens)) > 1e-3          # it does move
    for hd in hs.values():
        hd.destroy()
    h0.destroy()


def _batch_setup(torch, L, pbs, seed):
    hs = [L.dmrg_create(pb) for pb in pbs]
    phis = [I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + seed + i)) for i, h in enumerate(hs)]
    pds = [_dev(torch, p) for p in phis]
    tds = [torch.full((8 * h.n,), float("nan"), dtype=torch.float64, device="cuda") for h in hs]
    return hs, phis, pds, tds


def test_batch_tst_parity_small(env):
    """Eight chain superblocks (m 100..300, L 16..48) and one of odd vector length: batched
    targets against the oracle (<= 1e-10) and bit for bit against each handle's own call."""
    torch, L = env
    say("batch small")
    pbs = I.batch_workloads(8, seed_offset=300, m_lo=100, m_hi=300) + [problem("chain8_m17_odd")]
    hs, phis, pds, tds = _batch_setup(torch, L, pbs, 500)
    tau, kdim = 0.05, 15
    b = L.Batch(hs)
    w, infos = b.batch_tst_targets(pds, tau, kdim, tds)
    for i, (pb, h) in enumerate(zip(pbs, hs)):
        n = h.n
        t = _host(tds[i])
        ys, wref, _ = K.tst_targets(lambda v: M.matvec_sector(pb, v), phis[i], tau, kdim)
        assert np.array_equal(w, wref)
        errs = [rel(t[2 * n * x:2 * n * (x + 1)], ys[x]) for x in range(4)]
        say("  problem", i, "n", n, "max rel err", max(errs), infos[i])
        assert max(errs) <= KR_TOL
        one = torch.empty_like(tds[i])
        _, inf1 = h.tst_targets(pds[i], tau, kdim, one)
        assert torch.equal(one, tds[i])
        assert inf1 == infos[i]
    b.destroy()
    for h in hs:
        h.destroy()


def test_batch64_matches_per_problem(env):
    """The 64-superblock workload (chains, m 100..1000): batched with graphs, batched without,
    and the per-problem loop agree bit for bit; a second call with other inputs and a call with
    another kdim (new graph) agree too."""
    torch, L = env
    say("batch 64")
    pbs = I.batch_workloads(64)
    hs, phis, pds, tds = _batch_setup(torch, L, pbs, 600)
    b = L.Batch(hs)
    for call, (kdim, tau) in enumerate([(15, 0.05), (15, 0.05), (10, 0.1)]):
        say("  call", call, kdim, tau)
        if call == 1:
            for p in pds:
                p.mul_(-0.5)
        b.set_graph(True)
        _, inf_g = b.batch_tst_targets(pds, tau, kdim, tds)
        ref = [torch.empty_like(t) for t in tds]
        for h, p, r in zip(hs, pds, ref):
            h.tst_targets(p, tau, kdim, r, info=False)
        torch.cuda.synchronize()
        for i in range(len(hs)):
            assert torch.equal(tds[i], ref[i]), i
        b.set_graph(False)
        for t in tds:
            t.fill_(float("nan"))
        _, inf_e = b.batch_tst_targets(pds, tau, kdim, tds)
        assert inf_e == inf_g
        for i in range(len(hs)):
            assert torch.equal(tds[i], ref[i]), i
        norms = [float(torch.linalg.vector_norm(t[:2 * h.n])) for t, h in zip(tds, hs)]
        assert all(abs(x - (1.0 if call == 0 else 0.5)) < 1e-12 for x in norms)
    b.destroy()
    for h in hs:
        h.destroy()


def test_graph_replays_match_eager(env):
    """A single handle with captured Lanczos iterations: several replays, with eager work and
    synchronisations between them, each equal to the eager result; chained Krylov steps and a
    new kdim (second graph) too."""
    torch, L = env
    say("graph replays")
    pb = problem("chain32_m400")
    h = L.dmrg_create(pb)
    n = h.n
    xs = [_dev(torch, I.random_psi(n, np.random.default_rng(I.SEED_BASE + 700 + i))) for i in range(3)]
    eager = []
    for x in xs:
        t = torch.empty(8 * n, dtype=torch.float64, device="cuda")
        h.tst_targets(x, 0.05, 15, t, info=False)
        eager.append(t)
    ye = torch.empty_like(xs[0])
    inf_e = h.krylov_expm(xs[0], ye, 0.1, 12, 3)
    h.set_graph(True)
    tmp = torch.empty_like(xs[0])
    for rep in range(2):
        for i, x in enumerate(xs):
            t = torch.full((8 * n,), float("nan"), dtype=torch.float64, device="cuda")
            h.tst_targets(x, 0.05, 15, t, info=False)
            h.matvec(x, tmp)                      # eager work between replays
            torch.cuda.synchronize()
            say("  replay", rep, i)
            assert torch.equal(t, eager[i])
    yg = torch.full_like(xs[0], float("nan"))
    inf_g = h.krylov_expm(xs[0], yg, 0.1, 12, 3)
    assert torch.equal(yg, ye) and inf_g == inf_e
    h.set_graph(False)
    h.destroy()


def test_batch_rejects_mixed_precisions(env):
    torch, L = env
    say("batch precision check")
    hs = [L.dmrg_create(problem("chain12_m30")), L.dmrg_create(problem("chain14_m25_off"))]
    b = L.Batch(hs)
    hs[1].set_precision(L.DMRG_FP32)
    pds = [torch.zeros(2 * h.n, dtype=torch.float64, device="cuda") for h in hs]
    tds = [torch.zeros(8 * h.n, dtype=torch.float64, device="cuda") for h in hs]
    with pytest.raises(L.DmrgError) as e:
        b.batch_tst_targets(pds, 0.1, 8, tds)
    assert "precision" in str(e.value)
    hs[1].set_precision(L.DMRG_FP64)
    b.batch_tst_targets(pds, 0.1, 8, tds)          # zero inputs: zero targets, no error
    assert all(torch.count_nonzero(t).item() == 0 for t in tds)
    b.destroy()
    for h in hs:
        h.destroy()


def test_precision_switch_after_fp64_runs(env):
    """Switching arithmetic on a handle that already ran FP64 products (and back) keeps every
    result finite and within its tolerance: the workspace is re-laid out for the element size."""
    torch, L = env
    say("precision switch")
    pb = problem("chain32_m400")
    h = L.dmrg_create(pb)
    x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 41))
    xd = _dev(torch, x)
    yd = torch.empty_like(xd)
    yref = M.matvec_sector(pb, x)
    for prec in (L.DMRG_FP64, L.DMRG_FP32, L.DMRG_BF16X3, L.DMRG_FP64, L.DMRG_BF16X6, L.DMRG_FP32):
        h.set_precision(prec)
        h.matvec(xd, yd)
        err = rel(_host(yd), yref)
        say("  prec", prec, err)
        assert err <= (MV_TOL if prec == L.DMRG_FP64 else MIXED_TOL[prec])
    h.destroy()


@pytest.mark.parametrize("prec", [0, 1, 2, 3], ids=["fp64", "fp32", "bf16x3", "bf16x6"])
def test_autotune_and_variants_agree(env, prec):
    """The autotuner keeps the faster family of each stage; every family gives the product to
    the arithmetic's tolerance on the headline ladder, and the Krylov step is unchanged beyond
    rounding."""
    torch, L = env
    say("autotune", prec)
    pb = problem("ladder16_m1000")
    h = L.dmrg_create(pb)
    h.set_precision(prec)
    t = h.autotune(reps=3)
    say("  ", t)
    assert all(t[k] > 0 for k in ("stage1_register", "stage1_lds", "stage2_register", "stage2_lds",
                                  "stage1_narrow", "stage2_narrow"))
    s1 = min([(t["stage1_register"], 0), (t["stage1_lds"], L.DMRG_GEMM_STAGE1_LDS),
              (t["stage1_narrow"], L.DMRG_GEMM_STAGE1_NARROW)], key=lambda p: p[0])[1]
    s2 = min([(t["stage2_register"], 0), (t["stage2_lds"], L.DMRG_GEMM_STAGE2_LDS),
              (t["stage2_narrow"], L.DMRG_GEMM_STAGE2_NARROW)], key=lambda p: p[0])[1]
    want = s1 | s2
    best = (min(t["stage1_register"], t["stage1_lds"], t["stage1_narrow"]) +
            min(t["stage2_register"], t["stage2_lds"], t["stage2_narrow"]))
    if prec == 0 and t["stage1_x"] > 0 and t["stage1_x"] + t["stage2_x"] < best:
        want = L.DMRG_GEMM_X
        best = t["stage1_x"] + t["stage2_x"]
    if prec == 0 and t["stage1_k"] > 0 and t["stage1_k"] + t["stage2_k"] < best:
        want = L.DMRG_GEMM_K
    assert t["variant"] == want
    x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 91))
    xd = _dev(torch, x)
    yref = M.matvec_sector(pb, x)
    tol = MV_TOL if prec == 0 else MIXED_TOL[prec]
    for v in (0, 1, 2, 3, 4, 6, 8, 9, 12, 16, 32):
        h.set_gemm(v)
        yd = torch.empty_like(xd)
        h.matvec(xd, yd)
        err = rel(_host(yd), yref)
        say("  variant", v, err)
        assert err <= tol
    for bad in (L.DMRG_GEMM_STAGE1_LDS | L.DMRG_GEMM_STAGE1_NARROW,
                L.DMRG_GEMM_STAGE2_LDS | L.DMRG_GEMM_STAGE2_NARROW, 64,
                L.DMRG_GEMM_X | L.DMRG_GEMM_STAGE1_NARROW, L.DMRG_GEMM_K | L.DMRG_GEMM_X,
                L.DMRG_GEMM_K | L.DMRG_GEMM_STAGE2_NARROW):
        with pytest.raises(L.DmrgError):
            h.set_gemm(bad)
    h.destroy()
