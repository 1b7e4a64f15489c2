"""Pins of the oracle's local operators (oracle/observables.py) against the Fock-space
operators of the exact diagonalisation (Jordan-Wigner signs on bit strings), and of the
holon-doublon state built through the superblock against the paper's t = 0 values."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import ed
from oracle import krylov as K
from oracle import matvec as M
from oracle import observables as O
from paper_1103_5391_amd import inputs as I

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
KINDS = ["cdag_0", "cdag_1", "c_0", "c_1", "n_0", "n_1", "n", "nn", "holon_0", "holon_1",
         "doublon_0", "doublon_1"]
ODD = {"cdag_0", "cdag_1", "c_0", "c_1", "holon_0", "holon_1", "doublon_0", "doublon_1"}
DQ = {"cdag_0": (1, 0), "cdag_1": (0, 1), "c_0": (-1, 0), "c_1": (0, -1), "holon_0": (-1, 0),
      "holon_1": (0, -1), "doublon_0": (1, 0), "doublon_1": (0, 1)}


def to_fock(pb, x):
    """Superblock vector of an exact problem as the ED vector of its sector."""
    nS = len(pb.Sblk.sites)
    sec = ed.Sector(pb.L, *pb.target)
    v = np.zeros(sec.dim, dtype=complex)
    for p, blk in M.unpack(pb, x).items():
        q = pb.E.space.index[(pb.target[0] - int(pb.S.space.qn[p, 0]), pb.target[1] - int(pb.S.space.qn[p, 1]))]
        ms, me = pb.S.space.occ[p], pb.E.space.occ[q]
        masks = (ms[:, None] | (me[None, :] << (2 * nS))).reshape(-1)
        v[sec.index_of(masks)] = blk.reshape(-1)
    return sec, v


def ed_apply(kind, site, src, v):
    """The operator on a Fock vector; returns (destination sector, vector)."""
    dq = DQ.get(kind, (0, 0))
    dst = ed.Sector(src.L, src.nup + dq[0], src.ndn + dq[1]) if dq != (0, 0) else src
    if kind.startswith("n"):
        if kind == "n":
            return src, v * (ed.number(src, site, 0) + ed.number(src, site, 1))
        if kind == "nn":
            return src, v * ed.number(src, site, 0) * ed.number(src, site, 1)
        return src, v * ed.number(src, site, int(kind[-1]))
    s = int(kind[-1])
    mode = 2 * site + s
    if kind.startswith("cdag"):
        return dst, ed.create(src, dst, mode) @ v
    if kind.startswith("c_"):
        return dst, ed.annihilate(src, dst, mode) @ v
    if kind.startswith("holon"):
        return dst, ed.annihilate(src, dst, mode) @ (v * (1.0 - ed.number(src, site, 1 - s)))
    return dst, ed.create(src, dst, mode) @ (v * ed.number(src, site, 1 - s))


def _term_for(pb, site, kind):
    """(term, dq) of one site operator on the half that carries the site."""
    if site in pb.Sblk.sites:
        return (1.0, I.site_ops(pb.Sblk, site)[kind], None, 0)
    return (1.0, None, I.site_ops(pb.Eblk, site)[kind], 1 if kind in ODD else 0)


@pytest.mark.parametrize("L,target,bonds", [(6, (3, 3), None), (8, (4, 4), "ladder")])
def test_single_site_operators_match_fock_space(L, target, bonds):
    bl = I.ladder_bonds(L // 2, 1.0, 0.5) if bonds == "ladder" else None
    pb = I.exact_problem(L, 4.0, target, bonds=bl)
    lay, n = M.layout(pb)
    rng = np.random.default_rng(I.SEED_BASE + 601 + L)
    x = I.random_psi(n, rng)
    sec, v = to_fock(pb, x)
    checked = 0
    for site in range(L):
        for kind in KINDS:
            term = _term_for(pb, site, kind)
            dq = DQ.get(kind, (0, 0))
            tgt = (target[0] + dq[0], target[1] + dq[1])
            pd = I.with_ops(pb, target=tgt)[0]
            y = O.apply_terms(pb, pd, [term], x)
            dsec, w = ed_apply(kind, site, sec, v)
            _, wy = to_fock(pd, y)
            assert np.max(np.abs(wy - w)) < 1e-13, (site, kind)
            checked += 1
    assert checked == L * len(KINDS)


@pytest.mark.parametrize("i,j", [(1, 5), (5, 1), (0, 2), (6, 7), (3, 4)])
def test_holon_doublon_pair_matches_fock_space(i, j):
    """c_{i s}(1 - n_{i sbar}) c+_{j s'} n_{j s'bar} on the 2x4 ladder, for the sites on either
    half or across (the parity of the system between them)."""
    L = 8
    pb = I.exact_problem(L, 10.0, (4, 4), bonds=I.ladder_bonds(4, 1.0, 0.5))
    lay, n = M.layout(pb)
    rng = np.random.default_rng(I.SEED_BASE + 611 + 10 * i + j)
    x = I.random_psi(n, rng)
    sec, v = to_fock(pb, x)
    for s, s2 in itertools.product((0, 1), (0, 1)):
        hol, dbl = f"holon_{s}", f"doublon_{s2}"
        iS, jS = i in pb.Sblk.sites, j in pb.Sblk.sites
        if iS and jS:
            ops = I.site_ops(pb.Sblk, i)[hol], I.site_ops(pb.Sblk, j)[dbl]
            term = (1.0, I._op_mul(ops[0], ops[1], pb.S.space), None, 0)
        elif not iS and not jS:
            ops = I.site_ops(pb.Eblk, i)[hol], I.site_ops(pb.Eblk, j)[dbl]
            term = (1.0, None, I._op_mul(ops[0], ops[1], pb.E.space), 0)
        elif iS:        # c_i on S (left), c+_j on E (odd, passes S)
            term = (1.0, I.site_ops(pb.Sblk, i)[hol], I.site_ops(pb.Eblk, j)[dbl], 1)
        else:           # c_i on E applied after c+_j on S: c_i c+_j = -c+_j c_i
            term = (-1.0, I.site_ops(pb.Sblk, j)[dbl], I.site_ops(pb.Eblk, i)[hol], 1)
        dq = (DQ[dbl][0] + DQ[hol][0], DQ[dbl][1] + DQ[hol][1])
        pd = I.with_ops(pb, target=(4 + dq[0], 4 + dq[1]))[0]
        y = O.apply_terms(pb, pd, [term], x)
        s1, w1 = ed_apply(dbl, j, sec, v)
        s2_, w2 = ed_apply(hol, i, s1, w1)
        _, wy = to_fock(pd, y)
        assert np.max(np.abs(wy - w2)) < 1e-13, (s, s2)


@pytest.mark.parametrize("U", GOLDEN["holon_doublon_density_t0"]["U_values"])
def test_holon_doublon_t0_values_through_the_superblock(U):
    """Fig. 3/5 ladder: the superblock ground state (restarted Lanczos of the oracle, not the
    ED), the holon-doublon operator applied as superblock terms into its three sectors, and
    the densities and double occupations measured as superblock expectations."""
    g, gd = GOLDEN["holon_doublon_density_t0"], GOLDEN["double_occupation_t0"]
    L, i, j = 8, 2, 4
    pb = I.exact_problem(L, U, (4, 4), bonds=I.ladder_bonds(4, 1.0, 0.5))
    lay, n = M.layout(pb)
    x0 = I.random_psi(n, np.random.default_rng(I.SEED_BASE + 621), complex_=False)
    psi, info = K.ground_state(lambda v: M.matvec_sector(pb, v), x0, 40, 40, 1e-12)
    assert info.residual_est <= 1e-10
    parts = {}
    for s, s2 in itertools.product((0, 1), (0, 1)):
        term = (1.0, I.site_ops(pb.Sblk, i)[f"holon_{s}"], I.site_ops(pb.Eblk, j)[f"doublon_{s2}"], 1)
        dq = (DQ[f"doublon_{s2}"][0] + DQ[f"holon_{s}"][0], DQ[f"doublon_{s2}"][1] + DQ[f"holon_{s}"][1])
        tgt = (4 + dq[0], 4 + dq[1])
        pd = I.with_ops(pb, target=tgt)[0]
        y = O.apply_terms(pb, pd, [term], psi)
        parts[tgt] = (pd, parts[tgt][1] + y) if tgt in parts else (pd, y)
    assert sorted(parts) == [(3, 5), (4, 4), (5, 3)]
    norm = sum(float(np.dot(y, y)) for (_, y) in parts.values())
    dens, docc = np.zeros(L), np.zeros(L)
    for (pd, y) in parts.values():
        for p in range(L):
            dens[p] += O.expect(pd, [_term_for(pd, p, "n")], y).real
            docc[p] += O.expect(pd, [_term_for(pd, p, "nn")], y).real
    dens /= norm
    docc /= norm
    expect = np.full(L, g["other_site_value"])
    expect[i], expect[j] = g["holon_site_value"], g["doublon_site_value"]
    assert np.allclose(dens, expect, atol=1e-9), dens
    assert abs(docc[j] - gd["doublon_site_value"]) < 1e-9
    assert abs(docc[i] - gd["holon_site_value"]) < 1e-9
