"""Pins of the ED and of the closed forms (CPU only)."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import closed_forms as CF
from oracle import ed
from paper_1103_5391_amd import inputs as I

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _free_spectrum(eps, nup, ndn):
    ups = [sum(c) for c in itertools.combinations(eps, nup)]
    dns = [sum(c) for c in itertools.combinations(eps, ndn)]
    return np.sort(np.add.outer(ups, dns).reshape(-1))


def test_chain_closed_form_matches_hopping_eigh():
    for L in (4, 7, 12):
        E, U = CF.chain_levels(L)
        h = CF.hopping_matrix(L, I.chain_bonds(L))
        w, v = np.linalg.eigh(h)
        assert np.allclose(E, w, atol=1e-13)
        # modes are orthonormal eigenvectors
        assert np.allclose(h @ U, U * E[None, :], atol=1e-13)
        assert np.allclose(U.T @ U, np.eye(L), atol=1e-13)


@pytest.mark.parametrize("lattice", ["chain6", "ladder2x3"])
def test_ed_free_spectrum_is_sum_of_levels(lattice):
    """At U = 0 the many-body levels are sums of single-particle levels; a wrong Jordan-Wigner
    sign on hops that pass other modes breaks this."""
    if lattice == "chain6":
        L, bonds = 6, I.chain_bonds(6)
    else:
        L, bonds = 6, I.ladder_bonds(3, 1.0, 0.5)
    eps = np.linalg.eigvalsh(CF.hopping_matrix(L, bonds))
    for (nu, nd) in [(3, 3), (2, 3), (1, 4)]:
        sec, H = ed.hamiltonian(L, bonds, 0.0, nu, nd)
        w = np.linalg.eigvalsh(H.toarray())
        assert np.allclose(w, _free_spectrum(eps, nu, nd), atol=1e-10)


def test_ed_ground_energy_free_chain8():
    E, U = CF.chain_levels(8)
    sec, H = ed.hamiltonian(8, I.chain_bonds(8), 0.0, 4, 4)
    e0, _ = ed.ground_state(H)
    assert abs(e0 - CF.free_ground_energy(E, 4, 4)) < 1e-10


def _holon_doublon(L, bonds, U, i, j):
    """phi = sum_{s,s'} c_{i s}(1 - n_{i sbar}) c+_{j s'} n_{j s'bar} |psi>, per sector."""
    sec0, H0 = ed.hamiltonian(L, bonds, U, L // 2, L // 2)
    _, gs = ed.ground_state(H0)
    parts = {}
    for s, s2 in itertools.product((0, 1), (0, 1)):
        v = gs * ed.number(sec0, j, 1 - s2)
        d1 = [L // 2, L // 2]
        d1[s2] += 1
        sec1 = ed.Sector(L, *d1)
        v = ed.create(sec0, sec1, 2 * j + s2) @ v
        v = v * (1.0 - ed.number(sec1, i, 1 - s))
        d2 = list(d1)
        d2[s] -= 1
        sec2 = ed.Sector(L, *d2)
        v = ed.annihilate(sec1, sec2, 2 * i + s) @ v
        key = tuple(d2)
        if key in parts:
            parts[key] = (sec2, parts[key][1] + v)
        else:
            parts[key] = (sec2, v)
    return parts


@pytest.mark.parametrize("U", GOLDEN["holon_doublon_density_t0"]["U_values"])
def test_holon_doublon_t0_values(U):
    """Eq. (nd) and Sec. III.B.2 on the Fig. 3 ladder: density 0 / 2 / 1 and double occupation
    0 / 1 at t = 0, for U = 0 and U = 10 (paper values in tests/golden)."""
    g = GOLDEN["holon_doublon_density_t0"]
    gd = GOLDEN["double_occupation_t0"]
    L, i, j = 8, 2, 4
    bonds = I.ladder_bonds(4, 1.0, 0.5)
    parts = _holon_doublon(L, bonds, U, i, j)
    norm = sum(float(np.vdot(v, v).real) for (_, v) in parts.values())
    assert norm > 1e-3
    dens = np.zeros(L)
    docc = np.zeros(L)
    for (sec, v) in parts.values():
        w = np.abs(v) ** 2
        for p in range(L):
            dens[p] += np.sum(w * (ed.number(sec, p, 0) + ed.number(sec, p, 1)))
            docc[p] += np.sum(w * ed.number(sec, p, 0) * ed.number(sec, p, 1))
    dens /= norm
    docc /= norm
    expect = np.full(L, g["other_site_value"])
    expect[i] = g["holon_site_value"]
    expect[j] = g["doublon_site_value"]
    assert np.allclose(dens, expect, atol=1e-9), dens
    assert abs(docc[j] - gd["doublon_site_value"]) < 1e-9
    assert abs(docc[i] - gd["holon_site_value"]) < 1e-9


def test_onesite_excitation_closed_form_at_t0_matches_ed():
    """App. A at t = 0 against the ED: X_ij(0) = <psi| c+_i n_j c_i |psi>, and X_ii(0) = 0."""
    L = 8
    E, U = CF.chain_levels(L)
    sec0, H0 = ed.hamiltonian(L, I.chain_bonds(L), 0.0, 4, 4)
    _, gs = ed.ground_state(H0)
    sec1 = ed.Sector(L, 3, 4)
    i = 3
    phi = ed.annihilate(sec0, sec1, 2 * i) @ gs
    for j in range(L):
        x_ed = float(np.sum(np.abs(phi) ** 2 * ed.number(sec1, j, 0)))
        x_cf = CF.onesite_excitation(E, U, 4, i, j, 0.0)[0]
        assert abs(x_ed - x_cf) < 1e-10
    assert abs(CF.onesite_excitation(E, U, 4, i, i, 0.0)[0] - GOLDEN["onesite_excitation_t0"]["X_ii_t0"]) < 1e-12
