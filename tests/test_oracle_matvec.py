"""Pins of the oracle H_sb . psi (CPU only)."""
import numpy as np
import pytest

from oracle import ed
from oracle import matvec as M
from paper_1103_5391_amd import inputs as I
from tests.helpers import superblock_to_ed_perm


EXACT_CASES = [
    ("chain6_U4", 6, 4.0, (3, 3), None),
    ("chain8_U4", 8, 4.0, (4, 4), None),
    ("chain8_U4_3_4", 8, 4.0, (3, 4), None),
    ("ladder2x4_U10", 8, 10.0, (4, 4), I.ladder_bonds(4, 1.0, 0.5)),
    ("ladder2x4_U0_3_5", 8, 0.0, (3, 5), I.ladder_bonds(4, 1.0, 0.5)),
]


@pytest.mark.parametrize("name,L,U,target,bonds", EXACT_CASES)
def test_exact_blocks_equal_ed(name, L, U, target, bonds):
    """On untruncated blocks H_sb restricted to the target sector is the Hubbard Hamiltonian:
    equal to the bit-string ED matrix after a permutation of basis states (no signs, since
    both bases are normal-ordered in the same mode order)."""
    lat = I.chain_bonds(L) if bonds is None else bonds
    pb = I.exact_problem(L, U, target, bonds=lat)
    sec, H = ed.hamiltonian(L, lat, U, *target)
    perm = superblock_to_ed_perm(pb, sec)
    assert len(np.unique(perm)) == sec.dim
    Hed = H[perm][:, perm]
    lay, n = M.layout(pb)
    rng = np.random.default_rng(0)
    # random probes plus a random subset of unit vectors: a differing entry shows in both
    probes = [I.random_psi(n, rng) for _ in range(4)]
    for k in rng.choice(n, size=min(n, 40), replace=False):
        e = np.zeros(2 * n)
        e[k] = 1.0
        probes.append(e)
    for x in probes:
        y = M.matvec_sector(pb, x)
        z = x[:n] + 1j * x[n:]
        yz = Hed @ z
        assert np.max(np.abs(y - np.concatenate([yz.real, yz.imag]))) < 1e-12
    if n <= 400:
        assert np.max(np.abs(M.superblock_matrix(pb) - Hed.toarray())) < 1e-12


def _small_synthetic():
    return [
        I.synthetic_problem(12, 30, 4.0, I.chain_bonds(12), 7, name="chain12_m30"),
        I.synthetic_problem(12, 40, 8.0, I.ladder_bonds(6), 8, name="ladder2x6_m40"),
        I.synthetic_problem(14, 25, 2.0, I.chain_bonds(14), 9, name="chain14_m25_off",
                            target=(6, 8)),
    ]


@pytest.mark.parametrize("pb", _small_synthetic(), ids=lambda p: p.name)
def test_dense_definition_equals_sector_form(pb):
    lay, n = M.layout(pb)
    rng = np.random.default_rng(3)
    x = I.random_psi(n, rng)
    y1 = M.matvec_sector(pb, x)
    y2 = M.matvec_dense(pb, x)
    assert np.linalg.norm(y1 - y2) <= 1e-13 * np.linalg.norm(y2)


@pytest.mark.parametrize("pb", _small_synthetic(), ids=lambda p: p.name)
def test_hermitian(pb):
    lay, n = M.layout(pb)
    rng = np.random.default_rng(4)
    x, y = I.random_psi(n, rng), I.random_psi(n, rng)
    zx = x[:n] + 1j * x[n:]
    zy = y[:n] + 1j * y[n:]
    hx, hy = M.matvec_sector(pb, x), M.matvec_sector(pb, y)
    zhx, zhy = hx[:n] + 1j * hx[n:], hy[:n] + 1j * hy[n:]
    assert abs(np.vdot(zx, zhy) - np.vdot(zhx, zy)) < 1e-12 * np.linalg.norm(zhx)


def test_hopping_sign_gauge_invariance():
    """t -> -t on a bipartite lattice is the gauge c_j -> (-1)^j c_j: same spectrum."""
    L = 6
    pb1 = I.exact_problem(L, 4.0, (3, 3), bonds=I.chain_bonds(L, 1.0))
    pb2 = I.exact_problem(L, 4.0, (3, 3), bonds=I.chain_bonds(L, -1.0))
    w1 = np.linalg.eigvalsh(M.superblock_matrix(pb1))
    w2 = np.linalg.eigvalsh(M.superblock_matrix(pb2))
    assert np.allclose(w1, w2, atol=1e-10)


def test_linear_and_real():
    """H_sb is real: it maps the real and imaginary planes independently."""
    pb = _small_synthetic()[0]
    lay, n = M.layout(pb)
    rng = np.random.default_rng(5)
    x = I.random_psi(n, rng)
    xr = x.copy(); xr[n:] = 0
    xi = x.copy(); xi[:n] = 0
    y, yr, yi = M.matvec_sector(pb, x), M.matvec_sector(pb, xr), M.matvec_sector(pb, xi)
    assert np.allclose(y, yr + yi, atol=1e-13)
    assert np.all(yr[n:] == 0) and np.all(yi[:n] == 0)


def test_flop_count_chain8():
    """Algorithmic flop count of the exact L=8 chain superblock (fixed by the block dims)."""
    pb = I.exact_problem(8, 4.0, (4, 4))
    lay, n = M.layout(pb)
    # brute force: count multiply-adds of the naive per-block products in the cheaper order
    F = 0
    for (p, q, r, c, off) in lay:
        F += 2 * 2 * (r * r * c + r * c * c)
    assert M.flop_count(pb) > F and n == 4900
