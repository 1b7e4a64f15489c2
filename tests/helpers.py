"""Shared test helpers: mapping between the superblock product basis of exact blocks and the
bit-string basis of the ED, and measurement of site densities on ED vectors."""
from __future__ import annotations

import numpy as np

from oracle import ed
from oracle import matvec as M


def superblock_to_ed_perm(pb, sec: "ed.Sector") -> np.ndarray:
    """perm[k] = ED index of the k-th superblock basis vector (flat block layout); exact blocks
    only (the halves carry occupation masks)."""
    lay, n = M.layout(pb)
    nS = len(pb.S.sites)
    perm = np.zeros(n, dtype=np.int64)
    for (p, q, r, c, off) in lay:
        occS = np.asarray(pb.S.space.occ[p], dtype=np.int64)
        occE = np.asarray(pb.E.space.occ[q], dtype=np.int64)
        masks = (occS[:, None] | (occE[None, :] << (2 * nS)))      # r x c
        perm[off:off + r * c] = sec.index_of(masks.T.reshape(-1))
    return perm


def ed_to_flat(z_ed: np.ndarray, perm: np.ndarray) -> np.ndarray:
    z = z_ed[perm]
    return np.concatenate([z.real, z.imag]).astype(float)


def flat_to_ed(x: np.ndarray, perm: np.ndarray, dim: int) -> np.ndarray:
    n = x.shape[0] // 2
    out = np.zeros(dim, dtype=complex)
    out[perm] = x[:n] + 1j * x[n:]
    return out


def density(sec, z: np.ndarray, site: int, spin: int) -> float:
    return float(np.sum(np.abs(z) ** 2 * ed.number(sec, site, spin)))


def double_occ(sec, z: np.ndarray, site: int) -> float:
    return float(np.sum(np.abs(z) ** 2 * ed.number(sec, site, 0) * ed.number(sec, site, 1)))


_CASES = {}


def exact_case(L, U, target, bonds=None):
    """(problem, ED sector, sparse H_sb in the superblock ordering, perm) for exact blocks;
    the sparse matrix is the ED Hamiltonian permuted, which test_oracle_matvec pins equal to
    the oracle's H_sb."""
    key = (L, U, tuple(target), None if bonds is None else tuple(bonds))
    if key not in _CASES:
        from paper_1103_5391_amd import inputs as I
        lat = I.chain_bonds(L) if bonds is None else bonds
        pb = I.exact_problem(L, U, target, bonds=lat)
        sec, H = ed.hamiltonian(L, lat, U, *target)
        perm = superblock_to_ed_perm(pb, sec)
        Hsb = H[perm][:, perm].tocsr()
        _CASES[key] = (pb, sec, Hsb, perm)
    return _CASES[key]


def expm_flat(Hsp, x, tau):
    """exp(-i tau H) x for a sparse real symmetric H (scipy's expm_multiply), flat layout."""
    from scipy.sparse.linalg import expm_multiply
    n = Hsp.shape[0]
    z = x[:n] + 1j * x[n:]
    y = expm_multiply(-1j * tau * Hsp, z)
    return np.concatenate([y.real, y.imag])
