"""Exact diagonalisation of the Hubbard model in a bit-string Fock basis (oracle, test only).

H = -sum_<ij> sum_s t_ij (c+_is c_js + h.c.) + U sum_i n_i,up n_i,dn   (model of Sec. III.B;
the paper writes the hopping with a plus sign and symmetric t_ij: on the bipartite chain and
ladder the two signs are related by c_j -> (-1)^j c_j, so densities do not depend on it).

Fermion mode of (site i, spin s) is bit 2*i + s (s = 0 up, 1 down); basis states are
normal-ordered products of creation operators in increasing mode order.  Written without
reference to the block construction used by the input generator, so that agreement of the
two (up to a permutation of basis states) checks the fermion signs of both.

Pins: at U = 0 the many-body spectrum is sums of the tight-binding levels (closed_forms);
the holon-doublon t = 0 identities of App. B; the double occupation identities of Sec. III.B.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp


def _states_with(L: int, nup: int, ndn: int) -> np.ndarray:
    ups = [sum(1 << (2 * i) for i in c) for c in combinations(range(L), nup)]
    dns = [sum(1 << (2 * i + 1) for i in c) for c in combinations(range(L), ndn)]
    s = np.array([u | d for u in ups for d in dns], dtype=np.int64)
    return np.sort(s)


class Sector:
    """Fock states of L sites with fixed (N_up, N_dn), sorted by integer value."""

    def __init__(self, L: int, nup: int, ndn: int):
        self.L, self.nup, self.ndn = L, nup, ndn
        self.states = _states_with(L, nup, ndn)
        self.dim = len(self.states)

    def index_of(self, s: np.ndarray) -> np.ndarray:
        idx = np.searchsorted(self.states, s)
        assert np.all(self.states[np.minimum(idx, self.dim - 1)] == s)
        return idx


def _popcount(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64)
    c = np.zeros(x.shape, dtype=np.int64)
    while np.any(x):
        c += (x & np.uint64(1)).astype(np.int64)
        x = x >> np.uint64(1)
    return c


def _between_mask(a: int, b: int) -> int:
    lo, hi = min(a, b), max(a, b)
    return ((1 << hi) - 1) & ~((1 << (lo + 1)) - 1)


def hop_matrix(sec: Sector, a: int, b: int):
    """Sparse matrix of c+_a c_b (modes a != b) on one sector (it stays in the sector when a and
    b carry the same spin)."""
    s = sec.states
    ok = ((s >> b) & 1).astype(bool) & ~((s >> a) & 1).astype(bool)
    src = np.nonzero(ok)[0]
    s0 = s[src]
    s1 = s0 ^ (1 << b) ^ (1 << a)
    sign = 1.0 - 2.0 * (_popcount(s0 & _between_mask(a, b)) % 2)
    dst = sec.index_of(s1)
    return sp.csr_matrix((sign, (dst, src)), shape=(sec.dim, sec.dim))


def hamiltonian(L: int, bonds, U: float, nup: int, ndn: int):
    """Sparse Hubbard Hamiltonian on the (nup, ndn) sector; bonds = [(i, j, t), ...]."""
    sec = Sector(L, nup, ndn)
    H = sp.csr_matrix((sec.dim, sec.dim))
    for (i, j, t) in bonds:
        for spin in (0, 1):
            a, b = 2 * i + spin, 2 * j + spin
            h = hop_matrix(sec, a, b)
            H = H - t * (h + h.T)
    s = sec.states
    docc = np.zeros(sec.dim)
    for i in range(L):
        docc += (((s >> (2 * i)) & 1) & ((s >> (2 * i + 1)) & 1)).astype(float)
    H = H + sp.diags(U * docc)
    return sec, H.tocsr()


def number(sec: Sector, site: int, spin: int) -> np.ndarray:
    """Diagonal of n_{site,spin} on a sector."""
    return ((sec.states >> (2 * site + spin)) & 1).astype(float)


def annihilate(src: Sector, dst: Sector, mode: int):
    """Sparse matrix of c_mode from sector src to sector dst (one fewer particle of that spin)."""
    s = src.states
    ok = ((s >> mode) & 1).astype(bool)
    cols = np.nonzero(ok)[0]
    s0 = s[cols]
    sign = 1.0 - 2.0 * (_popcount(s0 & ((1 << mode) - 1)) % 2)
    rows = dst.index_of(s0 ^ (1 << mode))
    return sp.csr_matrix((sign, (rows, cols)), shape=(dst.dim, src.dim))


def create(src: Sector, dst: Sector, mode: int):
    """Sparse matrix of c+_mode from sector src to sector dst."""
    return annihilate(dst, src, mode).T.tocsr()


def ground_state(H) -> tuple:
    """Lowest eigenpair of a sparse symmetric matrix (dense for small dimensions)."""
    n = H.shape[0]
    if n <= 2000:
        w, v = np.linalg.eigh(H.toarray())
        return w[0], v[:, 0]
    from scipy.sparse.linalg import eigsh
    w, v = eigsh(H, k=1, which="SA", tol=1e-14, ncv=40)
    return w[0], v[:, 0]
