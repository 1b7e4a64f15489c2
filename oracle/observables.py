"""Local operators on the superblock, in FP64 (oracle, test infrastructure only).

Sec. II.B, Eq. (b): the state phi is built from the ground state by local operators B acting on
sites of the superblock; Sec. III.B measures the density n_p and the double occupation
n_p,up n_p,dn.  With the system's modes before the environment's, a product O_S O_E of an
operator on each half acts on |alpha>|beta> as (O_S P_S) (x) O_E when O_E is odd (it passes the
system's creation operators), P_S the fermion parity of the system state.  A term is
(coef, A, B, fermionic): coef (A P_S^fermionic) (x) B, A or B None for the identity, so on the
block matrix Psi (system rows, environment columns) it is coef A Psi B^T with the sign of every
source system sector.

Pins (tests): on exact blocks, every one- and two-site operator (c+, c, n, n_up n_dn, the
holon and doublon factors, on either half and across them) equals the operator applied to the
Fock-space vector with Jordan-Wigner signs; the holon-doublon state of the Fig. 3 ladder built
through the superblock gives the paper's t = 0 densities and double occupations.
"""
from __future__ import annotations

import numpy as np

from oracle import matvec as M


def apply_terms(pb_src, pb_dst, terms, x: np.ndarray) -> np.ndarray:
    """sum_t coef_t (A_t P_S^f_t (x) B_t) x, from pb_src's layout to pb_dst's (flat [Re | Im])."""
    S, E = pb_src.S.space, pb_src.E.space
    blocks = M.unpack(pb_src, x)
    lay_src, _ = M.layout(pb_src)
    lay_dst, _ = M.layout(pb_dst)
    out = {p: np.zeros((r, c), dtype=complex) for (p, q, r, c, off) in lay_dst}
    cols = {p: q for (p, q, r, c, off) in lay_dst}
    for (coef, A, B, fermionic) in terms:
        for (p, q, r, c, off) in lay_src:
            p2 = p if A is None else S.shift(p, A.dq)
            q2 = q if B is None else E.shift(q, B.dq)
            if p2 is None or q2 is None or (A is not None and p not in A.blocks) or \
                    (B is not None and q not in B.blocks):
                continue
            if cols.get(p2) != q2:
                continue
            blk = blocks[p]
            if B is not None:
                blk = blk @ B.blocks[q].T
            if A is not None:
                blk = A.blocks[p] @ blk
            sign = S.parity(p) if fermionic else 1.0
            out[p2] += coef * sign * blk
    return M.pack(pb_dst, out)


def expect(pb, terms, x: np.ndarray) -> complex:
    """<x| sum of terms |x> for terms that keep the sector."""
    n = x.size // 2
    y = apply_terms(pb, pb, terms, x)
    return complex(np.vdot(x[:n] + 1j * x[n:], y[:n] + 1j * y[n:]))

