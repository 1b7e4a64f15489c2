"""Wave-function transformation for a move of the centre one site to the right, in FP64
(oracle, test infrastructure only).

Sec. II.B: as the sweep moves the central sites, the targets are carried from one superblock
basis to the next by the wave-function transformation.  For
    S (x) E = (A (x) s1) (x) (s2 (x) R)   ->   S' (x) E' = (A' (x) s2) (x) (s3 (x) R'')
(A' the kept states of S, R = W^T-image of s3 (x) R''), the transformed vector is
    psi'[(alpha', a), gamma] = sum_{alpha, beta} conj(U[alpha, alpha']) psi[alpha, (a, beta)] W[gamma, beta]
with U the kept eigenvectors of the density matrix of S (as columns) and W_r the states of R
sector r written in the product basis of s3 (x) R''.  The modes of s2 follow those of A' in both
orderings, and every basis is normal-ordered, so the regrouping carries no sign.

Pins (tests): on exact blocks with every state kept, the Fock-space vector of psi equals that of
psi' with U undone (a complex unitary, so a missing conjugate or a transposed factor fails);
with truncation, psi' with U undone is (P (x) 1) psi, P the projector on the kept states, and
|psi'|^2 = 1 - the discarded weight of psi's own density matrix; the isometries W keep norms.
"""
from __future__ import annotations

import numpy as np

from oracle import matvec as M


def wft_right(pb, mv, U: dict, x: np.ndarray) -> np.ndarray:
    """psi' (flat [Re | Im] in the layout of mv.layout) for psi = x on pb.
    U: {S sector p: complex d_p x d_p matrix whose first mv.kept[b] columns are kept}."""
    blocks = M.unpack(pb, x)
    lay, _ = M.layout(pb)
    new_lay, _ = M.layout(mv.layout)
    out = {pp: np.zeros((r, c), dtype=complex) for (pp, qq, r, c, off) in new_lay}
    col_sector = {pp: qq for (pp, qq, r, c, off) in new_lay}
    for b, (p, q, r, c, off) in enumerate(lay):
        k = mv.kept[b]
        if k == 0:
            continue
        phi = U[p][:, :k].conj().T @ blocks[p]                  # kept states x E columns
        for (qq, a, rr, coff) in mv.esub:
            if qq != q:
                continue
            pp, roff = mv.ssub[(b, a)]
            j = mv.r_to_enew[rr]
            assert col_sector[pp] == j
            out[pp][roff:roff + k, :] += phi[:, coff:coff + mv.r_dim[rr]] @ mv.W[rr].T
    return M.pack(mv.layout, out)


def undo_system(pb, mv, U: dict, xnew: np.ndarray) -> dict:
    """(U_kept (x) 1) applied to the rows of psi': per new block p', the rows of sub-block (b, a)
    mapped back to the d_b states of S.  Returns {(b, a, j): complex d_b x d_E'(j)} (test aid)."""
    blocks = M.unpack(mv.layout, xnew)
    lay, _ = M.layout(pb)
    new_lay, _ = M.layout(mv.layout)
    col_sector = {pp: qq for (pp, qq, r, c, off) in new_lay}
    out = {}
    for (b, a), (pp, roff) in mv.ssub.items():
        if pp not in blocks:
            continue
        p = lay[b][0]
        k = mv.kept[b]
        out[(b, a, col_sector[pp])] = U[p][:, :k] @ blocks[pp][roff:roff + k, :]
    return out
