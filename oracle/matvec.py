"""H_sb . psi on the CPU in FP64 (oracle, test only).

The superblock is S (x) E, S = left block + site s1, E = site s2 + right block.  A vector
psi of the target sector (N_up, N_dn) is a set of blocks Psi_p of shape dim_S(p) x dim_E(q),
q = target - p.  The flat layout is 2n doubles: all real parts, then all imaginary parts,
blocks in S-sector order, each block column-major.

The Hamiltonian (Sec. IV calls its cross terms the "Hamiltonian connections" between system
and environment) is

    H_sb = H_S (x) 1 + 1 (x) H_E
           - sum_bonds t sum_s [ c+_{a s} c_{b s} + c+_{b s} c_{a s} ],     a in S, b in E.

With S modes ordered before E modes, c_{b s} = P_S (x) c_b on the superblock, so
c+_a c_b = (C+_a P_S) (x) C_b and c+_b c_a = (P_S C_a) (x) C+_b, P_S the fermion parity of S.
Using (A (x) B) vec(X) = A X B^T for the (s, e)-indexed coefficient matrix X:

    Y = H_S X + X H_E^T - sum t [ (C+_a P_S) X C+_b + (P_S C+_a^T) X C+_b^T ].

Two structurally different implementations:
  matvec_dense   the line above, literally, on dense m_S x m_E matrices;
  matvec_sector  per symmetry block, with P_S folded into a sign of the source S sector.
Pins: on exact blocks the superblock matrix equals the bit-string ED Hamiltonian up to a
permutation of basis states (tests); Hermiticity; the two implementations agree.
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------------------------------------
# layout
# ------------------------------------------------------------------------------------------
def layout(pb):
    """Blocks of the target sector: list of (p, q, rows, cols, offset)."""
    out, off = [], 0
    Sqn, Eidx = pb.S.space.qn, pb.E.space.index
    for p in range(len(pb.S.space.dim)):
        q = Eidx.get((pb.target[0] - int(Sqn[p, 0]), pb.target[1] - int(Sqn[p, 1])))
        if q is None:
            continue
        r, c = int(pb.S.space.dim[p]), int(pb.E.space.dim[q])
        out.append((p, q, r, c, off))
        off += r * c
    return out, off


def unpack(pb, x: np.ndarray) -> dict:
    """Flat [Re | Im] vector -> {p: complex block}."""
    lay, n = layout(pb)
    assert x.shape == (2 * n,), (x.shape, n)
    z = x[:n] + 1j * x[n:]
    return {p: z[off:off + r * c].reshape(c, r).T for (p, q, r, c, off) in lay}


def pack(pb, blocks: dict) -> np.ndarray:
    lay, n = layout(pb)
    z = np.zeros(n, dtype=complex)
    for (p, q, r, c, off) in lay:
        z[off:off + r * c] = blocks[p].T.reshape(-1)
    return np.concatenate([z.real, z.imag])


# ------------------------------------------------------------------------------------------
# connection terms (hopping bonds)
# ------------------------------------------------------------------------------------------
def terms(pb, extra_terms=()):
    """Expand every bond into its four Kronecker terms coef * (A P_S) (x) B.

    c+_a c_b   -> coef -t, A = C+_a,   B = C_b = (C+_b)^T
    c+_b c_a   -> (P_S C_a) (x) C+_b = -(C_a P_S) (x) C+_b  (C_a flips the parity of S),
                  so coef +t, A = (C+_a)^T, B = C+_b.
    extra_terms: generic terms (coef, S-op, S transposed?, E-op, E transposed?, fermionic?).
    Each entry: (coef, S-op index, S transposed?, E-op index, E transposed?, fermionic?)."""
    out = []
    for bd in pb.bonds:
        for s in (0, 1):
            out.append((-bd.t, bd.opS[s], False, bd.opE[s], True, True))
            out.append((+bd.t, bd.opS[s], True, bd.opE[s], False, True))
    for t in extra_terms:
        out.append((float(t[0]), int(t[1]), bool(t[2]), int(t[3]), bool(t[4]), bool(t[5])))
    return out


def _op_block(space, op, src: int, transposed: bool):
    """Block of op (or op^T) leaving sector src: returns (dst, block) or None."""
    if not transposed:
        if src not in op.blocks:
            return None
        return space.shift(src, op.dq), op.blocks[src]
    pre = space.shift(src, (-op.dq[0], -op.dq[1]))
    if pre is None or pre not in op.blocks:
        return None
    return pre, op.blocks[pre].T


def matvec_sector(pb, x: np.ndarray, extra_terms=()) -> np.ndarray:
    """Y = H_sb X per symmetry block.  Source block p (E sector q) contributes
        Y_p           += H_S[p] X_p + X_p H_E[q]^T
        Y_{p'}        += coef * (-1)^{N(p)} * A[p' <- p] X_p B[q' <- q]^T   for each term
    (the sign only for fermionic terms)."""
    X = unpack(pb, x)
    lay, n = layout(pb)
    qof = {p: q for (p, q, r, c, off) in lay}
    Y = {p: np.zeros_like(X[p]) for p in X}
    for p, Xp in X.items():
        q = qof[p]
        Y[p] += pb.S.H[p] @ Xp + Xp @ pb.E.H[q].T
    for (coef, a, ta, b, tb, ferm) in terms(pb, extra_terms):
        for p, Xp in X.items():
            A = _op_block(pb.S.space, pb.S.ops[a], p, ta)
            B = _op_block(pb.E.space, pb.E.ops[b], qof[p], tb)
            if A is None or B is None:
                continue
            p2, Ab = A
            q2, Bb = B
            if p2 not in Y:
                continue
            assert qof[p2] == q2
            sign = pb.S.space.parity(p) if ferm else 1.0
            Y[p2] += (coef * sign) * (Ab @ Xp @ Bb.T)
    return pack(pb, Y)


# ------------------------------------------------------------------------------------------
# dense-halves definition
# ------------------------------------------------------------------------------------------
def _offsets(dims):
    return np.concatenate([[0], np.cumsum(dims)]).astype(int)


def dense_half(space, H):
    off = _offsets(space.dim)
    M = np.zeros((off[-1], off[-1]))
    for p, h in enumerate(H):
        M[off[p]:off[p + 1], off[p]:off[p + 1]] = h
    return M


def dense_op(space, op):
    off = _offsets(space.dim)
    M = np.zeros((off[-1], off[-1]))
    for p, b in op.blocks.items():
        p2 = space.shift(p, op.dq)
        M[off[p2]:off[p2 + 1], off[p]:off[p + 1]] = b
    return M


def dense_parity(space):
    return np.concatenate([np.full(int(d), space.parity(p)) for p, d in enumerate(space.dim)])


def matvec_dense(pb, x: np.ndarray) -> np.ndarray:
    """Y = H_S X + X H_E^T - sum_bonds t sum_s [(C+_a P_S) X C+_b + (P_S C+_a^T) X C+_b^T]
    on dense m_S x m_E matrices, X zero outside the target-sector blocks."""
    lay, n = layout(pb)
    offS, offE = _offsets(pb.S.space.dim), _offsets(pb.E.space.dim)
    Xb = unpack(pb, x)
    X = np.zeros((offS[-1], offE[-1]), dtype=complex)
    for (p, q, r, c, off) in lay:
        X[offS[p]:offS[p + 1], offE[q]:offE[q + 1]] = Xb[p]
    HS, HE = dense_half(pb.S.space, pb.S.H), dense_half(pb.E.space, pb.E.H)
    PS = np.diag(dense_parity(pb.S.space))
    Y = HS @ X + X @ HE.T
    for bd in pb.bonds:
        for s in (0, 1):
            Ca = dense_op(pb.S.space, pb.S.ops[bd.opS[s]])
            Cb = dense_op(pb.E.space, pb.E.ops[bd.opE[s]])
            Y -= bd.t * ((Ca @ PS) @ X @ Cb + (PS @ Ca.T) @ X @ Cb.T)
    out = {p: Y[offS[p]:offS[p + 1], offE[q]:offE[q + 1]] for (p, q, r, c, off) in lay}
    return pack(pb, out)


def superblock_matrix(pb, matvec=matvec_sector) -> np.ndarray:
    """Dense real matrix of H_sb restricted to the target sector (columns = H e_k), for tiny
    problems only."""
    lay, n = layout(pb)
    M = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(2 * n)
        e[k] = 1.0
        M[:, k] = matvec(pb, e)[:n]
    return M


def flop_count(pb) -> int:
    """Algorithmic flops of one H_sb . psi for complex psi with real operators, cheaper
    contraction order per connection term, blocks never densified or padded, terms whose
    operator block is exactly zero not counted (they contribute nothing):
    F = 2 * sum_blocks [2 d_p^2 e_q + 2 d_p e_q^2
                        + sum_nonzero_terms 2 min(d' d e + d' e e', d e e' + d' d e')]."""
    lay, n = layout(pb)
    qof = {p: q for (p, q, r, c, off) in lay}
    dS, dE = pb.S.space.dim, pb.E.space.dim
    F = 0
    for (p, q, r, c, off) in lay:
        F += 2 * (2 * r * r * c + 2 * r * c * c)
    for (coef, a, ta, b, tb, ferm) in terms(pb):
        for (p, q, r, c, off) in lay:
            A = _op_block(pb.S.space, pb.S.ops[a], p, ta)
            B = _op_block(pb.E.space, pb.E.ops[b], q, tb)
            if A is None or B is None or A[0] not in qof or qof[A[0]] != B[0]:
                continue
            if not (np.any(A[1]) and np.any(B[1])):
                continue
            r2, c2 = int(dS[A[0]]), int(dE[B[0]])
            F += 2 * 2 * min(r2 * r * c + r2 * c * c2, r * c * c2 + r2 * r * c2)
    return F
