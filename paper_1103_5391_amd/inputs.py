"""Seeded inputs for the superblock Hamiltonian H_sb = H_S x 1 + 1 x H_E + connection terms.

This module only *constructs* what both the HIP library and the CPU oracle consume:
sector tables, block operators of the two superblock halves, the list of hopping bonds
that cross between the halves, and random vectors.  It contains none of the method's
arithmetic: no product H_sb.psi, no Lanczos, no exponential.

Conventions (the paper leaves them open; it only says operator reordering costs at most a
sign, Sec. II.B):
  * fermion modes are ordered along the DMRG path (left-block sites, s1, s2, right-block
    sites) with spin up before spin down on each site;
  * every basis is a normal-ordered Fock basis of its own modes, so the product basis of the
    two halves is the normal-ordered Fock basis of the whole lattice;
  * site basis |0>, |dn>, |up>, |updn> = c+_up c+_dn |0>, sorted by (N_up, N_dn);
  * the Hubbard model is H = -sum_<ij>,s t_ij (c+_is c_js + h.c.) + U sum_i n_i,up n_i,dn
    (Sec. III.B); ladders are labelled rung-major, sites 2r and 2r+1 forming rung r.

Sectors are labelled by (N_up, N_dn) and sorted lexicographically.  A block operator that
changes the quantum numbers by dq stores, for every source sector p whose image p+dq
exists, a dense block of shape dim(p+dq) x dim(p).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import comb

import numpy as np

SEED_BASE = 11035391
UP, DN = 0, 1
E_SIGMA = ((1, 0), (0, 1))

# single-site basis, sorted by (N_up, N_dn): |0>, |dn>, |up>, |updn>
_SITE_QN = np.array([[0, 0], [0, 1], [1, 0], [1, 1]], dtype=np.int32)
_SITE_OCC = [0b00, 0b10, 0b01, 0b11]          # bit 0 = up mode, bit 1 = dn mode


def _site_cdag(spin: int) -> np.ndarray:
    """4x4 matrix of c+_spin on one site, rows = destination, in the sorted site basis."""
    m = np.zeros((4, 4))
    if spin == UP:
        m[2, 0] = 1.0       # c+_up |0>  = |up>
        m[3, 1] = 1.0       # c+_up |dn> = c+_up c+_dn |0> = |updn>
    else:
        m[1, 0] = 1.0       # c+_dn |0>  = |dn>
        m[3, 2] = -1.0      # c+_dn |up> = c+_dn c+_up |0> = -|updn>
    return m


_SITE_PARITY = np.array([1.0, -1.0, -1.0, 1.0])
_SITE_NUPDN = np.diag([0.0, 0.0, 0.0, 1.0])


# --------------------------------------------------------------------------------------------
# sectored spaces and block-sparse operators
# --------------------------------------------------------------------------------------------
@dataclass
class Space:
    qn: np.ndarray                  # int32 [nsec, 2]
    dim: np.ndarray                 # int32 [nsec]
    occ: list | None = None         # exact blocks: per sector, int array of occupation masks

    def __post_init__(self):
        self.index = {(int(a), int(b)): i for i, (a, b) in enumerate(self.qn)}

    @property
    def nsec(self) -> int:
        return len(self.dim)

    @property
    def total(self) -> int:
        return int(np.sum(self.dim))

    def parity(self, i: int) -> float:
        return -1.0 if (int(self.qn[i, 0]) + int(self.qn[i, 1])) % 2 else 1.0

    def shift(self, i: int, dq) -> int | None:
        return self.index.get((int(self.qn[i, 0]) + dq[0], int(self.qn[i, 1]) + dq[1]))


@dataclass
class BlockOp:
    """Block-sparse operator on a Space; blocks[p] maps sector p to sector p+dq."""
    dq: tuple
    blocks: dict = field(default_factory=dict)

    def scaled(self, s: float) -> "BlockOp":
        return BlockOp(self.dq, {p: s * b for p, b in self.blocks.items()})


def _site_space() -> Space:
    return Space(_SITE_QN.copy(), np.ones(4, dtype=np.int32),
                 occ=[np.array([o]) for o in _SITE_OCC])


def _site_op_as_blockop(m: np.ndarray, dq) -> BlockOp:
    out = BlockOp(tuple(dq))
    for src in range(4):
        for dst in range(4):
            if m[dst, src] != 0.0:
                out.blocks[src] = np.array([[m[dst, src]]])
    return out


def _transpose(op: BlockOp, sp: Space) -> BlockOp:
    out = BlockOp((-op.dq[0], -op.dq[1]))
    for p, b in op.blocks.items():
        out.blocks[sp.shift(p, op.dq)] = b.T.copy()
    return out


def _right_parity(op: BlockOp, sp: Space) -> BlockOp:
    """op * P (P = fermion parity of the space), i.e. columns scaled by the source parity."""
    return BlockOp(op.dq, {p: sp.parity(p) * b for p, b in op.blocks.items()})


def _left_parity(op: BlockOp, sp: Space) -> BlockOp:
    """P * op, rows scaled by the destination parity."""
    return BlockOp(op.dq, {p: sp.parity(sp.shift(p, op.dq)) * b for p, b in op.blocks.items()})


# --------------------------------------------------------------------------------------------
# blocks: a sectored space with H and the c+ operators of the sites it still needs
# --------------------------------------------------------------------------------------------
@dataclass
class Block:
    space: Space
    H: list                          # per-sector dense symmetric matrices
    cdag: dict                       # site -> (BlockOp up, BlockOp dn)
    sites: list                      # lattice sites contained, in mode order
    # enlarged blocks: the two factors (first, second) and the composition
    # (sector of the first factor, sector of the second) -> (sector, offset in it)
    parts: tuple | None = None
    comp: dict | None = None


class _Product:
    """Product space A (x) B where one factor is a single site; sub-blocks are (a, b) pairs."""

    def __init__(self, spA: Space, spB: Space):
        subs = {}
        for a in range(spA.nsec):
            for b in range(spB.nsec):
                q = (int(spA.qn[a, 0] + spB.qn[b, 0]), int(spA.qn[a, 1] + spB.qn[b, 1]))
                subs.setdefault(q, []).append((a, b))
        keys = sorted(subs)
        self.spA, self.spB = spA, spB
        self.sub_off = {}
        dims = []
        for si, q in enumerate(keys):
            off = 0
            for (a, b) in subs[q]:
                self.sub_off[(a, b)] = (si, off)
                off += int(spA.dim[a]) * int(spB.dim[b])
            dims.append(off)
        self.keys = keys
        self.subs = subs
        self.space_qn = np.array(keys, dtype=np.int32).reshape(-1, 2)
        self.space_dim = np.array(dims, dtype=np.int32)

    def kron(self, opA: BlockOp, opB: BlockOp) -> BlockOp:
        """(opA (x) opB) on the product space.  One of the two factors has 1x1 sub-blocks."""
        dq = (opA.dq[0] + opB.dq[0], opA.dq[1] + opB.dq[1])
        out = BlockOp(dq)
        sp_dim = self.space_dim
        for (a, b), (si, off) in self.sub_off.items():
            if a not in opA.blocks or b not in opB.blocks:
                continue
            a2 = self.spA.shift(a, opA.dq)
            b2 = self.spB.shift(b, opB.dq)
            sj, off2 = self.sub_off[(a2, b2)]
            blk = np.kron(opA.blocks[a], opB.blocks[b])
            if si not in out.blocks:
                out.blocks[si] = np.zeros((int(sp_dim[sj]), int(sp_dim[si])))
            out.blocks[si][off2:off2 + blk.shape[0], off:off + blk.shape[1]] += blk
        return out


def _identity(sp: Space) -> BlockOp:
    return BlockOp((0, 0), {p: np.eye(int(sp.dim[p])) for p in range(sp.nsec)})


def _parity_op(sp: Space) -> BlockOp:
    return BlockOp((0, 0), {p: sp.parity(p) * np.eye(int(sp.dim[p])) for p in range(sp.nsec)})


def _add_into(H: list, op: BlockOp, sp_dim):
    assert op.dq == (0, 0)
    for p, b in op.blocks.items():
        H[p] = H[p] + b


def _enlarge(block: Block, site: int, U: float, bonds, site_first: bool, keep_sites) -> Block:
    """Add one lattice site to a block: block (x) site (append) or site (x) block (prepend).

    bonds: iterable of (i, j, t) meaning -t sum_s (c+_is c_js + h.c.); only bonds between
    `site` and a site carried by `block` are used.  keep_sites: sites whose c+ the new block
    keeps (others are dropped).
    """
    sB = block.space
    sS = _site_space()
    prod = _Product(sS, sB) if site_first else _Product(sB, sS)
    space = Space(prod.space_qn, prod.space_dim)
    # occupation masks for exact blocks (site-local mode numbering)
    if sB.occ is not None:
        occ = []
        nB = len(block.sites)
        for si, q in enumerate(prod.keys):
            masks = []
            for (a, b) in prod.subs[q]:
                if site_first:
                    masks.extend(int(_SITE_OCC[a]) | (int(m) << 2) for m in sB.occ[b])
                else:
                    masks.extend(int(m) | (int(_SITE_OCC[b]) << (2 * nB)) for m in sB.occ[a])
            occ.append(np.array(masks, dtype=np.int64))
        space.occ = occ

    site_eye = _site_op_as_blockop(np.eye(4), (0, 0))
    site_par = _site_op_as_blockop(np.diag(_SITE_PARITY), (0, 0))

    def on_block(op: BlockOp, fermionic: bool) -> BlockOp:
        """Operator of the old block embedded in the product; a fermionic one picks up the
        parity of the site when the site modes come first."""
        if site_first:
            return prod.kron(site_par if fermionic else site_eye, op)
        return prod.kron(op, site_eye)

    def on_site(m: np.ndarray, dq, fermionic: bool) -> BlockOp:
        """Single-site operator embedded in the product; a fermionic one picks up the parity
        of the old block when the block modes come first."""
        sop = _site_op_as_blockop(m, dq)
        if site_first:
            return prod.kron(sop, _identity(sB))
        return prod.kron(_parity_op(sB) if fermionic else _identity(sB), sop)

    # Hamiltonian: old H + on-site U + hopping between the new site and carried sites
    H = [np.zeros((int(d), int(d))) for d in space.dim]
    _add_into(H, on_block(BlockOp((0, 0), {p: block.H[p] for p in range(sB.nsec)}), False), space.dim)
    _add_into(H, on_site(U * _SITE_NUPDN, (0, 0), False), space.dim)
    new_cdag = {}
    for spin in (UP, DN):
        new_cdag.setdefault(site, [None, None])[spin] = on_site(_site_cdag(spin), E_SIGMA[spin], True)
    for (i, j, t) in bonds:
        other = j if i == site else (i if j == site else None)
        if other is None or other not in block.cdag:
            continue
        for spin in (UP, DN):
            cb = block.cdag[other][spin]
            cs = _site_cdag(spin)
            dq = E_SIGMA[spin]
            if site_first:
                # c+_site c_b = (c+_s P_s) (x) C_b ;  c+_b c_site = (P_s c_s) (x) C+_b
                t1 = prod.kron(_site_op_as_blockop(cs @ np.diag(_SITE_PARITY), dq), _transpose(cb, sB))
                t2 = prod.kron(_site_op_as_blockop(np.diag(_SITE_PARITY) @ cs.T, (-dq[0], -dq[1])), cb)
            else:
                # c+_b c_site = (C+_b P_B) (x) c_s ;  c+_site c_b = (P_B C_b) (x) c+_s
                t1 = prod.kron(_right_parity(cb, sB), _site_op_as_blockop(cs.T, (-dq[0], -dq[1])))
                t2 = prod.kron(_left_parity(_transpose(cb, sB), sB), _site_op_as_blockop(cs, dq))
            _add_into(H, t1.scaled(-t), space.dim)
            _add_into(H, t2.scaled(-t), space.dim)
    cdag = {}
    for s in keep_sites:
        if s == site:
            cdag[s] = tuple(new_cdag[site])
        elif s in block.cdag:
            cdag[s] = tuple(on_block(block.cdag[s][spin], True) for spin in (UP, DN))
    sites = ([site] + block.sites) if site_first else (block.sites + [site])
    parts = (sS, block) if site_first else (block, sS)
    return Block(space, H, cdag, sites, parts=parts, comp=dict(prod.sub_off))


def _site_block(site: int, U: float) -> Block:
    sp = _site_space()
    H = [np.array([[U * _SITE_NUPDN[i, i]]]) for i in range(4)]
    cdag = {site: tuple(_site_op_as_blockop(_site_cdag(s), E_SIGMA[s]) for s in (UP, DN))}
    return Block(sp, H, cdag, [site])


# --------------------------------------------------------------------------------------------
# lattices
# --------------------------------------------------------------------------------------------
def chain_bonds(L: int, t: float = 1.0):
    return [(i, i + 1, t) for i in range(L - 1)]


def ladder_bonds(Lx: int, t_leg: float = 1.0, t_rung: float = 1.0):
    """Two-leg ladder, rung-major labelling: site 2r+l is rung r, leg l."""
    b = []
    for r in range(Lx):
        b.append((2 * r, 2 * r + 1, t_rung))
        if r + 1 < Lx:
            b.append((2 * r, 2 * r + 2, t_leg))
            b.append((2 * r + 1, 2 * r + 3, t_leg))
    return sorted(b)


# --------------------------------------------------------------------------------------------
# superblock problem
# --------------------------------------------------------------------------------------------
@dataclass
class Half:
    """One superblock half: sectors, per-sector H, and the c+ operators of its edge sites."""
    space: Space
    H: list
    ops: list            # BlockOp list (c+ operators)
    op_label: list       # (site, spin) per op
    sites: list


@dataclass
class Bond:
    """-t sum_s (c+_{a s} c_{b s} + h.c.), a on S, b on E; op indices per spin."""
    opS: tuple
    opE: tuple
    t: float
    sites: tuple


@dataclass
class Problem:
    S: Half
    E: Half
    target: tuple
    bonds: list
    name: str = ""
    L: int = 0
    U: float = 0.0
    lattice_bonds: list = field(default_factory=list)
    Sblk: Block | None = None        # the blocks the halves were built from
    Eblk: Block | None = None


def _half_from_block(blk: Block, edge_sites) -> Half:
    ops, labels = [], []
    for s in edge_sites:
        for spin in (UP, DN):
            ops.append(blk.cdag[s][spin])
            labels.append((s, spin))
    return Half(blk.space, blk.H, ops, labels, blk.sites)


def _assemble(Sblk: Block, Eblk: Block, lattice_bonds, target, name, L, U) -> Problem:
    Ssites, Esites = set(Sblk.sites), set(Eblk.sites)
    cross = [(i, j, t) for (i, j, t) in lattice_bonds
             if (i in Ssites and j in Esites) or (j in Ssites and i in Esites)]
    cross = [(min(i, j), max(i, j), t) for (i, j, t) in cross]
    sedge = sorted({i for (i, j, t) in cross})
    eedge = sorted({j for (i, j, t) in cross})
    S = _half_from_block(Sblk, sedge)
    E = _half_from_block(Eblk, eedge)
    bonds = []
    for (i, j, t) in cross:
        a = S.op_label.index((i, UP))
        b = E.op_label.index((j, UP))
        bonds.append(Bond((a, a + 1), (b, b + 1), float(t), (i, j)))
    return Problem(S, E, tuple(target), bonds, name=name, L=L, U=U, lattice_bonds=lattice_bonds,
                   Sblk=Sblk, Eblk=Eblk)


def exact_problem(L: int, U: float, target, bonds=None, name="") -> Problem:
    """Exact (untruncated) blocks: left block sites 0..l-1, s1 = l, s2 = l+1, right block
    l+2..L-1, with l = (L-2)/2.  bonds default to the open chain with t = 1."""
    assert L % 2 == 0 and L >= 4
    bonds = chain_bonds(L) if bonds is None else bonds
    l = (L - 2) // 2
    s1, s2 = l, l + 1
    all_sites = set(range(L))
    left = _site_block(0, U)
    for k in range(1, l + 1):
        left = _enlarge(left, k, U, bonds, site_first=False, keep_sites=all_sites)
    right = _site_block(L - 1, U)
    for k in range(L - 2, s2 - 1, -1):
        right = _enlarge(right, k, U, bonds, site_first=True, keep_sites=all_sites)
    return _assemble(left, right, bonds, target, name, L, U)


def _largest_remainder(w: np.ndarray, m: int, cap: np.ndarray) -> np.ndarray:
    x = m * w / w.sum()
    d = np.floor(x).astype(np.int64)
    rem = int(m - d.sum())
    order = np.argsort(-(x - d), kind="stable")
    d[order[:rem]] += 1
    return np.minimum(d, cap)


def synthetic_block(l: int, m: int, sites, edge_sites, rng, width: float = 8.0,
                    spread: float = 32.0) -> Block:
    """Truncated block of l sites with about m states, synthetic:
    sector weights exp(-|n - l/2|^2 / width), largest-remainder rounding capped by the true
    sector size; per-sector H = Q diag(lambda) Q^T with lambda ~ U[-spread, spread] and Haar Q;
    c+ blocks between adjacent sectors ~ N(0, 1/m)."""
    qn, w, cap = [], [], []
    for nu in range(l + 1):
        for nd in range(l + 1):
            qn.append((nu, nd))
            w.append(np.exp(-((nu - l / 2) ** 2 + (nd - l / 2) ** 2) / width))
            cap.append(comb(l, nu) * comb(l, nd))
    d = _largest_remainder(np.array(w), m, np.array(cap))
    keep = d > 0
    qn = np.array(qn, dtype=np.int32)[keep]
    d = d[keep].astype(np.int32)
    sp = Space(qn, d)
    H = []
    for p in range(sp.nsec):
        n = int(d[p])
        g = rng.standard_normal((n, n))
        q, r = np.linalg.qr(g)
        q = q * np.sign(np.diag(r))[None, :]
        lam = rng.uniform(-spread, spread, size=n)
        h = (q * lam[None, :]) @ q.T
        H.append(0.5 * (h + h.T))
    cdag = {}
    sd = 1.0 / np.sqrt(m)
    for s in edge_sites:
        pair = []
        for spin in (UP, DN):
            op = BlockOp(E_SIGMA[spin])
            for p in range(sp.nsec):
                p2 = sp.shift(p, E_SIGMA[spin])
                if p2 is not None:
                    op.blocks[p] = sd * rng.standard_normal((int(d[p2]), int(d[p])))
            pair.append(op)
        cdag[s] = tuple(pair)
    return Block(sp, H, cdag, list(sites))


def synthetic_problem(L: int, m: int, U: float, lattice_bonds, seed: int, name="",
                      target=None, width: float = 8.0) -> Problem:
    """Superblock at the lattice centre from two synthetic truncated blocks of m states,
    each enlarged by one exact site: m_S = m_E = 4m.  width: spread of the sector weights
    (smaller concentrates the states in fewer, larger sectors)."""
    rng = np.random.default_rng(seed)
    l = (L - 2) // 2
    s1, s2 = l, l + 1
    Lsites = list(range(l))
    Rsites = list(range(s2 + 1, L))
    pairs = [(i, j) for (i, j, t) in lattice_bonds] + [(j, i) for (i, j, t) in lattice_bonds]
    Ledge = sorted({i for (i, j) in pairs if i in Lsites and j not in Lsites})
    Redge = sorted({i for (i, j) in pairs if i in Rsites and j not in Rsites})
    left = synthetic_block(l, m, Lsites, Ledge, rng, width=width)
    right = synthetic_block(L - l - 2, m, Rsites, Redge, rng, width=width)
    all_sites = set(range(L))
    S = _enlarge(left, s1, U, lattice_bonds, site_first=False, keep_sites=all_sites)
    E = _enlarge(right, s2, U, lattice_bonds, site_first=True, keep_sites=all_sites)
    if target is None:
        target = (L // 2, L // 2)
    return _assemble(S, E, lattice_bonds, target, name, L, U)


# --------------------------------------------------------------------------------------------
# local operators of the halves (operator application and observables)
# --------------------------------------------------------------------------------------------
def _op_mul(A: BlockOp, B: BlockOp, sp: Space) -> BlockOp:
    """The block operator A B (B applied first) on one space."""
    out = BlockOp((A.dq[0] + B.dq[0], A.dq[1] + B.dq[1]))
    for p, b in B.blocks.items():
        p2 = sp.shift(p, B.dq)
        if p2 is not None and p2 in A.blocks:
            out.blocks[p] = A.blocks[p2] @ b
    return out


def _op_add(A: BlockOp, B: BlockOp, sb: float = 1.0) -> BlockOp:
    """A + sb B for operators with the same dq."""
    assert A.dq == B.dq
    out = BlockOp(A.dq, {p: b.copy() for p, b in A.blocks.items()})
    for p, b in B.blocks.items():
        out.blocks[p] = out.blocks[p] + sb * b if p in out.blocks else sb * b
    return out


def site_ops(blk: Block, site: int) -> dict:
    """Operators of one lattice site carried by a block (exact blocks carry every site), as
    block operators of the block's space: cdag_s, c_s, n_s (s = 0 up, 1 down), n (both
    spins), nn = n_up n_dn, holon_s = c_s (1 - n_sbar) and doublon_s = c+_s n_sbar (the two
    factors of the holon-doublon operator, Sec. III.B)."""
    sp = blk.space
    out = {}
    for s in (UP, DN):
        cd = blk.cdag[site][s]
        out[f"cdag_{s}"] = cd
        out[f"c_{s}"] = _transpose(cd, sp)
        out[f"n_{s}"] = _op_mul(cd, out[f"c_{s}"], sp)
    out["n"] = _op_add(out["n_0"], out["n_1"])
    out["nn"] = _op_mul(out["n_0"], out["n_1"], sp)
    for s in (UP, DN):
        sb = 1 - s
        out[f"holon_{s}"] = _op_add(out[f"c_{s}"], _op_mul(out[f"c_{s}"], out[f"n_{sb}"], sp), -1.0)
        out[f"doublon_{s}"] = _op_mul(out[f"cdag_{s}"], out[f"n_{sb}"], sp)
    return out


def with_ops(pb: Problem, extra_S=(), extra_E=(), target=None) -> tuple:
    """A copy of pb whose halves also carry the given block operators (after the operators of
    its bonds), optionally for another target sector; returns (problem, indices of extra_S in
    S.ops, indices of extra_E in E.ops)."""
    S, E = pb.S, pb.E
    S2 = Half(S.space, S.H, list(S.ops) + list(extra_S), list(S.op_label) + [("x", k) for k in range(len(extra_S))], S.sites)
    E2 = Half(E.space, E.H, list(E.ops) + list(extra_E), list(E.op_label) + [("x", k) for k in range(len(extra_E))], E.sites)
    out = Problem(S2, E2, tuple(target) if target is not None else pb.target, pb.bonds, name=pb.name,
                  L=pb.L, U=pb.U, lattice_bonds=pb.lattice_bonds, Sblk=pb.Sblk, Eblk=pb.Eblk)
    return out, list(range(len(S.ops), len(S2.ops))), list(range(len(E.ops), len(E2.ops)))


# --------------------------------------------------------------------------------------------
# moving the centre one site to the right: the bases involved (wave-function transformation)
# --------------------------------------------------------------------------------------------
@dataclass
class WftMove:
    """Bases of a move of the centre one site to the right, for a superblock
    S (x) E = (A (x) s1) (x) (s2 (x) R):

      new system       S' = A' (x) s2, A' the kept states of S (per psi-layout sector of S, the
                       first kept[b] columns of its eigenvector matrix U_b);
      new environment  E' = s3 (x) R'', R expressed in it by W_r (d_E'(r) x d_R(r), one per
                       sector r of R; the identity for exact blocks, where R = s3 (x) R'').

    esub: (q, a, r, col offset) per sub-block of E = s2 (x) R (q: E sector, a: site state of s2,
    r: R sector); ssub: {(b, a): (p', row offset)} per sub-block of S' (b: psi-layout block of
    the kept S sector, a: site state of s2); layout: a Problem with the new halves' spaces and
    the same target (its block operators are empty: it only carries the vector layout)."""
    kept: list
    esub: list
    ssub: dict
    r_dim: list
    r_to_enew: list
    W: list
    layout: Problem
    exact: bool


def _haar_isometry(rows: int, cols: int, rng) -> np.ndarray:
    g = rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def wft_move(pb: Problem, kept, seed: int = 0) -> WftMove:
    """The bases of the move for pb (built by exact_problem or synthetic_problem) with kept[b]
    states of psi-layout block b.  Synthetic problems get a synthetic R'' (as many states as R,
    doubled until every sector of R fits) and Haar-random isometries W_r (seeded)."""
    S, E = pb.Sblk, pb.Eblk
    assert S is not None and E is not None and S.comp is not None and E.comp is not None
    R = E.parts[1]
    blocks = psi_blocks(pb)
    assert len(kept) == len(blocks)
    # old environment E = s2 (x) R
    esub = sorted((q, a, r, off) for (a, r), (q, off) in E.comp.items())
    # new system S' = A' (x) s2
    kb = [b for b in range(len(blocks)) if kept[b] > 0]
    Aqn = np.array([S.space.qn[blocks[b][0]] for b in kb], dtype=np.int32).reshape(-1, 2)
    Adim = np.array([kept[b] for b in kb], dtype=np.int32)
    prodS = _Product(Space(Aqn, Adim), _site_space())
    ssub = {(kb[i], a): so for (i, a), so in prodS.sub_off.items()}
    Snew = Space(prodS.space_qn, prodS.space_dim)
    # new environment E' = s3 (x) R''
    rng = np.random.default_rng(SEED_BASE + 7000 + seed)
    if R.comp is not None:                       # exact: R is s3 (x) R'' itself
        Enew = R.space
        W = [np.eye(int(d), dtype=complex) for d in R.space.dim]
        r_to_enew = list(range(R.space.nsec))
        exact = True
    else:
        nsites = len(R.sites) - 1
        m2 = int(R.space.total)
        while True:
            Rpp = synthetic_block(nsites, m2, R.sites[1:], [], rng)
            prodE = _Product(_site_space(), Rpp.space)
            Enew = Space(prodE.space_qn, prodE.space_dim)
            r_to_enew = [Enew.index.get((int(a), int(b))) for (a, b) in R.space.qn]
            if all(j is not None and Enew.dim[j] >= R.space.dim[r] for r, j in enumerate(r_to_enew)):
                break
            m2 *= 2
        W = [_haar_isometry(int(Enew.dim[j]), int(R.space.dim[r]), rng) for r, j in enumerate(r_to_enew)]
        exact = False
    lay = Problem(Half(Snew, [], [], [], []), Half(Enew, [], [], [], []), pb.target, [],
                  name=pb.name + "_moved", L=pb.L, U=pb.U)
    return WftMove(list(kept), esub, ssub, [int(d) for d in R.space.dim], r_to_enew, W, lay, exact)


# --------------------------------------------------------------------------------------------
# vectors
# --------------------------------------------------------------------------------------------
def psi_blocks(pb: Problem):
    """Blocks of a vector in the target sector: list of (p, q, rows, cols) in S-sector order,
    p an S sector, q = target - p the matching E sector."""
    out = []
    for p in range(pb.S.space.nsec):
        qn = (pb.target[0] - int(pb.S.space.qn[p, 0]), pb.target[1] - int(pb.S.space.qn[p, 1]))
        q = pb.E.space.index.get(qn)
        if q is not None:
            out.append((p, q, int(pb.S.space.dim[p]), int(pb.E.space.dim[q])))
    return out


def psi_size(pb: Problem) -> int:
    return sum(r * c for (_, _, r, c) in psi_blocks(pb))


def random_psi(n: int, rng, complex_=True) -> np.ndarray:
    """Flat vector of 2n doubles (all real parts, then all imaginary parts), Re and Im iid
    N(0,1) (zero Im if complex_ is False), normalised to unit 2-norm."""
    re = rng.standard_normal(n)
    im = rng.standard_normal(n) if complex_ else np.zeros(n)
    v = np.concatenate([re, im])
    return v / np.linalg.norm(v)


# --------------------------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------------------------
WORKLOADS = {
    # name: (kind, L, m, U, lattice, kdim, tau, nsteps, seed offset)
    "chain8_exact":  dict(kind="exact", L=8, U=4.0, lattice="chain", kdim=12, tau=0.1, nsteps=10, seed=1),
    "chain32_m400":  dict(kind="synthetic", L=32, m=400, U=4.0, lattice="chain", kdim=15, tau=0.1, nsteps=10, seed=2),
    "ladder16_m800": dict(kind="synthetic", L=32, m=800, U=8.0, lattice="ladder", kdim=15, tau=0.05, nsteps=10, seed=3),
    "ladder16_m1000": dict(kind="synthetic", L=32, m=1000, U=8.0, lattice="ladder", kdim=15, tau=0.05, nsteps=10, seed=10),
    "ladder32_m2000": dict(kind="synthetic", L=64, m=2000, U=8.0, lattice="ladder", kdim=20, tau=0.05, nsteps=50, seed=5),
}


def _lattice(kind: str, L: int):
    if kind == "chain":
        return chain_bonds(L)
    return ladder_bonds(L // 2)


def make_workload(name: str, m: int | None = None) -> Problem:
    """Problem for a named workload; m overrides the block size for scaled-down variants."""
    w = WORKLOADS[name]
    seed = SEED_BASE + w["seed"]
    if w["kind"] == "exact":
        return exact_problem(w["L"], w["U"], (w["L"] // 2, w["L"] // 2), name=name)
    return synthetic_problem(w["L"], m if m is not None else w["m"], w["U"],
                             _lattice(w["lattice"], w["L"]), seed, name=name)


def batch_workloads(count: int = 64, seed_offset: int = 100, m_lo=100, m_hi=1000):
    """Independent chain superblocks: m ~ U{m_lo..m_hi}, L ~ U{16,18,..,48}, U in {2,4,8}."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(SEED_BASE + seed_offset + i)
        m = int(rng.integers(m_lo, m_hi + 1))
        L = int(rng.choice(np.arange(16, 49, 2)))
        U = float(rng.choice([2.0, 4.0, 8.0]))
        out.append(synthetic_problem(L, m, U, chain_bonds(L), SEED_BASE + seed_offset + 1000 + i,
                                     name=f"batch{i}"))
    return out
