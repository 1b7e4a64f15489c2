"""Pins of the oracle's wave-function transformation (oracle/wft.py) against what the bases fix:
the Fock-space vector on exact blocks, the projector on the kept states, the discarded weight of
the density matrix, and isometries with a known action."""
import numpy as np
import pytest

from oracle import density as D
from oracle import matvec as M
from oracle import wft as W
from paper_1103_5391_amd import inputs as I


def _haar_unitary(d, rng):
    g = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    q, r = np.linalg.qr(g)
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def _fock_old(pb, x):
    """{Fock mask: amplitude} of psi on exact blocks S (x) E (masks of S, then E shifted)."""
    nS = len(pb.Sblk.sites)
    blocks = M.unpack(pb, x)
    lay, _ = M.layout(pb)
    out = {}
    for (p, q, r, c, off) in lay:
        ms, me = pb.S.space.occ[p], pb.E.space.occ[q]
        for i in range(r):
            for j in range(c):
                out[int(ms[i]) | (int(me[j]) << (2 * nS))] = blocks[p][i, j]
    return out


def _fock_new(pb, mv, U, xn):
    """{Fock mask: amplitude} of psi' with U undone: rows are states of S (x) s2, columns states
    of R (exact: E' = R)."""
    nS = len(pb.Sblk.sites)
    R = pb.Eblk.parts[1]
    lay, _ = M.layout(pb)
    out = {}
    site_occ = [0b00, 0b10, 0b01, 0b11]
    for (b, a, j), blk in W.undo_system(pb, mv, U, xn).items():
        p = lay[b][0]
        ms, mr = pb.S.space.occ[p], R.space.occ[j]
        for i in range(blk.shape[0]):
            for g in range(blk.shape[1]):
                out[int(ms[i]) | (site_occ[a] << (2 * nS)) | (int(mr[g]) << (2 * nS + 2))] = blk[i, g]
    return out


def _compare(fa, fb, tol):
    keys = set(fa) | set(fb)
    return max(abs(fa.get(k, 0.0) - fb.get(k, 0.0)) for k in keys)


@pytest.mark.parametrize("L,target", [(6, (3, 3)), (8, (4, 4)), (8, (5, 3))])
def test_exact_blocks_keep_everything_is_the_same_state(L, target):
    pb = I.exact_problem(L, 4.0, target)
    lay, n = M.layout(pb)
    rng = np.random.default_rng(I.SEED_BASE + 501 + L)
    U = {p: _haar_unitary(r, rng) for (p, q, r, c, off) in lay}
    kept = [r for (p, q, r, c, off) in lay]
    mv = I.wft_move(pb, kept)
    assert mv.exact
    x = I.random_psi(n, rng)
    xn = W.wft_right(pb, mv, U, x)
    assert abs(np.linalg.norm(xn) - 1.0) < 1e-13
    fo, fn = _fock_old(pb, x), _fock_new(pb, mv, U, xn)
    assert len(fo) == n
    assert _compare(fo, fn, 0) < 1e-14
    # a plausible mistake: U transposed instead of conjugate-transposed
    Ut = {p: u.conj() for p, u in U.items()}
    bad = _fock_new(pb, mv, U, W.wft_right(pb, mv, Ut, x))
    assert _compare(fo, bad, 0) > 1e-3


def test_exact_blocks_truncation_is_the_projector_and_discarded_weight():
    pb = I.exact_problem(8, 4.0, (4, 4))
    lay, n = M.layout(pb)
    rng = np.random.default_rng(I.SEED_BASE + 511)
    x = I.random_psi(n, rng)
    tr = D.truncate(pb, [x], [1.0], keep=40)
    kept = [tr.kept[p] for p in tr.sectors]
    assert 0 < sum(kept) < sum(r for (p, q, r, c, off) in lay)
    mv = I.wft_move(pb, kept)
    xn = W.wft_right(pb, mv, tr.evecs, x)
    # norm: the kept weight of psi's own density matrix
    assert abs(np.linalg.norm(xn) ** 2 - (1.0 - tr.trunc_err)) < 1e-13
    # with U undone: (P (x) 1) psi, P the projector on the kept states of every sector
    blocks = M.unpack(pb, x)
    proj = {}
    for b, (p, q, r, c, off) in enumerate(lay):
        Uk = tr.evecs[p][:, :kept[b]]
        proj[p] = Uk @ (Uk.conj().T @ blocks[p])
    xp = M.pack(pb, proj)
    assert _compare(_fock_old(pb, xp), _fock_new(pb, mv, tr.evecs, xn), 0) < 1e-14


def test_synthetic_isometries_act_as_defined():
    """W_r replaced by phase-permutation isometries: state beta of R is exp(i theta) |pi(beta)>
    of s3 (x) R'', so its amplitude must reappear at pi(beta) times exp(i theta)."""
    pb = I.synthetic_problem(12, 30, 4.0, I.chain_bonds(12), 7)
    lay, n = M.layout(pb)
    kept = [max(1, r // 2) for (p, q, r, c, off) in lay]
    mv = I.wft_move(pb, kept, seed=3)
    assert not mv.exact
    rng = np.random.default_rng(I.SEED_BASE + 521)
    perm, phase = [], []
    for r, w in enumerate(mv.W):
        de, dr = w.shape
        pi = rng.permutation(de)[:dr]
        th = rng.uniform(0, 2 * np.pi, dr)
        Wr = np.zeros((de, dr), dtype=complex)
        Wr[pi, np.arange(dr)] = np.exp(1j * th)
        mv.W[r] = Wr
        perm.append(pi)
        phase.append(np.exp(1j * th))
    U = {p: _haar_unitary(r, rng) for (p, q, r, c, off) in lay}
    x = I.random_psi(n, rng)
    xn = W.wft_right(pb, mv, U, x)
    new = M.unpack(mv.layout, xn)
    blocks = M.unpack(pb, x)
    checked = 0
    for b, (p, q, r, c, off) in enumerate(lay):
        phi = U[p][:, :kept[b]].conj().T @ blocks[p]
        for (qq, a, rr, coff) in mv.esub:
            if qq != q:
                continue
            pp, roff = mv.ssub[(b, a)]
            got = new[pp][roff:roff + kept[b], :]
            for beta in range(mv.r_dim[rr]):
                want = phi[:, coff + beta] * phase[rr][beta]
                assert np.max(np.abs(got[:, perm[rr][beta]] - want)) < 1e-14
                checked += 1
            # columns that no state of R maps to stay zero
            free = np.setdiff1d(np.arange(got.shape[1]), perm[rr])
            assert np.max(np.abs(got[:, free]), initial=0.0) == 0.0
    assert checked > 0
    # Haar isometries keep the norm of the kept part
    mv2 = I.wft_move(pb, kept, seed=3)
    xn2 = W.wft_right(pb, mv2, U, x)
    kept_norm2 = sum(np.linalg.norm(U[p][:, :kept[b]].conj().T @ blocks[p]) ** 2
                     for b, (p, q, r, c, off) in enumerate(lay))
    assert abs(np.linalg.norm(xn2) ** 2 - kept_norm2) < 1e-13
