"""Pins of the oracle reduced density matrix and truncation (CPU only)."""
import numpy as np

from oracle import density as D
from oracle import krylov as K
from oracle import matvec as M
from paper_1103_5391_amd import inputs as I


def _case(seed=3):
    pb = I.synthetic_problem(12, 30, 4.0, I.chain_bonds(12), 7, name="chain12_m30")
    lay, n = M.layout(pb)
    rng = np.random.default_rng(seed)
    vecs = [I.random_psi(n, rng) for _ in range(5)]
    return pb, lay, n, vecs, K.tst_weights()


def test_trace_hermitian_psd_and_svd_spectrum():
    pb, lay, n, vecs, w = _case()
    rho = D.density_blocks(pb, vecs, w)
    tr = sum(np.trace(r).real for r in rho.values())
    assert abs(tr - sum(wi * np.linalg.norm(v) ** 2 for wi, v in zip(w, vecs))) < 1e-14
    for p, r in rho.items():
        assert np.allclose(r, r.conj().T, atol=1e-15)
        # eigenvalues = squared singular values of the stacked, weighted blocks
        X = np.hstack([np.sqrt(wi) * M.unpack(pb, v)[p] for wi, v in zip(w, vecs)])
        sv = np.sort(np.linalg.svd(X, compute_uv=False) ** 2)[::-1]
        ev = np.sort(np.linalg.eigvalsh(r))[::-1]
        k = min(len(sv), len(ev))
        assert np.allclose(ev[:k], sv[:k], atol=1e-14)
        assert np.all(ev > -1e-14)
        assert np.all(np.abs(ev[k:]) < 1e-14)


def test_truncation_counts_and_error():
    pb, lay, n, vecs, w = _case()
    total_states = sum(r for (p, q, r, c, off) in lay)
    t_all = D.truncate(pb, vecs, w, keep=total_states)
    assert t_all.trunc_err < 1e-14 and abs(t_all.trace - 1.0) < 1e-14
    keep = total_states // 3
    t = D.truncate(pb, vecs, w, keep=keep)
    assert sum(t.kept.values()) == keep
    allv = np.sort(np.concatenate([t.evals[p] for p in t.sectors]))[::-1]
    assert abs(t.trunc_err - allv[keep:].sum()) < 1e-14
    # the kept states of a sector are its largest eigenvalues, and eigen-pairs hold
    rho = D.density_blocks(pb, vecs, w)
    for p in t.sectors:
        lam, U = t.evals[p], t.evecs[p]
        assert np.all(np.diff(lam) <= 1e-15)
        assert np.allclose(rho[p] @ U, U * lam, atol=1e-13)
        if t.kept[p] < len(lam):
            assert lam[t.kept[p]] <= allv[keep - 1] + 1e-15


def test_product_state_has_rank_one_blocks():
    """A target whose blocks are outer products u v^T gives rank-one rho_p per sector."""
    pb, lay, n, vecs, w = _case()
    rng = np.random.default_rng(5)
    blocks = {p: np.outer(rng.standard_normal(r) + 1j * rng.standard_normal(r),
                          rng.standard_normal(c) + 1j * rng.standard_normal(c))
              for (p, q, r, c, off) in lay}
    x = M.pack(pb, blocks)
    x = x / np.linalg.norm(x)
    rho = D.density_blocks(pb, [x], [1.0])
    for r in rho.values():
        ev = np.sort(np.linalg.eigvalsh(r))[::-1]
        assert np.all(np.abs(ev[1:]) < 1e-14 * max(1.0, ev[0]))
