"""Pins of the oracle Krylov exponential and time-step targeting (CPU only)."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import closed_forms as CF
from oracle import ed
from oracle import krylov as K
from oracle import matvec as M
from paper_1103_5391_amd import inputs as I
from tests.helpers import ed_to_flat, exact_case, expm_flat, flat_to_ed, superblock_to_ed_perm

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _apply(pb):
    return lambda v: M.matvec_sector(pb, v)


def _dense_expm_flat(Hreal, x, tau):
    n = Hreal.shape[0]
    z = x[:n] + 1j * x[n:]
    y = sla.expm(-1j * tau * Hreal) @ z
    return np.concatenate([y.real, y.imag])


def test_full_krylov_equals_dense_expm():
    """kdim = dim of the space: the Krylov step is the exact exponential (library expm)."""
    pb = I.exact_problem(4, 4.0, (2, 2))           # 36 states
    H = M.superblock_matrix(pb)
    lay, n = M.layout(pb)
    x = I.random_psi(n, np.random.default_rng(1))
    for tau in (0.1, 1.0, 3.0):
        y, info = K.krylov_expm(_apply(pb), x, tau, kdim=n)
        yref = _dense_expm_flat(H, x, tau)
        assert np.linalg.norm(y - yref) < 1e-11, tau
        assert info.k_eff[0] <= n


def test_eigenvector_input_breaks_down_exactly():
    pb = I.exact_problem(6, 4.0, (3, 3))
    H = M.superblock_matrix(pb)
    w, v = np.linalg.eigh(H)
    x = np.concatenate([v[:, 5], np.zeros_like(v[:, 5])])
    y, info = K.krylov_expm(_apply(pb), x, 0.3, kdim=12)
    assert info.k_eff == [1] and info.breakdown
    z = np.exp(-1j * w[5] * 0.3) * v[:, 5]
    assert np.linalg.norm(y - np.concatenate([z.real, z.imag])) < 1e-12


def test_tau_zero_identity_and_zero_vector():
    pb = I.exact_problem(6, 4.0, (3, 3))
    lay, n = M.layout(pb)
    x = I.random_psi(n, np.random.default_rng(2))
    y, _ = K.krylov_expm(_apply(pb), x, 0.0, kdim=10)
    assert np.linalg.norm(y - x) < 1e-13
    y0, info = K.krylov_expm(_apply(pb), np.zeros(2 * n), 0.3, kdim=10)
    assert np.all(y0 == 0) and info.k_eff == [0]


def test_chain8_config_against_dense_expm_and_invariants():
    """Chain L=8, U=4, exact blocks, complex psi, kdim=12, tau=0.1, 10 steps: against the dense
    exponential of the ED-equal matrix; norm and energy conserved."""
    pb, sec, H, perm = exact_case(8, 4.0, (4, 4))
    lay, n = M.layout(pb)
    x = I.random_psi(n, np.random.default_rng(I.SEED_BASE + 1))
    y, info = K.krylov_expm(_apply(pb), x, 0.1, kdim=12, nsteps=10)
    yref = expm_flat(H, x, 1.0)
    assert np.linalg.norm(y - yref) < 1e-9
    z, zy = x[:n] + 1j * x[n:], y[:n] + 1j * y[n:]
    assert abs(np.linalg.norm(zy) - 1.0) < 1e-12
    e0 = np.vdot(z, H @ z).real
    e1 = np.vdot(zy, H @ zy).real
    assert abs(e1 - e0) < 1e-10 * max(1.0, abs(e0))
    assert all(k == 12 for k in info.k_eff)


def test_error_decreases_with_tau():
    """Sec. II.A: at fixed n_l the Krylov accuracy increases as t decreases."""
    pb, sec, H, perm = exact_case(8, 4.0, (4, 4))
    lay, n = M.layout(pb)
    x = I.random_psi(n, np.random.default_rng(9))
    errs = []
    for tau in (0.8, 0.4, 0.2, 0.1):
        y, _ = K.krylov_expm(_apply(pb), x, tau, kdim=6)
        errs.append(np.linalg.norm(y - expm_flat(H, x, tau)))
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs


@pytest.mark.parametrize("L,i,nsteps", [(8, 3, 8), (10, 4, 8), (12, 5, 4)])
def test_onesite_excitation_closed_form(L, i, nsteps):
    """App. A: X_ij(t) = R_i R_j - |T_ij(t)|^2 for U = 0, half filling, phi = c_{i up}|GS>,
    evolved by repeated Krylov steps on exact blocks (the closed form is even in t, so the
    evolution sign convention does not enter).  L = 12: 731,808 states, four steps."""
    E, U = CF.chain_levels(L)
    sec0, H0 = ed.hamiltonian(L, I.chain_bonds(L), 0.0, L // 2, L // 2)
    _, gs = ed.ground_state(H0)
    sec1 = ed.Sector(L, L // 2 - 1, L // 2)
    phi = ed.annihilate(sec0, sec1, 2 * i) @ gs
    pb = I.exact_problem(L, 0.0, (L // 2 - 1, L // 2))
    perm = superblock_to_ed_perm(pb, sec1)
    x = ed_to_flat(phi.astype(complex), perm)
    tau = 0.25
    y = x
    for s in range(1, nsteps + 1):
        y, _ = K.krylov_expm(_apply(pb), y, tau, kdim=14)
        z = flat_to_ed(y, perm, sec1.dim)
        for j in range(L):
            x_num = float(np.sum(np.abs(z) ** 2 * ed.number(sec1, j, 0)))
            x_cf = CF.onesite_excitation(E, U, L // 2, i, j, s * tau)[0]
            assert abs(x_num - x_cf) < 1e-8, (s, j, x_num, x_cf)


def test_holon_doublon_small_time_expansion():
    """Fig. 4: O(t) = O(0) + a t^2 + O(t^4) with a = <phi|H n H - H^2 n|phi>/<phi|phi> (real
    phi), on the 2x4 ladder with U = 10; evolution by the Krylov step per sector."""
    from tests.test_oracle_ed import _holon_doublon
    L, i, j, U = 8, 2, 4, 10.0
    bonds = I.ladder_bonds(4, 1.0, 0.5)
    parts = _holon_doublon(L, bonds, U, i, j)
    norm = sum(float(np.vdot(v, v).real) for (_, v) in parts.values())
    for t in (0.01, 0.02, 0.04):
        O = np.zeros(L)
        O0 = np.zeros(L)
        a = np.zeros(L)
        for key, (sec, v) in parts.items():
            _, H = ed.hamiltonian(L, bonds, U, *key)
            pb = I.exact_problem(L, U, key, bonds=bonds)
            perm = superblock_to_ed_perm(pb, sec)
            y, _ = K.krylov_expm(_apply(pb), ed_to_flat(v.astype(complex), perm), t, kdim=10)
            z = flat_to_ed(y, perm, sec.dim)
            hv = H @ v
            h2v = H @ hv
            for p in range(L):
                n_p = ed.number(sec, p, 0) + ed.number(sec, p, 1)
                O[p] += np.sum(np.abs(z) ** 2 * n_p)
                O0[p] += np.sum(np.abs(v) ** 2 * n_p)
                a[p] += np.sum(hv * n_p * hv) - np.sum(h2v * n_p * v)
        O, O0, a = O / norm, O0 / norm, a / norm
        resid = np.abs(O - O0 - a * t * t)
        assert np.max(resid) < 50 * t ** 4 + 1e-10, (t, resid)


def test_tst_targets_and_weights():
    pb, sec, H, perm = exact_case(8, 4.0, (4, 4))
    lay, n = M.layout(pb)
    phi = I.random_psi(n, np.random.default_rng(11))
    tau = 0.1
    ys, w, b = K.tst_targets(_apply(pb), phi, tau, kdim=12)
    g = GOLDEN["tst_weights"]
    assert np.array_equal(w * 8, np.array(g["weights_times_8"], dtype=float))
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.linalg.norm(ys[0] - phi) < 1e-13
    y_step, _ = K.krylov_expm(_apply(pb), phi, tau, kdim=12)
    assert np.linalg.norm(ys[3] - y_step) < 1e-14
    for x, t in zip(ys, K.tst_times(tau)):
        assert np.linalg.norm(x - expm_flat(H, phi, t)) < 1e-10


def test_tst_chains_against_dense_expm():
    """The per-target chains: four different vectors (here the shared-basis targets), each
    advanced by tau, against the dense exponential; chains are independent of each other (the
    same vector gives the same result whatever the others are)."""
    pb, sec, H, perm = exact_case(8, 4.0, (4, 4))
    lay, n = M.layout(pb)
    phi = I.random_psi(n, np.random.default_rng(13))
    tau = 0.1
    starts, _, _ = K.tst_targets(_apply(pb), phi, tau, kdim=12)
    ys, w, infos = K.tst_chains(_apply(pb), starts, tau, kdim=12)
    assert np.array_equal(w * 8, np.array(GOLDEN["tst_weights"]["weights_times_8"], dtype=float))
    for x0, y, info in zip(starts, ys, infos):
        assert np.linalg.norm(y - expm_flat(H, x0, tau)) < 1e-10
        assert abs(np.linalg.norm(y) - np.linalg.norm(x0)) < 1e-13
        assert info.err_est < 1e-8
    other = [starts[0], phi, phi, phi]
    ys2, _, _ = K.tst_chains(_apply(pb), other, tau, kdim=12)
    assert np.array_equal(ys2[0], ys[0])


def test_ground_state_against_sparse_eigensolver_and_closed_form():
    """Restarted Lanczos ground state: the exact-block chain (L = 8, U = 4, sector (4,4))
    against ARPACK's lowest eigenpair of the sector Hamiltonian (a library routine on the ED
    matrix); at U = 0 against the closed form 2 sum_{k<=4} -2 cos(k pi / 9); the Ritz residual."""
    import scipy.sparse.linalg as spla
    for U in (4.0, 0.0):
        pb, sec, H, perm = exact_case(8, U, (4, 4))
        lay, n = M.layout(pb)
        x0 = I.random_psi(n, np.random.default_rng(14))
        y, info = K.ground_state(_apply(pb), x0, kdim=30, max_restarts=60, tol=1e-12)
        evals, evecs = spla.eigsh(H, k=2, which="SA", tol=1e-14)
        order = np.argsort(evals)
        evals, evecs = evals[order], evecs[:, order]
        assert abs(info.energy - evals[0]) < 1e-10 * max(1.0, abs(evals[0]))
        hy = M.matvec_sector(pb, y)
        assert np.linalg.norm(hy - info.energy * y) < 1e-8
        assert abs(np.linalg.norm(y) - 1.0) < 1e-12
        if U == 0.0:
            closed = 2.0 * sum(-2.0 * np.cos(k * np.pi / 9.0) for k in range(1, 5))
            assert abs(info.energy - closed) < 1e-10
        else:
            assert evals[1] - evals[0] > 1e-3        # non-degenerate: the vector is unique
            yc = y[:n] + 1j * y[n:]
            assert abs(abs(np.vdot(evecs[:, 0], yc)) - 1.0) < 1e-8


def test_error_estimate_bounds_true_error():
    pb, sec, H, perm = exact_case(8, 4.0, (4, 4))
    lay, n = M.layout(pb)
    x = I.random_psi(n, np.random.default_rng(12))
    for tau in (0.3, 0.6):
        y, info = K.krylov_expm(_apply(pb), x, tau, kdim=8)
        err = np.linalg.norm(y - expm_flat(H, x, tau))
        assert err <= info.err_est * 1.01 + 1e-15
