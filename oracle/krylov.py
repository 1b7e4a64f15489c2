"""Krylov (Lanczos) time evolution and time-step-targeting targets in FP64 (oracle, test only).

Sec. II.A: start the Lanczos recursion from phi itself, so H ~ V^T T V with the first Lanczos
vector proportional to phi; diagonalise the small tridiagonal T = S D S^T and use
    phi(t) ~ V^T exp(-i T t) V phi = beta0 V^T S exp(-i D t) S^T e_1
(the library evolves with exp(-i tau H); the paper's exp(+iHt) is tau -> -tau.  Eq.
(lanczosevolution) as printed also carries factors T^dagger and T around the exponential, which
would not give the evolution of phi; the form above, the one the text states before it, is
used).
Sec. II.C: larger times by repeating the step from the evolved vector, Eq. (lanczosevolution2).
Sec. II.B/II.C: time-step targeting keeps n_v = 4 equally spaced times 0, tau/3, 2tau/3, tau
from one Krylov basis, with weights 2W for the ground state and the first and last time
vector and W for the others, W = 1/(n + 3), n = 5 targets including the ground state.
Ground-state targeting (Sec. II.B, the ground state is a target of weight 2W): the same
Lanczos basis, with the lowest eigenpair of T in place of its exponential, restarted from the
Ritz vector until the residual estimate beta_k |z_{k-1}| is small.
Per-target (4-RHS) variant of the seeding of the next interval (Sec. II.C leaves it open): each
target is its own chain, advanced by one Krylov step exp(-i tau H) from its current vector; it
agrees with the shared-basis targets only to Krylov error, so it has its own oracle function.

The recursion, step by step, on complex vectors (flat [Re | Im] layout outside):
  beta0 = ||x||; v_0 = x / beta0
  for j = 0 .. k-1:
      w = H v_j;  alpha_j = Re(v_j^H w);  w -= alpha_j v_j + beta_j v_{j-1}
      twice: h = V_{0..j}^H w;  w -= V_{0..j} h      (full reorthogonalisation, h discarded)
      beta_{j+1} = ||w||
      if j < k-1: stop with k_eff = j+1 if beta_{j+1} <= 1e-12 max(1, |alpha_i|, beta_i),
                  else v_{j+1} = w / beta_{j+1}
Pins: k = dim gives the dense exponential; eigenvector input gives exp(-i E tau) x with
k_eff = 1; tau = 0 is the identity; norm and <H> are conserved; App. A closed form.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.linalg import eigh_tridiagonal

BREAKDOWN_REL = 1e-12


def _cplx(x: np.ndarray) -> np.ndarray:
    n = x.shape[0] // 2
    return x[:n] + 1j * x[n:]


def _flat(z: np.ndarray) -> np.ndarray:
    return np.concatenate([z.real, z.imag])


@dataclass
class Basis:
    V: np.ndarray          # k_eff x n complex, rows are Lanczos vectors
    alpha: np.ndarray      # k_eff
    beta: np.ndarray       # k_eff + 1: beta[0] = beta0 = ||x||, beta[j] couples v_{j-1}, v_j
    k_eff: int
    breakdown: bool


def lanczos(apply_h, x: np.ndarray, kdim: int) -> Basis:
    """Lanczos basis of span{x, Hx, ..., H^{k-1} x} started from x (apply_h acts on flat
    [Re | Im] vectors)."""
    z = _cplx(x)
    n = z.shape[0]
    beta0 = float(np.linalg.norm(z))
    V = np.zeros((kdim, n), dtype=complex)
    alpha = np.zeros(kdim)
    beta = np.zeros(kdim + 1)
    beta[0] = beta0
    if beta0 == 0.0:
        return Basis(V[:0], alpha[:0], beta[:1], 0, False)
    V[0] = z / beta0
    k_eff, broke = kdim, False
    scale = 1.0
    for j in range(kdim):
        w = _cplx(apply_h(_flat(V[j])))
        alpha[j] = float(np.real(np.vdot(V[j], w)))
        w = w - alpha[j] * V[j]
        if j > 0:
            w = w - beta[j] * V[j - 1]
        for _ in range(2):
            h = V[: j + 1].conj() @ w
            w = w - V[: j + 1].T @ h
        beta[j + 1] = float(np.linalg.norm(w))
        scale = max(scale, abs(alpha[j]), beta[j] if j > 0 else 0.0)
        if j < kdim - 1:
            if beta[j + 1] <= BREAKDOWN_REL * scale:
                k_eff, broke = j + 1, True
                break
            V[j + 1] = w / beta[j + 1]
    return Basis(V[:k_eff], alpha[:k_eff], beta[: k_eff + 1], k_eff, broke)


def tridiag_coeffs(b: Basis, times) -> np.ndarray:
    """c(t) = beta0 S exp(-i D t) S^T e_1 for each t (rows), T = tridiag(alpha; beta_1..)."""
    k = b.k_eff
    if k == 0:
        return np.zeros((len(times), 0), dtype=complex)
    D, S = eigh_tridiagonal(b.alpha[:k], b.beta[1:k])
    out = []
    for t in times:
        out.append(b.beta[0] * (S @ (np.exp(-1j * D * t) * S[0, :])))
    return np.array(out)


def combine(b: Basis, c: np.ndarray) -> np.ndarray:
    """y = V^T c as a flat [Re | Im] vector."""
    n = b.V.shape[1]
    if b.k_eff == 0:
        return np.zeros(2 * n)
    return _flat(b.V.T @ c)


def error_estimate(b: Basis, tau: float) -> float:
    """beta_k |c_{k-1}(tau)|, the norm of the first neglected Krylov component (a known
    overestimate); zero after breakdown."""
    if b.k_eff == 0 or b.breakdown:
        return 0.0
    c = tridiag_coeffs(b, [tau])[0]
    return float(b.beta[b.k_eff] * abs(c[-1]))


@dataclass
class StepInfo:
    k_eff: list
    beta0: float
    beta_last: float
    err_est: float
    breakdown: bool


def krylov_expm(apply_h, x: np.ndarray, tau: float, kdim: int, nsteps: int = 1):
    """(exp(-i tau H))^nsteps x, each step from a fresh Lanczos basis of the current vector
    (Eq. (lanczosevolution2))."""
    y = x.copy()
    info = StepInfo([], 0.0, 0.0, 0.0, False)
    for s in range(nsteps):
        b = lanczos(apply_h, y, kdim)
        c = tridiag_coeffs(b, [tau])
        if s == 0:
            info.beta0 = float(b.beta[0])
        info.k_eff.append(b.k_eff)
        info.beta_last = float(b.beta[b.k_eff]) if b.k_eff > 0 else 0.0
        info.err_est = error_estimate(b, tau)
        info.breakdown = info.breakdown or b.breakdown
        y = combine(b, c[0]) if b.k_eff > 0 else np.zeros_like(x)
    return y, info


def tst_times(tau: float, nv: int = 4):
    return [tau * x / (nv - 1) for x in range(nv)]


def tst_weights(nv: int = 4) -> np.ndarray:
    """[ground state, phi(t_0), ..., phi(t_{nv-1})]: 2W for the ground state and the first and
    last time vectors, W for the rest, W = 1/(n+3) with n = nv + 1 targets."""
    n = nv + 1
    W = 1.0 / (n + 3)
    w = np.full(n, W)
    w[0] = w[1] = w[-1] = 2 * W
    return w


def tst_targets(apply_h, phi: np.ndarray, tau: float, kdim: int, nv: int = 4):
    """The nv time-step-targeting vectors phi(t_x), t_x = x tau / (nv-1), from one Krylov basis
    started at phi, and the nv + 1 weights."""
    b = lanczos(apply_h, phi, kdim)
    c = tridiag_coeffs(b, tst_times(tau, nv))
    ys = [combine(b, c[i]) if b.k_eff > 0 else np.zeros_like(phi) for i in range(nv)]
    return ys, tst_weights(nv), b


def tst_chains(apply_h, phis, tau: float, kdim: int):
    """Per-target chains: each vector advanced by one Krylov step exp(-i tau H) with a basis of
    its own (the 4-RHS variant of Sec. II.C), and the time-step-targeting weights."""
    ys, infos = [], []
    for phi in phis:
        y, info = krylov_expm(apply_h, phi, tau, kdim)
        ys.append(y)
        infos.append(info)
    return ys, tst_weights(len(phis)), infos


@dataclass
class GroundInfo:
    energy: float
    restarts: int
    residual_est: float
    k_eff: int


def ground_state(apply_h, x0: np.ndarray, kdim: int, max_restarts: int = 20, tol: float = 1e-10):
    """Lowest eigenpair of H by restarted Lanczos: basis of kdim vectors from the current vector,
    the lowest eigenpair (lam, z) of T (z real, unit, its largest entry positive), Ritz vector
    y = V^T z; restart from y until beta_k |z_{k-1}| <= tol max(1, |lam|) or max_restarts bases."""
    x = x0
    for r in range(max_restarts):
        b = lanczos(apply_h, x, kdim)
        k = b.k_eff
        D, S = eigh_tridiagonal(b.alpha[:k], b.beta[1:k])
        z = S[:, 0]
        z = z * (1.0 if z[np.argmax(np.abs(z))] > 0 else -1.0)
        y = combine(b, z.astype(complex))
        res = 0.0 if b.breakdown else float(b.beta[k] * abs(z[-1]))
        if res <= tol * max(1.0, abs(D[0])) or r == max_restarts - 1 or b.breakdown:
            return y, GroundInfo(float(D[0]), r + 1, res, k)
        x = y
