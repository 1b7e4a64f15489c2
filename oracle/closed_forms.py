"""Non-interacting (U = 0) closed forms used as pins (oracle, test only).

* Open-chain tight-binding levels e_k = -2 t cos(k pi / (L+1)) with modes
  phi_k(j) = sqrt(2/(L+1)) sin(k pi j / (L+1)), j = 1..L (site index + 1).
* App. A: one-site excitation of the half-filled non-interacting ground state,
  X_ij(t) = R_i R_j - |T_ij(t)|^2 with R_i = sum' |U_il|^2 and
  T_ij(t) = sum' conj(U_il) U_jl exp(-i E_l t), the prime restricting to occupied levels.
* App. B / Eq. (nd): holon-doublon density at t = 0 is 0 on the holon site, 2 on the doublon
  site and 1 elsewhere; Sec. III.B.2: double occupation at t = 0 is 1 on the doublon site and 0
  on the holon site.
"""
from __future__ import annotations

import numpy as np


def chain_levels(L: int, t: float = 1.0):
    """Tight-binding levels and modes of the open chain with -t hopping, ascending energy.
    Returns (E[L], U[L, L]) with U[j, k] = phi_k(j) (site j is 0-based here)."""
    k = np.arange(1, L + 1)
    E = -2.0 * t * np.cos(k * np.pi / (L + 1))
    j = np.arange(1, L + 1)
    Umat = np.sqrt(2.0 / (L + 1)) * np.sin(np.outer(j, k) * np.pi / (L + 1))
    order = np.argsort(E)
    return E[order], Umat[:, order]


def hopping_matrix(L: int, bonds) -> np.ndarray:
    """Single-particle matrix of -sum t_ij (c+_i c_j + h.c.)."""
    h = np.zeros((L, L))
    for (i, j, t) in bonds:
        h[i, j] -= t
        h[j, i] -= t
    return h


def free_ground_energy(E: np.ndarray, nup: int, ndn: int) -> float:
    Es = np.sort(E)
    return float(Es[:nup].sum() + Es[:ndn].sum())


def onesite_excitation(E: np.ndarray, Umat: np.ndarray, nocc: int, i: int, j: int, t):
    """App. A: X_ij(t) = R_i R_j - |T_ij(t)|^2 for the half-filled free ground state."""
    occ = slice(0, nocc)
    R = np.sum(np.abs(Umat[:, occ]) ** 2, axis=1)
    t = np.atleast_1d(np.asarray(t, dtype=float))
    T = np.array([np.sum(np.conj(Umat[i, occ]) * Umat[j, occ] * np.exp(-1j * E[occ] * tt))
                  for tt in t])
    return R[i] * R[j] - np.abs(T) ** 2


def holon_doublon_density_t0(L: int, i: int, j: int) -> np.ndarray:
    """Eq. (nd): O_{j,i,p}(0) summed over spin, for every site p."""
    out = np.ones(L)
    out[i] = 0.0
    out[j] = 2.0
    return out
