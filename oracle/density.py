"""Reduced density matrix of the time-step targets and its truncation, in FP64 (oracle, test only).

Sec. II.B: the density matrix that decides which system states to keep is built from every
target vector with its weight,
    rho = sum_l w_l Tr_E |phi_l><phi_l|,
and the m eigenvectors of rho with the largest eigenvalues are kept; the sum of the discarded
eigenvalues is the truncation error.  The weights are those of time-step targeting (the ground
state and the four time vectors; see oracle.krylov.tst_weights).

Every target lies in one (N_up, N_dn) sector, so a target is a set of blocks Psi_{l,p}
(dim_S(p) x dim_E(q), q = target - p) and rho is block diagonal over the system sectors p:
    rho_p = sum_l w_l Psi_{l,p} Psi_{l,p}^H.
(The printed density-matrix equation places the conjugate transpose first, which would give the
complex conjugate of this matrix; the spectrum is the same, and this form is the one whose
eigenvectors span the system states.)

Truncation: the eigenvalues of all sectors are ranked together (largest first; equal values
by sector, then by position in the sector's descending order) and the first m are kept;
kept[p] counts them per sector.
Pins (tests): trace rho = sum_l w_l ||phi_l||^2; rho_p Hermitian and positive semidefinite; its
eigenvalues equal the squared singular values of [sqrt(w_l) Psi_{l,p}]_l (an SVD, not an
eigensolver); a single product-state target gives one non-zero eigenvalue; keeping every state
discards nothing.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from oracle import matvec as M


def density_blocks(pb, vecs, weights) -> dict:
    """{p: rho_p} (complex Hermitian dim_S(p) x dim_S(p)) for flat [Re | Im] target vectors."""
    rho = {}
    for x, w in zip(vecs, weights):
        for p, blk in M.unpack(pb, x).items():
            term = w * (blk @ blk.conj().T)
            rho[p] = rho[p] + term if p in rho else term
    return rho


@dataclass
class Truncation:
    sectors: list          # system sectors p in layout order
    evals: dict            # p -> eigenvalues, descending
    evecs: dict            # p -> eigenvectors as columns, in the order of evals
    kept: dict             # p -> number kept
    trunc_err: float       # sum of the discarded eigenvalues
    trace: float


def truncate(pb, vecs, weights, keep: int) -> Truncation:
    """Eigen-decomposition of every rho_p and the global choice of the `keep` largest states."""
    rho = density_blocks(pb, vecs, weights)
    lay, _ = M.layout(pb)
    sectors = [p for (p, q, r, c, off) in lay]
    evals, evecs, cand = {}, {}, []
    for p in sectors:
        lam, vec = np.linalg.eigh(rho[p])            # ascending
        lam, vec = lam[::-1], vec[:, ::-1]           # descending
        evals[p], evecs[p] = lam, vec
        for i, v in enumerate(lam):
            cand.append((-v, p, i))
    cand.sort()
    kept = {p: 0 for p in sectors}
    for (_, p, i) in cand[:keep]:
        kept[p] += 1
    total = float(sum(np.sum(evals[p]) for p in sectors))
    kept_sum = float(sum(np.sum(evals[p][:kept[p]]) for p in sectors))
    return Truncation(sectors, evals, evecs, kept, total - kept_sum, total)
