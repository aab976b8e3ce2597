"""Beamspace interference nulling (Sec. VIII, "Interference cancellation") in
float64 on the CPU.  Test infrastructure only: the product path never
imports this package.

For interferer directions q (beams of the problem's own grid), the nulled
Fourier coefficients of beam b are (eq. interfer_beam_space)

    tilde beta_b = A_b^{-1} (w_b - sum_q G_{b,q} w_q),
    G_{b,q} = F_b^H F_q (F_q^H F_q + delta I)^{-1} = C_{b,q} A_q^{-1},

with w = F^H y the beamspace vectors of Sec. IV, and the nulled beam is
F_u tilde beta_b (eq. bhatls).  Equivalently (the paper derives the
beamspace form from it) it is the FBST of the array data with each
interferer's regularised least-squares fit removed,
y - sum_q F_q A_q^{-1} F_q^H y; ``nulled_beams_dense`` takes that route with
explicit matrices for tiny sizes, which pins the beamspace form.

Reading: for several interferers the paper sums the separate projections
(its footnote calls the projection approximate); so does this oracle.

Interferers off the beam grid (Sec. VIII, closing paragraph of interference
cancellation): the expressions need only the interferer's beam vector w_q
and G_{b,q} at its direction.  ``nulled_beams`` takes such a direction as an
extra beam of an extended problem and either projects w_q = F_q^H y exactly
or takes it from the caller; ``nulled_beams_interp`` takes it the paper's
way, spline-interpolated from the beamspace vectors of the grid beams around
the interferer (oracle.interp).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import direct as od
from . import interp as oi

__all__ = ["cross_gram", "nulled_beams", "nulled_beams_dense", "extended_problem",
           "nulled_beams_interp"]


def cross_gram(p: od.Problem, b: int, q: int) -> np.ndarray:
    """C_{b,q} = F_b^H F_q, L x L (Sec. VIII).

    [F_b^H F_q]_{l,k} = sum_{m,n} exp(-j (omega_l - omega_k) t_n)
                                  exp(j ((2 pi f_c + omega_l) tau_{b,m} - (2 pi f_c + omega_k) tau_{q,m}))
    (from the entries of F in eq. FthetaH); the exponent splits into a time
    part and a sensor part, so the double sum is the product of the time sum
    and the sensor sum.  For q = b it is the Gram matrix of Sec. V."""
    w = od.omegas(p.L, p.eps, p.ts)
    tau = od.delays(p)
    a = 2.0 * np.pi * p.fc + w                                   # [L]
    dw = np.subtract.outer(w, w)                                 # omega_l - omega_k
    time_sum = np.exp(-1j * np.multiply.outer(dw, p.t)).sum(axis=-1)          # [L, L]
    Eb = np.exp(1j * np.multiply.outer(tau[b], a))               # [M, L]: e^{j a_l tau_{b,m}}
    Eq = np.exp(1j * np.multiply.outer(tau[q], a))               # [M, L]
    sensor_sum = Eb.T @ np.conj(Eq)                              # sum over m
    return time_sum * sensor_sum


def nulled_beams(y: np.ndarray, p: od.Problem, interferers, beam_idx=None,
                 return_parts: bool = False, interferer_vectors=None):
    """Beams with the interferers nulled in beamspace (eq. interfer_beam_space),
    shape [len(beam_idx), N].  interferer_vectors: the w_q to use, one row per
    interferer (default: F_q^H y projected from y)."""
    idx = np.arange(p.B) if beam_idx is None else np.asarray(beam_idx)
    interferers = [int(q) for q in interferers]
    need = sorted(set(int(b) for b in idx) | set(interferers))
    W = dict(zip(need, od.project(y, p, need)))
    if interferer_vectors is not None:
        for q, wq in zip(interferers, np.asarray(interferer_vectors)):
            W[q] = np.asarray(wq, dtype=np.complex128)
    beta_q = {q: od.solve(od.toeplitz_system(p, q), W[q]) for q in interferers}
    wt = np.empty((len(idx), p.L), dtype=np.complex128)
    beta = np.empty_like(wt)
    for i, b in enumerate(idx):
        b = int(b)
        wt[i] = W[b] - sum((cross_gram(p, b, q) @ beta_q[q] for q in interferers),
                           np.zeros(p.L, dtype=np.complex128))
        beta[i] = od.solve(od.toeplitz_system(p, b), wt[i])
    out = od.reconstruct(beta, p)
    if return_parts:
        return out, wt, beta
    return out


def nulled_beams_dense(y: np.ndarray, p: od.Problem, interferers) -> np.ndarray:
    """The array-space route with explicit matrices (tiny sizes): remove from y
    each interferer's fit F_q (F_q^H F_q + delta I)^{-1} F_q^H y, then the
    dense FBST of the result."""
    yv = np.asarray(y, dtype=np.complex128).reshape(-1)           # m' = m * N + n
    fit = np.zeros_like(yv)
    for q in interferers:
        F = od.F_matrix(p, int(q))
        A = F.conj().T @ F + p.delta * np.eye(p.L)
        fit += F @ np.linalg.solve(A, F.conj().T @ yv)
    return od.beams_dense((yv - fit).reshape(p.M, p.N), p)


def extended_problem(p: od.Problem, uq, vq=None) -> od.Problem:
    """p with the directions (uq, vq) appended as beams B, B + 1, ..."""
    uq = np.atleast_1d(np.asarray(uq, dtype=np.float64))
    vq = np.zeros_like(uq) if vq is None else np.atleast_1d(np.asarray(vq, dtype=np.float64))
    return dataclasses.replace(p, u=np.r_[p.u, uq], v=np.r_[p.v, vq])


def nulled_beams_interp(y: np.ndarray, p: od.Problem, grid_u, uq, grid_v=None, vq=None,
                        beam_idx=None, W=None, centre="array", return_parts: bool = False):
    """Grid beams of p with interferers at directions (uq, vq) nulled the
    paper's way (Sec. VIII): each w_q is the spline estimate from the
    beamspace vectors of the 8 (8 x 8) grid beams around it, G_{b,q} is taken
    at the interferer's direction, then eq. interfer_beam_space.  W: the
    grid's beamspace vectors [B, L] (default: projected from y); centre as
    in oracle.interp.vector_interp_beams."""
    if W is None:
        W = od.project(y, p)
    c = oi.array_centre(p) if centre == "array" else (None if centre == "origin" else centre)
    wq = oi.interp_vectors(W, grid_u, uq, grid_v, vq, p=p, centre=c)
    pe = extended_problem(p, uq, vq)
    idx = np.arange(p.B) if beam_idx is None else np.asarray(beam_idx)
    return nulled_beams(y, pe, list(range(p.B, pe.B)), beam_idx=idx, return_parts=return_parts,
                        interferer_vectors=wq)
