"""Bias and variance of the FBST beam (Sec. VII), test oracle only.

The paper states both on the continuous interval [0, T].  The pins use two
forms:
* the paper's closed form of the variance, 2 sigma^2 sum_{k,l} Q_{kl}
  e^{j(w_k - w_l)T/2} sin((w_k - w_l)T/2)/(w_k - w_l), with
  Q = A^{-1} F^H F A^{-1} (A = F^H F + delta I);
* the same quantities at the N output times t_n (reading: the beam is only
  ever evaluated there), variance sigma^2 tr(F_u Q F_u^H) and, for a source
  that is a zero-mean band-limited Gaussian process with covariance
  P sinc(2 Omega tau) (the flat-spectrum process of Sec. VII), the mean squared
  bias tr(K C_yy K^H) - 2 Re tr(K C_ys) + tr(C_ss) with K = F_u A^{-1} F^H.
"""
from __future__ import annotations

import numpy as np

from .direct import F_matrix, Fu_matrix, omegas, Problem

__all__ = ["Q_matrix", "variance_discrete", "variance_continuous", "bias_discrete",
           "estimator_matrix"]


def Q_matrix(p: Problem, b: int) -> np.ndarray:
    """Q = (F^H F + delta I)^{-1} F^H F (F^H F + delta I)^{-1} (Sec. VII)."""
    F = F_matrix(p, b)
    T = F.conj().T @ F
    A = T + p.delta * np.eye(p.L)
    Ai = np.linalg.inv(A)
    return Ai @ T @ Ai


def estimator_matrix(p: Problem, b: int) -> np.ndarray:
    """K = F_u (F^H F + delta I)^{-1} F^H, the N x MN map from samples to beam."""
    F = F_matrix(p, b)
    A = F.conj().T @ F + p.delta * np.eye(p.L)
    return Fu_matrix(p) @ np.linalg.solve(A, F.conj().T)


def variance_discrete(p: Problem, b: int, sigma2: float) -> float:
    """E sum_n |noise part of b[n]|^2 = sigma^2 tr(F_u Q F_u^H)."""
    Fu = Fu_matrix(p)
    return float(sigma2 * np.real(np.trace(Fu @ Q_matrix(p, b) @ Fu.conj().T)))


def variance_continuous(p: Problem, b: int, sigma2: float, T: float) -> float:
    """The paper's closed form for E ||F^* A^{-1} F^H n||^2 over [0, T]."""
    Q = Q_matrix(p, b)
    w = omegas(p.L, p.eps, p.ts)
    dw = w[:, None] - w[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        kern = np.where(dw == 0.0, T / 2.0,
                        np.exp(1j * dw * T / 2.0) * np.sin(dw * T / 2.0) / np.where(dw == 0, 1.0, dw))
    return float(np.real(2.0 * sigma2 * np.sum(Q * kern)))


def _cov(tau: np.ndarray, omega: float, power: float) -> np.ndarray:
    """Covariance P sinc(2 Omega tau) of a flat-spectrum process on [-Omega, Omega]."""
    return power * np.sinc(2.0 * omega * tau)


def bias_discrete(p: Problem, b: int, u_src: float, v_src: float = 0.0,
                  power: float = 1.0) -> float:
    """E sum_n |b[n] - s(t_n)|^2 for a noise-free band-limited Gaussian source
    arriving from (u_src, v_src), with the beam steered at beam b."""
    tau = u_src * p.px + v_src * p.py                             # true delays [M]
    t = p.t
    # sample times and carrier phases of y_{m,n} = e^{-j2pi fc tau_m} s(t_n - tau_m)
    st = (t[None, :] - tau[:, None]).reshape(-1)                  # [MN]
    ph = np.repeat(np.exp(-2j * np.pi * p.fc * tau), p.N)         # [MN]
    Cyy = ph[:, None] * _cov(st[:, None] - st[None, :], p.omega, power) * ph.conj()[None, :]
    Cys = ph[:, None] * _cov(st[:, None] - t[None, :], p.omega, power)
    Css = _cov(t[:, None] - t[None, :], p.omega, power)
    K = estimator_matrix(p, b)
    val = (np.trace(K @ Cyy @ K.conj().T) - 2.0 * np.real(np.trace(K @ Cys))
           + np.trace(Css))
    return float(np.real(val))
