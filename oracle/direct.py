"""The FBST beam from its definition, in float64 on the CPU (test oracle only).

Every function cites the passage of the paper (Singh, DeLude, Davenport,
Romberg, "A Fast Broadband Beamspace Transformation") it follows.  Nothing
here uses an FFT or a chirp-z transform: sums are evaluated as written, with
matrix products as the only library primitive, and the linear system is
solved by a dense Cholesky factorisation (LAPACK).

Conventions (readings where the paper is silent or garbled):
* t_n = n T_s with n = 0..N-1.  The beams do not depend on the time origin
  (a shift multiplies F and F_u by the same unitary diagonal); a test pins it.
* l = 1..L and l' = l - L/2 as printed (Sec. III-A, eq. stfourierapprox);
  arrays store l at index l - 1.  L must be even.
* The reference point of the delays is the coordinate origin: element 0 of
  a line, element (0, 0) of a grid, unless the array gives offsets.
* Beam grid: odd B uses eq. (thetab); for even B the printed formula exceeds 1
  at b = B, so the symmetric rule sin(theta_b) = (2b - B - 1)/B is used.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np
import scipy.linalg as sla

__all__ = [
    "Problem", "beam_grid", "omegas", "delays", "F_matrix", "Fu_matrix",
    "stage1a", "project", "gram_column", "toeplitz_system", "generator",
    "solve", "reconstruct", "beams", "beams_dense",
]


@dataclass(frozen=True)
class Problem:
    """One array, band, basis and beam set.

    px, py: per-element delay coordinates in seconds per unit direction
    cosine, so tau_{b,m} = u_b px_m + v_b py_m (Sec. III, tau = p_m^T theta).
    u, v: direction cosines of the B beams.
    """
    N: int
    L: int
    eps: float
    delta: float
    fc: float
    omega: float
    ts: float
    px: np.ndarray
    py: np.ndarray
    u: np.ndarray
    v: np.ndarray
    t0: float = 0.0          # time origin: t_n = (t0 + n) T_s

    @property
    def M(self) -> int:
        return len(self.px)

    @property
    def B(self) -> int:
        return len(self.u)

    @property
    def t(self) -> np.ndarray:
        return (self.t0 + np.arange(self.N, dtype=np.float64)) * self.ts


def beam_grid(B: int) -> np.ndarray:
    """sin(theta_b) for b = 1..B: eq. (thetab), (2b - B - 1)/(B - 1) for odd B;
    (2b - B - 1)/B for even B (symmetric reading of the garbled even rule)."""
    b = np.arange(1, B + 1, dtype=np.float64)
    if B == 1:
        return np.zeros(1)
    den = (B - 1) if (B % 2 == 1) else B
    return (2.0 * b - B - 1.0) / den


def omegas(L: int, eps: float, ts: float) -> np.ndarray:
    """omega_l = 2 pi eps (l - L/2) / (L T_s), l = 1..L (eq. stfourierapprox)."""
    l = np.arange(1, L + 1, dtype=np.float64)
    return 2.0 * np.pi * eps * (l - L / 2.0) / (L * ts)


def delays(p: Problem) -> np.ndarray:
    """tau_{b,m} = p_m^T theta_b (Sec. III), shape [B, M]."""
    return np.multiply.outer(p.u, p.px) + np.multiply.outer(p.v, p.py)


def F_matrix(p: Problem, b: int) -> np.ndarray:
    """The MN x L matrix of eq. (FthetaH) for beam b; row m' = m * N + n.

    [F]_{(m,n),l} = exp(-j 2 pi f_c tau_m) exp(j omega_l (t_n - tau_m)).
    Tiny sizes only (brute-force pin)."""
    tau = delays(p)[b]                                        # [M]
    w = omegas(p.L, p.eps, p.ts)                              # [L]
    tt = (p.t[None, :] - tau[:, None]).reshape(-1)            # [M*N]
    car = np.repeat(np.exp(-2j * np.pi * p.fc * tau), p.N)    # [M*N]
    return car[:, None] * np.exp(1j * np.multiply.outer(tt, w))


def Fu_matrix(p: Problem) -> np.ndarray:
    """[F_u]_{n,l} = exp(j omega_l t_n) (eq. bhatls), shape [N, L]."""
    return np.exp(1j * np.multiply.outer(p.t, omegas(p.L, p.eps, p.ts)))


def stage1a(y: np.ndarray, p: Problem) -> np.ndarray:
    """hat y_{m,l} = sum_n y_{m,n} exp(-j omega_l t_n)  (Sec. IV, the first of
    the two sums of eq. (DFT_1)), shape [M, L]."""
    E = np.exp(-1j * np.multiply.outer(p.t, omegas(p.L, p.eps, p.ts)))   # [N, L]
    return np.asarray(y, dtype=np.complex128) @ E


def project(y: np.ndarray, p: Problem, beam_idx=None, yhat=None) -> np.ndarray:
    """w_b = F_b^H y for the requested beams, shape [len(beam_idx), L].

    Eq. (sum_1): [F^H y]_l = sum_{n,m} y_m[n] exp(j (2 pi f_c tau_m
    - omega_l t_n + omega_l tau_m)); the sum over n is taken first (stage1a)
    and the sum over m second, which only regroups the double sum."""
    if yhat is None:
        yhat = stage1a(y, p)
    idx = np.arange(p.B) if beam_idx is None else np.asarray(beam_idx)
    tau = delays(p)
    w = omegas(p.L, p.eps, p.ts)
    out = np.empty((len(idx), p.L), dtype=np.complex128)
    for i, b in enumerate(idx):
        ph = np.exp(1j * np.multiply.outer(tau[b], 2.0 * np.pi * p.fc + w))   # [M, L]
        out[i] = np.sum(ph * yhat, axis=0)
    return out


def gram_column(p: Problem, b: int) -> np.ndarray:
    """c_b(d) = [F_b^H F_b]_{l+d, l}, d = 0..L-1 (Sec. V, Fast Inverse).

    The entry is sum_{m,n} exp(-j (omega_l - omega_k)(t_n - tau_{b,m})) with
    l - k = d, i.e. a function of d alone (Toeplitz); the exponent splits into
    a time factor and a sensor factor, so the double sum is the product of
    the two single sums."""
    tau = delays(p)[b]
    dw = 2.0 * np.pi * p.eps * np.arange(p.L, dtype=np.float64) / (p.L * p.ts)   # omega_l - omega_k
    st = np.exp(-1j * np.multiply.outer(dw, p.t)).sum(axis=1)
    ss = np.exp(1j * np.multiply.outer(dw, tau)).sum(axis=1)
    return st * ss


def toeplitz_system(p: Problem, b: int) -> np.ndarray:
    """A_b = F_b^H F_b + delta I (Sec. V), Hermitian Toeplitz, L x L."""
    c = gram_column(p, b)
    A = sla.toeplitz(c, np.conj(c))
    A[np.diag_indices(p.L)] += p.delta
    return A


def solve(A: np.ndarray, w: np.ndarray) -> np.ndarray:
    """beta = A^{-1} w by dense Cholesky (A is Hermitian positive definite
    for delta > 0), eq. (betahatls)."""
    cf = sla.cho_factor(A, lower=True, check_finite=False)
    return sla.cho_solve(cf, w, check_finite=False)


def generator(p: Problem, b: int) -> np.ndarray:
    """First column of A_b^{-1} (the generating vector x of the
    Gohberg-Semencul representation in Sec. V)."""
    e0 = np.zeros(p.L, dtype=np.complex128)
    e0[0] = 1.0
    return solve(toeplitz_system(p, b), e0)


def reconstruct(beta: np.ndarray, p: Problem) -> np.ndarray:
    """b = F_u beta (eq. bhatls); beta may be [L] or [B', L]."""
    return np.asarray(beta) @ Fu_matrix(p).T


def beams(y: np.ndarray, p: Problem, beam_idx=None, return_parts: bool = False):
    """All (or the requested) beams, shape [len(beam_idx), N].

    hat beta_b = (F_b^H F_b + delta I)^{-1} F_b^H y and b_b = F_u hat beta_b
    (eqs. betahatls, bhatls)."""
    idx = np.arange(p.B) if beam_idx is None else np.asarray(beam_idx)
    W = project(y, p, idx)
    beta = np.empty_like(W)
    for i, b in enumerate(idx):
        beta[i] = solve(toeplitz_system(p, int(b)), W[i])
    out = reconstruct(beta, p)
    if return_parts:
        return out, W, beta
    return out


def beams_dense(y: np.ndarray, p: Problem) -> np.ndarray:
    """Brute force with explicit matrices (eqs. FthetaH, betahatls, bhatls);
    tiny sizes only."""
    yv = np.asarray(y, dtype=np.complex128).reshape(-1)          # m' = m * N + n
    Fu = Fu_matrix(p)
    out = np.empty((p.B, p.N), dtype=np.complex128)
    for b in range(p.B):
        F = F_matrix(p, b)
        A = F.conj().T @ F + p.delta * np.eye(p.L)
        out[b] = Fu @ np.linalg.solve(A, F.conj().T @ yv)
    return out


def make_problem(*, N, L, eps, delta, fc, omega, ts, px, py=None, u, v=None, t0=0.0) -> Problem:
    px = np.asarray(px, dtype=np.float64)
    py = np.zeros_like(px) if py is None else np.asarray(py, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    v = np.zeros_like(u) if v is None else np.asarray(v, dtype=np.float64)
    if L % 2:
        raise ValueError("L must be even (Sec. III-A)")
    return Problem(N=N, L=L, eps=eps, delta=delta, fc=fc, omega=omega, ts=ts,
                   px=px, py=py, u=u, v=v, t0=t0)


def line_problem(M, N, B, *, fc, omega=0.5, ts=1.0, eps=1.01, gamma=2, delta=1e-5,
                 x0=0.0, spacing=None, u=None) -> Problem:
    """Uniform line, lambda/2 spacing at f_c + Omega (Sec. IV), on the beam grid
    of eq. (thetab) unless u is given."""
    d = 1.0 / (2.0 * (fc + omega)) if spacing is None else spacing
    px = (x0 + np.arange(M, dtype=np.float64)) * d
    uu = beam_grid(B) if u is None else np.asarray(u, dtype=np.float64)
    return make_problem(N=N, L=int(round(gamma * N)), eps=eps, delta=delta, fc=fc,
                        omega=omega, ts=ts, px=px, u=uu)


def grid_problem(mx, my, bu, bv, N, *, fc, omega=0.5, ts=1.0, eps=1.01, gamma=2,
                 delta=1e-5) -> Problem:
    """mx x my grid with lambda/2 spacing at f_c + Omega on both axes (App. B),
    beams on the separable (u, v) grid, each axis by the rule of eq. (thetab);
    element m = k * my + k2 and beam b = a * bv + c."""
    d = 1.0 / (2.0 * (fc + omega))
    k = np.arange(mx, dtype=np.float64)
    k2 = np.arange(my, dtype=np.float64)
    px = np.repeat(k * d, my)
    py = np.tile(k2 * d, mx)
    ua = beam_grid(bu)
    vc = beam_grid(bv)
    u = np.repeat(ua, bv)
    v = np.tile(vc, bu)
    return make_problem(N=N, L=int(round(gamma * N)), eps=eps, delta=delta, fc=fc,
                        omega=omega, ts=ts, px=px, py=py, u=u, v=v)
