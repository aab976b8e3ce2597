"""The FBST itself, in float64 with numpy FFTs (test oracle only).

A second oracle, independent of ``oracle.direct``: where ``direct`` evaluates
the regularised least-squares beam b = F_u (F_b^H F_b + delta I)^{-1} F_b^H y
(eqs. betahatls, bhatls) from its sums and a dense Cholesky solve, this module
takes the paper's fast route step by step, so that every beam of a full-size
block can be checked in seconds:

* stage 1a (Sec. IV, first sum of eq. DFT_1): per element a chirp-z transform
  from N time samples to the L basis frequencies, by Bluestein's identity
  nk = (n^2 + k^2 - (k - n)^2) / 2 and one FFT convolution;
* stage 1b (Sec. IV, eq. DFT_1; App. B per axis of a grid): per frequency a
  chirp-z transform from the elements to the beams, whose rate depends on the
  frequency; elements at arbitrary positions (Sec. IX) take the plain sum;
* stage 2 (Sec. V, Fast Inverse): the Gram column c_b(d) in closed form (a
  time Dirichlet kernel times a sensor Dirichlet kernel; plain sums for
  arbitrary positions), the generator x_b = A_b^{-1} e_0 by Levinson's
  recursion (scipy.linalg.solve_toeplitz, on the real symmetric matrix left
  once the linear phase of c_b(d) is taken out where the array is uniform),
  the Gohberg-Semencul product A^{-1} w = (1/x_0)[L(x) L(x)^H w - L(y~) L(y~)^H w]
  with y~ = (0, conj x_{L-1}, ..., conj x_1), each triangular Toeplitz product
  by circulant embedding (numpy FFTs of 2L points), and F_u as a chirp-z
  transform.

It shares no code with ``direct`` or with the GPU library.  Its own rounding
is of the order of cond(A_b) times float64's unit roundoff, so it is the
all-beam check for noise-level ridges (cond ~ 1e3..1e5); the Cholesky route of
``direct`` stays the reference of record, and the two are pinned against each
other in tests/test_oracle_fbst64.py.

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see oracle/__init__.py).
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

__all__ = ["Layout", "layout_of", "czt", "stage1a", "project", "gram_column", "generator",
           "gs_apply", "reconstruct", "beams"]


def _pow2(n: int) -> int:
    return 1 << max(0, int(n - 1).bit_length())


def czt(x: np.ndarray, K: int, a, b) -> np.ndarray:
    """X[..., k] = sum_n x[..., n] exp(j (a n + b n k)), k = 0..K-1.

    Bluestein: exp(j b n k) = exp(j b n^2/2) exp(j b k^2/2) exp(-j b (k-n)^2/2),
    so X is a chirp times the linear convolution of the chirped input with the
    conjugate chirp, computed by FFTs of P >= Nin + K - 1 points.  a and b are
    scalars or arrays broadcasting over the leading axes of x (one rate per
    row, as in stage 1b)."""
    x = np.asarray(x, dtype=np.complex128)
    nin = x.shape[-1]
    P = _pow2(nin + K - 1)
    a = np.asarray(a, dtype=np.float64)[..., None]
    b = np.asarray(b, dtype=np.float64)[..., None]
    n = np.arange(nin, dtype=np.float64)
    k = np.arange(K, dtype=np.float64)
    u = x * np.exp(1j * (a * n + 0.5 * b * n * n))
    # kernel h[d] = exp(-j b d^2 / 2) for d = -(nin-1) .. K-1, placed circularly
    d = np.concatenate([np.arange(K, dtype=np.float64), np.arange(-(nin - 1), 0, dtype=np.float64)])
    h = np.exp(-0.5j * b * d * d)
    hp = np.zeros(h.shape[:-1] + (P,), dtype=np.complex128)
    hp[..., :K] = h[..., :K]
    if nin > 1:
        hp[..., P - (nin - 1):] = h[..., K:]
    conv = np.fft.ifft(np.fft.fft(u, P, axis=-1) * np.fft.fft(hp, axis=-1), axis=-1)[..., :K]
    return conv * np.exp(0.5j * b * k * k)


@dataclass(frozen=True)
class Layout:
    """Affine description of a uniform array and beam grid (Sec. IV; App. B):
    element (k, k2) at px = px0 + k dpx, py = py0 + k2 dpy (m = k my + k2), beam
    (a, c) at u = u0 + a du, v = v0 + c dv (b = a bv + c).  kind 'arbitrary'
    keeps the explicit coordinates."""
    kind: str
    mx: int = 0
    my: int = 1
    px0: float = 0.0
    dpx: float = 0.0
    py0: float = 0.0
    dpy: float = 0.0
    bu: int = 0
    bv: int = 1
    u0: float = 0.0
    du: float = 0.0
    v0: float = 0.0
    dv: float = 0.0


def _affine(v: np.ndarray):
    if len(v) == 1:
        return float(v[0]), 0.0
    step = (v[-1] - v[0]) / (len(v) - 1)
    fit = v[0] + step * np.arange(len(v))
    scale = max(np.max(np.abs(v)), 1e-300)
    return (float(v[0]), float(step)) if np.max(np.abs(fit - v)) <= 1e-12 * scale else None


def layout_of(p, shape=None) -> Layout:
    """The Layout of an oracle.direct Problem: shape = (mx, my, bu, bv) for a
    grid (element m = k my + k2, beam b = a bv + c); None for a line.  Arrays
    whose coordinates are not affine per axis are 'arbitrary'."""
    M, B = len(p.px), len(p.u)
    mx, my, bu, bv = shape if shape is not None else (M, 1, B, 1)
    px = p.px.reshape(mx, my)
    py = p.py.reshape(mx, my)
    u = p.u.reshape(bu, bv)
    v = p.v.reshape(bu, bv)
    ax, ay = _affine(px[:, 0]), _affine(py[0, :])
    au, av = _affine(u[:, 0]), _affine(v[0, :])
    uniform = (ax is not None and ay is not None and au is not None and av is not None
               and np.allclose(px, px[:, :1], rtol=0, atol=1e-15 * (1 + np.abs(px).max()))
               and np.allclose(py, py[:1, :], rtol=0, atol=1e-15 * (1 + np.abs(py).max()))
               and np.allclose(u, u[:, :1]) and np.allclose(v, v[:1, :]))
    if not uniform:
        return Layout("arbitrary")
    return Layout("grid" if shape is not None else "line", mx, my, ax[0], ax[1], ay[0], ay[1],
                  bu, bv, au[0], au[1], av[0], av[1])


def _omega(p) -> np.ndarray:
    """omega_l = 2 pi eps (l - L/2)/(L T_s), l = 1..L (eq. stfourierapprox)."""
    l = np.arange(1, p.L + 1, dtype=np.float64)
    return 2.0 * np.pi * p.eps * (l - 0.5 * p.L) / (p.L * p.ts)


def stage1a(y: np.ndarray, p) -> np.ndarray:
    """Yhat[m, l] = sum_n y[m, n] exp(-j omega_l t_n), t_n = (t0 + n) T_s, as a
    chirp-z transform per element (Sec. IV): omega_l t_n = kappa (l' + i)(t0 + n)
    with l = i + 1, l' = 1 - L/2 and kappa = 2 pi eps / L."""
    kappa = 2.0 * np.pi * p.eps / p.L
    l0 = 1.0 - 0.5 * p.L
    X = czt(y, p.L, -kappa * l0, -kappa)          # sum_n y[n] exp(-j kappa (l0 + i) n)
    i = np.arange(p.L, dtype=np.float64)
    return X * np.exp(-1j * kappa * (l0 + i) * p.t0)


def _axis_czt(Z: np.ndarray, a_l: np.ndarray, pos0: float, dpos: float, c0: float, dc: float,
              n_out: int, axis: int) -> np.ndarray:
    """out[..., c, ..., l] = sum_k Z[..., k, ..., l] exp(j a_l (pos0 + k dpos)(c0 + c dc))
    along `axis` (frequency last): one chirp-z per frequency l (App. B applies
    it per axis).  The exponent splits into a_l c0 (pos0 + k dpos) (premultiply),
    a_l dpos dc k c (the chirp-z rate of frequency l) and a_l pos0 dc c
    (postmultiply)."""
    Zt = np.moveaxis(Z, axis, -1)                                          # [..., L, k]
    k = np.arange(Zt.shape[-1], dtype=np.float64)
    c = np.arange(n_out, dtype=np.float64)
    pre = np.exp(1j * a_l[:, None] * c0 * (pos0 + k * dpos)[None, :])      # [L, k]
    X = czt(Zt * pre, n_out, 0.0, a_l * dpos * dc)
    post = np.exp(1j * a_l[:, None] * pos0 * dc * c[None, :])              # [L, c]
    return np.moveaxis(X * post, -1, axis)


def project(y: np.ndarray, p, lay: Layout | None = None, yhat=None) -> np.ndarray:
    """W[b, l] = [F_b^H y]_l = sum_m Yhat[m, l] exp(j (2 pi f_c + omega_l) tau_{b,m})
    (eq. sum_1, regrouped as eq. DFT_1): for uniform arrays one chirp-z per
    frequency and axis (Sec. IV; App. B), else the plain sum over elements
    (Sec. IX)."""
    lay = layout_of(p) if lay is None else lay
    if yhat is None:
        yhat = stage1a(y, p)
    a_l = 2.0 * np.pi * p.fc + _omega(p)                      # [L]
    if lay.kind == "arbitrary":
        tau = np.multiply.outer(p.u, p.px) + np.multiply.outer(p.v, p.py)  # [B, M]
        out = np.empty((len(p.u), p.L), dtype=np.complex128)
        for b in range(len(p.u)):
            out[b] = np.sum(np.exp(1j * np.multiply.outer(tau[b], a_l)) * yhat, axis=0)
        return out
    Z = yhat.reshape(lay.mx, lay.my, p.L)
    # x axis: tau_x = (u0 + a du)(px0 + k dpx); y axis: (v0 + c dv)(py0 + k2 dpy)
    Z = _axis_czt(Z, a_l, lay.px0, lay.dpx, lay.u0, lay.du, lay.bu, axis=0)   # [bu, my, L]
    if lay.my > 1 or lay.bv > 1 or lay.py0 != 0.0:
        Z = _axis_czt(Z, a_l, lay.py0, lay.dpy, lay.v0, lay.dv, lay.bv, axis=1)  # [bu, bv, L]
    return Z.reshape(lay.bu * lay.bv, p.L)


def _dirichlet(x: np.ndarray, K: int) -> np.ndarray:
    """The real factor D_K(x) of sum_{k<K} exp(j k x) = exp(j x (K-1)/2) D_K(x),
    D_K(x) = sin(K x/2) / sin(x/2).  With x = r + 2 pi m, |r| <= pi, it equals
    (-1)^(m (K-1)) sin(K r/2) / sin(r/2), evaluated on the reduced r (K at r = 0)
    so that the ratio stays accurate near multiples of 2 pi."""
    x = np.asarray(x, dtype=np.float64)
    m = np.round(x / (2.0 * np.pi))
    r = x - 2.0 * np.pi * m
    sign = np.where((m.astype(np.int64) * (K - 1)) % 2 == 0, 1.0, -1.0)
    out = np.empty_like(r)
    tiny = np.abs(r) < 1e-8
    out[tiny] = K * (1.0 - (K * K - 1.0) * r[tiny] ** 2 / 24.0)
    rr = r[~tiny]
    out[~tiny] = np.sin(0.5 * K * rr) / np.sin(0.5 * rr)
    return sign * out


def gram_column(p, b: int, lay: Layout | None = None):
    """c_b(d) = [F_b^H F_b]_{l+d, l}, d = 0..L-1 (Sec. V): the time sum
    sum_n exp(-j w_d t_n) times the sensor sum sum_m exp(j w_d tau_{b,m}),
    w_d = 2 pi eps d / (L T_s).  For uniform arrays both are Dirichlet kernels
    and c_b(d) = exp(j d phi) R(d) with R real; returns (R, phi), or (c, None)
    for arbitrary positions (plain sums)."""
    lay = layout_of(p) if lay is None else lay
    d = np.arange(p.L, dtype=np.float64)
    wd = 2.0 * np.pi * p.eps * d / p.L                         # per sample (T_s units)
    # time: sum_n exp(-j wd (t0 + n)) = exp(-j wd (t0 + (N-1)/2)) D_N(wd)
    rt = _dirichlet(wd, p.N)
    phi = -2.0 * np.pi * p.eps / p.L * (p.t0 + 0.5 * (p.N - 1))
    wdt = wd / p.ts                                            # rad per second of delay
    if lay.kind == "arbitrary":
        tau = p.u[b] * p.px + p.v[b] * p.py
        ss = np.exp(1j * np.multiply.outer(wdt, tau)).sum(axis=1)
        return rt * np.exp(1j * d * phi) * ss, None
    a, c = divmod(b, lay.bv)
    u, v = lay.u0 + a * lay.du, lay.v0 + c * lay.dv
    # x: sum_k exp(j wd u (px0 + k dpx)); y: sum_k2 exp(j wd v (py0 + k2 dpy))
    rx = _dirichlet(wdt * u * lay.dpx, lay.mx)
    ry = _dirichlet(wdt * v * lay.dpy, lay.my)
    phi += 2.0 * np.pi * p.eps / (p.L * p.ts) * (u * (lay.px0 + 0.5 * (lay.mx - 1) * lay.dpx)
                                                 + v * (lay.py0 + 0.5 * (lay.my - 1) * lay.dpy))
    return rt * rx * ry, phi


def generator(p, b: int, lay: Layout | None = None) -> np.ndarray:
    """x_b = A_b^{-1} e_0, A_b = F_b^H F_b + delta I (Sec. V), by Levinson's
    recursion.  Uniform arrays: A_b = D (R + delta I) D^H with D = diag(exp(j l phi)),
    so x_b[l] = exp(j l phi) [(R + delta I)^{-1} e_0][l] (a real solve)."""
    c, phi = gram_column(p, b, lay)
    c = c.copy()
    c[0] += p.delta
    e0 = np.zeros(p.L)
    e0[0] = 1.0
    if phi is None:
        return sla.solve_toeplitz((c, np.conj(c)), e0.astype(np.complex128), check_finite=False)
    xr = sla.solve_toeplitz(c, e0, check_finite=False)
    return xr * np.exp(1j * phi * np.arange(p.L))


def gs_apply(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """A^{-1} w for Hermitian Toeplitz A with first inverse column x (Sec. V):
    (1/x_0) [L(x) L(x)^H w - L(y~) L(y~)^H w], y~ = (0, conj x_{L-1}, ..., conj x_1),
    L(.) lower-triangular Toeplitz; L(g)^H w is a correlation and L(g) p a
    convolution, both by circulant embedding in 2L points.  x, w: [..., L]."""
    L = x.shape[-1]
    P = 2 * L
    yt = np.zeros_like(x)
    yt[..., 1:] = np.conj(x[..., :0:-1])
    W = np.fft.fft(w, P, axis=-1)
    out = np.zeros(np.broadcast_shapes(x.shape, w.shape), dtype=np.complex128)
    for g, sign in ((x, 1.0), (yt, -1.0)):
        G = np.fft.fft(g, P, axis=-1)
        corr = np.fft.ifft(np.conj(G) * W, axis=-1)[..., :L]          # L(g)^H w
        conv = np.fft.ifft(G * np.fft.fft(corr, P, axis=-1), axis=-1)[..., :L]
        out += sign * conv
    return out / x[..., :1]


def reconstruct(beta: np.ndarray, p) -> np.ndarray:
    """b[n] = sum_l beta[l] exp(j omega_l t_n) (eq. bhatls), F_u as a chirp-z
    transform in n (Sec. V, last paragraph)."""
    kappa = 2.0 * np.pi * p.eps / p.L
    l0 = 1.0 - 0.5 * p.L
    i = np.arange(p.L, dtype=np.float64)
    pre = np.exp(1j * kappa * (l0 + i) * p.t0)
    X = czt(beta * pre, p.N, 0.0, kappa)                    # sum_i beta_i exp(j kappa i n)
    n = np.arange(p.N, dtype=np.float64)
    return X * np.exp(1j * kappa * l0 * n)


def _generators(p, lay: Layout, idx) -> np.ndarray:
    idx = list(idx)
    cost = len(idx) * p.L * p.L
    workers = min(16, os.cpu_count() or 1)
    if cost < 4e9 or workers < 2:
        return np.stack([generator(p, int(b), lay) for b in idx])
    # large systems: Levinson per beam in worker processes (spawned, so they
    # start from a fresh interpreter with no device state)
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        return np.stack(list(ex.map(_generator_job, [(p, int(b), lay) for b in idx],
                                    chunksize=max(1, len(idx) // (4 * workers)))))


def _generator_job(args):
    p, b, lay = args
    return generator(p, b, lay)


def beams(y: np.ndarray, p, shape=None, beam_idx=None, return_parts: bool = False):
    """All (or the requested) beams [B', N]: stage 1a, stage 1b, then per beam
    the Gohberg-Semencul product and F_u (Secs. IV and V).  shape = (mx, my,
    bu, bv) for a grid."""
    lay = layout_of(p, shape)
    W = project(y, p, lay)
    idx = np.arange(len(p.u)) if beam_idx is None else np.asarray(beam_idx)
    Wi = W[idx]
    X = _generators(p, lay, idx)
    beta = gs_apply(X, Wi)
    out = reconstruct(beta, p)
    if return_parts:
        return out, Wi, beta
    return out
