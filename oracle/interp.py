"""Off-grid beams by spline interpolation of grid beams (Sec. VIII, "Off-grid
angle interpolation") in float64 on the CPU.  Test infrastructure only: the
product path never imports this package.

The paper forms the beam at an off-grid direction theta* by interpolating the
beams of the few grid directions around it (8 of the 256 beams of its 128-
element line) with a spline, for every time sample.  Readings taken here
(the paper names neither the spline nor the coordinate):

* the interpolation variable is the direction cosine u = sin(theta), in
  which the beam grid of eq. (thetab) is uniform;
* the 8 neighbours are the grid beams j-3 .. j+4, where u_j <= u* < u_{j+1}
  (so u* lies in the middle interval), the window shifted inward where it
  would leave the grid; u* outside [u_0, u_{B-1}] is rejected (no
  extrapolation);
* the spline is the cubic interpolating spline with not-a-knot end
  conditions (the third derivative is continuous at the second and the
  second-to-last node), applied to the real and imaginary parts alike, so
  the interpolated beam is a real-weighted sum of the 8 beams.

For a planar (u, v) beam grid (beam b = a * bv + c at (u_a, v_c)) the same
reading is applied per axis: the tensor-product spline over the 8 x 8 grid
beams around (u*, v*), i.e. the 1-D spline along u of the 1-D splines along
v, whose weights are the products of the two axes' weights.

Two forms are written out.  ``interp_beams`` interpolates the finished
time-domain beams b_b.  The paper's own text (Sec. VIII) interpolates the
beamspace vectors instead: the stage-1 outputs w_b = F_b^H y of the grid
beams around theta* give an estimate of w* = F_*^H y, and the beam at theta*
is then formed from it like any grid beam, b* = F_u A_*^{-1} w*, with A_* the
Toeplitz system of theta* itself (``vector_interp_beams``).  The two differ
because A_b changes from beam to beam; at a grid node both return the grid
beam, and both approach the beam formed at theta* as the grid is refined.
The vectors are interpolated with their reference point at the centre of
the array (``interp_vectors``), a reading: the paper does not say where.

``spline_weights`` writes that spline out from its definition: one cubic per
interval, 4 (n - 1) unknown coefficients, fixed by interpolation at both
ends of every interval, continuity of the first and second derivatives at
the interior nodes and the two not-a-knot conditions, solved as one dense
linear system.  Since the spline is linear in the node values, the weight
of node i is the spline through the unit vector e_i, evaluated at u*.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import direct as od

__all__ = ["NEIGHBOURS", "neighbour_window", "spline_coefficients", "spline_eval",
           "spline_weights", "interp_weights", "interp_beams", "interp_weights_2d",
           "interp_beams_2d", "array_centre", "interp_vectors", "direction_problem",
           "vector_interp_beams"]

NEIGHBOURS = 8


def neighbour_window(grid_u: np.ndarray, u: float, k: int = NEIGHBOURS) -> int:
    """First index of the k grid beams used for direction u (grid_u ascending)."""
    g = np.asarray(grid_u, dtype=np.float64)
    if len(g) < k:
        raise ValueError(f"need at least {k} grid beams")
    if not (g[0] <= u <= g[-1]):
        raise ValueError("direction outside the beam grid (no extrapolation)")
    j = int(np.searchsorted(g, u, side="right")) - 1          # g[j] <= u < g[j+1]
    j = min(j, len(g) - 1)
    return int(min(max(j - (k // 2 - 1), 0), len(g) - k))


def spline_coefficients(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Coefficients [n-1, 4] (a, b, c, d) of the not-a-knot cubic spline through
    (x_i, y_i): on [x_k, x_{k+1}], S(t) = a + b s + c s^2 + d s^3 with s = t - x_k.
    Needs n >= 4 strictly increasing nodes."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(x)
    if n < 4 or np.any(np.diff(x) <= 0):
        raise ValueError("need >= 4 strictly increasing nodes")
    m = n - 1                                   # intervals
    A = np.zeros((4 * m, 4 * m))
    r = np.zeros(4 * m)
    row = 0

    def col(k, p):                              # coefficient p of interval k
        return 4 * k + p

    for k in range(m):
        h = x[k + 1] - x[k]
        A[row, col(k, 0)] = 1.0                 # S_k(x_k) = y_k
        r[row] = y[k]
        row += 1
        for p in range(4):                      # S_k(x_{k+1}) = y_{k+1}
            A[row, col(k, p)] = h ** p
        r[row] = y[k + 1]
        row += 1
    for k in range(m - 1):                      # interior node x_{k+1}
        h = x[k + 1] - x[k]
        # S_k'(x_{k+1}) - S_{k+1}'(x_{k+1}) = 0
        A[row, col(k, 1)] = 1.0
        A[row, col(k, 2)] = 2.0 * h
        A[row, col(k, 3)] = 3.0 * h * h
        A[row, col(k + 1, 1)] = -1.0
        row += 1
        # S_k''(x_{k+1}) - S_{k+1}''(x_{k+1}) = 0
        A[row, col(k, 2)] = 2.0
        A[row, col(k, 3)] = 6.0 * h
        A[row, col(k + 1, 2)] = -2.0
        row += 1
    # not-a-knot: S''' continuous at x_1 and x_{n-2}
    A[row, col(0, 3)] = 1.0
    A[row, col(1, 3)] = -1.0
    row += 1
    A[row, col(m - 2, 3)] = 1.0
    A[row, col(m - 1, 3)] = -1.0
    row += 1
    assert row == 4 * m
    return np.linalg.solve(A, r).reshape(m, 4)


def spline_eval(x: np.ndarray, coef: np.ndarray, t: float) -> float:
    """Value of the spline (nodes x, coefficients from spline_coefficients) at t
    in [x_0, x_{n-1}]."""
    x = np.asarray(x, dtype=np.float64)
    k = int(np.searchsorted(x, t, side="right")) - 1
    k = min(max(k, 0), len(x) - 2)
    s = t - x[k]
    a, b, c, d = coef[k]
    return float(a + b * s + c * s * s + d * s ** 3)


def spline_weights(x: np.ndarray, t: float) -> np.ndarray:
    """w with S(t) = sum_i w_i y_i for every data vector y: w_i is the spline
    through the unit vector e_i evaluated at t."""
    n = len(x)
    w = np.empty(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        w[i] = spline_eval(x, spline_coefficients(x, e), t)
    return w


def interp_weights(grid_u: np.ndarray, u: float, k: int = NEIGHBOURS):
    """(first neighbour index, k weights) for direction u on beam grid grid_u."""
    g = np.asarray(grid_u, dtype=np.float64)
    j0 = neighbour_window(g, u, k)
    return j0, spline_weights(g[j0:j0 + k], u)


def interp_beams(beams: np.ndarray, grid_u: np.ndarray, us) -> np.ndarray:
    """Interpolated beams at directions us from grid beams [..., B, N]:
    out[..., d, :] = sum_i w_{d,i} beams[..., j0_d + i, :]."""
    bm = np.asarray(beams)
    out = np.empty(bm.shape[:-2] + (len(us), bm.shape[-1]), dtype=np.complex128)
    for d, u in enumerate(us):
        j0, w = interp_weights(grid_u, float(u))
        out[..., d, :] = np.tensordot(w, bm[..., j0:j0 + len(w), :], axes=([0], [-2]))
    return out


def interp_weights_2d(grid_u: np.ndarray, grid_v: np.ndarray, u: float, v: float,
                      k: int = NEIGHBOURS) -> np.ndarray:
    """Weights over all bu * bv grid beams (beam b = a * bv + c) of the
    tensor-product spline at (u, v): W[a, c] = w_u[a - a0] w_v[c - c0] inside
    the two windows, zero elsewhere; returned flattened to [bu * bv]."""
    a0, wu = interp_weights(grid_u, u, k)
    c0, wv = interp_weights(grid_v, v, k)
    W = np.zeros((len(grid_u), len(grid_v)))
    W[a0:a0 + k, c0:c0 + k] = np.outer(wu, wv)
    return W.reshape(-1)


def interp_beams_2d(beams: np.ndarray, grid_u: np.ndarray, grid_v: np.ndarray, us, vs) -> np.ndarray:
    """Interpolated beams at directions (us[d], vs[d]) from planar-grid beams
    [..., bu * bv, N]."""
    bm = np.asarray(beams)
    W = np.stack([interp_weights_2d(grid_u, grid_v, float(u), float(v)) for u, v in zip(us, vs)])
    return np.moveaxis(np.tensordot(W, bm, axes=([1], [-2])), 0, -2)


def array_centre(p: od.Problem):
    """Centre of the array's extent (delay coordinates, seconds per unit
    direction cosine): the midpoints of px and of py."""
    return (0.5 * (float(np.min(p.px)) + float(np.max(p.px))),
            0.5 * (float(np.min(p.py)) + float(np.max(p.py))))


def _reference_phase(p: od.Problem, u, v, centre) -> np.ndarray:
    """exp(j (2 pi f_c + omega_l) (u c_x + v c_y)) for directions (u, v),
    shape [D, L]: the phase that moves a beamspace vector's reference point
    from the origin to the point c (eq. FthetaH: w_b[l] carries
    exp(j (2 pi f_c + omega_l) tau_{b,m}) for element m)."""
    a = 2.0 * np.pi * p.fc + od.omegas(p.L, p.eps, p.ts)
    arg = np.asarray(u, dtype=np.float64) * centre[0] + np.asarray(v, dtype=np.float64) * centre[1]
    return np.exp(1j * np.multiply.outer(arg, a))


def interp_vectors(W: np.ndarray, grid_u: np.ndarray, us, grid_v=None, vs=None,
                   p: od.Problem | None = None, centre=None) -> np.ndarray:
    """Spline estimates of beamspace vectors at directions from the grid ones
    (Sec. VIII): W [B, L] (grid beam b = a * bv + c on a plane, at p.u[b],
    p.v[b]) -> [D, L].

    Reading: the vectors are interpolated with their reference point moved
    to `centre` (p required; default None keeps the origin): w_b[l] is
    multiplied by conj(_reference_phase) of its grid direction, interpolated
    with the real spline weights, and the result multiplied by the phase of
    the target direction.  Referred to the array's centre the vectors vary
    more slowly with u (their phase no longer turns with the full aperture
    measured from one end), so the spline is more accurate; with the origin
    it is the plain interpolation of the w_b."""
    us = np.atleast_1d(np.asarray(us, dtype=np.float64))
    vs = np.zeros_like(us) if vs is None else np.atleast_1d(np.asarray(vs, dtype=np.float64))
    Wc = np.asarray(W, dtype=np.complex128)
    if centre is not None:
        Wc = Wc * np.conj(_reference_phase(p, p.u, p.v, centre))
    if grid_v is None or len(grid_v) == 1:
        out = interp_beams(Wc, grid_u, us)
    else:
        out = interp_beams_2d(Wc, grid_u, grid_v, us, vs)
    if centre is not None:
        out = out * _reference_phase(p, us, vs, centre)
    return out


def direction_problem(p: od.Problem, us, vs=None) -> od.Problem:
    """The problem of p with its beam set replaced by the directions (us, vs)."""
    u = np.atleast_1d(np.asarray(us, dtype=np.float64))
    v = np.zeros_like(u) if vs is None else np.atleast_1d(np.asarray(vs, dtype=np.float64))
    return dataclasses.replace(p, u=u, v=v)


def vector_interp_beams(y: np.ndarray, p: od.Problem, grid_u: np.ndarray, us, grid_v=None,
                        vs=None, W=None, centre="array", return_parts: bool = False):
    """The paper's off-grid beam (Sec. VIII): w* spline-interpolated from the
    beamspace vectors of the 8 (8 x 8 on a plane) grid beams around each
    direction (``interp_vectors``), then beta* = A_*^{-1} w* (A_* = F_*^H F_*
    + delta I, the Toeplitz system of the direction itself, Sec. V) and
    b* = F_u beta* (eq. bhatls).  W: the grid's beamspace vectors [B, L]
    (default: projected from y by the oracle).  centre: "array" (reference
    point of the interpolation at the array's centre), "origin", or a pair
    (c_x, c_y).  Returns [D, N] (and w*, beta* on request)."""
    if W is None:
        W = od.project(y, p)
    c = array_centre(p) if centre == "array" else (None if centre == "origin" else centre)
    ws = interp_vectors(W, grid_u, us, grid_v, vs, p=p, centre=c)
    pd = direction_problem(p, us, vs)
    beta = np.empty_like(ws)
    for d in range(pd.B):
        beta[d] = od.solve(od.toeplitz_system(pd, d), ws[d])
    out = od.reconstruct(beta, pd)
    if return_parts:
        return out, ws, beta
    return out
