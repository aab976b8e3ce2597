"""Pins of the spline interpolation oracle (Sec. VIII, off-grid angle
interpolation) against things other than itself: scipy's cubic spline with
the same end conditions, exact reproduction of cubics (a property of the
not-a-knot spline), interpolation at the nodes, and the paper's Fig. 3(d)
setting (a 128-element line, 256 beams, theta* = pi/3), where the beam
interpolated from 8 grid beams must be close to the beam formed at theta*."""
import numpy as np
import pytest
from scipy.interpolate import CubicSpline, RectBivariateSpline

from oracle import direct as od
from oracle import interp as oi


def test_matches_scipy_not_a_knot():
    rng = np.random.default_rng(11)
    for n in (4, 5, 8, 11):
        x = np.cumsum(rng.uniform(0.2, 1.5, n))
        y = rng.standard_normal(n)
        coef = oi.spline_coefficients(x, y)
        ref = CubicSpline(x, y, bc_type="not-a-knot")
        for t in np.concatenate([rng.uniform(x[0], x[-1], 25), x]):
            assert abs(oi.spline_eval(x, coef, t) - float(ref(t))) < 1e-12 * (1 + abs(ref(t)))
        w = oi.spline_weights(x, float(x[1] + 0.3 * (x[2] - x[1])))
        assert abs(w @ y - float(ref(x[1] + 0.3 * (x[2] - x[1])))) < 1e-12


def test_reproduces_cubics_exactly():
    rng = np.random.default_rng(12)
    x = np.sort(rng.uniform(-1, 1, 8))
    c = rng.standard_normal(4)
    f = lambda t: c[0] + c[1] * t + c[2] * t * t + c[3] * t ** 3
    for t in rng.uniform(x[0], x[-1], 20):
        assert abs(oi.spline_weights(x, t) @ f(x) - f(t)) < 1e-12
    # a quartic is not reproduced: the pin would catch a wrong end condition
    g = lambda t: t ** 4
    errs = [abs(oi.spline_weights(x, t) @ g(x) - g(t)) for t in rng.uniform(x[0], x[-1], 20)]
    assert max(errs) > 1e-6


def test_nodes_and_partition_of_unity():
    x = np.linspace(0.0, 7.0, 8)
    for i in range(8):
        w = oi.spline_weights(x, x[i])
        assert np.allclose(w, np.eye(8)[i], atol=1e-13)
    for t in np.linspace(0.0, 7.0, 29):
        assert abs(oi.spline_weights(x, t).sum() - 1.0) < 1e-13


def test_neighbour_window():
    g = od.beam_grid(32)
    du = g[1] - g[0]
    assert oi.neighbour_window(g, g[10] + 0.5 * du) == 7          # j = 10: 7 .. 14
    assert oi.neighbour_window(g, g[10]) == 7                     # on a node
    assert oi.neighbour_window(g, g[0]) == 0                      # shifted inward
    assert oi.neighbour_window(g, g[1] + 0.2 * du) == 0
    assert oi.neighbour_window(g, g[-1]) == 24                    # last node
    assert oi.neighbour_window(g, g[-2] + 0.9 * du) == 24
    with pytest.raises(ValueError):
        oi.neighbour_window(g, g[-1] + 1e-9)
    with pytest.raises(ValueError):
        oi.neighbour_window(od.beam_grid(7), 0.0)


def test_interp_beams_is_weighted_sum():
    rng = np.random.default_rng(13)
    g = od.beam_grid(16)
    bm = rng.standard_normal((2, 16, 5)) + 1j * rng.standard_normal((2, 16, 5))
    us = [g[3] + 0.37 * (g[4] - g[3]), g[0], g[15]]
    out = oi.interp_beams(bm, g, us)
    for d, u in enumerate(us):
        j0, w = oi.interp_weights(g, u)
        for blk in range(2):
            ref = sum(w[i] * bm[blk, j0 + i] for i in range(8))
            assert np.allclose(out[blk, d], ref, atol=1e-14)
    assert np.allclose(out[:, 1], bm[:, 0], atol=1e-13)
    assert np.allclose(out[:, 2], bm[:, 15], atol=1e-13)


def test_fig3d_interpolated_beam_close_to_true_beam():
    """128-element line, 256 beams, theta* = pi/3 (Fig. 3(d)): a broadband
    plane wave from theta*; the beam interpolated from 8 grid beams agrees
    with the beam formed at theta* to within 10 % relative L2 (6.4 % here,
    against 25 % for the nearest grid beam alone)."""
    M, N, B, fc, omega = 128, 32, 256, 1.0, 0.5
    u_star = np.sin(np.pi / 3)
    grid = od.beam_grid(B)
    p = od.line_problem(M, N, B, fc=fc, omega=omega, delta=1e-3)
    rng = np.random.default_rng(14)
    # band-limited source: a sum of tones in [-omega, omega] (baseband)
    freqs = rng.uniform(-omega, omega, 12)
    amps = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    tau = u_star * p.px
    t = p.t
    y = np.zeros((M, N), dtype=np.complex128)
    for f, a in zip(freqs, amps):
        y += a * np.exp(-2j * np.pi * fc * tau)[:, None] * np.exp(
            2j * np.pi * f * (t[None, :] - tau[:, None]))
    j0 = oi.neighbour_window(grid, u_star)
    near = od.beams(y, p, beam_idx=np.arange(j0, j0 + 8))
    interp = oi.interp_beams(near[None], grid[j0:j0 + 8], [u_star])[0, 0]
    p_star = od.line_problem(M, N, 1, fc=fc, omega=omega, delta=1e-3, u=[u_star])
    true = od.beams(y, p_star)[0]
    err = np.linalg.norm(interp - true) / np.linalg.norm(true)
    assert err < 0.1, err
    # and far better than the nearest grid beam alone
    nearest = near[int(np.argmin(np.abs(grid[j0:j0 + 8] - u_star)))]
    assert err < 0.5 * np.linalg.norm(nearest - true) / np.linalg.norm(true)


def test_2d_matches_scipy_bivariate_interpolating_spline():
    """FITPACK's interpolating bicubic spline (s = 0) keeps the interior knots
    at all but the second and second-to-last nodes of each axis: the
    tensor-product not-a-knot spline."""
    rng = np.random.default_rng(15)
    gu = od.beam_grid(12)
    gv = od.beam_grid(9)
    Z = rng.standard_normal((12, 9))
    for _ in range(10):
        u = rng.uniform(gu[0], gu[-1])
        v = rng.uniform(gv[0], gv[-1])
        a0 = oi.neighbour_window(gu, u)
        c0 = oi.neighbour_window(gv, v)
        ref = RectBivariateSpline(gu[a0:a0 + 8], gv[c0:c0 + 8], Z[a0:a0 + 8, c0:c0 + 8],
                                  kx=3, ky=3, s=0)(u, v)[0, 0]
        assert abs(oi.interp_weights_2d(gu, gv, u, v) @ Z.reshape(-1) - ref) < 1e-12


def test_2d_reproduces_bicubics_and_nodes():
    rng = np.random.default_rng(16)
    gu = od.beam_grid(10)
    gv = od.beam_grid(8)
    c = rng.standard_normal((4, 4))
    f = lambda u, v: sum(c[p, q] * u ** p * v ** q for p in range(4) for q in range(4))
    vals = np.array([[f(a, b) for b in gv] for a in gu]).reshape(-1)
    for _ in range(10):
        u = rng.uniform(gu[0], gu[-1])
        v = rng.uniform(gv[0], gv[-1])
        assert abs(oi.interp_weights_2d(gu, gv, u, v) @ vals - f(u, v)) < 1e-11
    W = oi.interp_weights_2d(gu, gv, gu[3], gv[5])
    assert np.allclose(W, np.eye(80)[3 * 8 + 5], atol=1e-13)
    bm = rng.standard_normal((2, 80, 4)) + 1j * rng.standard_normal((2, 80, 4))
    out = oi.interp_beams_2d(bm, gu, gv, [gu[3], 0.1], [gv[5], -0.2])
    assert out.shape == (2, 2, 4)
    assert np.allclose(out[:, 0], bm[:, 3 * 8 + 5], atol=1e-13)
    ref = np.tensordot(oi.interp_weights_2d(gu, gv, 0.1, -0.2), bm, axes=([0], [1]))
    assert np.allclose(out[:, 1], ref, atol=1e-14)
