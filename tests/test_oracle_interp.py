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


# ---- the paper's form: interpolate the beamspace vectors w, then solve at the
# ---- direction itself (Sec. VIII)

def _plane_wave_line(p, u, fc, omega, rng, tones=12):
    y = np.zeros((p.M, p.N), dtype=np.complex128)
    tau = u * p.px
    for f, a in zip(rng.uniform(-omega, omega, tones),
                    rng.standard_normal(tones) + 1j * rng.standard_normal(tones)):
        y += a * np.exp(-2j * np.pi * fc * tau)[:, None] * np.exp(
            2j * np.pi * f * (p.t[None, :] - tau[:, None]))
    return y


@pytest.mark.parametrize("centre", ["array", "origin"])
def test_vector_interp_at_nodes_is_the_grid_beam(centre):
    rng = np.random.default_rng(40)
    M, N, B = 8, 32, 16
    p = od.line_problem(M, N, B, fc=2.0, delta=1.0)
    y = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    g = od.beam_grid(B)
    nodes = [0, 5, 11, 15]
    out = oi.vector_interp_beams(y, p, g, g[nodes], centre=centre)
    ref = od.beams(y, p, beam_idx=nodes)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("centre", ["array", "origin"])
def test_vector_interp_converges_at_fourth_order(centre):
    """Refining the beam grid moves the interpolated w* to F_*^H y at the
    rate of a cubic spline, h^4, and the beam with it, since A_* is the
    direction's own system; solving with a neighbouring grid beam's system
    instead would leave an O(h) error."""
    rng = np.random.default_rng(41)
    M, N = 8, 32
    y = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    us = 0.3137
    true = od.beams(y, oi.direction_problem(od.line_problem(M, N, 1, fc=1.0, delta=1e-2), [us]))[0]
    errs = []
    for B in (32, 64, 128):
        p = od.line_problem(M, N, B, fc=1.0, delta=1e-2)
        out = oi.vector_interp_beams(y, p, od.beam_grid(B), [us], centre=centre)[0]
        errs.append(np.linalg.norm(out - true) / np.linalg.norm(true))
    assert errs[0] / errs[1] > 10 and errs[1] / errs[2] > 10, errs


def test_vectors_reproduce_referenced_cubics():
    """Beamspace vectors whose reference-moved form is a cubic in u come out
    exactly: pins the sign and size of the reference phase, which a plain
    cubic (centre at the origin) would not see."""
    rng = np.random.default_rng(42)
    M, N, B = 6, 16, 12
    p = od.line_problem(M, N, B, fc=2.0, delta=1.0)
    g = od.beam_grid(B)
    c = oi.array_centre(p)
    a = 2 * np.pi * p.fc + od.omegas(p.L, p.eps, p.ts)
    coef = rng.standard_normal((4, p.L)) + 1j * rng.standard_normal((4, p.L))
    cubic = lambda u: sum(coef[k] * u ** k for k in range(4))
    W = np.stack([cubic(u) * np.exp(1j * a * u * c[0]) for u in g])
    us = [g[2] + 0.41 * (g[3] - g[2]), g[9] + 0.77 * (g[10] - g[9])]
    got = oi.interp_vectors(W, g, us, p=p, centre=c)
    for d, u in enumerate(us):
        want = cubic(u) * np.exp(1j * a * u * c[0])
        assert np.max(np.abs(got[d] - want)) < 1e-11 * np.max(np.abs(want))
    # the same vectors interpolated without moving the reference are not exact
    plain = oi.interp_vectors(W, g, us)
    assert np.max(np.abs(plain[0] - cubic(us[0]) * np.exp(1j * a * us[0] * c[0]))) > 1e-6


def test_vectors_reproduce_referenced_bicubics_on_a_plane():
    rng = np.random.default_rng(43)
    mx, my, bu, bv, N = 3, 4, 9, 10, 8
    p = od.grid_problem(mx, my, bu, bv, N, fc=2.0, delta=1.0)
    gu, gv = od.beam_grid(bu), od.beam_grid(bv)
    c = oi.array_centre(p)
    a = 2 * np.pi * p.fc + od.omegas(p.L, p.eps, p.ts)
    coef = rng.standard_normal((4, 4, p.L))
    f = lambda u, v: sum(coef[i, k] * u ** i * v ** k for i in range(4) for k in range(4))
    W = np.stack([f(u, v) * np.exp(1j * a * (u * c[0] + v * c[1])) for u, v in zip(p.u, p.v)])
    us, vs = [0.13, -0.61], [0.27, 0.05]
    got = oi.interp_vectors(W, gu, us, gv, vs, p=p, centre=c)
    for d, (u, v) in enumerate(zip(us, vs)):
        want = f(u, v) * np.exp(1j * a * (u * c[0] + v * c[1]))
        assert np.max(np.abs(got[d] - want)) < 1e-10 * np.max(np.abs(want))
    # nodes of the plane give the grid beams
    y = rng.standard_normal((p.M, N)) + 1j * rng.standard_normal((p.M, N))
    b = [3 * bv + 4, 8 * bv + 9]
    out = oi.vector_interp_beams(y, p, gu, p.u[b], gv, p.v[b])
    ref = od.beams(y, p, beam_idx=b)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-12


def test_fig3d_vector_interp_close_to_true_beam():
    """The Fig. 3(d) setting (128 elements, 256 beams, theta* = pi/3) in the
    paper's form: 1.6e-3 relative L2 from the beam formed at theta* with the
    reference at the array's centre (6.4e-2 with the reference at element 0,
    25 % for the nearest grid beam alone)."""
    M, N, B, fc, omega = 128, 32, 256, 1.0, 0.5
    u_star = np.sin(np.pi / 3)
    grid = od.beam_grid(B)
    p = od.line_problem(M, N, B, fc=fc, omega=omega, delta=1e-3)
    y = _plane_wave_line(p, u_star, fc, omega, np.random.default_rng(14))
    j0 = oi.neighbour_window(grid, u_star)
    W = np.zeros((B, p.L), dtype=np.complex128)
    W[j0:j0 + 8] = od.project(y, p, np.arange(j0, j0 + 8))
    true = od.beams(y, oi.direction_problem(p, [u_star]))[0]
    err = {c: np.linalg.norm(oi.vector_interp_beams(y, p, grid, [u_star], W=W, centre=c)[0] - true)
           / np.linalg.norm(true) for c in ("array", "origin")}
    assert err["array"] < 5e-3, err
    assert err["origin"] < 0.1, err
