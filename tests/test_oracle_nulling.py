"""Pins of the beamspace nulling oracle (Sec. VIII, eq. interfer_beam_space)."""
import numpy as np

from oracle import direct as od
from oracle import nulling as on
import synth
from tests.helpers import rel, crandn


def test_cross_gram_brute_force_and_gram():
    """C_{b,q} = F_b^H F_q against the explicit matrices of eq. (FthetaH), and
    C_{b,b} + delta I against the Toeplitz system of Sec. V."""
    p = od.line_problem(5, 12, 6, fc=2.0, delta=0.3)
    for b, q in [(0, 3), (4, 1), (2, 2), (5, 5)]:
        C = on.cross_gram(p, b, q)
        E = od.F_matrix(p, b).conj().T @ od.F_matrix(p, q)
        assert np.abs(C - E).max() < 1e-10 * np.abs(E).max()
    A = od.toeplitz_system(p, 3)
    assert np.abs(on.cross_gram(p, 3, 3) + p.delta * np.eye(p.L) - A).max() < 1e-10 * np.abs(A).max()
    pg = od.grid_problem(3, 2, 2, 3, 10, fc=2.5, delta=0.1)
    C = on.cross_gram(pg, 1, 4)
    E = od.F_matrix(pg, 1).conj().T @ od.F_matrix(pg, 4)
    assert np.abs(C - E).max() < 1e-10 * np.abs(E).max()


def test_beamspace_equals_array_space_projection():
    """The beamspace form equals the FBST of the array data minus each
    interferer's regularised fit (the derivation in Sec. VIII), for one and
    for two interferers; with none it is the plain beam."""
    rng = np.random.default_rng(1)
    p = od.line_problem(6, 10, 7, fc=2.0, delta=0.05)
    y = crandn(rng, p.M, p.N)
    for qs in ([2], [1, 5]):
        a = on.nulled_beams(y, p, qs)
        d = on.nulled_beams_dense(y, p, qs)
        assert rel(a, d) < 1e-9, qs
    assert rel(on.nulled_beams(y, p, []), od.beams(y, p)) < 1e-14


def test_interferer_removed_source_kept():
    """A strong source on beam q and a weaker one on beam s: after nulling q,
    every beam's power from the interferer drops by more than 40 dB, and the
    source at s still comes out of its beam (Sec. VIII)."""
    M, N, B = 32, 128, 32
    band = synth.band_from_fb(0.5)
    arr = synth.ula(M, band)
    p = od.line_problem(M, N, B, fc=band.fc, omega=band.omega, delta=1e-3)
    q, s = 8, 21
    rng = np.random.default_rng(7)
    fi, ai = synth._draw_waveform(rng, band, 100.0, 256)
    fs, as_ = synth._draw_waveform(rng, band, 1.0, 256)
    interf = synth.Source(u=float(p.u[q]), v=0.0, freqs=fi, amps=ai)
    src = synth.Source(u=float(p.u[s]), v=0.0, freqs=fs, amps=as_)
    y_i = synth.Scene(arr, band, [interf], 0.0, 0, N).clean_block(0)
    sc = synth.Scene(arr, band, [interf, src], 0.0, 0, N)
    y = sc.clean_block(0)
    before = np.sum(np.abs(od.beams(y_i, p)) ** 2)
    after = np.sum(np.abs(on.nulled_beams(y_i, p, [q])) ** 2)
    assert after < 1e-4 * before
    out = on.nulled_beams(y, p, [q], beam_idx=[s])[0]
    assert rel(out, sc.source_samples(1)) < 1e-2


def test_nulling_on_random_positions():
    """Non-uniform arrays (Sec. IX: the beamspace applications are unchanged):
    on a random planar layout the cross-Gram equals the explicit product and
    the beamspace form equals the array-space projection, for interferers at a
    grid beam and at an off-grid direction."""
    rng = np.random.default_rng(12)
    px = rng.uniform(0.0, 1.0, 7)
    py = rng.uniform(0.0, 0.8, 7)
    u = np.array([-0.6, -0.1, 0.3, 0.75, 0.2])
    v = np.array([0.1, -0.4, 0.25, 0.0, 0.55])
    p = od.make_problem(N=8, L=16, eps=1.01, delta=0.05, fc=2.0, omega=0.5, ts=1.0, px=px, py=py,
                        u=u, v=v)
    for b, q in [(0, 3), (4, 1), (2, 2)]:
        C = on.cross_gram(p, b, q)
        E = od.F_matrix(p, b).conj().T @ od.F_matrix(p, q)
        assert np.abs(C - E).max() < 1e-10 * np.abs(E).max()
    y = crandn(rng, p.M, p.N)
    for qs in ([1], [0, 4]):
        assert rel(on.nulled_beams(y, p, qs), on.nulled_beams_dense(y, p, qs)) < 1e-9, qs


# ---- off-grid interferers the paper's way: w_q spline-interpolated from the
# ---- grid's beamspace vectors (Sec. VIII)

def test_interpolated_interferer_on_a_node_is_the_on_grid_nulling():
    rng = np.random.default_rng(50)
    M, N, B = 8, 32, 16
    p = od.line_problem(M, N, B, fc=2.0, delta=1.0)
    y = crandn(rng, M, N)
    for centre in ("array", "origin"):
        a = on.nulled_beams_interp(y, p, p.u, [p.u[11]], centre=centre)
        assert rel(a, on.nulled_beams(y, p, [11])) < 1e-12


def test_interpolated_interferer_given_exact_vector_is_the_direction_nulling():
    """The interpolation enters only through w_q: handing nulled_beams the
    exact F_q^H y of the extended problem reproduces its own projection."""
    rng = np.random.default_rng(51)
    M, N, B = 7, 24, 12
    p = od.line_problem(M, N, B, fc=2.0, delta=1.0)
    y = crandn(rng, M, N)
    uq = [0.2113]
    pe = on.extended_problem(p, uq)
    wq = od.project(y, pe, [B])
    a = on.nulled_beams(y, pe, [B], beam_idx=np.arange(B), interferer_vectors=wq)
    assert rel(a, on.nulled_beams(y, pe, [B], beam_idx=np.arange(B))) < 1e-13


def test_interpolated_interferer_converges_to_the_direction_nulling():
    rng = np.random.default_rng(52)
    M, N = 8, 32
    y = crandn(rng, M, N)
    uq = 0.4137
    errs = []
    for B in (24, 48, 96):
        p = od.line_problem(M, N, B, fc=2.0, delta=1.0)
        idx = np.arange(0, B, B // 8)
        a = on.nulled_beams_interp(y, p, p.u, [uq], beam_idx=idx)
        b = on.nulled_beams(y, on.extended_problem(p, [uq]), [B], beam_idx=idx)
        errs.append(rel(a, b))
    assert errs[0] / errs[1] > 8 and errs[1] / errs[2] > 8, errs


def test_interpolated_off_grid_null_is_deep():
    """The paper's nulling setting (Fig. 4(b)): a 128-element line, 256 beams,
    N = 64, a source at 60 degrees and a 20 dB interferer at 20 degrees (off
    the grid), its beam vector interpolated from 8 grid beams.  In the four
    beams around the interferer its power drops by more than 35 dB (about
    40 dB, as deep as with the exact w_q within a factor 1.3)."""
    M, N, B, fc, omega = 128, 64, 256, 1.0, 0.5
    p = od.line_problem(M, N, B, fc=fc, omega=omega, delta=0.1 * 2 * N)
    u_i, u_s = np.sin(np.deg2rad(20.0)), np.sin(np.deg2rad(60.0))
    rng = np.random.default_rng(31)

    def source(u, power):
        f = rng.uniform(-omega, omega, 64)
        a = crandn(rng, 64) * np.sqrt(power / 64)
        tau = u * p.px
        return sum(ai * np.exp(-2j * np.pi * fc * tau)[:, None]
                   * np.exp(2j * np.pi * fi * (p.t[None, :] - tau[:, None])) for fi, ai in zip(f, a))

    y = source(u_s, 1.0) + source(u_i, 100.0) + 0.1 * crandn(rng, M, N)
    j = int(np.searchsorted(p.u, u_i)) - 1
    idx = [j - 1, j, j + 1, j + 2]
    W = od.project(y, p)
    plain = od.beams(y, p, beam_idx=idx)
    a = on.nulled_beams_interp(y, p, p.u, [u_i], beam_idx=idx, W=W)
    ex = on.nulled_beams(y, on.extended_problem(p, [u_i]), [B], beam_idx=idx)
    drop = np.sum(np.abs(a) ** 2) / np.sum(np.abs(plain) ** 2)
    drop_exact = np.sum(np.abs(ex) ** 2) / np.sum(np.abs(plain) ** 2)
    assert drop < 10 ** -3.5, drop
    assert drop < 1.3 * drop_exact, (drop, drop_exact)
