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
