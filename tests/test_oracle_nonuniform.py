"""Pins of the FP64 oracle for non-uniform arrays (Sec. IX, eq. DFT_non_unif).

With arbitrary element positions the fan sum over m no longer has chirp-z
structure, but the beam is still the regularised least-squares fit of
eqs. (FthetaH, betahatls, bhatls): these tests check the oracle's factored
sums and its Toeplitz Gram matrix against the explicit matrices, and the
physics of a plane wave, on randomly perturbed arrays.
"""
import numpy as np
import pytest

from oracle import direct as od
import synth
from helpers import crandn, oracle_problem, perturbed_cfg, rel


def _random_line(M, N, B, seed, delta=1e-3):
    rng = np.random.default_rng(seed)
    d = 1.0 / (2.0 * 2.5)
    px = (np.arange(M) + rng.uniform(-0.4, 0.4, M)) * d
    return od.make_problem(N=N, L=2 * N, eps=1.01, delta=delta, fc=2.0, omega=0.5, ts=1.0,
                           px=px, u=od.beam_grid(B))


@pytest.mark.parametrize("M,N,B,seed", [(3, 4, 3, 1), (5, 8, 4, 2), (4, 8, 6, 3)])
def test_bruteforce_random_line(M, N, B, seed):
    p = _random_line(M, N, B, seed)
    y = crandn(np.random.default_rng(seed + 10), M, N)
    assert rel(od.beams(y, p), od.beams_dense(y, p)) < 1e-9
    for b in range(B):
        F = od.F_matrix(p, b)
        G = F.conj().T @ F
        # the Gram matrix stays Toeplitz for any positions (its entries depend
        # on omega_l - omega_k only) and equals the oracle's closed product
        assert np.allclose(G[1:, 1:], G[:-1, :-1], atol=1e-12 * abs(G[0, 0]))
        assert rel(od.toeplitz_system(p, b), G + p.delta * np.eye(p.L)) < 1e-12
        assert rel(od.project(y, p, [b])[0], F.conj().T @ y.reshape(-1)) < 1e-12


def test_bruteforce_random_plane():
    rng = np.random.default_rng(4)
    d = 0.2
    px = rng.uniform(0.0, 3 * d, 6)
    py = rng.uniform(0.0, 2 * d, 6)
    p = od.make_problem(N=4, L=8, eps=1.01, delta=1e-3, fc=2.0, omega=0.5, ts=1.0, px=px, py=py,
                        u=np.repeat(od.beam_grid(3), 2), v=np.tile(od.beam_grid(2), 3))
    y = crandn(rng, 6, 4)
    assert rel(od.beams(y, p), od.beams_dense(y, p)) < 1e-9


def test_plane_wave_on_perturbed_line():
    """A noise-free plane wave from a grid direction, on a line whose elements
    are moved by up to a quarter spacing, is recovered in its own beam at the
    bias level (Sec. IX: the rest of the method is unchanged)."""
    cfg = perturbed_cfg("ula", 48, 256, 48, index=93)
    p = oracle_problem(cfg, delta=1e-5)
    b0 = 31
    rng = np.random.default_rng(6)
    f, a = synth._draw_waveform(rng, cfg.band, 1.0, 256)
    sc = synth.Scene(cfg.array, cfg.band, [synth.Source(u=float(p.u[b0]), v=0.0, freqs=f, amps=a)],
                     0.0, 0, cfg.N)
    out = od.beams(sc.clean_block(0), p)
    assert int(np.argmax(np.sum(np.abs(out) ** 2, axis=1))) == b0
    assert rel(out[b0], sc.source_samples(0)) < 1e-5


def test_perturbed_positions_are_seeded_and_bounded():
    cfg = synth.config("nula256")
    a = cfg.array
    px, py = a.positions()
    px2, _ = cfg.array.positions()
    assert np.array_equal(px, px2) and not np.any(py)
    off = px / a.dx - np.arange(cfg.M)
    assert np.all(np.abs(off) <= cfg.perturb) and np.std(off) > 0.1
    g = synth.config("nura16").array
    gx, gy = g.positions()
    assert np.all(np.abs(gx / g.dx - np.repeat(np.arange(16), 16)) <= 0.25)
    assert np.all(np.abs(gy / g.dy - np.tile(np.arange(16), 16)) <= 0.25)
