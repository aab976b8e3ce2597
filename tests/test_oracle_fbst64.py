"""Pins of the second FP64 oracle, oracle/fbst64.py (the FBST itself with numpy
FFTs), against library routines and the direct oracle (the definition with a
dense Cholesky solve), step by step and on whole blocks: the chirp-z helper
against scipy.signal.czt, each stage against its plain sum, the closed-form
Gram column and the Levinson generator against the direct ones, the
Gohberg-Semencul product against a dense solve, and every beam of small
blocks plus sampled beams of the 256-element line."""
import numpy as np
import pytest
import scipy.signal as ss

import synth
from oracle import direct as od
from oracle import fbst64 as fb


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("nin,K", [(37, 53), (64, 16), (1, 9), (100, 100)])
def test_czt_matches_scipy(nin, K):
    """czt(x, K, a, b)[k] = sum_n x[n] exp(j(a n + b n k)) is scipy's chirp-z
    with A = exp(-j a), W = exp(j b) (z_k = A W^-k, X_k = sum x[n] z_k^-n)."""
    rng = np.random.default_rng(nin * 1000 + K)
    x = _rand(rng, nin)
    for a, b in [(0.3, -0.07), (-1.1, 0.013), (0.0, 2 * np.pi / K)]:
        ref = ss.czt(x, K, w=np.exp(1j * b), a=np.exp(-1j * a))
        assert _rel(fb.czt(x, K, a, b), ref) < 1e-12
    # one rate per row (stage 1b): row r against its own scipy transform
    X = _rand(rng, (3, nin))
    rates = np.array([0.01, -0.2, 0.7])
    got = fb.czt(X, K, 0.0, rates)
    for r in range(3):
        assert _rel(got[r], ss.czt(X[r], K, w=np.exp(1j * rates[r]), a=1.0)) < 1e-12


@pytest.mark.parametrize("t0,eps", [(0.0, 1.01), (3.5, 1.01), (0.0, 1.0), (-7.0, 1.3)])
def test_stages_against_direct_line(t0, eps):
    rng = np.random.default_rng(5)
    M, N, B = 9, 40, 11
    p = od.line_problem(M, N, B, fc=2.0, eps=eps, delta=0.8, x0=0.5)
    p = od.make_problem(N=p.N, L=p.L, eps=p.eps, delta=p.delta, fc=p.fc, omega=p.omega,
                        ts=p.ts, px=p.px, u=p.u, t0=t0)
    y = _rand(rng, (M, N))
    assert _rel(fb.stage1a(y, p), od.stage1a(y, p)) < 1e-12
    assert _rel(fb.project(y, p), od.project(y, p)) < 1e-12
    beta = _rand(rng, (3, p.L))
    assert _rel(fb.reconstruct(beta, p), od.reconstruct(beta, p)) < 1e-12


def test_project_grid_and_arbitrary():
    rng = np.random.default_rng(6)
    pg = od.grid_problem(4, 3, 5, 2, 24, fc=2.5, delta=1.0)
    y = _rand(rng, (12, 24))
    lay = fb.layout_of(pg, (4, 3, 5, 2))
    assert lay.kind == "grid"
    assert _rel(fb.project(y, pg, lay), od.project(y, pg)) < 1e-12
    px = (np.arange(7) + rng.uniform(-0.3, 0.3, 7)) * 0.2
    py = rng.uniform(-0.5, 0.5, 7)
    pa = od.make_problem(N=24, L=48, eps=1.01, delta=1.0, fc=2.0, omega=0.5, ts=1.0, px=px, py=py,
                         u=od.beam_grid(6), v=np.linspace(-0.3, 0.4, 6))
    y = _rand(rng, (7, 24))
    assert fb.layout_of(pa).kind == "arbitrary"
    assert _rel(fb.project(y, pa), od.project(y, pa)) < 1e-12


@pytest.mark.parametrize("kind", ["line", "grid", "arbitrary"])
def test_gram_and_generator_against_direct(kind):
    rng = np.random.default_rng(7)
    if kind == "line":
        p, shape = od.line_problem(10, 32, 10, fc=2.0, delta=0.5, x0=-1.5), None
    elif kind == "grid":
        p, shape = od.grid_problem(3, 4, 3, 3, 32, fc=2.5, delta=0.5), (3, 4, 3, 3)
    else:
        px = rng.uniform(0, 2, 8)
        p, shape = od.make_problem(N=32, L=64, eps=1.01, delta=0.5, fc=2.0, omega=0.5, ts=1.0,
                                   px=px, py=rng.uniform(0, 1, 8), u=od.beam_grid(5),
                                   v=np.full(5, 0.2)), None
    lay = fb.layout_of(p, shape)
    d = np.arange(p.L)
    for b in range(len(p.u)):
        c, phi = fb.gram_column(p, b, lay)
        if phi is not None:
            c = c * np.exp(1j * phi * d)
        assert _rel(c, od.gram_column(p, b)) < 1e-12, b
        assert _rel(fb.generator(p, b, lay), od.generator(p, b)) < 1e-10, b


def test_gohberg_semencul_product_is_the_dense_solve():
    """gs_apply(x, w) = A^{-1} w with x = A^{-1} e_0 (Sec. V), several rows at once."""
    rng = np.random.default_rng(8)
    p = od.line_problem(12, 48, 12, fc=2.0, delta=2.0)
    X, W, ref = [], [], []
    for b in (0, 5, 11):
        A = od.toeplitz_system(p, b)
        w = _rand(rng, p.L)
        X.append(od.generator(p, b))
        W.append(w)
        ref.append(np.linalg.solve(A, w))
    got = fb.gs_apply(np.array(X), np.array(W))
    assert _rel(got, np.array(ref)) < 1e-10


def test_every_beam_of_the_small_line_and_a_grid():
    cfg = synth.config("ula16")
    y = cfg.scene().block(0)
    p = od.line_problem(cfg.M, cfg.N, cfg.B, fc=cfg.band.fc, omega=cfg.band.omega,
                        ts=cfg.band.ts, eps=cfg.eps, gamma=cfg.gamma, delta=cfg.delta_noise)
    got, ref = fb.beams(y, p), od.beams(y, p)
    per_beam = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert per_beam.max() < 1e-10, per_beam.max()
    rng = np.random.default_rng(9)
    pg = od.grid_problem(4, 4, 5, 3, 64, fc=2.5, delta=3.0)
    yg = _rand(rng, (16, 64))
    got, ref = fb.beams(yg, pg, shape=(4, 4, 5, 3)), od.beams(yg, pg)
    per_beam = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert per_beam.max() < 1e-10, per_beam.max()


def test_sampled_beams_of_the_256_element_line():
    """16 beams of a 256-element line block (M = B = 256, N = 1024, L = 2048):
    both grid ends, broadside and 13 seeded beams, against the Cholesky route."""
    cfg = synth.config("ula256")
    y = cfg.scene().block(0)
    p = od.line_problem(cfg.M, cfg.N, cfg.B, fc=cfg.band.fc, omega=cfg.band.omega,
                        ts=cfg.band.ts, eps=cfg.eps, gamma=cfg.gamma, delta=cfg.delta_noise)
    rng = np.random.default_rng(10)
    idx = np.unique(np.concatenate([[0, cfg.B - 1, cfg.B // 2], rng.choice(cfg.B, 13, replace=False)]))
    got = fb.beams(y, p, beam_idx=idx)
    ref = od.beams(y, p, beam_idx=idx)
    per_beam = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert per_beam.max() < 1e-10, per_beam.max()
