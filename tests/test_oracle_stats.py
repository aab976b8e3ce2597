"""Sec. VII pins: the oracle's beams on Monte-Carlo noise and Monte-Carlo
band-limited Gaussian sources against the paper's variance and bias formulas."""
import numpy as np

from oracle import direct as od
from oracle import analysis as oa
import synth


def test_variance_closed_form_matches_quadrature():
    """The paper's closed form of int_0^T r(t,t) dt equals a fine quadrature of
    sigma^2 sum Q_kl e^{j (w_k - w_l) t}."""
    p = od.line_problem(6, 16, 5, fc=2.0, delta=1e-3)
    T = 15.0
    Q = oa.Q_matrix(p, 3)
    w = od.omegas(p.L, p.eps, 1.0)
    tt = np.linspace(0.0, T, 20001)
    r = np.einsum("kl,tk,tl->t", Q, np.exp(1j * np.outer(tt, w)), np.exp(-1j * np.outer(tt, w))).real
    quad = np.trapezoid(r, tt)
    assert abs(oa.variance_continuous(p, 3, 1.0, T) - quad) < 1e-6 * abs(quad)


def test_variance_monte_carlo():
    """Mean energy of the beam of pure noise = sigma^2 tr(F_u Q F_u^H)."""
    M, N, B, sigma2 = 8, 32, 8, 1.0
    p = od.line_problem(M, N, B, fc=2.0, delta=1e-5)
    b = 6
    rng = np.random.default_rng(11)
    trials = 400
    e = np.empty(trials)
    for i in range(trials):
        n = synth.noise(rng, (M, N), sigma2)
        e[i] = np.sum(np.abs(od.beams(n, p, [b])[0]) ** 2)
    pred = oa.variance_discrete(p, b, sigma2)
    se = e.std(ddof=1) / np.sqrt(trials)
    assert abs(e.mean() - pred) < 4 * se


def test_variance_approaches_array_gain():
    """Per-sample variance falls towards sigma^2 / M as N grows (Sec. VII)."""
    M, sigma2 = 8, 1.0
    vals = []
    for N in (16, 32, 64, 128):
        p = od.line_problem(M, N, 8, fc=2.0, delta=1e-5)
        vals.append(oa.variance_discrete(p, 6, sigma2) / N)
    assert all(a > b for a, b in zip(vals, vals[1:]))
    assert vals[-1] < 1.2 * sigma2 / M
    assert vals[-1] > sigma2 / M


def test_bias_monte_carlo():
    """Mean squared error of a noise-free beam on band-limited Gaussian sources
    (sum of sinusoids with uniform frequencies; covariance sinc(2 Omega tau))
    equals the closed-form bias."""
    M, N, B = 6, 16, 6
    band = synth.band_from_fb(0.5)
    p = od.line_problem(M, N, B, fc=band.fc, omega=band.omega, gamma=1.25, delta=1e-4)
    b = 4
    arr = synth.ula(M, band)
    rng = np.random.default_rng(12)
    trials = 600
    e = np.empty(trials)
    for i in range(trials):
        f, a = synth._draw_waveform(rng, band, 1.0, 32)
        sc = synth.Scene(arr, band, [synth.Source(u=float(p.u[b]), v=0.0, freqs=f, amps=a)], 0.0, 0, N)
        e[i] = np.sum(np.abs(od.beams(sc.clean_block(0), p, [b])[0] - sc.source_samples(0)) ** 2)
    pred = oa.bias_discrete(p, b, float(p.u[b]))
    se = e.std(ddof=1) / np.sqrt(trials)
    assert abs(e.mean() - pred) < 4 * se
    assert pred > 0


def test_bias_falls_with_extension_factor():
    """Bias drops steeply once gamma exceeds its lower bound (Sec. VII, Fig. 3c)."""
    M, N = 8, 32
    band = synth.band_from_fb(0.5)
    vals = []
    for gamma in (1.0, 1.25, 1.5, 2.0):
        p = od.line_problem(M, N, 8, fc=band.fc, omega=band.omega, gamma=gamma, delta=1e-8)
        vals.append(oa.bias_discrete(p, 6, float(p.u[6])))
    assert all(a > b for a, b in zip(vals, vals[1:]))
    assert vals[-1] < 1e-3 * vals[0]
