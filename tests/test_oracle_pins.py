"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's
own formula: they use the explicit matrices, the paper's other printed forms
(eq. DFT_1), library routines (scipy czt, numpy FFT), limits with textbook
answers, physics of a plane wave, and the Sec. VII statistics.
"""
import numpy as np
import pytest
import scipy.signal

from oracle import direct as od
import synth


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


# --------------------------------------------------------------------------
# T1: brute force with the explicit MN x L matrices (eqs. FthetaH, betahatls,
# bhatls) vs the factored sums, Toeplitz Gram matrix and Cholesky solve.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("M,N,B,gamma", [(2, 4, 2, 2), (3, 8, 3, 2), (5, 4, 4, 3),
                                         (5, 8, 5, 3), (3, 4, 5, 2), (2, 8, 4, 3)])
def test_bruteforce_tiny(M, N, B, gamma):
    rng = np.random.default_rng(M * 100 + N * 10 + B)
    p = od.line_problem(M, N, B, fc=2.0, gamma=gamma, delta=1e-3)
    y = crandn(rng, M, N)
    ref = od.beams_dense(y, p)
    got = od.beams(y, p)
    assert rel(got, ref) < 1e-9
    # the projection and the Gram matrix separately
    for b in range(B):
        F = od.F_matrix(p, b)
        assert rel(od.project(y, p, [b])[0], F.conj().T @ y.reshape(-1)) < 1e-12
        A = F.conj().T @ F + p.delta * np.eye(p.L)
        assert rel(od.toeplitz_system(p, b), A) < 1e-12


def test_bruteforce_grid_tiny():
    rng = np.random.default_rng(7)
    p = od.grid_problem(2, 3, 3, 2, 4, fc=2.5, gamma=2, delta=1e-3)
    y = crandn(rng, p.M, p.N)
    assert rel(od.beams(y, p), od.beams_dense(y, p)) < 1e-9


# --------------------------------------------------------------------------
# T2: the fan form, eq. (DFT_1), with the printed zeta, xi, b' and l'.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("B", [5, 6])
def test_fan_identity(B):
    M, N, gamma, eps = 7, 16, 2, 1.01
    fc, omega, ts = 2.0, 0.5, 1.0
    L = gamma * N
    p = od.line_problem(M, N, B, fc=fc, omega=omega, ts=ts, eps=eps, gamma=gamma)
    rng = np.random.default_rng(B)
    y = crandn(rng, M, N)
    D = (B - 1) if B % 2 else B        # even B: the symmetric grid rule
    ft = fc + omega
    zeta = 2 * fc / (D * ft)
    xi = 2 * eps / (D * L * ts * ft)
    w = np.zeros((B, L), complex)
    for b in range(1, B + 1):
        bp = b - (B + 1) / 2
        for l in range(1, L + 1):
            lp = l - L / 2
            acc = 0j
            for m in range(M):
                for n in range(N):
                    acc += y[m, n] * np.exp(1j * np.pi * (zeta + xi * lp) * bp * m) \
                        * np.exp(-2j * np.pi * eps / L * lp * n)
            w[b - 1, l - 1] = acc
    assert rel(od.project(y, p), w) < 1e-12


# --------------------------------------------------------------------------
# T5: each chirp-z of Sec. IV against scipy.signal.czt.
# --------------------------------------------------------------------------
def test_stage1a_czt():
    M, N, L, eps = 3, 40, 80, 1.01
    p = od.line_problem(M, N, 4, fc=2.0, eps=eps, gamma=2)
    rng = np.random.default_rng(1)
    y = crandn(rng, M, N)
    lp0 = 1 - L / 2
    W = np.exp(-2j * np.pi * eps / L)
    A = np.exp(2j * np.pi * eps * lp0 / L)
    ref = np.stack([scipy.signal.czt(y[m], m=L, w=W, a=A) for m in range(M)])
    assert rel(od.stage1a(y, p), ref) < 1e-11


def test_stage1b_czt():
    M, N, B, eps, fc, omega = 12, 16, 9, 1.01, 2.0, 0.5
    p = od.line_problem(M, N, B, fc=fc, omega=omega, eps=eps, gamma=2)
    rng = np.random.default_rng(2)
    y = crandn(rng, M, N)
    yh = od.stage1a(y, p)
    d = 1.0 / (2 * (fc + omega))
    u = od.beam_grid(B)
    u0, du = u[0], u[1] - u[0]
    om = od.omegas(p.L, eps, 1.0)
    ref = np.empty((B, p.L), complex)
    for l in range(p.L):
        rho = (2 * np.pi * fc + om[l]) * d
        ref[:, l] = scipy.signal.czt(yh[:, l], m=B, w=np.exp(1j * rho * du), a=np.exp(-1j * rho * u0))
    assert rel(od.project(y, p), ref) < 1e-11


# --------------------------------------------------------------------------
# T4: epsilon = 1 makes stage 1a a zero-padded L-point DFT (Sec. III-A).
# --------------------------------------------------------------------------
def test_eps1_is_dft():
    M, N, L = 4, 32, 64
    p = od.line_problem(M, N, 4, fc=2.0, eps=1.0, gamma=2)
    rng = np.random.default_rng(3)
    y = crandn(rng, M, N)
    X = np.fft.fft(y, n=L, axis=1)
    lp = np.arange(1, L + 1) - L // 2
    assert rel(od.stage1a(y, p), X[:, lp % L]) < 1e-12


# --------------------------------------------------------------------------
# T3: narrowband limit (Sec. I): with FB -> 0 the delays vanish and every
# beam is (1/M) times a spatial DFT of the snapshot.
# --------------------------------------------------------------------------
def test_narrowband_limit_is_spatial_fft():
    M = B = 16
    N = 64
    fc = 1e9                                 # FB = 2 Omega / f_c = 1e-9
    p = od.line_problem(M, N, B, fc=fc, omega=0.5, eps=1.01, gamma=2, delta=1e-5)
    rng = np.random.default_rng(4)
    y = crandn(rng, M, N)
    m = np.arange(M)
    pre = y * np.exp(-1j * np.pi * (B + 1) * m / B)[:, None]
    sp = B * np.fft.ifft(pre, axis=0) / M            # sum_m y_m e^{j 2 pi b m / B} / M
    ref = sp[np.arange(1, B + 1) % B]                # b' = b - (B+1)/2
    assert rel(od.beams(y, p), ref) < 1e-6


# --------------------------------------------------------------------------
# T7: a noise-free plane wave from a grid direction is recovered at the bias
# level and peaks in its own beam (Sec. III, delay-and-sum ideal; Sec. VI).
# --------------------------------------------------------------------------
def test_plane_wave_on_grid():
    M, N, B = 64, 256, 64
    band = synth.band_from_fb(0.5)
    arr = synth.ula(M, band)
    p = od.line_problem(M, N, B, fc=band.fc, omega=band.omega, delta=1e-5)
    b0 = 41
    rng = np.random.default_rng(5)
    f, a = synth._draw_waveform(rng, band, 1.0, 256)
    src = synth.Source(u=float(p.u[b0]), v=0.0, freqs=f, amps=a)
    sc = synth.Scene(arr, band, [src], 0.0, 0, N)
    y = sc.clean_block(0)
    out = od.beams(y, p)
    power = np.sum(np.abs(out) ** 2, axis=1)
    assert int(np.argmax(power)) == b0
    assert rel(out[b0], sc.source_samples(0)) < 5e-6


# --------------------------------------------------------------------------
# T15: no beam squint (Sec. VI, beam pattern across the band): a single tone at
# any of 20 frequencies across [-Omega, Omega] from the steered direction comes
# out of that beam with unit gain and zero phase.
# --------------------------------------------------------------------------
def test_flat_response_across_band():
    M, N, B = 32, 128, 32
    band = synth.band_from_fb(0.5)
    arr = synth.ula(M, band)
    p = od.line_problem(M, N, B, fc=band.fc, omega=band.omega, delta=1e-5)
    b0 = 24
    px, _ = arr.positions()
    tau = p.u[b0] * px
    t = np.arange(N, dtype=float)
    for f in np.linspace(-band.omega, band.omega, 20):
        y = np.exp(-2j * np.pi * band.fc * tau)[:, None] * np.exp(2j * np.pi * f * (t[None, :] - tau[:, None]))
        out = od.beams(y, p, [b0])[0]
        assert rel(out, np.exp(2j * np.pi * f * t)) < 2e-3


# --------------------------------------------------------------------------
# T10: invariances of the definition.
# --------------------------------------------------------------------------
def test_time_origin_invariance():
    rng = np.random.default_rng(6)
    p0 = od.line_problem(8, 32, 8, fc=2.0, delta=1e-4)
    p1 = od.make_problem(N=p0.N, L=p0.L, eps=p0.eps, delta=p0.delta, fc=p0.fc, omega=p0.omega,
                         ts=p0.ts, px=p0.px, u=p0.u, t0=1.0)     # n = 1..N as printed
    y = crandn(rng, 8, 32)
    assert rel(od.beams(y, p1), od.beams(y, p0)) < 1e-8


def test_linearity():
    rng = np.random.default_rng(8)
    p = od.line_problem(8, 32, 6, fc=2.0, delta=1e-4)
    y1, y2 = crandn(rng, 8, 32), crandn(rng, 8, 32)
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    assert rel(od.beams(a * y1 + b * y2, p), a * od.beams(y1, p) + b * od.beams(y2, p)) < 1e-9


def test_reference_point_is_delay_and_phase():
    """Moving the reference point by tau0 along the beam turns the beam into
    exp(j 2 pi f_c tau0) times the old expansion evaluated at t_n + tau0."""
    rng = np.random.default_rng(9)
    fc, om = 2.0, 0.5
    p0 = od.line_problem(8, 32, 6, fc=fc, omega=om, delta=1e-4)
    x0 = -3.5
    p1 = od.line_problem(8, 32, 6, fc=fc, omega=om, delta=1e-4, x0=x0)
    y = crandn(rng, 8, 32)
    got = od.beams(y, p1)
    _, _, beta = od.beams(y, p0, return_parts=True)
    d = 1.0 / (2 * (fc + om))
    w = od.omegas(p0.L, p0.eps, 1.0)
    t = np.arange(p0.N, dtype=float)
    for b in range(p0.B):
        tau0 = p0.u[b] * x0 * d
        ref = np.exp(2j * np.pi * fc * tau0) * (np.exp(1j * np.multiply.outer(t + tau0, w)) @ beta[b])
        assert rel(got[b], ref) < 1e-7
