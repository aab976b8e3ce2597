"""Seeded synthetic array workloads.

This module makes the *inputs* of the fast broadband beamspace transformation:
baseband samples of band-limited plane waves on uniform linear and rectangular
arrays, plus white sensor noise.  It implements only the physical signal model
of Sec. III (eq. (1): the demodulated output of sensor m is the source, delayed
by the plane-wave delay tau_m = p_m . theta, times the carrier phase
exp(-j 2 pi f_c tau_m)), and holds none of the transformation's arithmetic.
It is shared by the tests, the benchmark and the smoke check, and is the only
code the CPU oracle and the GPU library both see.

Units: everything is expressed with the sample period T_s = 1 and the baseband
half-bandwidth Omega = 1/2 (critical sampling, as in the experiments of
Sec. VI), so a fractional bandwidth FB = 2 Omega / f_c gives f_c = 1 / FB.

Source waveforms follow the sum-of-sinusoids model the paper uses for its
experiments (Sec. VI, footnote on the source model): s(t) = sum_i a_i
exp(j 2 pi f_i t) with f_i uniform on [-Omega, Omega] and a_i circular complex
Gaussian with total power P.  Its covariance is exactly P sinc(2 Omega tau)
for any number of terms, so it is the band-limited Gaussian process of Sec. VII
in expectation, and it can be evaluated exactly at fractional delays.

Random draws: numpy PCG64.  A scene draws, per source and in this order, its
direction, its power, then its K frequencies and K amplitudes; block k of a
scene draws its noise from an independent stream seeded (seed, k).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = [
    "Band", "Array", "Source", "Scene", "band_from_fb", "ula", "ura",
    "draw_sources_ula", "draw_sources_ura", "CONFIGS", "config",
]

SEED_BASE = 2512_08887


@dataclass(frozen=True)
class Band:
    """Carrier f_c, baseband half-bandwidth Omega and sample period T_s."""
    fc: float
    omega: float
    ts: float = 1.0

    @property
    def f_top(self) -> float:
        """Top band edge f_c + Omega, where the array is lambda/2 spaced."""
        return self.fc + self.omega


def band_from_fb(fb: float) -> Band:
    """Critically sampled band (T_s = 1, Omega = 1/2) of fractional bandwidth fb."""
    return Band(fc=1.0 / fb, omega=0.5, ts=1.0)


@dataclass(frozen=True)
class Array:
    """Uniform linear (my == 1) or rectangular array, optionally perturbed.

    Element (k, k2), flattened as m = k * my + k2, sits at delay-per-direction-
    cosine coordinates px = (x0 + k) * dx and py = (y0 + k2) * dy (seconds),
    so a plane wave with direction cosines (u, v) reaches it with delay
    tau = u * px + v * py relative to the reference point (the origin).

    perturb > 0 makes the array non-uniform as in Sec. IX's experiments:
    every coordinate is moved by an independent offset uniform in
    [-perturb, perturb] times its spacing (a line moves along x only), drawn
    from PCG64 seeded with perturb_seed (x offsets first, then y).
    """
    mx: int
    my: int
    dx: float
    dy: float
    x0: float = 0.0
    y0: float = 0.0
    perturb: float = 0.0
    perturb_seed: int = 0

    @property
    def M(self) -> int:
        return self.mx * self.my

    def positions(self) -> tuple[np.ndarray, np.ndarray]:
        k = np.arange(self.mx, dtype=np.float64)
        k2 = np.arange(self.my, dtype=np.float64)
        px = np.repeat((self.x0 + k) * self.dx, self.my)
        py = np.tile((self.y0 + k2) * self.dy, self.mx)
        if self.perturb > 0.0:
            rng = np.random.default_rng(self.perturb_seed)
            px = px + rng.uniform(-self.perturb, self.perturb, px.shape) * self.dx
            if self.my > 1:
                py = py + rng.uniform(-self.perturb, self.perturb, py.shape) * self.dy
        return px, py


def ula(M: int, band: Band, x0: float = 0.0) -> Array:
    """M-element line, half-wavelength spacing at the top band edge."""
    d = 1.0 / (2.0 * band.f_top)
    return Array(mx=M, my=1, dx=d, dy=0.0, x0=x0)


def ura(mx: int, my: int, band: Band) -> Array:
    """mx x my grid, half-wavelength spacing at the top band edge on both axes."""
    d = 1.0 / (2.0 * band.f_top)
    return Array(mx=mx, my=my, dx=d, dy=d)


@dataclass
class Source:
    """One plane wave: direction cosines (u, v) and a sum of K sinusoids."""
    u: float
    v: float
    freqs: np.ndarray          # Hz, in [-Omega, Omega]
    amps: np.ndarray           # complex amplitudes
    power: float = 1.0

    def waveform(self, t: np.ndarray) -> np.ndarray:
        """s(t) at arbitrary (fractional) times t."""
        t = np.asarray(t, dtype=np.float64)
        ph = np.exp(2j * np.pi * np.multiply.outer(t, self.freqs))
        return ph @ self.amps


def _draw_waveform(rng: np.random.Generator, band: Band, power: float, K: int):
    freqs = rng.uniform(-band.omega, band.omega, size=K)
    amps = (rng.standard_normal(K) + 1j * rng.standard_normal(K)) * np.sqrt(power / (2.0 * K))
    return freqs, amps


def draw_sources_ula(rng, band: Band, n: int, *, max_deg: float = 60.0,
                     power_db_range: float = 0.0, K: int = 256) -> list[Source]:
    """n sources at angles uniform in [-max_deg, max_deg] (u = sin theta),
    powers 10^(-U(0, power_db_range)/10)."""
    out = []
    for _ in range(n):
        theta = np.deg2rad(rng.uniform(-max_deg, max_deg))
        p = 10.0 ** (-rng.uniform(0.0, power_db_range) / 10.0) if power_db_range > 0 else 1.0
        f, a = _draw_waveform(rng, band, p, K)
        out.append(Source(u=float(np.sin(theta)), v=0.0, freqs=f, amps=a, power=p))
    return out


def draw_sources_ura(rng, band: Band, n: int, *, el_deg=(10.0, 90.0),
                     power_db_range: float = 0.0, K: int = 256) -> list[Source]:
    """n sources with azimuth uniform in [0, 2 pi) and elevation (from the
    array plane) uniform in el_deg; u = cos(el) cos(az), v = cos(el) sin(az)."""
    out = []
    for _ in range(n):
        az = rng.uniform(0.0, 2.0 * np.pi)
        el = np.deg2rad(rng.uniform(*el_deg))
        p = 10.0 ** (-rng.uniform(0.0, power_db_range) / 10.0) if power_db_range > 0 else 1.0
        f, a = _draw_waveform(rng, band, p, K)
        out.append(Source(u=float(np.cos(el) * np.cos(az)), v=float(np.cos(el) * np.sin(az)),
                          freqs=f, amps=a, power=p))
    return out


def noise(rng, shape, sigma2: float) -> np.ndarray:
    """Circular complex white Gaussian noise with E|n|^2 = sigma2."""
    if sigma2 <= 0.0:
        return np.zeros(shape, dtype=np.complex128)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(sigma2 / 2.0)


@dataclass
class Scene:
    """Sources impinging on an array; blocks are consecutive N-sample windows.

    block(k) samples t_n = k * N + n (n = 0..N-1) at every sensor; the noise of
    block k is drawn from its own stream so any block can be made alone.
    """
    array: Array
    band: Band
    sources: list
    sigma2: float
    seed: int
    N: int

    def clean_block(self, k: int = 0) -> np.ndarray:
        """Noise-free y[m, n] = sum_sources exp(-j 2 pi f_c tau_m) s(t_n - tau_m)."""
        px, py = self.array.positions()
        t = (k * self.N + np.arange(self.N, dtype=np.float64)) * self.band.ts
        y = np.zeros((self.array.M, self.N), dtype=np.complex128)
        for s in self.sources:
            tau = s.u * px + s.v * py                                    # [M]
            # s(t_n - tau_m) = sum_i a_i e^{j2pi f_i t_n} e^{-j2pi f_i tau_m}
            left = np.exp(-2j * np.pi * np.multiply.outer(tau, s.freqs)) * s.amps    # [M, K]
            right = np.exp(2j * np.pi * np.multiply.outer(s.freqs, t))                # [K, N]
            carrier = np.exp(-2j * np.pi * self.band.fc * tau)                        # [M]
            y += carrier[:, None] * (left @ right)
        return y

    def block(self, k: int = 0) -> np.ndarray:
        y = self.clean_block(k)
        rng = np.random.default_rng([self.seed, k + 1])
        return y + noise(rng, y.shape, self.sigma2)

    def source_samples(self, i: int, k: int = 0) -> np.ndarray:
        """s_i(t_n) at the reference point for block k."""
        t = (k * self.N + np.arange(self.N, dtype=np.float64)) * self.band.ts
        return self.sources[i].waveform(t)


# ---------------------------------------------------------------------------
# Named workloads, shaped like the experiments of Sec. VI (critical sampling,
# f_c / f_s = 2 at fractional bandwidth 0.5, lambda/2 spacing at f_c + Omega,
# N at least twice the aperture in samples), epsilon = 1.01 and gamma = 2.
# ---------------------------------------------------------------------------

@dataclass
class Config:
    name: str
    kind: str                 # "ula" or "ura"
    M: int                    # sensors (mx * my for a ura)
    N: int
    B: int                    # beams (bu * bv for a ura)
    fb: float
    n_sources: int
    power_db_range: float
    sigma2: float
    n_blocks: int = 1
    mx: int = 0
    my: int = 0
    bu: int = 0
    bv: int = 0
    eps: float = 1.01
    gamma: int = 2
    index: int = 0
    perturb: float = 0.0      # > 0: non-uniform array (random offsets, fraction of the spacing)
    extra: dict = field(default_factory=dict)

    @property
    def L(self) -> int:
        return self.gamma * self.N

    @property
    def band(self) -> Band:
        return band_from_fb(self.fb)

    @property
    def array(self) -> Array:
        a = ura(self.mx, self.my, self.band) if self.kind == "ura" else ula(self.M, self.band)
        if self.perturb > 0.0:
            a = Array(a.mx, a.my, a.dx, a.dy, a.x0, a.y0, perturb=self.perturb,
                      perturb_seed=SEED_BASE + 1000 * self.index + 500)
        return a

    @property
    def delta_noise(self) -> float:
        """Ridge value sigma^2 * L: the MAP weight for a unit-power source whose
        L coefficients each carry prior variance 1/L."""
        return self.sigma2 * self.L

    def scene(self, seed_offset: int = 0) -> Scene:
        seed = SEED_BASE + 1000 * self.index + seed_offset
        rng = np.random.default_rng(seed)
        if self.kind == "ura":
            srcs = draw_sources_ura(rng, self.band, self.n_sources,
                                    power_db_range=self.power_db_range)
        else:
            srcs = draw_sources_ula(rng, self.band, self.n_sources,
                                    power_db_range=self.power_db_range)
        return Scene(self.array, self.band, srcs, self.sigma2, seed, self.N)


CONFIGS = {
    # small linear array: 3 unit-power sources, 20 dB SNR, one block
    "ula16": Config("ula16", "ula", M=16, N=256, B=16, fb=0.5, n_sources=3,
                    power_db_range=0.0, sigma2=0.01, index=0),
    # large linear array streamed as 64 consecutive blocks: 8 sources over 30 dB, 10 dB SNR
    "ula256": Config("ula256", "ula", M=256, N=1024, B=256, fb=0.5, n_sources=8,
                     power_db_range=30.0, sigma2=0.1, n_blocks=64, index=1),
    # 32 x 32 planar array, 32 x 32 (u, v) beams, FB 0.4, 16 sources, 10 dB SNR
    "ura32": Config("ura32", "ura", M=1024, N=2048, B=1024, fb=0.4, n_sources=16,
                    power_db_range=0.0, sigma2=0.1, mx=32, my=32, bu=32, bv=32, index=2),
    # precision study: 1024-element line, 32 sources over 40 dB, 0 dB SNR
    "ula1024": Config("ula1024", "ula", M=1024, N=4096, B=1024, fb=0.5, n_sources=32,
                      power_db_range=40.0, sigma2=1.0, index=4),
    # the paper's experimental operating point (128-element line, N = 64 snapshots per
    # block) streamed as 1024 short blocks: 3 unit-power sources, 10 dB SNR
    "ula128n64": Config("ula128n64", "ula", M=128, N=64, B=128, fb=0.5, n_sources=3,
                        power_db_range=0.0, sigma2=0.1, n_blocks=1024, index=5),
    # non-uniform arrays (Sec. IX): the 256-element line and a 16 x 16 grid with every
    # element moved by up to a quarter of the spacing
    "nula256": Config("nula256", "ula", M=256, N=1024, B=256, fb=0.5, n_sources=8,
                      power_db_range=30.0, sigma2=0.1, n_blocks=64, index=6, perturb=0.25),
    "nura16": Config("nura16", "ura", M=256, N=512, B=256, fb=0.5, n_sources=8,
                     power_db_range=0.0, sigma2=0.1, mx=16, my=16, bu=16, bv=16, n_blocks=16,
                     index=7, perturb=0.25),
}


def config(name: str) -> Config:
    return CONFIGS[name]


def serving_arrays(n_arrays: int = 64, seed: int = SEED_BASE + 3000):
    """The heterogeneous serving mix: n_arrays independent lines with M drawn
    from {64, 128, 256, 512}, N from {512, 1024, 2048, 4096}, B = M and a
    fractional bandwidth uniform in [0.2, 0.8], fixed per array."""
    rng = np.random.default_rng(seed)
    out = []
    for a in range(n_arrays):
        M = int(rng.choice([64, 128, 256, 512]))
        N = int(rng.choice([512, 1024, 2048, 4096]))
        fb = float(rng.uniform(0.2, 0.8))
        out.append(Config(f"serve{a}", "ula", M=M, N=N, B=M, fb=fb,
                          n_sources=int(rng.integers(1, 9)), power_db_range=0.0,
                          sigma2=0.1, index=3, extra={"array": a}))
    return out
