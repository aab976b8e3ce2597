"""Shared helpers of the test-suite (inputs, oracle problems, error measures)."""
import numpy as np

from oracle import direct as od
import synth


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def oracle_problem(cfg, delta, eps=None):
    """The oracle's Problem for a synth.Config (its own geometry and grid code)."""
    band = cfg.band
    e = cfg.eps if eps is None else eps
    if cfg.perturb > 0.0:
        px, py = cfg.array.positions()
        if cfg.kind == "ura":
            u = np.repeat(od.beam_grid(cfg.bu), cfg.bv)
            v = np.tile(od.beam_grid(cfg.bv), cfg.bu)
        else:
            u, v = od.beam_grid(cfg.B), None
        return od.make_problem(N=cfg.N, L=cfg.L, eps=e, delta=delta, fc=band.fc, omega=band.omega,
                               ts=band.ts, px=px, py=py, u=u, v=v)
    if cfg.kind == "ura":
        return od.grid_problem(cfg.mx, cfg.my, cfg.bu, cfg.bv, cfg.N, fc=band.fc, omega=band.omega,
                               ts=band.ts, eps=e, gamma=cfg.gamma, delta=delta)
    return od.line_problem(cfg.M, cfg.N, cfg.B, fc=band.fc, omega=band.omega, ts=band.ts, eps=e,
                           gamma=cfg.gamma, delta=delta)


def line_cfg(M, N, B, fb=0.5, sigma2=0.1, n_sources=2, index=90):
    return synth.Config(f"line{M}x{N}x{B}", "ula", M=M, N=N, B=B, fb=fb, n_sources=n_sources,
                        power_db_range=0.0, sigma2=sigma2, index=index)


def grid_cfg(mx, my, bu, bv, N, fb=0.4, sigma2=0.1, n_sources=2, index=91):
    return synth.Config(f"grid{mx}x{my}", "ura", M=mx * my, N=N, B=bu * bv, fb=fb,
                        n_sources=n_sources, power_db_range=0.0, sigma2=sigma2, mx=mx, my=my,
                        bu=bu, bv=bv, index=index)


def perturbed_cfg(kind, M, N, B, *, mx=0, my=0, bu=0, bv=0, perturb=0.25, fb=0.5, sigma2=0.1,
                  n_sources=2, index=92):
    """A non-uniform array (synth's perturbed line or grid)."""
    return synth.Config(f"n{kind}{M}x{N}x{B}", kind, M=M, N=N, B=B, fb=fb, n_sources=n_sources,
                        power_db_range=0.0, sigma2=sigma2, mx=mx, my=my, bu=bu, bv=bv,
                        index=index, perturb=perturb)


_FBST64_CACHE = {}


def fbst64_beams(cfg, block=0, delta=None):
    """Every beam of one block of a synth.Config by the second FP64 oracle
    (oracle.fbst64) on the complex64-rounded input the GPU sees; cached for
    the test session (the large configurations take tens of seconds)."""
    from oracle import fbst64 as fb
    d = cfg.delta_noise if delta is None else delta
    key = (cfg.name, block, d)
    if key not in _FBST64_CACHE:
        y = cfg.scene().block(block).astype(np.complex64).astype(np.complex128)
        p = oracle_problem(cfg, d)
        shape = (cfg.mx, cfg.my, cfg.bu, cfg.bv) if cfg.kind == "ura" else None
        _FBST64_CACHE[key] = fb.beams(y, p, shape=shape)
    return _FBST64_CACHE[key]
