"""The accuracy claim behind the non-uniform stage 1b's parameters (Sec. IX).

The plan spreads with an exponential-of-semicircle kernel of width w = 8
(float32 plans) or 16 (float64) on a grid of nf = next power of two >= 2 K
points for K modes, beta = 0.98 pi (1 - 1/(2 sigma)) w, sigma = nf / K, and
divides by the kernel's Fourier transform (Gauss-Legendre quadrature).  This
check evaluates a type-1 non-uniform FFT with exactly those choices in numpy
float64 and compares it with the direct sum over random points: the error
must sit below the float32 target of the path (1e-7 with w = 8) and near
float64 rounding (1e-12 with w = 16).  It is a check of the design's numbers,
independent of the GPU code and of the oracle.
"""
import numpy as np
import pytest


def type1(c, s, K, w):
    nf = max(32, 1 << (2 * K - 1).bit_length())
    beta = 0.98 * np.pi * (1.0 - 0.5 / (nf / K)) * w
    ka = K // 2
    g = (s % 1.0) * nf                                  # points in grid units
    j0 = np.floor(g).astype(int) - w // 2 + 1
    f = g - np.floor(g)
    grid = np.zeros(nf, complex)
    for t in range(w):
        z = (t - w // 2 + 1 - f) * 2.0 / w
        kv = np.exp(beta * (np.sqrt(np.maximum(1.0 - z * z, 0.0)) - 1.0))
        np.add.at(grid, (j0 + t) % nf, c * kv)
    X = np.fft.ifft(grid) * nf                          # sum_j grid_j e^{+2 pi i k j / nf}
    zq, wq = np.polynomial.legendre.leggauss(4 * w + 32)
    k = np.arange(K) - ka
    phi = np.exp(beta * (np.sqrt(1.0 - zq ** 2) - 1.0))
    psi = 0.5 * w * (wq * phi * np.cos(np.multiply.outer(k, zq) * np.pi * w / nf)).sum(axis=1)
    return X[k % nf] / psi


@pytest.mark.parametrize("K,w,bar", [(37, 8, 1e-7), (64, 8, 2e-7), (256, 8, 2e-7), (100, 16, 1e-12)])
def test_type1_accuracy(K, w, bar):
    rng = np.random.default_rng(K + w)
    M = 3 * K
    s = rng.uniform(-3.0, 3.0, M)                       # cycles: wraps the grid several times
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    k = np.arange(K) - K // 2
    exact = np.exp(2j * np.pi * np.multiply.outer(k, s)) @ c
    err = np.linalg.norm(type1(c, s, K, w) - exact) / np.linalg.norm(exact)
    assert err < bar, err
