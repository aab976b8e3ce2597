"""FP64 CPU oracle of the fast broadband beamspace transformation (FBST).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke check in
``__graft_entry__.smoke`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or run anything under ``oracle/``.  The GPU library never calls it, and
the oracle shares no code, tables or constants with the GPU library: it
computes every beam straight from the paper's least-squares definition.

Modules
-------
direct
    The regularised least-squares beam of Sec. III-A, written out:
    beta = (F^H F + delta I)^{-1} F^H y  (eq. betahatls, with F from
    eq. FthetaH) and b = F_u beta (eq. bhatls), in float64, with the
    projection F^H y evaluated as the double sum of eq. (sum_1), the Gram
    matrix from the entry formula of Sec. V and a dense Cholesky solve.
    Also the explicit-matrix form for tiny sizes.
analysis
    The bias and variance expressions of Sec. VII (discrete-time reading) used
    by the Monte-Carlo pins.
nulling
    Beamspace interference nulling of Sec. VIII (eq. interfer_beam_space) and
    the array-space projection it is derived from (explicit matrices).
fbst64
    The FBST itself in float64 with numpy FFTs (Secs. IV and V: chirp-z
    stages by Bluestein, closed-form Gram column, Levinson generator,
    Gohberg-Semencul product by circulant embedding, F_u as a chirp-z): the
    fast all-beam check at full size, pinned to ``direct``.
interp
    Off-grid interpolation of Sec. VIII (not-a-knot cubic spline weights).

Pins (tests/test_oracle_*.py, run with ``-m "not gpu"``)
------------------------------------------------------
* explicit MN x L matrices vs the factored sums on tiny inputs (brute force);
* the fan form eq. (DFT_1) with its printed zeta, xi, b' and l';
* scipy.signal.czt for each of the two chirp-z stages of Sec. IV;
* numpy FFT for epsilon = 1 (stage 1a becomes a zero-padded DFT);
* the narrowband limit (FB -> 0): beams become a spatial DFT (numpy FFT);
* a noise-free on-grid plane wave is recovered to the bias level and peaks
  in its own beam;
* Monte-Carlo noise vs the variance formula of Sec. VII, and Monte-Carlo
  band-limited Gaussian sources vs the bias formula of Sec. VII;
* invariances: time origin, linearity, and the pure phase/delay effect of a
  moved reference point.

Readings of the paper that the oracle takes (where it is silent or garbled)
are listed in the project design notes; each function cites the passage it
follows.
"""
from . import direct, analysis, nulling, fbst64  # noqa: F401
