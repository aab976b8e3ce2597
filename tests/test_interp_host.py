"""The host table of the spline-interpolated off-grid beams (fbst_interp_*,
Sec. VIII) on host-only plans, against the oracle's weights, and its argument
errors; runs without a GPU."""
import numpy as np
import pytest

from oracle import direct as od
from oracle import interp as oi

from paper_2512_08887_amd import fbst as F

HOST = F.FBST_FLAG_HOST_ONLY


def host_plan(M, N, B, geometry=None, grid=None):
    return F.fbst_plan_create(M, N, B, geometry, F.make_band(2.0, 0.5, 1.0), grid,
                              F.make_options(6.4, flags=HOST))


def table_dense(h, D, bu, bv):
    first, w = F.fbst_interp_table(h, D)
    out = np.zeros((D, bu, bv))
    tv = 8 if bv > 1 else 1
    for d, ((a0, c0), (wu, wv)) in enumerate(zip(first, w)):
        out[d, a0:a0 + 8, c0:c0 + tv] = np.outer(wu, wv[:tv])
    return out.reshape(D, -1)


def test_line_weights_match_oracle():
    B = 23                                               # odd: grid (2b - B - 1) / (B - 1)
    plan = host_plan(8, 32, B)
    g = od.beam_grid(B)
    du = g[1] - g[0]
    rng = np.random.default_rng(51)
    us = list(rng.uniform(g[0], g[-1], 40)) + [g[0], g[-1], g[11], g[0] + 0.5 * du,
                                               g[-1] - 0.3 * du]
    h = F.fbst_interp_create(plan, us)
    ref = np.zeros((len(us), B))
    for d, u in enumerate(us):
        j0, w = oi.interp_weights(g, u)
        ref[d, j0:j0 + 8] = w
    err = np.abs(table_dense(h, len(us), B, 1) - ref).max()
    assert err < 1e-12, err
    F.fbst_interp_destroy(h)
    F.fbst_destroy(plan)


def test_plane_weights_match_oracle():
    bu, bv = 9, 16
    plan = host_plan(16, 32, bu * bv, F.make_grid_geometry(4, 4), F.make_beam_grid(bu, bv))
    gu, gv = od.beam_grid(bu), od.beam_grid(bv)
    rng = np.random.default_rng(52)
    us = list(rng.uniform(gu[0], gu[-1], 20)) + [gu[0], gu[-1]]
    vs = list(rng.uniform(gv[0], gv[-1], 20)) + [gv[-1], gv[3]]
    h = F.fbst_interp_create(plan, us, vs)
    ref = np.stack([oi.interp_weights_2d(gu, gv, u, v) for u, v in zip(us, vs)])
    err = np.abs(table_dense(h, len(us), bu, bv) - ref).max()
    assert err < 1e-12, err
    with pytest.raises(F.FbstError) as ei:               # host-only: no execution
        F.fbst_execute_interp(h, 1, 1, 1)
    assert ei.value.status == F.FBST_E_INVALID
    F.fbst_interp_destroy(h)
    F.fbst_destroy(plan)


def test_argument_errors():
    plan = host_plan(8, 32, 16)
    g = od.beam_grid(16)
    for bad in ([g[-1] + 1e-3], [g[0] - 1e-3], [float("nan")]):
        with pytest.raises(F.FbstError) as ei:
            F.fbst_interp_create(plan, bad)
        assert ei.value.status == F.FBST_E_INVALID
    with pytest.raises(F.FbstError) as ei:
        F.fbst_interp_create(plan, [])
    assert ei.value.status == F.FBST_E_INVALID
    F.fbst_destroy(plan)
    few = host_plan(8, 32, 7)
    with pytest.raises(F.FbstError) as ei:
        F.fbst_interp_create(few, [0.0])
    assert ei.value.status == F.FBST_E_UNSUPPORTED
    F.fbst_destroy(few)
    grid = host_plan(12, 32, 12, F.make_grid_geometry(4, 3), F.make_beam_grid(4, 3))
    with pytest.raises(F.FbstError) as ei:
        F.fbst_interp_create(grid, [0.0], [0.0])
    assert ei.value.status == F.FBST_E_UNSUPPORTED
    with pytest.raises(F.FbstError) as ei:
        F.fbst_interp_create(grid, [0.0])                # a planar grid needs v
    assert ei.value.status == F.FBST_E_INVALID
    F.fbst_destroy(grid)
    with pytest.raises(F.FbstError):
        F.fbst_interp_table(None, 1)
