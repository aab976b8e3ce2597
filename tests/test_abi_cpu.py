"""CPU tests of the C ABI: the library loads, exports every declared symbol,
validates its arguments, and its FP64 host plan tables (beam grid, Toeplitz
generator c_b(d) + delta, Levinson generator x_b = A_b^{-1} e_0) agree with the
oracle.  No GPU call is made: plans are created host-only."""
import ctypes

import numpy as np
import pytest
import scipy.linalg

from paper_2512_08887_amd import fbst as F
from oracle import direct as od


def test_library_exports_every_declared_symbol():
    lib = F.lib()
    names = F.header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert F.fbst_version().startswith("fbst")


def host_plan(M, N, B, *, fc=2.0, omega=0.5, delta=1e-3, eps=1.01, L=0, geometry=None, grid=None,
              precision="fp64"):
    band = F.make_band(fc, omega, 1.0)
    opts = F.make_options(delta, eps=eps, L=L, precision=precision, flags=F.FBST_FLAG_HOST_ONLY)
    return F.fbst_plan_create(M, N, B, geometry, band, grid, opts)


@pytest.mark.parametrize("M,N,B", [(8, 32, 8), (7, 20, 5), (16, 64, 12)])
def test_host_tables_match_oracle_line(M, N, B):
    h = host_plan(M, N, B, delta=1e-3)
    try:
        info = F.fbst_plan_info(h)
        L = info.L
        assert L == 2 * N
        u = F.fbst_plan_table(h, F.FBST_TABLE_BEAM_U, np.zeros(B))
        p = od.line_problem(M, N, B, fc=2.0, omega=0.5, delta=1e-3)
        assert np.allclose(u, p.u, atol=1e-15)
        gram = F.fbst_plan_table(h, F.FBST_TABLE_GRAM, np.zeros((B, L), complex))
        gen = F.fbst_plan_table(h, F.FBST_TABLE_GENERATOR, np.zeros((B, L), complex))
        for b in range(B):
            A = od.toeplitz_system(p, b)
            assert np.allclose(gram[b], A[:, 0], rtol=0, atol=1e-12 * np.abs(A[0, 0]))
            x = od.generator(p, b)
            assert np.linalg.norm(gen[b] - x) < 1e-8 * np.linalg.norm(x)
    finally:
        F.fbst_destroy(h)


def test_host_tables_match_oracle_grid():
    geom = F.make_grid_geometry(3, 4)
    grid = F.make_beam_grid(3, 2)
    h = host_plan(12, 16, 6, fc=2.5, geometry=geom, grid=grid)
    try:
        L = F.fbst_plan_info(h).L
        p = od.grid_problem(3, 4, 3, 2, 16, fc=2.5, delta=1e-3)
        u = F.fbst_plan_table(h, F.FBST_TABLE_BEAM_U, np.zeros(6))
        v = F.fbst_plan_table(h, F.FBST_TABLE_BEAM_V, np.zeros(6))
        assert np.allclose(u, p.u) and np.allclose(v, p.v)
        gen = F.fbst_plan_table(h, F.FBST_TABLE_GENERATOR, np.zeros((6, L), complex))
        for b in range(6):
            x = od.generator(p, b)
            assert np.linalg.norm(gen[b] - x) < 1e-8 * np.linalg.norm(x)
    finally:
        F.fbst_destroy(h)


def test_gohberg_semencul_from_plan_generator():
    """The plan's generator reproduces A^{-1} w through the Gohberg-Semencul
    form (Sec. V) with circulant-embedded FFTs, as the stage-2 kernel uses it."""
    M, N, B = 8, 24, 6
    h = host_plan(M, N, B, delta=1e-2)
    try:
        L = F.fbst_plan_info(h).L
        gen = F.fbst_plan_table(h, F.FBST_TABLE_GENERATOR, np.zeros((B, L), complex))
        p = od.line_problem(M, N, B, fc=2.0, delta=1e-2)
        rng = np.random.default_rng(0)
        P = 2 * L
        for b in range(B):
            x = gen[b]
            yt = np.zeros(L, complex)
            yt[1:] = np.conj(x[:0:-1])
            w = rng.standard_normal(L) + 1j * rng.standard_normal(L)
            G1 = np.fft.fft(x, P)
            G2 = np.fft.fft(yt, P)
            V = np.fft.fft(w, P)
            p1 = np.fft.ifft(np.conj(G1) * V)[:L]
            p2 = np.fft.ifft(np.conj(G2) * V)[:L]
            beta = np.fft.ifft(G1 * np.fft.fft(p1, P) - G2 * np.fft.fft(p2, P))[:L] / x[0].real
            ref = od.solve(od.toeplitz_system(p, b), w)
            assert np.linalg.norm(beta - ref) < 1e-9 * np.linalg.norm(ref)
    finally:
        F.fbst_destroy(h)


def test_invalid_arguments():
    band = F.make_band(2.0, 0.5, 1.0)
    opts = F.make_options(1e-3, flags=F.FBST_FLAG_HOST_ONLY)
    bad = [
        dict(M=0, N=8, B=4, band=band, opts=opts),
        dict(M=4, N=8, B=4, band=None, opts=opts),
        dict(M=4, N=8, B=4, band=F.make_band(2.0, 0.5, 2.0), opts=opts),                  # ts > 1/(2 omega)
        dict(M=4, N=8, B=4, band=band, opts=F.make_options(0.0, flags=1)),                # delta <= 0
        dict(M=4, N=8, B=4, band=band, opts=F.make_options(1e-3, L=7, flags=1)),          # odd L
        dict(M=4, N=8, B=4, band=band, opts=opts, geom=F.make_line(5)),                   # mx != M
        dict(M=6, N=8, B=4, band=band, opts=opts, geom=F.make_grid_geometry(2, 3)),       # grid without beam grid
        dict(M=6, N=8, B=4, band=band, opts=opts, geom=F.make_grid_geometry(2, 3),
             grid=F.make_beam_grid(3, 2)),                                                # bu*bv != B
        dict(M=4, N=8, B=4, band=band, opts=F.make_options(1e-3, precision=9, flags=1)),
    ]
    for case in bad:
        st, hnd = F.fbst_plan_create_status(case["M"], case["N"], case["B"], case.get("geom"),
                                            case["band"], case.get("grid"), case["opts"])
        assert st == F.FBST_E_INVALID, (case, st)
        assert hnd is None
        assert F.fbst_last_error() != ""
    # an FFT size beyond one workgroup's LDS is reported as unsupported
    st, hnd = F.fbst_plan_create_status(4, 8192, 4, None, band, None,
                                        F.make_options(1e-3, flags=F.FBST_FLAG_HOST_ONLY))
    assert st == F.FBST_E_UNSUPPORTED and hnd is None


def test_stage2_size_limit_follows_the_stage2_precision():
    """Stage 2 takes P3 = 16384 (M = B = 1024, N = 4096, L = 8192) in every
    precision: in float32 in one workgroup's LDS, in float64 with each
    transform split into two 8192-point halves and a fixed scratch of
    256 workgroups x 2 x 16384 complex128 (128 MiB) added to the workspace
    of every launch.  A float64 stage 1 holds 8192 points: FBST_PREC_FP64 runs
    here with stage 1a in split-output form (p1_split = 8192), and is refused
    where that form does not apply (FBST_FLAG_NO_SPLIT)."""
    band = F.make_band(2.0, 0.5, 1.0)
    delta = 1.0 * 2 * 4096
    for prec in ("fp32", "bf16_split", "fp16_split", "fp64_stage2"):
        h = F.fbst_plan_create(1024, 4096, 1024, None, band, None,
                               F.make_options(delta, precision=prec, flags=F.FBST_FLAG_HOST_ONLY))
        info = F.fbst_plan_info(h)
        ws1, ws3 = F.fbst_workspace_bytes(h, 1), F.fbst_workspace_bytes(h, 3)
        F.fbst_destroy(h)
        assert info.p3 == 16384, (prec, info.p3)
        fixed = 256 * 2 * 16384 * 16 if prec == "fp64_stage2" else 0
        assert info.workspace_fixed == fixed, (prec, info.workspace_fixed)
        assert ws1 == info.workspace_per_block + fixed
        assert ws3 == 3 * info.workspace_per_block + fixed
    h = F.fbst_plan_create(1024, 4096, 1024, None, band, None,
                           F.make_options(delta, precision="fp64", flags=F.FBST_FLAG_HOST_ONLY))
    info = F.fbst_plan_info(h)
    F.fbst_destroy(h)
    assert info.p1 == 16384 and info.p1_split == 8192 and info.p3 == 16384
    st, hnd = F.fbst_plan_create_status(
        1024, 4096, 1024, None, band, None,
        F.make_options(delta, precision="fp64",
                       flags=F.FBST_FLAG_HOST_ONLY | F.FBST_FLAG_NO_SPLIT))
    assert st == F.FBST_E_UNSUPPORTED and hnd is None
    # a float64 plan with a float64 stage 1 of 8192 points and P3 = 16384
    h = F.fbst_plan_create(8, 2400, 8, None, band, None,
                           F.make_options(1.0, precision="fp64", flags=F.FBST_FLAG_HOST_ONLY))
    info = F.fbst_plan_info(h)
    F.fbst_destroy(h)
    assert info.p3 == 16384 and info.p1 <= 8192 and info.workspace_fixed == 256 * 2 * 16384 * 16


def test_steer_needs_a_device_plan():
    """fbst_plan_steer (a new beam grid in place) rejects NULL and host-only
    plans without touching them."""
    band = F.make_band(2.0, 0.5, 1.0)
    h = F.fbst_plan_create(8, 32, 8, None, band, None,
                           F.make_options(1.0, flags=F.FBST_FLAG_HOST_ONLY))
    g = F.make_beam_grid(8, 1, -0.5, 0.1)
    assert F.lib().fbst_plan_steer(h, g, None) == F.FBST_E_INVALID
    assert F.lib().fbst_plan_steer(None, g, None) == F.FBST_E_INVALID
    assert F.fbst_plan_info(h).B == 8
    F.fbst_destroy(h)


def test_null_and_host_only_plan_calls():
    lib = F.lib()
    lib.fbst_destroy(None)                                  # no-op
    assert lib.fbst_workspace_bytes(None, 1) == 0
    assert lib.fbst_plan_device_bytes(None) == 0
    assert lib.fbst_execute(None, None, None, None, None) == F.FBST_E_INVALID
    assert lib.fbst_graph_launch(None, None) == F.FBST_E_INVALID
    lib.fbst_graph_destroy(None)                            # no-op
    h = host_plan(8, 16, 4)
    try:
        assert lib.fbst_execute(h, ctypes.c_void_p(16), ctypes.c_void_p(16), None, None) == F.FBST_E_INVALID
        assert lib.fbst_execute_stage(h, 3, 1, ctypes.c_void_p(16), ctypes.c_void_p(16), None, None) == F.FBST_E_INVALID
        g = ctypes.c_void_p(1)
        assert lib.fbst_graph_create(h, 1, 1, ctypes.c_void_p(16), ctypes.c_void_p(16), None,
                                     ctypes.byref(g)) == F.FBST_E_INVALID
        assert g.value is None                              # *out cleared on failure
        c, ms = ctypes.c_int(), ctypes.c_float()
        assert lib.fbst_autotune(h, 4, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16),
                                 None, 0, ctypes.byref(c), ctypes.byref(ms)) == F.FBST_E_INVALID
        info = F.fbst_plan_info(h)
        assert (info.p1, info.p2x, info.p3) == (64, 32, 64)
        assert F.fbst_workspace_bytes(h, 3) == 3 * (8 + 4) * 32 * 16     # complex128 (FBST_PREC_FP64)
    finally:
        F.fbst_destroy(h)


def test_generator_accurate_at_paper_delta():
    """At the paper's delta = 1e-5 (cond(A) ~ 8e8 here) the plan's generator
    x_b = A_b^{-1} e_0 is accurate to float64 working precision: it matches a
    Cholesky solve of the plan's own Toeplitz matrix polished by iterative
    refinement with long-double residuals (a plain Levinson recursion misses
    by cond(A) * u ~ 1e-7..1e-5), and that matrix matches the oracle's A_b to
    rounding."""
    M, N, B = 16, 256, 16
    h = host_plan(M, N, B, delta=1e-5)
    try:
        L = F.fbst_plan_info(h).L
        gen = F.fbst_plan_table(h, F.FBST_TABLE_GENERATOR, np.zeros((B, L), complex))
        gram = F.fbst_plan_table(h, F.FBST_TABLE_GRAM, np.zeros((B, L), complex))
        p = od.line_problem(M, N, B, fc=2.0, delta=1e-5)
        e0 = np.zeros(L, complex)
        e0[0] = 1.0
        for b in (0, 5, 8, 15):
            A = od.toeplitz_system(p, b)
            assert np.abs(gram[b] - A[:, 0]).max() < 1e-13 * np.abs(A[0, 0])
            Ap = scipy.linalg.toeplitz(gram[b], np.conj(gram[b]))
            x = od.solve(Ap, e0)
            Al = Ap.astype(np.clongdouble)
            for _ in range(3):
                r = (e0 - Al @ x.astype(np.clongdouble)).astype(complex)
                x = x + od.solve(Ap, r)
            assert np.linalg.norm(gen[b] - x) < 1e-9 * np.linalg.norm(x)
    finally:
        F.fbst_destroy(h)


def test_server_argument_validation():
    """Server options and null arguments are rejected before any device work."""
    lib = F.lib()
    h = ctypes.c_void_p()
    bad = [F.fbst_server_options(0, 4, 16, -1), F.fbst_server_options(1 << 20, 0, 16, -1),
           F.fbst_server_options(1 << 20, 17, 16, -1), F.fbst_server_options(1 << 20, 4, 0, -1),
           F.fbst_server_options(1 << 20, 4, F.MAX_LAUNCH_BLOCKS + 1, -1)]
    for o in bad:
        assert lib.fbst_server_create(ctypes.byref(o), ctypes.byref(h)) == F.FBST_E_INVALID
        assert h.value is None
    assert lib.fbst_server_create(None, None) == F.FBST_E_INVALID
    assert lib.fbst_server_submit(None, None, None, None, 0) == F.FBST_E_INVALID
    assert lib.fbst_server_poll(None, None, 0) == F.FBST_E_INVALID
    assert lib.fbst_server_drain(None, 0.0) == F.FBST_E_INVALID
    lib.fbst_server_destroy(None)


@pytest.mark.parametrize("N,L,flags,prec,expect", [
    (1024, 2048, 0, "fp32", (4096, 2048)),       # L = 2N: half-size convolutions
    (100, 256, 0, "fp32", (512, 256)),           # L != 2N, still 3 p1s < 2 p1
    (100, 100, 0, "fp32", (256, 0)),             # p1s = 256 = p1: no gain, one convolution
    (1024, 2048, 4, "fp32", (4096, 0)),          # FBST_FLAG_NO_SPLIT
    (1024, 2048, 0, "bf16_split", (4096, 0)),    # the matrix-core stage 1a has no split form
    (1024, 2048, 0, "fp64", (4096, 2048)),
])
def test_stage1a_split_selection(N, L, flags, prec, expect):
    """Which stage-1a form a plan selects (fbst_info.p1 / p1_split)."""
    band = F.make_band(2.0, 0.5, 1.0)
    opts = F.make_options(0.1 * L, L=L, precision=prec, flags=flags | F.FBST_FLAG_HOST_ONLY)
    h = F.fbst_plan_create(4, N, 4, None, band, None, opts)
    try:
        info = F.fbst_plan_info(h)
        assert (info.p1, info.p1_split) == expect
    finally:
        F.fbst_destroy(h)


def test_precompute_flag_validation():
    """FBST_FLAG_PRECOMPUTE needs complex64 data and a K of at most 16 GiB."""
    band = F.make_band(2.0, 0.5, 1.0)
    host = F.FBST_FLAG_HOST_ONLY | F.FBST_FLAG_PRECOMPUTE
    st, h = F.fbst_plan_create_status(8, 32, 8, None, band, None,
                                      F.make_options(1.0, precision="fp64", flags=host))
    assert st == F.FBST_E_UNSUPPORTED and h is None
    assert "complex64" in F.fbst_last_error()
    # 1024 beams x N = 4096 x L = 8192 x 8 B = 256 GiB (and P3 = 16384)
    st, h = F.fbst_plan_create_status(4, 4096, 1024, None, band, None,
                                      F.make_options(1.0, flags=host))
    assert st == F.FBST_E_UNSUPPORTED and h is None
    # 4096 beams x N = 2048 x L = 4096 x 8 B = 256 GiB at P3 = 8192
    st, h = F.fbst_plan_create_status(4, 2048, 4096, None, band, None,
                                      F.make_options(1.0, flags=host))
    assert st == F.FBST_E_UNSUPPORTED and h is None and "GiB" in F.fbst_last_error()
    for prec in ("fp32", "fp64_stage2", "bf16_split"):
        st, h = F.fbst_plan_create_status(8, 512, 8, None, band, None,
                                          F.make_options(1.0, precision=prec, flags=host))
        assert st == F.FBST_OK, prec
        F.fbst_destroy(h)


@pytest.mark.parametrize("two_d", [False, True])
def test_host_tables_match_oracle_arbitrary(two_d):
    """Non-uniform arrays (Sec. IX): the plan's direct-sum Gram column and its
    complex-Levinson generator against the oracle's dense solve."""
    rng = np.random.default_rng(11 + two_d)
    d = 0.2
    if two_d:
        M, N, bu, bv = 12, 16, 3, 2
        px = (np.repeat(np.arange(3), 4) + rng.uniform(-0.3, 0.3, M)) * d
        py = (np.tile(np.arange(4), 3) + rng.uniform(-0.3, 0.3, M)) * d
        grid = F.make_beam_grid(bu, bv)
        u, v = np.repeat(od.beam_grid(bu), bv), np.tile(od.beam_grid(bv), bu)
    else:
        M, N, bu, bv = 9, 16, 7, 1
        px = (np.arange(M) + rng.uniform(-0.3, 0.3, M)) * d
        py, grid = None, None
        u, v = od.beam_grid(bu), None
    B = bu * bv
    h = host_plan(M, N, B, geometry=F.make_arbitrary(px, py), grid=grid)
    try:
        info = F.fbst_plan_info(h)
        L = info.L
        assert info.nu_width == 16            # float64 plan (float32 plans take 8)
        assert info.p2x == max(32, 1 << (2 * bu - 1).bit_length())
        assert info.p2y == (max(32, 1 << (2 * bv - 1).bit_length()) if two_d else 0)
        p = od.make_problem(N=N, L=L, eps=1.01, delta=1e-3, fc=2.0, omega=0.5, ts=1.0, px=px,
                            py=py, u=u, v=v)
        assert np.allclose(F.fbst_plan_table(h, F.FBST_TABLE_BEAM_U, np.zeros(B)), p.u)
        assert np.allclose(F.fbst_plan_table(h, F.FBST_TABLE_BEAM_V, np.zeros(B)), p.v)
        gram = F.fbst_plan_table(h, F.FBST_TABLE_GRAM, np.zeros((B, L), complex))
        gen = F.fbst_plan_table(h, F.FBST_TABLE_GENERATOR, np.zeros((B, L), complex))
        for b in range(B):
            A = od.toeplitz_system(p, b)
            assert np.allclose(gram[b], A[:, 0], rtol=0, atol=1e-12 * np.abs(A[0, 0]))
            x = od.generator(p, b)
            assert np.linalg.norm(gen[b] - x) < 1e-8 * np.linalg.norm(x)
    finally:
        F.fbst_destroy(h)


def test_arbitrary_geometry_validation():
    band = F.make_band(2.0, 0.5, 1.0)
    host = F.make_options(1e-3, flags=F.FBST_FLAG_HOST_ONLY)
    g = F.make_arbitrary(np.arange(4) * 0.2)
    g.px = None                                         # no coordinates
    with pytest.raises(F.FbstError) as e:
        F.fbst_plan_create(4, 8, 4, g, band, None, host)
    assert e.value.status == F.FBST_E_INVALID
    bad = np.arange(4) * 0.2
    bad[2] = np.nan
    with pytest.raises(F.FbstError) as e:
        F.fbst_plan_create(4, 8, 4, F.make_arbitrary(bad), band, None, host)
    assert e.value.status == F.FBST_E_INVALID
    # a 2-D oversampled grid of 256 x 256 cells does not fit one workgroup's LDS
    xy = np.arange(16) * 0.2
    with pytest.raises(F.FbstError) as e:
        F.fbst_plan_create(16, 8, 128 * 128, F.make_arbitrary(xy, xy), band,
                           F.make_beam_grid(128, 128), host)
    assert e.value.status == F.FBST_E_UNSUPPORTED
    # float64 plans spread with 16 points; p2x covers twice the modes
    h = F.fbst_plan_create(4, 8, 20, F.make_arbitrary(xy[:4]), band, None,
                           F.make_options(1e-3, precision="fp64", flags=F.FBST_FLAG_HOST_ONLY))
    try:
        info = F.fbst_plan_info(h)
        assert info.nu_width == 16 and info.p2x == 64 and info.p2y == 0
    finally:
        F.fbst_destroy(h)


def test_device_generator_flag_validation():
    band = F.make_band(2.0, 0.5, 1.0)
    with pytest.raises(F.FbstError) as e:
        F.fbst_plan_create(8, 32, 8, None, band, None,
                           F.make_options(1.0, flags=F.FBST_FLAG_DEVICE_GENERATORS | F.FBST_FLAG_HOST_ONLY))
    assert e.value.status == F.FBST_E_INVALID
    with pytest.raises(F.FbstError) as e:
        F.fbst_plan_create(8, 5000, 8, None, band, None,
                           F.make_options(1.0, flags=F.FBST_FLAG_DEVICE_GENERATORS))
    assert e.value.status == F.FBST_E_UNSUPPORTED


def test_nonuniform_spread_lanes_choice():
    """The plan spreads R elements per frequency at once only where their
    kernel supports are disjoint at every frequency: 16 for the perturbed
    256-element line (elements in order, about 25 grid cells between the
    elements taken together), 1 for an unordered aperture that wraps the
    oversampled grid many times, and 0 (not used) for a 2-D beam grid."""
    import synth
    band = F.make_band(2.0, 0.5, 1.0)
    cfg = synth.config("nula256")
    px, _ = cfg.array.positions()
    host = F.FBST_FLAG_HOST_ONLY
    h = F.fbst_plan_create(cfg.M, cfg.N, cfg.B, F.make_arbitrary(px), band, None,
                           F.make_options(cfg.delta_noise, L=cfg.L, flags=host))
    try:
        assert F.fbst_plan_info(h).nu_lanes == 16
    finally:
        F.fbst_destroy(h)
    rng = np.random.default_rng(0)
    h = F.fbst_plan_create(64, 128, 64, F.make_arbitrary(rng.uniform(0.0, 40.0, 64)), band, None,
                           F.make_options(25.6, flags=host))
    try:
        assert F.fbst_plan_info(h).nu_lanes == 1
    finally:
        F.fbst_destroy(h)
    xy = np.arange(16) * 0.2
    h = F.fbst_plan_create(16, 32, 16, F.make_arbitrary(xy, xy[::-1]), band, F.make_beam_grid(4, 4),
                           F.make_options(6.4, flags=host))
    try:
        assert F.fbst_plan_info(h).nu_lanes == 0
    finally:
        F.fbst_destroy(h)


def test_conditioning_guard():
    """fbst_plan_create refuses a plan whose stage-2 precision cannot hold
    cond(A_b) (Sec. V: A_b = F_b^H F_b + delta I): float32 at the paper's
    delta = 1e-5 would return beams off by O(1).  The reported bound
    1 + M lambda_max(T)/delta must cover every beam's condition number (the
    oracle's Gram, dense eigenvalues) and be tight at broadside."""
    M, N, B = 16, 64, 16
    for prec in ("fp32", "bf16_split", "fp16_split"):
        st, hnd = F.fbst_plan_create_status(M, N, B, None, F.make_band(2.0, 0.5, 1.0), None,
                                            F.make_options(1e-5, precision=prec,
                                                           flags=F.FBST_FLAG_HOST_ONLY))
        if prec != "fp32" and st == F.FBST_E_UNSUPPORTED and "1024 points" in F.fbst_last_error():
            continue          # the matrix-core stage 1a needs larger FFTs: refused earlier
        assert st == F.FBST_E_UNSUPPORTED and hnd is None, (prec, st)
        assert "too small" in F.fbst_last_error()
    # float64 at the same delta is accepted and reports its bound
    h = host_plan(M, N, B, delta=1e-5, precision="fp64")
    try:
        bound = F.fbst_plan_info(h).cond_bound
    finally:
        F.fbst_destroy(h)
    p = od.line_problem(M, N, B, fc=2.0, omega=0.5, delta=1e-5)
    conds = []
    for b in range(B):
        ev = np.linalg.eigvalsh(od.toeplitz_system(p, b))
        conds.append(ev[-1] / ev[0])
    assert max(conds) <= bound * (1 + 1e-6), (max(conds), bound)
    assert max(conds) >= 0.9 * bound, (max(conds), bound)
    # float32 at a noise-level delta (sigma^2 L) is accepted; float64 at an
    # absurdly small delta is not
    h = host_plan(M, N, B, delta=0.01 * 2 * N, precision="fp32")
    F.fbst_destroy(h)
    st, hnd = F.fbst_plan_create_status(M, N, B, None, F.make_band(2.0, 0.5, 1.0), None,
                                        F.make_options(1e-12, precision="fp64",
                                                       flags=F.FBST_FLAG_HOST_ONLY))
    assert st == F.FBST_E_UNSUPPORTED and hnd is None


def test_null_options_default_is_float64():
    """NULL options select the paper's delta = 1e-5 with FBST_PREC_FP64, a
    combination whose conditioning bound passes the guard: without a GPU the
    call gets past validation and the tables and fails only at the device."""
    st, hnd = F.fbst_plan_create_status(16, 64, 16, None, F.make_band(2.0, 0.5, 1.0), None, None)
    if hnd is not None:                      # a GPU is present
        try:
            info = F.fbst_plan_info(hnd)
            assert info.precision == F.PRECISIONS["fp64"] and info.io_elem_bytes == 16
        finally:
            F.fbst_destroy(hnd)
    else:
        assert st == F.FBST_E_DEVICE, (st, F.fbst_last_error())


def test_stage2_refine_flag():
    """FBST_FLAG_STAGE2_REFINE: accepted with a float32 stage 2 (its workspace
    grows by beta_1, B L complex64 per block); refused with a float64 stage 2
    and with the precomputed stage 2."""
    band = F.make_band(2.0, 0.5, 1.0)
    M, N, B = 16, 64, 12
    delta = 0.1 * 2 * N
    host = F.FBST_FLAG_HOST_ONLY
    base = F.fbst_plan_create(M, N, B, None, band, None, F.make_options(delta, flags=host))
    ref = F.fbst_plan_create(M, N, B, None, band, None,
                             F.make_options(delta, flags=host | F.FBST_FLAG_STAGE2_REFINE))
    try:
        w0 = F.fbst_plan_info(base).workspace_per_block
        w1 = F.fbst_plan_info(ref).workspace_per_block
        assert w1 - w0 == B * 2 * N * 8, (w0, w1)
    finally:
        F.fbst_destroy(base)
        F.fbst_destroy(ref)
    for prec, extra in (("fp64_stage2", 0), ("fp64", 0), ("fp32", F.FBST_FLAG_PRECOMPUTE)):
        st, h = F.fbst_plan_create_status(M, N, B, None, band, None,
                                          F.make_options(delta, precision=prec,
                                                         flags=host | extra | F.FBST_FLAG_STAGE2_REFINE))
        assert st == F.FBST_E_UNSUPPORTED and h is None, (prec, st)
        assert "REFINE" in F.fbst_last_error()


@pytest.mark.parametrize("shape", ["line", "ragged", "grid", "arbitrary", "paper_delta"])
def test_superfast_generators_host(shape):
    """FBST_FLAG_SUPERFAST_GENERATORS on a host-only plan: the generators
    x_b = A_b^{-1} e_0 by the doubling Schur algorithm against the oracle's
    Cholesky solve of the same Toeplitz matrix (Sec. V), to Levinson's bound
    L cond(A) u at a noise-level delta; at the paper's delta = 1e-5 the plan's
    refinement brings it back within that bound.  Bar: 10 L cond(A) u (the
    doubling algorithm is weakly stable: its error carries a larger constant
    than Levinson's, 4e-11 against a Levinson bound of 1e-11 on the ragged
    line)."""
    band = F.make_band(2.0, 0.5, 1.0)
    geom = grid = None
    if shape == "line":
        M, N, B, delta = 16, 256, 16, 51.2
        p = od.line_problem(M, N, B, fc=2.0, delta=delta)
    elif shape == "ragged":
        M, N, B, delta = 13, 100, 9, 20.0
        p = od.line_problem(M, N, B, fc=2.0, delta=delta)
    elif shape == "grid":
        M, N, B, delta = 12, 128, 20, 25.6
        geom, grid = F.make_grid_geometry(4, 3), F.make_beam_grid(5, 4)
        p = od.grid_problem(4, 3, 5, 4, N, fc=2.0, delta=delta)
    elif shape == "arbitrary":
        M, N, B, delta = 10, 96, 8, 19.2
        rng = np.random.default_rng(5)
        px = (np.arange(M) + rng.uniform(-0.25, 0.25, M)) / (2 * 2.5)
        geom = F.make_arbitrary(px)
        p = od.make_problem(N=N, L=2 * N, eps=1.01, delta=delta, fc=2.0, omega=0.5, ts=1.0, px=px,
                            u=od.beam_grid(B))
    else:
        M, N, B, delta = 16, 128, 6, 1e-5
        p = od.line_problem(M, N, B, fc=2.0, delta=delta)
    flags = F.FBST_FLAG_HOST_ONLY | F.FBST_FLAG_KEEP_HOST_TABLES | F.FBST_FLAG_SUPERFAST_GENERATORS
    h = F.fbst_plan_create(M, N, B, geom, band, grid,
                           F.make_options(delta, precision="fp64", flags=flags))
    try:
        L = p.L
        gen = np.empty((B, L), dtype=np.complex128)
        F.fbst_plan_table(h, F.FBST_TABLE_GENERATOR, gen)
    finally:
        F.fbst_destroy(h)
    for b in range(B):
        A = od.toeplitz_system(p, b)
        ref = od.generator(p, b)
        cond = np.linalg.cond(A)
        e = np.linalg.norm(gen[b] - ref) / np.linalg.norm(ref)
        assert e < 10 * L * cond * 2.0 ** -52, (b, e, cond)
