"""Beamspace interference nulling (fbst_nulls_*, fbst_execute_nulled) against
the FP64 oracle of Sec. VIII (eq. interfer_beam_space), through the C ABI.
Float32 tolerance as for the plain beams: relative L2 error 1e-5."""
import numpy as np
import pytest

from oracle import direct as od
from oracle import nulling as on
import synth
from tests.helpers import rel, crandn, oracle_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2512_08887_amd import fbst as F  # noqa: E402

TOL32 = 1e-5


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("qs", [[3], [1, 8], [0, 4, 9]])
def test_line_random_data(qs):
    need_gpu()
    M, N, B = 12, 40, 10
    delta = 0.1 * 2 * N
    rng = np.random.default_rng(len(qs))
    plan = F.Plan(M, N, B, band=F.make_band(2.0, 0.5, 1.0), options=F.make_options(delta))
    nl = F.Nulls(plan, qs)
    nb = 3
    y = crandn(rng, nb, M, N)
    x = torch.from_numpy(y.astype(np.complex64)).cuda()
    out = nl.execute(x).cpu().numpy()
    torch.cuda.synchronize()
    p = od.line_problem(M, N, B, fc=2.0, delta=delta)
    y32 = x.cpu().numpy().astype(np.complex128)
    e = max(rel(out[k], on.nulled_beams(y32[k], p, qs)) for k in range(nb))
    print(f"line nulling {qs}: rel err {e:.2e}")
    assert e < TOL32
    nl.close()


def test_paper_operating_point_interferer():
    """128-element line, N = 64: a 20 dB interferer on beam 40 and the
    workload's sources; nulled beams against the oracle on sampled beams,
    the interferer's power removed from its own beam, batching-invariant."""
    need_gpu()
    cfg = synth.config("ula128n64")
    band = cfg.band
    arr = cfg.array
    p = oracle_problem(cfg, cfg.delta_noise)
    q = 40
    rng = np.random.default_rng(9)
    fi, ai = synth._draw_waveform(rng, band, 100.0, 256)
    interf = synth.Source(u=float(p.u[q]), v=0.0, freqs=fi, amps=ai)
    nb = 6
    base = cfg.scene()
    y = np.stack([base.block(k) + synth.Scene(arr, band, [interf], 0.0, 0, cfg.N).clean_block(k)
                  for k in range(nb)])
    plan = F.plan_for_config(cfg)
    nl = F.Nulls(plan, [q])
    x = torch.from_numpy(y).to(torch.complex64).cuda()
    a = nl.execute(x, max_chunk=4)
    c = nl.execute(x, max_chunk=6)
    plain = plan.execute_batched(x, max_chunk=6)
    torch.cuda.synchronize()
    assert torch.equal(a, c)
    a = a.cpu().numpy()
    y32 = x.cpu().numpy().astype(np.complex128)
    idx = [0, q - 1, q, q + 1, 77, 127]
    ref = on.nulled_beams(y32[2], p, [q], beam_idx=idx)
    plain = plain.cpu().numpy()
    # Nulling is a cancellation: near the interferer the nulled beam is 40 dB
    # below the data that produced it, so float32 rounding of the data is
    # measured against the un-nulled beams (the data scale), 1e-5 as elsewhere.
    e_data = np.linalg.norm(a[2][idx] - ref) / np.linalg.norm(plain[2][idx])
    e_rel = rel(a[2][idx], ref)
    pw_plain = np.sum(np.abs(plain[2, q]) ** 2)
    pw_null = np.sum(np.abs(a[2, q]) ** 2)
    print(f"ula128n64 nulling: error {e_data:.2e} of the data scale ({e_rel:.2e} of the nulled "
          f"beams); beam {q} power {pw_plain:.3e} -> {pw_null:.3e}")
    assert e_data < TOL32
    assert pw_null < 1e-3 * pw_plain
    nl.close()


def test_grid_and_precomputed_stage2():
    """A small planar grid, and a plan whose stage 2 is precomputed."""
    need_gpu()
    mx, my, bu, bv, N = 4, 3, 4, 3, 32
    M, B = mx * my, bu * bv
    delta = 0.1 * 2 * N
    band = F.make_band(2.0, 0.5, 1.0)
    rng = np.random.default_rng(4)
    y = crandn(rng, 2, M, N)
    x = torch.from_numpy(y.astype(np.complex64)).cuda()
    y32 = x.cpu().numpy().astype(np.complex128)
    pg = od.grid_problem(mx, my, bu, bv, N, fc=2.0, delta=delta)
    for flags in (0, F.FBST_FLAG_PRECOMPUTE):
        plan = F.Plan(M, N, B, band=band, geometry=F.make_grid_geometry(mx, my),
                      grid=F.make_beam_grid(bu, bv), options=F.make_options(delta, flags=flags))
        nl = F.Nulls(plan, [5, 7])
        out = nl.execute(x).cpu().numpy()
        e = max(rel(out[k], on.nulled_beams(y32[k], pg, [5, 7])) for k in range(2))
        print(f"grid nulling (flags {flags}): rel err {e:.2e}")
        assert e < TOL32
        nl.close()
        plan.close()


def test_nulling_arguments():
    need_gpu()
    plan = F.Plan(8, 32, 8, band=F.make_band(2.0, 0.5, 1.0), options=F.make_options(6.4))
    with pytest.raises(F.FbstError):
        F.fbst_nulls_create(plan.handle, [8])           # beam out of range
    with pytest.raises(F.FbstError):
        F.fbst_nulls_create(plan.handle, [])
    p64 = F.Plan(8, 32, 8, band=F.make_band(2.0, 0.5, 1.0),
                 options=F.make_options(6.4, precision="fp64"))
    with pytest.raises(F.FbstError) as ei:
        F.fbst_nulls_create(p64.handle, [1])
    assert ei.value.status == F.FBST_E_UNSUPPORTED
    other = F.Plan(8, 32, 8, band=F.make_band(2.0, 0.5, 1.0), options=F.make_options(6.4))
    nl = F.Nulls(plan, [2])
    x = torch.zeros((1, 8, 32), dtype=torch.complex64, device="cuda")
    out = torch.empty((1, 8, 32), dtype=torch.complex64, device="cuda")
    ws = nl.workspace(1)
    with pytest.raises(F.FbstError):                    # nulls of another plan
        F.fbst_execute_nulled(other.handle, nl.handle, 1, 1, x.data_ptr(), out.data_ptr(),
                              ws.data_ptr())
    nl.close()


def _extended(p, uq, vq=None):
    """The oracle problem with the interferer directions appended as beams."""
    import dataclasses
    vq = np.zeros(len(uq)) if vq is None else np.asarray(vq, float)
    return dataclasses.replace(p, u=np.r_[p.u, np.asarray(uq, float)], v=np.r_[p.v, vq])


def test_off_grid_directions_line():
    """Interferers between grid beams (Sec. VIII: no grid alignment needed):
    against the oracle on the problem extended by the interferer directions;
    a direction exactly on a grid beam gives the on-grid result."""
    need_gpu()
    M, N, B = 12, 40, 10
    delta = 0.1 * 2 * N
    rng = np.random.default_rng(21)
    plan = F.Plan(M, N, B, band=F.make_band(2.0, 0.5, 1.0), options=F.make_options(delta))
    p = od.line_problem(M, N, B, fc=2.0, delta=delta)
    uq = [0.5 * (p.u[2] + p.u[3]), p.u[7] + 0.013]
    nl = F.Nulls(plan, u=uq)
    y = crandn(rng, 2, M, N)
    x = torch.from_numpy(y.astype(np.complex64)).cuda()
    out = nl.execute(x).cpu().numpy()
    y32 = x.cpu().numpy().astype(np.complex128)
    pe = _extended(p, uq)
    e = max(rel(out[k], on.nulled_beams(y32[k], pe, [B, B + 1], beam_idx=np.arange(B)))
            for k in range(2))
    print(f"off-grid line nulling: rel err {e:.2e}")
    assert e < TOL32
    on_grid = F.Nulls(plan, [4])
    as_dir = F.Nulls(plan, u=[float(p.u[4])])
    a = on_grid.execute(x)
    b = as_dir.execute(x)
    torch.cuda.synchronize()
    d = rel(b.cpu().numpy(), a.cpu().numpy())
    print(f"grid beam as a direction vs on-grid: {d:.2e}")
    assert d < TOL32


def test_off_grid_direction_grid_and_physics():
    """A planar grid with an off-grid (u, v) interferer against the oracle; and
    the 128-element line at N = 64 with a 20 dB interferer at an off-grid
    angle: its power leaves the neighbouring beams, sampled beams agree with
    the oracle to 1e-5 of the data scale."""
    need_gpu()
    mx, my, bu, bv, N = 4, 3, 4, 3, 32
    M, B = mx * my, bu * bv
    delta = 0.1 * 2 * N
    rng = np.random.default_rng(22)
    plan = F.Plan(M, N, B, band=F.make_band(2.0, 0.5, 1.0), geometry=F.make_grid_geometry(mx, my),
                  grid=F.make_beam_grid(bu, bv), options=F.make_options(delta))
    pg = od.grid_problem(mx, my, bu, bv, N, fc=2.0, delta=delta)
    uq, vq = [0.31], [-0.22]
    nl = F.Nulls(plan, u=uq, v=vq)
    y = crandn(rng, M, N)
    x = torch.from_numpy(y.astype(np.complex64)).cuda()
    out = nl.execute(x).cpu().numpy()
    e = rel(out, on.nulled_beams(x.cpu().numpy().astype(np.complex128), _extended(pg, uq, vq),
                                 [B], beam_idx=np.arange(B)))
    print(f"off-grid grid nulling: rel err {e:.2e}")
    assert e < TOL32

    cfg = synth.config("ula128n64")
    band = cfg.band
    p = oracle_problem(cfg, cfg.delta_noise)
    u_i = float(0.5 * (p.u[40] + p.u[41]))
    rng = np.random.default_rng(23)
    fi, ai = synth._draw_waveform(rng, band, 100.0, 256)
    interf = synth.Source(u=u_i, v=0.0, freqs=fi, amps=ai)
    y = cfg.scene().block(0) + synth.Scene(cfg.array, band, [interf], 0.0, 0, cfg.N).clean_block(0)
    plan = F.plan_for_config(cfg)
    nl = F.Nulls(plan, u=[u_i])
    x = torch.from_numpy(y).to(torch.complex64).cuda()
    a = nl.execute(x).cpu().numpy()
    plain = plan.execute(x).cpu().numpy()
    idx = [0, 39, 40, 41, 42, 100]
    ref = on.nulled_beams(x.cpu().numpy().astype(np.complex128), _extended(p, [u_i]), [cfg.B],
                          beam_idx=idx)
    e_data = np.linalg.norm(a[idx] - ref) / np.linalg.norm(plain[idx])
    drop = np.sum(np.abs(a[[40, 41]]) ** 2) / np.sum(np.abs(plain[[40, 41]]) ** 2)
    print(f"ula128n64 off-grid nulling: error {e_data:.2e} of the data scale, "
          f"power in beams 40-41 x{drop:.1e}")
    assert e_data < TOL32
    assert drop < 1e-3
