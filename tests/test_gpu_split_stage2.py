"""Float64 stage 2 at P3 = 16384, where one float64 transform (256 KiB)
exceeds the LDS: each P3-point transform of the Gohberg-Semencul apply and of
F_u (Sec. V) runs as two 8192-point halves in LDS joined by one radix-2 step,
with the branch spectra of a beam in a fixed global scratch between them.

Every beam is compared with the FP64 oracle (oracle.fbst64, pinned to the
Cholesky oracle of record).  Bars:
  FBST_PREC_FP64 (float64 throughout): aggregate and every beam within
      1e-10 at a noise-level ridge (cond(A_b) ~ 1e2..1e3; the chirp phases,
      up to ~1e4 rad, carry ~1e4 u of absolute error on both sides), and
      within 10 cond u (u = 2^-53, cond the plan's bound on cond(A_b)) at the
      paper's conditioning;
  FBST_PREC_FP64_STAGE2 (float32 stage 1): aggregate <= 1e-5 and every
      beam err_b / max(|b_b|, RMS) <= 1e-5, the float64-stage-2 bar of the
      every-beam tests.
Small shapes reach P3 = 16384 through L = 2N > 4096: a ragged line
(N = 2800, L = 5600, not a multiple of the 512 threads of a half transform),
a float64 line with P1 = 8192, and a 4 x 4 grid."""
import numpy as np
import pytest

from tests.helpers import fbst64_beams, grid_cfg, line_cfg, oracle_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2512_08887_amd import fbst as F  # noqa: E402

SPLIT_SCRATCH = 256 * 2 * 16384 * 16
U64 = 2.0 ** -53


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def check_every_beam(name, got, ref, bar_beam, bar_agg):
    err = np.linalg.norm(got - ref, axis=1)
    norm = np.linalg.norm(ref, axis=1)
    scale = np.maximum(norm, np.sqrt(np.mean(norm ** 2)))
    agg = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    worst = (err / scale).max()
    print(f"{name}: aggregate {agg:.2e} (bar {bar_agg:.1e}); every beam on max(|b|, RMS) "
          f"{worst:.2e} (bar {bar_beam:.1e})", flush=True)
    assert agg < bar_agg and worst < bar_beam


CASES = {
    "line16_n2800_fp64_stage2": (lambda: line_cfg(16, 2800, 16, index=140), "fp64_stage2"),
    "line8_n2400_fp64": (lambda: line_cfg(8, 2400, 8, index=141), "fp64"),
    "grid4x4_n2400_fp64_stage2": (lambda: grid_cfg(4, 4, 4, 4, 2400, index=142), "fp64_stage2"),
}


@pytest.mark.parametrize("case", list(CASES))
def test_split_stage2_small_every_beam(case):
    need_gpu()
    make, prec = CASES[case]
    cfg = make()
    plan = F.plan_for_config(cfg, precision=prec)
    info = plan.info
    assert info.p3 == 16384 and info.workspace_fixed == SPLIT_SCRATCH
    # the oracle sees the complex64-rounded scene, so the float64 plan does too
    npdt = np.complex128 if prec == "fp64" else np.complex64
    ys = np.stack([cfg.scene().block(k) for k in range(3)]).astype(np.complex64).astype(npdt)
    x = torch.from_numpy(ys).cuda()
    print(f"[{case}] M = {cfg.M}, N = {cfg.N}, L = {cfg.L}, B = {cfg.B}, p1 = {info.p1}", flush=True)
    one = plan.execute(x[0]).cpu().numpy()
    many = plan.execute_batched(x, max_chunk=2).cpu().numpy()
    torch.cuda.synchronize()
    # the rows of a launch are independent: the same beams whatever the chunking
    assert np.array_equal(one, many[0])
    # stage 2 alone with the plan's own scratch (no workspace) equals the path
    w = plan.stage(1, plan.stage(0, x[:1]))
    s2 = plan.stage(2, w).cpu().numpy()[0]
    assert np.array_equal(s2, one)
    for k in (0, 2):
        ref = fbst64_beams(cfg, k)
        if prec == "fp64":
            check_every_beam(f"{case} block {k}", many[k], ref, 1e-10, 1e-10)
        else:
            check_every_beam(f"{case} block {k}", many[k], ref, 1e-5, 1e-5)
    plan.close()


@pytest.mark.parametrize("prec", ["fp64_stage2", "fp64"])
def test_split_stage2_ula1024_every_beam(prec):
    """M = B = 1024, N = 4096 (L = 8192) with a float64 stage 2 at the
    workload's noise ridge: every beam to the float64-stage-2 bar; float64
    throughout (stage 1a in split-output form at 8192 points, one LDS
    buffer) to 1e-10."""
    need_gpu()
    import synth
    cfg = synth.config("ula1024")
    plan = F.plan_for_config(cfg, precision=prec)
    assert plan.info.p3 == 16384 and plan.info.workspace_fixed == SPLIT_SCRATCH
    npdt = np.complex128 if prec == "fp64" else np.complex64
    y = cfg.scene().block(0).astype(np.complex64).astype(npdt)
    x = torch.from_numpy(y[None]).cuda()
    print(f"[ula1024 {prec}] executing", flush=True)
    out = plan.execute_batched(x).cpu().numpy()[0]
    ref = fbst64_beams(cfg)
    p = oracle_problem(cfg, cfg.delta_noise)
    assert out.shape == ref.shape == (p.B, cfg.N)
    bar = 1e-10 if prec == "fp64" else 1e-5
    check_every_beam(f"ula1024 {prec}", out, ref, bar, bar)
    plan.close()


def test_split_stage2_ula1024_paper_conditioning():
    """The paper's delta = 1e-5 belongs to M = 128, N = 64 (Sec. VI), where
    cond(A_b) ~ 2MN / delta = 1.6e9.  At M = 1024, N = 4096 the same absolute
    delta puts the bound at 1.6e12: the float64 Gram column's own rounding
    (about L u 2MN ~ delta) leaves A_b numerically indefinite and the plan is
    refused.  Scaled with MN (delta = 5.12e-3) the conditioning is the
    paper's; a float32 stage 2 is refused there, and float64 throughout is
    held to 10 cond u on sampled beams against beta_b = A_b^{-1} w_b by the
    direct oracle's dense Cholesky solve (w_b and F_u by the pinned FP64
    oracle): Levinson's forward error at this conditioning (oracle.fbst64's
    generators, up to ~5e-4) is well above cond u, while the plan refines its
    generators."""
    need_gpu()
    import synth
    from oracle import direct as od
    from oracle import fbst64 as fb
    cfg = synth.config("ula1024")
    band = F.make_band(cfg.band.fc, cfg.band.omega, cfg.band.ts)
    st, h = F.fbst_plan_create_status(
        cfg.M, cfg.N, cfg.B, None, band, None,
        F.make_options(1e-5, eps=cfg.eps, L=cfg.L, precision="fp64", flags=F.FBST_FLAG_HOST_ONLY))
    assert st != F.FBST_OK and h is None
    delta = 1e-5 * (cfg.M * cfg.N) / (128 * 64)
    st, h = F.fbst_plan_create_status(
        cfg.M, cfg.N, cfg.B, None, band, None,
        F.make_options(delta, eps=cfg.eps, L=cfg.L, precision="fp32", flags=F.FBST_FLAG_HOST_ONLY))
    assert st == F.FBST_E_UNSUPPORTED and h is None
    print(f"[ula1024 fp64 delta {delta:.3g}] planning", flush=True)
    plan = F.plan_for_config(cfg, delta=delta, precision="fp64")
    cond = plan.info.cond_bound
    y = cfg.scene().block(0).astype(np.complex64).astype(np.complex128)
    x = torch.from_numpy(y[None]).cuda()
    print(f"[ula1024 fp64 delta {delta:.3g}] cond bound {cond:.2e}; executing", flush=True)
    out = plan.execute_batched(x).cpu().numpy()[0]
    plan.close()
    p = oracle_problem(cfg, delta)
    W = fb.project(y, p)
    bar = 10.0 * cond * U64
    for b in (0, 300, 511, 1023):
        ref = fb.reconstruct(od.solve(od.toeplitz_system(p, b), W[b]), p)
        e = float(np.linalg.norm(out[b] - ref) / np.linalg.norm(ref))
        print(f"ula1024 fp64 delta {delta:.3g} (cond bound {cond:.2e}) beam {b}: {e:.2e} "
              f"(bar {bar:.1e})", flush=True)
        assert e < bar, (b, e)


def test_split_stage2_served_and_static():
    """The fixed scratch of the split stage 2 goes with every launch: the
    server reserves nblocks * per-block + fixed bytes (batches of 2 and 3
    blocks and a single one equal fbst_execute bit for bit; a budget below
    one block plus the scratch fails the request cleanly), and the
    allocation-free entry point, whose array is smaller than the scratch,
    refuses the plan."""
    need_gpu()
    cfg = line_cfg(16, 2800, 16, index=143)
    plan = F.plan_for_config(cfg, precision="fp64_stage2")
    info = plan.info
    ys = np.stack([cfg.scene().block(k) for k in range(5)]).astype(np.complex64)
    xs = [torch.from_numpy(y).cuda() for y in ys]
    outs = [torch.empty((cfg.B, cfg.N), dtype=torch.complex64, device="cuda") for _ in xs]
    torch.cuda.synchronize()
    budget = 3 * info.workspace_per_block + info.workspace_fixed + (1 << 20)
    srv = F.Server(workspace_bytes=budget, streams=2, max_batch=3)
    for tag, (x, o) in enumerate(zip(xs, outs)):
        srv.submit(plan, x, o, tag)
    srv.drain(timeout_s=60)
    comps = srv.poll(16)
    srv.close()
    assert sorted(c.tag for c in comps) == list(range(len(xs)))
    assert all(c.status == F.FBST_OK for c in comps)
    for x, o in zip(xs, outs):
        alone = plan.execute(x)
        torch.cuda.synchronize()
        assert torch.equal(alone, o)
    small = F.Server(workspace_bytes=info.workspace_per_block + info.workspace_fixed // 2,
                     streams=1, max_batch=1)
    small.submit(plan, xs[0], outs[0], 99)
    small.drain(timeout_s=30)
    c = small.poll(4)
    small.close()
    assert len(c) == 1 and c[0].status == F.FBST_E_NOMEM
    with pytest.raises(F.FbstError) as e:
        plan.execute_static(xs[0][None], outs[0][None])
    assert e.value.status == F.FBST_E_UNSUPPORTED
    plan.close()
