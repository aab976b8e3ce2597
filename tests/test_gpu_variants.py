"""Stage-2 kernel instances chosen at run time (fbst_plan_set_variant,
fbst_autotune_ex): the persistent-grid variants give the same beams bit for
bit as their one-workgroup-per-row forms, the single-buffer form agrees with
the dual-transform form to float32 rounding (it combines the two
Gohberg-Semencul branches in another rounding order), through direct launches
and captured graphs; the tuned instance agrees with the FP64 oracle."""
import numpy as np
import pytest

from oracle import direct as od
import synth
from tests.helpers import rel, crandn, oracle_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2512_08887_amd import fbst as F  # noqa: E402

VARIANTS = [0, F.FBST_VARIANT_K3_SINGLE, F.FBST_VARIANT_K3_PERSISTENT,
            F.FBST_VARIANT_K3_SINGLE | F.FBST_VARIANT_K3_PERSISTENT,
            F.FBST_VARIANT_K3_SINGLE | F.FBST_VARIANT_K3_WAVES3]


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _plans():
    band = F.make_band(2.0, 0.5, 1.0)
    return [
        ("ula256", F.plan_for_config(synth.config("ula256")), 16),
        ("line 100x300x70", F.Plan(100, 300, 70, band=band, options=F.make_options(0.1 * 2 * 300)), 5),
        ("grid 6x5", F.Plan(30, 512, 42, band=band, geometry=F.make_grid_geometry(6, 5),
                            grid=F.make_beam_grid(7, 6), options=F.make_options(0.1 * 2 * 512)), 3),
        # P3 = 8192: three LDS exchanges per transform, so the single form's
        # alternating buffers keep the barrier ahead of each transform's first
        # exchange
        ("line 16x2048x16", F.Plan(16, 2048, 16, band=band, options=F.make_options(0.1 * 2 * 2048)), 2),
    ]


def test_variants_agree():
    need_gpu()
    rng = np.random.default_rng(80)
    for name, plan, nb in _plans():
        x = torch.from_numpy(crandn(rng, nb, plan.M, plan.N)).to(torch.complex64).cuda()
        ws = plan.workspace(nb)
        outs = {}
        for var in VARIANTS:
            plan.variant = var
            assert plan.variant == var
            outs[var] = plan.execute_batched(x, workspace=ws)
            # one block alone (fewer rows than a persistent grid holds)
            one = plan.execute(x[0])
            torch.cuda.synchronize()
            assert torch.equal(one, outs[var][0]), (name, var)
        for var in VARIANTS:
            base = outs[var & F.FBST_VARIANT_K3_SINGLE]           # same form, not persistent
            if var & F.FBST_VARIANT_K3_WAVES3:                    # another register allocation
                assert rel(outs[var].cpu().numpy(), base.cpu().numpy()) < 1e-6, (name, var)
            else:
                assert torch.equal(outs[var], base), (name, var)
        d = rel(outs[F.FBST_VARIANT_K3_SINGLE].cpu().numpy(), outs[0].cpu().numpy())
        print(f"{name}: persistent = grid bit for bit; single vs dual {d:.1e}")
        assert d < 1e-6
        plan.close()


def test_variant_rules():
    need_gpu()
    band = F.make_band(2.0, 0.5, 1.0)
    small = F.Plan(8, 64, 8, band=band, options=F.make_options(12.8))          # P3 = 256
    fp64 = F.Plan(16, 512, 16, band=band, options=F.make_options(1e-2, precision="fp64"))
    ref = F.Plan(16, 512, 16, band=band,
                 options=F.make_options(102.4, flags=F.FBST_FLAG_STAGE2_REFINE))
    for p in (small, fp64, ref):
        assert p.variant == 0
        for var in VARIANTS[1:]:
            with pytest.raises(F.FbstError) as e:
                p.variant = var
            assert e.value.status == F.FBST_E_UNSUPPORTED
        assert p.variant == 0
        p.variant = 0
    line = F.Plan(64, 1024, 64, band=band, options=F.make_options(204.8))
    assert line.variant == F.FBST_VARIANT_K3_SINGLE                    # the default where compiled
    for bad in (F.FBST_VARIANT_K3_WAVES3, 6, 7, 8, -1):
        with pytest.raises(F.FbstError):
            line.variant = bad
    line.close()
    for p in (small, fp64, ref):
        p.close()


def test_stage1b_tiles_bit_identical():
    """The stage-1b instances with half and twice the frequencies per
    workgroup give the same beams bit for bit (each transform is the same
    arithmetic), on a line and a planar grid, combined with the stage-2
    variants; a float64 stage 1 and an arbitrary array have one instance."""
    need_gpu()
    rng = np.random.default_rng(81)
    band = F.make_band(2.0, 0.5, 1.0)
    line = F.Plan(64, 512, 48, band=band, options=F.make_options(102.4))
    grid = F.Plan(64, 256, 36, band=band, geometry=F.make_grid_geometry(8, 8),
                  grid=F.make_beam_grid(6, 6), options=F.make_options(51.2))
    for name, plan in (("line", line), ("grid", grid)):
        x = torch.from_numpy(crandn(rng, 3, plan.M, plan.N)).to(torch.complex64).cuda()
        ws = plan.workspace(3)
        base = plan.variant
        ref = plan.execute_batched(x, workspace=ws)
        for tile in (F.FBST_VARIANT_K2_TILE_HALF, F.FBST_VARIANT_K2_TILE_DOUBLE):
            plan.variant = base | tile
            assert plan.variant == base | tile
            out = plan.execute_batched(x, workspace=ws)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (name, tile)
        plan.variant = base
        plan.close()
    fp64 = F.Plan(16, 512, 16, band=band, options=F.make_options(1e-2, precision="fp64"))
    px = (np.arange(16) + 0.2 * np.sin(np.arange(16))) / 5.0
    arb = F.Plan(16, 256, 16, band=band, geometry=F.make_arbitrary(px),
                 options=F.make_options(51.2))
    for p in (fp64, arb):
        for tile in (F.FBST_VARIANT_K2_TILE_HALF, F.FBST_VARIANT_K2_TILE_DOUBLE):
            with pytest.raises(F.FbstError) as e:
                p.variant = p.variant | tile
            assert e.value.status == F.FBST_E_UNSUPPORTED
        p.close()


def test_tuned_variant_graph_and_oracle():
    """fbst_autotune_ex over chunk x variant on ula256 (64 blocks): the chosen
    variant is set on the plan and cached; each variant captured in a graph
    replays bit-identical to eager; the tuned plan's beams of block 0 agree
    with the oracle on sampled beams."""
    need_gpu()
    cfg = synth.config("ula256")
    plan = F.plan_for_config(cfg)
    y = np.stack([cfg.scene().block(k) for k in range(64)]).astype(np.complex64)
    x = torch.from_numpy(y).cuda()
    chunk, var, ms = plan.autotune_ex(x, force=True)
    print(f"ula256 tuned: {chunk} blocks per launch, variant {var}, {ms:.3f} ms")
    assert chunk in (1, 2, 4, 8, 16, 32, 64) and (var & 15) in VARIANTS and ms > 0
    assert (var & ~15) in (0, F.FBST_VARIANT_K2_TILE_HALF, F.FBST_VARIANT_K2_TILE_DOUBLE)
    assert plan.variant == var
    assert plan.autotune_ex(x)[:2] == (chunk, var)       # cached
    ws = plan.workspace(chunk)
    eager = plan.execute_batched(x, max_chunk=chunk, workspace=ws)
    torch.cuda.synchronize()
    for v in VARIANTS:
        plan.variant = v
        ev = plan.execute_batched(x, max_chunk=chunk, workspace=ws)
        torch.cuda.synchronize()
        out = torch.empty_like(eager)
        g = plan.graph(x, out, workspace=ws, max_chunk=chunk)
        for _ in range(3):
            out.zero_()
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(out, ev), v
        g.close()
    plan.variant = var
    p = oracle_problem(cfg, cfg.delta_noise)
    idx = [0, 77, 128, 255]
    e = rel(eager[0].cpu().numpy()[idx], od.beams(y[0].astype(np.complex128), p, idx))
    print(f"tuned plan vs oracle: {e:.2e}")
    assert e < 1e-5
    plan.close()
