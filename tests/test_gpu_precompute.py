"""Stage 2 in precomputed form (FBST_FLAG_PRECOMPUTE): K_b = F_u A_b^{-1}
built on the device in float64 arithmetic, applied as a per-beam complex
matrix product on the float32 matrix cores.  Against the FP64 oracle at the
float32 tolerance (and the float32 Gohberg-Semencul path is reported beside
it: at N = 64 its error is about cond(A) u, above the precomputed form's).
"""
import numpy as np
import pytest

from oracle import direct as od
import synth
from tests.helpers import rel, crandn, oracle_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2512_08887_amd import fbst as F  # noqa: E402

TOL32 = 1e-5


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_paper_operating_point_batched():
    """The 128-element line at N = 64 (L = 128, 128 beams): 40 blocks in
    launches of 32 and of 7 (ragged tiles) against the oracle; the beams of a
    block do not depend on how blocks are batched (bit-identical)."""
    need_gpu()
    cfg = synth.config("ula128n64")
    sc = cfg.scene()
    nb = 40
    y = np.stack([sc.block(k) for k in range(nb)])
    plan = F.plan_for_config(cfg, flags=F.FBST_FLAG_PRECOMPUTE)
    assert plan.info.stage2_precomputed == 1
    gs = F.plan_for_config(cfg)
    x = torch.from_numpy(y).to(torch.complex64).cuda()
    a = plan.execute_batched(x, max_chunk=32)
    c = plan.execute_batched(x, max_chunk=7)
    g = gs.execute_batched(x, max_chunk=32)
    one = plan.execute(x[5].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(a, c)
    assert torch.equal(a[5], one)
    p = oracle_problem(cfg, cfg.delta_noise)
    y32 = x.cpu().numpy().astype(np.complex128)
    a = a.cpu().numpy()
    g = g.cpu().numpy()
    refs = {k: od.beams(y32[k], p) for k in (0, 17, 39)}
    errs = [rel(a[k], r) for k, r in refs.items()]
    errg = [rel(g[k], r) for k, r in refs.items()]
    print(f"ula128n64: precomputed {max(errs):.2e}, float32 Gohberg-Semencul {max(errg):.2e}")
    assert max(errs) < TOL32


@pytest.mark.parametrize("M,N,B,L", [(13, 50, 7, 100), (5, 70, 66, 140), (9, 33, 3, 66)])
def test_ragged_shapes(M, N, B, L):
    """N, B and L off the 64 / 32 / 32 tiles of the product kernel."""
    need_gpu()
    rng = np.random.default_rng(M + N + B)
    band = F.make_band(2.0, 0.5, 1.0)
    delta = 0.1 * L
    plan = F.Plan(M, N, B, band=band,
                  options=F.make_options(delta, L=L, flags=F.FBST_FLAG_PRECOMPUTE))
    nb = 3
    y = crandn(rng, nb, M, N)
    x = torch.from_numpy(y.astype(np.complex64)).cuda()
    out = plan.execute_batched(x, max_chunk=nb).cpu().numpy()
    p = od.line_problem(M, N, B, fc=2.0, omega=0.5, delta=delta, gamma=L / N)
    y32 = x.cpu().numpy().astype(np.complex128)
    e = max(rel(out[k], od.beams(y32[k], p)) for k in range(nb))
    print(f"M={M} N={N} B={B} L={L} precomputed rel err {e:.2e}")
    assert e < TOL32


def test_grid_and_stage_entry():
    """A small planar grid; stage 2 alone through fbst_execute_stage uses K."""
    need_gpu()
    mx, my, bu, bv, N = 4, 3, 4, 2, 32
    M, B = mx * my, bu * bv
    band = F.make_band(2.0, 0.5, 1.0)
    geom = F.make_grid_geometry(mx, my)
    grid = F.make_beam_grid(bu, bv)
    delta = 0.1 * 2 * N
    rng = np.random.default_rng(4)
    plan = F.Plan(M, N, B, band=band, geometry=geom, grid=grid,
                  options=F.make_options(delta, flags=F.FBST_FLAG_PRECOMPUTE))
    y = crandn(rng, M, N)
    x = torch.from_numpy(y.astype(np.complex64)).cuda()
    w = plan.stage(1, plan.stage(0, x))
    b2 = plan.stage(2, w)
    full = plan.execute(x)
    torch.cuda.synchronize()
    assert torch.equal(b2[0], full)
    p = od.grid_problem(mx, my, bu, bv, N, fc=2.0, delta=delta)
    e = rel(full.cpu().numpy(), od.beams(x.cpu().numpy().astype(np.complex128), p))
    print(f"grid precomputed rel err {e:.2e}")
    assert e < TOL32


def test_fp64_stage2_precision():
    """With FBST_PREC_FP64_STAGE2 the plan's own float64 stage-2 tables build K."""
    need_gpu()
    M, N, B = 16, 64, 16
    delta = 0.1 * 2 * N
    band = F.make_band(2.0, 0.5, 1.0)
    rng = np.random.default_rng(8)
    y = crandn(rng, M, N)
    x = torch.from_numpy(y.astype(np.complex64)).cuda()
    p = od.line_problem(M, N, B, fc=2.0, delta=delta)
    ref = od.beams(x.cpu().numpy().astype(np.complex128), p)
    plan = F.Plan(M, N, B, band=band, options=F.make_options(
        delta, precision="fp64_stage2", flags=F.FBST_FLAG_PRECOMPUTE))
    out = plan.execute(x)
    torch.cuda.synchronize()
    e = rel(out.cpu().numpy(), ref)
    print(f"fp64-built K rel err {e:.2e}")
    assert e < TOL32
