"""Graph capture and autotuning of the batched execution, through the C ABI.

A captured graph replays the same launches as fbst_execute_batched, so every
replay must be bit-identical to the eager result.  The replays are interleaved
with eager work on the same buffers' neighbours and host synchronisations, and
the input is changed between replays to show that the graph reads the bound
buffers at replay time (not a snapshot taken at capture).
"""
import numpy as np
import pytest

from oracle import direct as od
import synth
from tests.helpers import rel, oracle_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2512_08887_amd import fbst as F  # noqa: E402


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("nblocks,chunk", [(5, 2), (3, 1), (4, 4)])
def test_graph_replays_match_eager(nblocks, chunk):
    need_gpu()
    cfg = synth.config("ula16")
    sc = cfg.scene()
    plan = F.plan_for_config(cfg)
    ys = [np.stack([sc.block(i + k) for i in range(nblocks)]) for k in range(3)]
    x = torch.from_numpy(ys[0]).to(torch.complex64).cuda()
    beams = torch.empty((nblocks, plan.B, plan.N), dtype=torch.complex64, device="cuda")
    g = plan.graph(x, beams, max_chunk=chunk)
    for k in range(3):
        x.copy_(torch.from_numpy(ys[k]).to(torch.complex64))
        eager = plan.execute_batched(x, max_chunk=chunk)
        torch.cuda.synchronize()
        beams.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(beams, eager), f"replay {k} differs from eager"
        # unrelated eager work on the same stream between replays
        _ = plan.execute(x[0])
        torch.cuda.synchronize()
    # the last replay against the oracle
    p = oracle_problem(cfg, cfg.delta_noise)
    y32 = x.cpu().numpy().astype(np.complex128)
    e = max(rel(beams[i].cpu().numpy(), od.beams(y32[i], p)) for i in range(nblocks))
    assert e < 1e-5
    g.close()


def test_graph_fp64():
    need_gpu()
    cfg = synth.config("ula16")
    plan = F.plan_for_config(cfg, delta=1e-5, precision="fp64")
    y = np.stack([cfg.scene().block(i) for i in range(3)])
    x = torch.from_numpy(y).cuda()
    beams = torch.empty((3, plan.B, plan.N), dtype=torch.complex128, device="cuda")
    g = plan.graph(x, beams, max_chunk=2)
    eager = plan.execute_batched(x, max_chunk=2)
    g.launch()
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(beams, eager)


def test_graph_rejects_bad_arguments():
    need_gpu()
    cfg = synth.config("ula16")
    plan = F.plan_for_config(cfg)
    x = torch.zeros((2, plan.M, plan.N), dtype=torch.complex64, device="cuda")
    with pytest.raises(F.FbstError):
        F.fbst_graph_create(plan.handle, 0, 1, x.data_ptr(), x.data_ptr(), 0)
    with pytest.raises(F.FbstError):
        F.fbst_graph_create(plan.handle, 2, 2, x.data_ptr(), x.data_ptr(), 0)  # chunk > 1 needs a workspace
    with pytest.raises(F.FbstError):
        F.fbst_graph_launch(0)


def test_autotune_picks_a_valid_chunk_and_caches():
    need_gpu()
    cfg = synth.config("ula16")
    plan = F.plan_for_config(cfg)
    nb = 12
    x = torch.from_numpy(np.stack([cfg.scene().block(i) for i in range(nb)])).to(torch.complex64).cuda()
    c1, ms1 = plan.autotune(x)
    assert c1 in (1, 2, 4, 8) and ms1 > 0
    c2, ms2 = plan.autotune(x)
    assert (c2, ms2) == (c1, ms1)        # served from the cache
    c3, ms3 = plan.autotune(x, force=True)
    assert c3 in (1, 2, 4, 8) and ms3 > 0
    # the tuned chunk computes the same beams as any other chunk
    a = plan.execute_batched(x, max_chunk=c3)
    b = plan.execute_batched(x, max_chunk=1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
