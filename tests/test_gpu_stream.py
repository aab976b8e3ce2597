"""Streaming over one recording with overlapping windows (fbst_execute_stream,
Sec. III streaming remark): each window's beams equal those of the window
taken out as a block (bit-identical: the same kernels read it in place), and
the oracle's beams of that window."""
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


@pytest.mark.parametrize("hop,chunk", [(128, 0), (256, 2), (77, 3)])
def test_overlapping_windows(hop, chunk):
    need_gpu()
    cfg = synth.config("ula16")
    plan = F.plan_for_config(cfg)
    sc = cfg.scene()
    T = 3 * cfg.N + 37
    rng = np.random.default_rng(hop)
    rec = np.concatenate([sc.block(k) for k in range(4)], axis=1)[:, :T] + 0.01 * crandn(rng, cfg.M, T)
    x = torch.from_numpy(rec).to(torch.complex64).cuda()
    out = plan.execute_stream(x, hop, max_chunk=chunk)
    nb = (T - cfg.N) // hop + 1
    assert out.shape[0] == nb
    p = oracle_problem(cfg, cfg.delta_noise)
    x64 = x.cpu().numpy().astype(np.complex128)
    for k in range(nb):
        win = x[:, k * hop:k * hop + cfg.N].contiguous()
        one = plan.execute(win)
        torch.cuda.synchronize()
        assert torch.equal(out[k], one), k
    for k in (0, nb - 1):
        e = rel(out[k].cpu().numpy(), od.beams(x64[:, k * hop:k * hop + cfg.N], p))
        print(f"hop {hop}: window {k} rel err {e:.2e}")
        assert e < TOL32


def test_stream_fp64_and_arguments():
    """complex128 recordings (FBST_PREC_FP64) at a noise-level ridge; bad
    lengths and hops are rejected."""
    need_gpu()
    M, N, B = 6, 64, 5
    delta = 0.1 * 2 * N
    band = F.make_band(2.0, 0.5, 1.0)
    plan = F.Plan(M, N, B, band=band, options=F.make_options(delta, precision="fp64"))
    rng = np.random.default_rng(3)
    T = 200
    rec = crandn(rng, M, T)
    x = torch.from_numpy(rec).cuda()
    out = plan.execute_stream(x, 40)
    p = od.line_problem(M, N, B, fc=2.0, delta=delta)
    for k in (0, 2, 3):
        e = rel(out[k].cpu().numpy(), od.beams(rec[:, k * 40:k * 40 + N], p))
        print(f"fp64 stream window {k}: rel err {e:.2e}")
        assert e < 1e-11
    beams = torch.empty((4, B, N), dtype=torch.complex128, device="cuda")
    with pytest.raises(F.FbstError):
        F.fbst_execute_stream(plan.handle, N - 1, 1, x.data_ptr(), beams.data_ptr())
    with pytest.raises(F.FbstError):
        F.fbst_execute_stream(plan.handle, T, 0, x.data_ptr(), beams.data_ptr())
