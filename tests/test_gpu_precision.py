"""Split-precision stage 1a on the matrix cores (bfloat16 / float16 hi-lo
products with float32 accumulation) against the FP64 oracle.

Tolerance for the low-precision forms: relative L2 error 1e-3 on the beams
(the stated target for BF16/FP16 with refinement); stage 1a alone is held to
the error of a 16-bit hi/lo operand pair, 1e-4 (bfloat16: 2^-16 per operand,
three radix-16 passes per transform and two transforms) and 1e-5 (float16).
"""
import numpy as np
import pytest

from oracle import direct as od
import synth
from tests.helpers import rel, oracle_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2512_08887_amd import fbst as F  # noqa: E402

STAGE1A_TOL = {"bf16_split": 1e-4, "fp16_split": 1e-5}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", ["bf16_split", "fp16_split"])
def test_small_line_split_precision(prec):
    need_gpu()
    cfg = synth.config("ula16")
    y = cfg.scene().block(0)
    plan = F.plan_for_config(cfg, precision=prec)
    p = oracle_problem(cfg, cfg.delta_noise)
    x = torch.from_numpy(y).to(torch.complex64).cuda()
    y32 = x.cpu().numpy().astype(np.complex128)
    yhat = plan.stage(0, x)
    out = plan.execute(x)
    torch.cuda.synchronize()
    e1 = rel(yhat[0].cpu().numpy(), od.stage1a(y32, p))
    eb = rel(out.cpu().numpy(), od.beams(y32, p))
    print(f"ula16 {prec}: stage 1a {e1:.2e}, beams {eb:.2e}")
    assert e1 < STAGE1A_TOL[prec]
    assert eb < 1e-3


@pytest.mark.parametrize("prec", ["bf16_split", "fp16_split"])
def test_large_line_split_precision_sampled(prec):
    """The 256-element line (P1 = 4096, three radix-16 matrix-core passes)."""
    need_gpu()
    cfg = synth.config("ula256")
    y = cfg.scene().block(0)
    plan = F.plan_for_config(cfg, precision=prec)
    p = oracle_problem(cfg, cfg.delta_noise)
    x = torch.from_numpy(y).to(torch.complex64).cuda()
    y32 = x.cpu().numpy().astype(np.complex128)
    out = plan.execute(x).cpu().numpy()
    idx = [3, 128, 250]
    eb = rel(out[idx], od.beams(y32, p, idx))
    print(f"ula256 {prec}: sampled beams {eb:.2e}")
    assert eb < 1e-3


def test_remainder_pass_sizes():
    """P1 = 2048 (two matrix-core passes + a radix-8 float32 pass) and
    P1 = 1024 (radix 16, 16, 4)."""
    need_gpu()
    rng = np.random.default_rng(2)
    for M, N, B in [(8, 512, 8), (8, 300, 6)]:
        band = F.make_band(2.0, 0.5)
        for prec in ("bf16_split", "fp16_split"):
            plan = F.Plan(M, N, B, band=band, options=F.make_options(0.1 * 2 * N, precision=prec))
            y = (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))).astype(np.complex64)
            x = torch.from_numpy(y).cuda()
            yhat = plan.stage(0, x)
            torch.cuda.synchronize()
            p = od.line_problem(M, N, B, fc=2.0, delta=0.1 * 2 * N)
            e1 = rel(yhat[0].cpu().numpy(), od.stage1a(y.astype(np.complex128), p))
            print(f"M={M} N={N} P1={plan.info.p1} {prec}: stage 1a {e1:.2e}")
            assert e1 < STAGE1A_TOL[prec]
