"""Full-size parity for the planar array (32 x 32 elements, 32 x 32 beams,
N = 2048) and the 1024-element line (N = 4096, L = 8192), in the launch
configuration of the library's batched path.

The dense oracle cannot finish every beam of these sizes in a test, so each
stage is checked against its definition on sampled outputs, taking the GPU's
own previous-stage output as input (so each check isolates one stage):
  stage 1a  sampled sensor rows of Yhat = y E, E[n, l] = exp(-j omega_l t_n);
  stage 1b  sampled beams of W from Yhat with the projection phases;
  stage 2   sampled beams: Cholesky solve of A_b and F_u, from the GPU's W;
plus the whole chain on the sampled beams against the oracle of record.
"""
import numpy as np
import pytest

from oracle import direct as od
import synth
from tests.helpers import rel, oracle_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2512_08887_amd import fbst as F  # noqa: E402

TOL32 = 1e-5


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def stage1a_rows(y, p, rows, chunk=1024):
    """Yhat rows by the definition, E built in chunks of frequencies."""
    w = od.omegas(p.L, p.eps, p.ts)
    out = np.empty((len(rows), p.L), complex)
    for c0 in range(0, p.L, chunk):
        E = np.exp(-1j * np.multiply.outer(p.t, w[c0:c0 + chunk]))
        out[:, c0:c0 + chunk] = y[rows] @ E
    return out


def check_large(cfg, beams_idx, rows):
    y = cfg.scene().block(0)
    plan = F.plan_for_config(cfg)
    p = oracle_problem(cfg, cfg.delta_noise)
    x = torch.from_numpy(y).to(torch.complex64).cuda()
    y32 = x.cpu().numpy().astype(np.complex128)
    ws = plan.workspace(1)
    yhat = plan.stage(0, x, workspace=ws)
    w = plan.stage(1, yhat, workspace=ws)
    b = plan.stage(2, w)
    full = plan.execute(x)
    torch.cuda.synchronize()
    yhat = yhat[0].cpu().numpy().astype(np.complex128)
    w = w[0].cpu().numpy().astype(np.complex128)
    b = b[0].cpu().numpy()
    assert np.array_equal(b, full.cpu().numpy())
    assert np.isfinite(b).all()
    e1 = rel(yhat[rows], stage1a_rows(y32, p, rows))
    e2 = rel(w[beams_idx], od.project(None, p, beams_idx, yhat=yhat))
    beta = np.stack([od.solve(od.toeplitz_system(p, int(k)), w[k]) for k in beams_idx])
    e3 = rel(b[beams_idx], od.reconstruct(beta, p))
    print(f"{cfg.name}: stage 1a {e1:.2e}  stage 1b {e2:.2e}  stage 2 {e3:.2e}")
    assert e1 < TOL32 and e2 < TOL32 and e3 < TOL32
    return y32, b, p


def test_planar_array_full_size():
    """32 x 32 grid, 32 x 32 (u, v) beams, N = 2048, L = 4096, FB 0.4."""
    need_gpu()
    cfg = synth.config("ura32")
    idx = [0, 31, 33 * 16, 1023, 517]
    y32, b, p = check_large(cfg, idx, [0, 100, 1023])
    # the whole chain against the oracle of record: physical beams (u^2 + v^2 < 1)
    # to the float32 tolerance; the corner beam (u = v = -31/32, outside the
    # visible region, App. B) carries only noise projected on an evanescent
    # direction, about 10x weaker, so its relative error is held to 1e-4
    phys = [528, 517]
    e_phys = rel(b[phys], od.beams(y32, p, phys))
    e_corner = rel(b[[0]], od.beams(y32, p, [0]))
    print(f"ura32 chain: physical beams {e_phys:.2e}, corner beam {e_corner:.2e}")
    assert e_phys < TOL32
    assert e_corner < 1e-4


def test_long_line_full_size():
    """1024-element line, 1024 beams, N = 4096, L = 8192, FB 0.5."""
    need_gpu()
    cfg = synth.config("ula1024")
    y32, b, p = check_large(cfg, [5, 700], [0, 511])
    assert rel(b[[700]], od.beams(y32, p, [700])) < TOL32
