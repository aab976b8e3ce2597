"""Generators solved on the GPU (FBST_FLAG_DEVICE_GENERATORS): the Levinson
recursion for x_b = A_b^{-1} e_0 (Sec. V) in float64, one workgroup per beam,
against the host's float64 solve of the same matrices and, through the beams,
against the oracle.

The Levinson recursion on a positive definite Toeplitz matrix is weakly
stable: its forward error is bounded by a modest multiple of L cond(A_b) u
(cond ~ 2MN/delta), and the host solves a real, centred form of the same
matrix while the device solves the complex one, so the two generators are
held to L cond u of each other.  Each device generator is also checked on its
own: its residual |A x - e_0| relative to |A| |x| stays at float64 rounding
times L.  With refinement (2MN/delta > 1e6) both are refined on the host."""
import time

import numpy as np
import pytest

from oracle import direct as od
import synth
from tests.helpers import rel, crandn, oracle_problem, grid_cfg, perturbed_cfg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2512_08887_amd import fbst as F  # noqa: E402

TOL32 = 1e-5


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def residual(col, x):
    """|A x - e_0| / (|A|_1 |x|) for the Hermitian Toeplitz A with first column col."""
    import scipy.linalg as sla
    A = sla.toeplitz(col, np.conj(col))
    r = A @ x
    r[0] -= 1.0
    return float(np.linalg.norm(r) / (np.abs(A).sum(axis=0).max() * np.linalg.norm(x)))


def generators(plan):
    return F.fbst_plan_table(plan.handle, F.FBST_TABLE_GENERATOR,
                             np.zeros((plan.B, plan.L), complex))


@pytest.mark.parametrize("name", ["ula16", "grid", "perturbed", "ula256"])
def test_device_generators_match_host(name):
    need_gpu()
    cfg = {"ula16": synth.config("ula16"), "grid": grid_cfg(4, 6, 5, 4, 64),
           "perturbed": perturbed_cfg("ula", 48, 128, 40, index=102),
           "ula256": synth.config("ula256")}[name]
    keep = F.FBST_FLAG_KEEP_HOST_TABLES
    host = F.plan_for_config(cfg, flags=keep)
    dev = F.plan_for_config(cfg, flags=keep | F.FBST_FLAG_DEVICE_GENERATORS)
    gh, gd = generators(host), generators(dev)
    cond = 2.0 * cfg.M * cfg.N / cfg.delta_noise
    d = max(rel(gd[b], gh[b]) for b in range(cfg.B))
    x, y32 = None, None
    y = cfg.scene().block(0)
    x = torch.from_numpy(y).to(torch.complex64).cuda()
    out = dev.execute(x).cpu().numpy()
    y32 = x.cpu().numpy().astype(np.complex128)
    idx = list(range(cfg.B)) if cfg.B <= 64 else [0, 1, 100, 200, 255]
    e = rel(out[idx], od.beams(y32, oracle_problem(cfg, cfg.delta_noise), idx))
    gram = F.fbst_plan_table(dev.handle, F.FBST_TABLE_GRAM, np.zeros((cfg.B, dev.L), complex))
    res = max(residual(gram[b], gd[b]) for b in (0, cfg.B // 3, cfg.B - 1))
    print(f"{name}: device vs host generators {d:.2e} (cond ~ {cond:.1e}); residual {res:.1e}; "
          f"beams vs oracle {e:.2e}")
    assert d < dev.L * cond * np.finfo(np.float64).eps
    assert res < dev.L * np.finfo(np.float64).eps
    assert e < TOL32


def test_device_generators_refined_at_paper_delta():
    """delta = 1e-5 (cond ~ 2MN/delta = 8e8): the device solve, refined on the
    host, gives float64 beams at the oracle's accuracy bound."""
    need_gpu()
    cfg = synth.config("ula16")
    plan = F.plan_for_config(cfg, delta=1e-5, precision="fp64",
                             flags=F.FBST_FLAG_DEVICE_GENERATORS)
    y = cfg.scene().block(0)
    x = torch.from_numpy(y).to(torch.complex128).cuda()
    out = plan.execute(x).cpu().numpy()
    e = rel(out, od.beams(x.cpu().numpy(), oracle_problem(cfg, 1e-5)))
    print(f"ula16 fp64 delta=1e-5 device generators: rel err {e:.2e}")
    assert e < 2.0 * cfg.M * cfg.N / 1e-5 * np.finfo(np.float64).eps


def test_device_generators_largest_L():
    """L = 8192 (the 1024-element line, N = 4096): the largest system the
    device solve holds; generators against the host solve."""
    need_gpu()
    cfg = synth.config("ula1024")
    keep = F.FBST_FLAG_KEEP_HOST_TABLES
    t0 = time.perf_counter()
    host = F.plan_for_config(cfg, flags=keep)
    t1 = time.perf_counter()
    dev = F.plan_for_config(cfg, flags=keep | F.FBST_FLAG_DEVICE_GENERATORS)
    t2 = time.perf_counter()
    gh, gd = generators(host), generators(dev)
    cond = 2.0 * cfg.M * cfg.N / cfg.delta_noise
    d = max(rel(gd[b], gh[b]) for b in range(0, cfg.B, 37))
    print(f"ula1024: device vs host generators {d:.2e} (cond ~ {cond:.1e}); plan build "
          f"{t1 - t0:.2f} s host, {t2 - t1:.2f} s with device generators")
    assert d < dev.L * cond * np.finfo(np.float64).eps


@pytest.mark.parametrize("name", ["ula16", "grid", "perturbed", "ula256", "ura32"])
def test_superfast_device_generators(name):
    """FBST_FLAG_SUPERFAST_GENERATORS with FBST_FLAG_DEVICE_GENERATORS: the
    doubling Schur algorithm on the GPU (O(L log^2 L) per beam, float64).
    Against the oracle's Cholesky generator (sampled beams) within 10 L cond u,
    against the host's superfast solve within the same bound (the host solves
    the real, centred form of a uniform array's matrix, the device the complex
    one; on the perturbed line both solve the same complex matrix and agree to
    1e-13), residual at float64 rounding, beams against the oracle; its GPU
    time beside the O(L^2) device Levinson's."""
    need_gpu()
    cfg = {"ula16": synth.config("ula16"), "grid": grid_cfg(4, 6, 5, 4, 64),
           "perturbed": perturbed_cfg("ula", 48, 128, 40, index=102),
           "ula256": synth.config("ula256"), "ura32": synth.config("ura32")}[name]
    keep = F.FBST_FLAG_KEEP_HOST_TABLES
    sf = F.FBST_FLAG_SUPERFAST_GENERATORS
    dev = F.plan_for_config(cfg, flags=keep | F.FBST_FLAG_DEVICE_GENERATORS | sf)
    lev = F.plan_for_config(cfg, flags=keep | F.FBST_FLAG_DEVICE_GENERATORS)
    t0 = time.perf_counter()
    host = F.plan_for_config(cfg, flags=keep | sf)
    host_s = time.perf_counter() - t0
    gd, gh = generators(dev), generators(host)
    p = oracle_problem(cfg, cfg.delta_noise)
    L = dev.L
    cond = 2.0 * cfg.M * cfg.N / cfg.delta_noise
    sample = sorted(set([0, cfg.B // 3, cfg.B // 2, cfg.B - 1]))
    err = max(rel(gd[b], od.generator(p, b)) for b in sample)
    same = max(rel(gd[b], gh[b]) for b in range(cfg.B))
    gram = F.fbst_plan_table(dev.handle, F.FBST_TABLE_GRAM, np.zeros((cfg.B, L), complex))
    res = max(residual(gram[b], gd[b]) for b in sample)
    y = cfg.scene().block(0)
    x = torch.from_numpy(y).to(torch.complex64).cuda()
    out = dev.execute(x).cpu().numpy()
    idx = sample
    e = rel(out[idx], od.beams(x.cpu().numpy().astype(np.complex128), p, idx))
    print(f"{name} (L = {L}, B = {cfg.B}): superfast device vs Cholesky {err:.2e} "
          f"(10 L cond u = {10 * L * cond * 2.0 ** -52:.1e}); device vs host superfast {same:.1e}; "
          f"residual {res:.1e}; beams {e:.2e}; GPU solve {dev.info.generator_ms:.2f} ms superfast, "
          f"{lev.info.generator_ms:.2f} ms Levinson; host superfast plan {host_s:.2f} s")
    assert err < 10 * L * cond * 2.0 ** -52
    assert same < 10 * L * cond * 2.0 ** -52
    assert res < 10 * L * np.finfo(np.float64).eps
    assert e < TOL32
    for h in (dev, lev, host):
        h.close()


def test_superfast_device_limits():
    need_gpu()
    cfg = synth.config("ula1024")                           # L = 8192 > 4096
    with pytest.raises(F.FbstError) as e:
        F.plan_for_config(cfg, flags=F.FBST_FLAG_DEVICE_GENERATORS | F.FBST_FLAG_SUPERFAST_GENERATORS)
    assert e.value.status == F.FBST_E_UNSUPPORTED
