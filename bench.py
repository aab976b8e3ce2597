#!/usr/bin/env python3
"""Throughput of the FBST hot path on one MI355X.

Workload: the large linear-array stream -- M = B = 256 sensors/beams,
N = 1024 complex64 samples per block, L = 2048 basis frequencies
(eps = 1.01, gamma = 2), fractional bandwidth 0.5, 8 seeded band-limited
sources over 30 dB, 10 dB SNR, streamed as 64 consecutive blocks.  One step
is one pass of the whole path (time chirp-z, space chirp-z, Toeplitz apply +
reconstruction) over the 64 blocks, with inputs already resident in HBM.

Prints one JSON line: beam-samples/s, ms per step, the roofline of the
dominant kernel (stage 2, timed with HIP events on its own stream inside the
timed region), p50/p99 latency of a single block, and the CPU oracle timed on
a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12      # MI355X vector FP32 (packed FMA), FLOP/s
PEAK_FP64 = 78.6e12
PEAK_HBM = 8.0e12


def fft_flops(P):
    return 5.0 * P * math.log2(P)


def stage_flops(info):
    """Algorithmic flops per block and per stage (5 P log2 P per FFT, 6 per
    complex product, 2 per complex add)."""
    M, N, B, L = info.M, info.N, info.B, info.L
    if info.p1_split:   # one forward and two inverse transforms of p1_split points
        s0 = M * (3 * fft_flops(info.p1_split) + 6 * (N + 2 * info.p1_split + L))
    else:
        s0 = M * (2 * fft_flops(info.p1) + 6 * (N + info.p1 + L))
    if info.bv > 1:
        s1 = (info.my * L * (2 * fft_flops(info.p2x) + 6 * (info.mx + info.p2x + info.bu))
              + info.bu * L * (2 * fft_flops(info.p2y) + 6 * (info.my + info.p2y + info.bv)))
    else:
        s1 = L * (2 * fft_flops(info.p2x) + 6 * (M + info.p2x + B))
    P = info.p3
    s2 = B * (8 * fft_flops(P) + 6 * (4 * P + L + P + N) + 2 * P)
    return s0, s1, s2


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, y, delta, n_beams=48, n_beams_1t=8):
    """The FP64 oracle on one block restricted to n_beams beams, on every BLAS
    thread the process may use, and on n_beams_1t beams with one thread."""
    from oracle import direct as od
    import threadpoolctl
    threads = max([d.get("num_threads", 1) for d in threadpoolctl.threadpool_info()] or [1])
    band = cfg.band
    p = od.line_problem(cfg.M, cfg.N, cfg.B, fc=band.fc, omega=band.omega, ts=band.ts, eps=cfg.eps,
                        gamma=cfg.gamma, delta=delta)
    idx = np.linspace(0, cfg.B - 1, n_beams).round().astype(int)
    t0 = time.perf_counter()
    ref = od.beams(y, p, idx)
    dt = time.perf_counter() - t0
    idx1 = idx[:: max(1, n_beams // n_beams_1t)][:n_beams_1t]
    with threadpoolctl.threadpool_limits(1):
        t1 = time.perf_counter()
        od.beams(y, p, idx1)
        dt1 = time.perf_counter() - t1
    return ({"value": n_beams * cfg.N / dt, "unit": "beam-samples/s", "cores": int(threads),
             "kind": "oracle",
             "sample": f"FP64 oracle (definition: dense projection sums + Cholesky), one block, "
                       f"{n_beams} of {cfg.B} beams, {dt:.1f} s",
             "cpu_model": _cpu_model(), "affinity_cores": len(os.sched_getaffinity(0)),
             "one_thread": {"value": len(idx1) * cfg.N / dt1, "unit": "beam-samples/s",
                            "sample": f"{len(idx1)} beams, {dt1:.1f} s, 1 BLAS thread"}},
            idx, ref)


def fbst64_baseline(names=("ula16", "ula256", "ura32", "ula1024")):
    """The second FP64 oracle (the FBST with numpy FFTs) on every beam of one
    block of each workload, on the host's cores (its Levinson solves run in
    up to 16 worker processes for the large ones)."""
    from oracle import fbst64 as fb
    import synth
    out, beams = {}, {}
    for name in names:
        c = synth.config(name)
        p = _oracle_problem(c)
        y = c.scene().block(0).astype(np.complex64).astype(np.complex128)
        shape = (c.mx, c.my, c.bu, c.bv) if c.kind == "ura" else None
        t0 = time.perf_counter()
        beams[name] = fb.beams(y, p, shape=shape)
        dt = time.perf_counter() - t0
        out[name] = {"blocks_per_s": 1.0 / dt, "beam_samples_per_s": c.B * c.N / dt,
                     "seconds": dt}
    out["workers"] = min(16, os.cpu_count() or 1)
    return out, beams


def large_bench(F, torch, *, steps=5, log=print):
    """Whole-path throughput of the planar array (32 x 32, N = 2048) and the
    1024-element line (N = 4096) in float32, and of the line with the
    bfloat16 / float16 split stage 1a and with a float64 stage 2 (P3 = 16384,
    split transforms) or float64 throughout; blocks of one step in one launch.
    Returns the results and block 0's beams of each (for the oracle check)."""
    import synth
    runs = [("ura32", "fp32", 8), ("ura32", "fp32_refine", 8), ("ula1024", "fp32", 4),
            ("ula1024", "bf16_split", 4), ("ula1024", "fp16_split", 4),
            ("ula1024", "fp64_stage2", 4), ("ula1024", "fp64", 4)]
    out, first = {}, {}
    for name, prec, nb in runs:
        c = synth.config(name)
        if prec == "fp32_refine":
            plan = F.plan_for_config(c, precision="fp32", flags=F.FBST_FLAG_STAGE2_REFINE)
        else:
            plan = F.plan_for_config(c, precision=prec)
        y = np.stack([c.scene().block(k) for k in range(nb)]).astype(np.complex64)
        if prec == "fp64":
            y = y.astype(np.complex128)
        x = torch.from_numpy(y).cuda()
        ws = plan.workspace(nb)
        bo = plan.execute_batched(x, workspace=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.execute_batched(x, beams=bo, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        key = f"{name}_{prec}"
        out[key] = {"workload": f"{name}: M={c.M}, B={c.B}, N={c.N}, L={c.L}, {nb} blocks per launch",
                    "precision": prec, "value": nb * c.B * c.N / (ms * 1e-3),
                    "unit": "beam-samples/s", "ms_per_step": ms}
        first[key] = (name, bo[0].cpu().numpy())
        log(f"[bench] {key}: {ms:.3f} ms per {nb} blocks, {out[key]['value']:.3e} beam-samples/s")
        plan.close()
        del x, ws, bo
    return out, first


def rocprof_summary(kt_dir, pmc_dirs, copy_dirs):
    """Text summary of rocprofv3 CSV output: per-kernel dispatch durations
    (kernel trace) and HBM counters per dispatch, scaled by what the same
    counters read for a plain copy of known size."""
    import csv
    import glob
    import re
    from collections import defaultdict

    def short(name):
        m = re.match(r"_ZN4fbst12_GLOBAL__N_1\d+(k_\w+?)ILi(\d+)EDv8_DF16(b|_)", name)
        if m:   # names the profiler leaves mangled (16-bit vector template arguments)
            return f"{m.group(1)}<{m.group(2)}, {'bf16x8' if m.group(3) == 'b' else 'f16x8'}>"
        n = name.replace("void ", "").replace("fbst::(anonymous namespace)::", "")
        return re.sub(r"\(.*", "", n)

    out = []
    dur = defaultdict(list)
    for f in glob.glob(os.path.join(kt_dir, "*kernel_trace.csv")):
        for r in csv.DictReader(open(f)):
            key = (short(r["Kernel_Name"]), int(r["Grid_Size_X"]))
            dur[key].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out.append("kernel | grid (work-items) | dispatches | avg us | min us | max us")
    out.append("---|---|---|---|---|---")
    for (k, g), v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"{k} | {g} | {len(v)} | {np.mean(v) / 1e3:.1f} | {np.min(v) / 1e3:.1f} | {np.max(v) / 1e3:.1f}")
    scale = {}
    for cdir in copy_dirs:
        for f in glob.glob(os.path.join(cdir, "*counter_collection.csv")):
            rows = [r for r in csv.DictReader(open(f)) if "copyBuffer" in r["Kernel_Name"]]
            for r in rows:
                scale.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    copy_bytes = None
    for cdir in copy_dirs:
        for f in glob.glob(os.path.join(cdir, "*.log")) + glob.glob(cdir + ".log"):
            m = re.search(r'"copy_calib_bytes_each_way": (\d+)', open(f).read())
            if m:
                copy_bytes = int(m.group(1))
    factors = {}
    if copy_bytes:
        for c, v in scale.items():
            factors[c] = copy_bytes / (np.median(v) * 1024.0)
    out.append("")
    out.append(f"copy calibration: {copy_bytes} bytes each way; counter KiB read per copy: "
               + ", ".join(f"{c} {np.median(v):.0f}" for c, v in scale.items())
               + "; scale factors (true bytes per counted byte): "
               + ", ".join(f"{c} {f:.3f}" for c, f in factors.items()))
    cnt = defaultdict(list)
    for pdir in pmc_dirs:
        for f in glob.glob(os.path.join(pdir, "*counter_collection.csv")):
            for r in csv.DictReader(open(f)):
                cnt[(short(r["Kernel_Name"]), int(r["Grid_Size"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
    out.append("")
    out.append("kernel | grid | counter | dispatches | KiB per dispatch | scaled MB per dispatch")
    out.append("---|---|---|---|---|---")
    scaled = {}
    for (k, g, c), v in sorted(cnt.items()):
        if not k.startswith("k_"):
            continue
        f = factors.get(c, 1.0)
        scaled.setdefault(f"{k} | {g}", {})[c] = float(np.median(v) * 1024 * f)
        out.append(f"{k} | {g} | {c} | {len(v)} | {np.median(v):.0f} | {np.median(v) * 1024 * f / 1e6:.1f}")
    return "\n".join(out), scaled


def sq_summary(pmc_dirs, kernels=("k_toeplitz_fu", "k_time_czt", "k_axis_czt")):
    """Per-wave SQ counters of the hot kernels from rocprofv3 --pmc runs
    (counter_collection.csv; several runs, each with its own counter set):
    median over dispatches of counter / SQ_WAVES, per (kernel, grid)."""
    import csv
    import glob
    import re
    from collections import defaultdict

    def short(name):
        m = re.match(r"_ZN4fbst12_GLOBAL__N_1\d+(k_\w+?)ILi(\d+)EDv8_DF16(b|_)", name)
        if m:
            return f"{m.group(1)}<{m.group(2)}, {'bf16x8' if m.group(3) == 'b' else 'f16x8'}>"
        n = name.replace("void ", "").replace("fbst::(anonymous namespace)::", "")
        return re.sub(r"\(.*", "", n)

    per = defaultdict(lambda: defaultdict(list))      # (kernel, grid) -> counter -> values
    for pdir in pmc_dirs:
        for f in glob.glob(os.path.join(pdir, "*counter_collection.csv")):
            rows = list(csv.DictReader(open(f)))
            by_dispatch = defaultdict(dict)
            for r in rows:
                k = short(r["Kernel_Name"])
                if not any(k.startswith(x) for x in kernels):
                    continue
                by_dispatch[(r.get("Dispatch_Id", ""), k, int(r["Grid_Size"]))][r["Counter_Name"]] = \
                    float(r["Counter_Value"])
            for (_, k, g), c in by_dispatch.items():
                waves = c.get("SQ_WAVES")
                for name, val in c.items():
                    if name != "SQ_WAVES" and waves:
                        per[(k, g)][name].append(val / waves)
                if waves:
                    per[(k, g)]["SQ_WAVES"].append(waves)
    names = sorted({n for d in per.values() for n in d})
    out = ["kernel | grid | " + " | ".join(n.replace("SQ_", "") for n in names),
           "---|---|" + "---|" * len(names)]
    for (k, g), d in sorted(per.items()):
        cells = []
        for n in names:
            v = d.get(n)
            cells.append(f"{np.median(v):.0f}" if v else "")
        out.append(f"{k} | {g} | " + " | ".join(cells))
    return "\n".join(out)


# Sources whose change invalidates stored HBM counter readings of the kernels.
KERNEL_SOURCES = ["cx.h", "fft_lds.h", "kernel_common.h", "kernels.h", "kernels.hip", "stage2.hip",
                  "mfma_czt.hip", "precompute.hip"]
COUNTERS_JSON = os.path.join(ROOT, "profiles", "hbm_counters_ula256.json")


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2512_08887_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "paper_2512_08887_amd", "build.py"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel, grid):
    """HBM bytes per dispatch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) of a
    kernel from the committed counter readings, or None when the kernel sources
    changed since they were taken."""
    try:
        with open(COUNTERS_JSON) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != kernel_source_digest():
        return None
    c = d.get("kernels", {}).get(f"{kernel} | {grid}")
    if not c or "FETCH_SIZE" not in c or "WRITE_SIZE" not in c:
        return None
    return c["FETCH_SIZE"] + c["WRITE_SIZE"]


def precompute_bench(F, torch, *, steps=10, warmup=2, nblk=1024, chunk=256, log=print, checks=None):
    """The paper's operating point (128-element line, N = 64, L = 128, 128
    beams; synthetic stand-in, 1024 blocks): stage 2 as the Gohberg-Semencul
    kernel against the precomputed per-beam product on the matrix cores.
    Accuracy against the oracle is appended to checks (run with the CPU
    baseline)."""
    import synth
    cfg = synth.config("ula128n64")
    sc = cfg.scene()
    base = np.stack([sc.block(k) for k in range(64)])
    x = torch.from_numpy(np.concatenate([base] * (nblk // 64))).to(torch.complex64).cuda()
    stream = torch.cuda.current_stream()
    out = {"workload": "ula128n64: line M=B=128, N=64, L=128, FB=0.5, 3 sources, 10 dB SNR, "
                       f"delta=sigma^2 L=12.8, {nblk} blocks per step, {chunk} per launch"}
    samples = nblk * cfg.B * cfg.N
    beams = {}
    for name, flags in (("gohberg_semencul", 0), ("precomputed", F.FBST_FLAG_PRECOMPUTE)):
        t0 = time.perf_counter()
        plan = F.plan_for_config(cfg, flags=flags)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        ws = plan.workspace(chunk)
        bo = torch.empty((nblk, cfg.B, cfg.N), dtype=torch.complex64, device="cuda")
        for _ in range(warmup):
            plan.execute_batched(x, beams=bo, workspace=ws, max_chunk=chunk)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            plan.execute_batched(x, beams=bo, workspace=ws, max_chunk=chunk)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        r = {"value": samples / (ms / 1e3), "unit": "beam-samples/s", "ms_per_step": ms,
             "plan_s": plan_s, "device_MiB": F.fbst_plan_device_bytes(plan.handle) / 2**20}
        # stage 2 alone, one launch of `chunk` blocks, on the stage-1 output
        w = plan.stage(1, plan.stage(0, x[:chunk].contiguous(), nblocks=chunk), nblocks=chunk)
        o2 = torch.empty((chunk, cfg.B, cfg.N), dtype=torch.complex64, device="cuda")
        plan.stage(2, w, nblocks=chunk, out=o2)
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a0.record(stream)
        for _ in range(20):
            plan.stage(2, w, nblocks=chunk, out=o2)
        a1.record(stream)
        torch.cuda.synchronize()
        r["stage2_ms_per_launch"] = a0.elapsed_time(a1) / 20
        if flags:
            flops = 8.0 * cfg.B * cfg.N * plan.L * chunk     # complex multiply-add = 8 flops
            ach = flops / (r["stage2_ms_per_launch"] / 1e3)
            r["roofline"] = {"kernel": "k_precomputed_apply (per-beam complex product, float32 MFMA)",
                             "bound": "mfma", "achieved": ach / 1e12, "peak": 157.3,
                             "unit": "TFLOP/s", "frac": ach / 157.3e12,
                             "flops_per_launch": flops}
        beams[name] = bo[0].cpu().numpy()
        out[name] = r
        log(f"[bench] n64 {name}: {ms:.3f} ms per {nblk} blocks, stage 2 "
            f"{r['stage2_ms_per_launch'] * 1e3:.1f} us per {chunk}-block launch, plan {plan_s:.2f} s")
        plan.close()
    x0 = x[0].cpu().numpy().astype(np.complex128)

    def problem():
        from oracle import direct as od
        return od.line_problem(cfg.M, cfg.N, cfg.B, fc=cfg.band.fc, omega=cfg.band.omega,
                               ts=cfg.band.ts, eps=cfg.eps, gamma=cfg.gamma, delta=cfg.delta_noise)

    def accuracy():
        from oracle import direct as od
        ref = od.beams(x0, problem())
        out["accuracy_vs_oracle"] = {k: float(np.linalg.norm(v - ref) / np.linalg.norm(ref))
                                     for k, v in beams.items()}
    if checks is not None:
        checks.append(accuracy)

    # beamspace nulling of interferers at 1 and 4 beams (Sec. VIII), precomputed stage 2
    plan = F.plan_for_config(cfg, flags=F.FBST_FLAG_PRECOMPUTE)
    nul = {}
    for qs in ([40], [20, 40, 60, 100]):
        t0 = time.perf_counter()
        nl = F.Nulls(plan, qs)
        build_s = time.perf_counter() - t0
        ws = nl.workspace(chunk)
        bo = torch.empty((nblk, cfg.B, cfg.N), dtype=torch.complex64, device="cuda")
        nl.execute(x, beams=bo, workspace=ws, max_chunk=chunk)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            nl.execute(x, beams=bo, workspace=ws, max_chunk=chunk)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        idx = [0, qs[0], 77]
        got = bo[0].cpu().numpy()[idx]
        r = {"value": samples / (ms / 1e3), "unit": "beam-samples/s", "ms_per_step": ms,
             "tables_build_s": build_s}
        nul[f"P={len(qs)}"] = r

        def nulling_accuracy(r=r, qs=qs, idx=idx, got=got):
            from oracle import nulling as on
            refn = on.nulled_beams(x0, problem(), qs, beam_idx=idx)
            r["rel_l2_vs_oracle"] = float(np.linalg.norm(got - refn) / np.linalg.norm(refn))
        if checks is not None:
            checks.append(nulling_accuracy)
        log(f"[bench] n64 nulling P={len(qs)}: {ms:.3f} ms per {nblk} blocks, tables {build_s:.2f} s")
        nl.close()
    plan.close()
    out["nulling"] = nul
    return out


def nonuniform_bench(F, torch, *, steps=10, warmup=2, log=print, checks=None):
    """Non-uniform arrays (Sec. IX): the 256-element line with every element
    moved by up to a quarter spacing (same band, blocks and delta as the
    uniform line) and the perturbed 16 x 16 grid.  Stage 1b is the type-1
    non-uniform FFT per frequency (spread kernel, then one FFT pass per axis);
    its roofline is HBM bandwidth over the algorithmic bytes of the two
    kernels."""
    import synth
    stream = torch.cuda.current_stream()
    out = {}
    for name in ("nula256", "nura16"):
        cfg = synth.config(name)
        nblk = cfg.n_blocks
        sc = cfg.scene()
        x = torch.from_numpy(np.stack([sc.block(k) for k in range(nblk)])).to(torch.complex64).cuda()
        t0 = time.perf_counter()
        plan = F.plan_for_config(cfg)
        plan_s = time.perf_counter() - t0
        info = plan.info
        ws = plan.workspace(nblk)
        bo = torch.empty((nblk, cfg.B, cfg.N), dtype=torch.complex64, device="cuda")
        for _ in range(warmup):
            plan.execute_batched(x, beams=bo, workspace=ws)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            plan.execute_batched(x, beams=bo, workspace=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        # stage 1b alone over the step's blocks (one launch of each kernel)
        yhat = plan.stage(0, x, nblocks=nblk)
        zws = plan.workspace(nblk)
        w = plan.stage(1, yhat, nblocks=nblk, workspace=zws)
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a0.record(stream)
        for _ in range(20):
            plan.stage(1, yhat, nblocks=nblk, out=w, workspace=zws)
        a1.record(stream)
        torch.cuda.synchronize()
        s1b = a0.elapsed_time(a1) / 20
        nfx, nfy = info.p2x, max(info.p2y, 1)
        cells, L, M, B = nfx * nfy, info.L, cfg.M, cfg.B
        fused = (info.p2y == 0 and 256 <= nfx <= 4096) or (nfx == 32 and info.p2y == 32)
        # Yhat in, tables (pre + positions per axis) once per launch, W out; the
        # two-kernel form also writes the oversampled grid and reads it back
        # (and, in 2-D, the x pass's output)
        tables = M * L * 8 * (2 + (1 if info.p2y else 0))
        byts = nblk * (M * L * 8 + B * L * 8) + tables
        if not fused:
            byts += nblk * 2 * cells * L * 8
            if info.p2y:
                byts += nblk * 2 * cfg.bu * nfy * L * 8
        ach = byts / (s1b / 1e3)
        idx = [0, 37, B // 2, B - 1]
        got = bo[0].cpu().numpy()[idx]
        x0 = x[0].cpu().numpy().astype(np.complex128)
        out[name] = {
            "workload": f"{name}: {'grid %dx%d' % (cfg.mx, cfg.my) if cfg.kind == 'ura' else 'line'} "
                        f"M={M}, B={B}, N={cfg.N}, L={L}, elements moved by up to {cfg.perturb} spacing, "
                        f"{nblk} blocks per step",
            "value": nblk * B * cfg.N / (ms / 1e3), "unit": "beam-samples/s", "ms_per_step": ms,
            "plan_s": plan_s, "oversampled_grid": [nfx, nfy], "kernel_width": info.nu_width,
            "stage1b_ms_per_launch": s1b,
            "stage1b_roofline": {"kernels": ("k_nu_plane_fused" if info.p2y else "k_nu_line_fused") if fused else
                                 ("k_nu_spread_plane + 2 x k_axis_dft" if info.p2y else
                                  "k_nu_spread_line + k_axis_dft"), "bound": "hbm",
                                 "achieved": ach / 1e9, "peak": 8000.0, "unit": "GB/s",
                                 "frac": ach / 8e12, "bytes_per_launch": byts},
        }

        def accuracy(r=out[name], cfg=cfg, idx=idx, got=got, x0=x0):
            from oracle import direct as od
            t0 = time.perf_counter()
            ref = od.beams(x0, _oracle_problem(cfg), idx)
            dt = time.perf_counter() - t0
            r["rel_l2_vs_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            r["oracle"] = {"value": len(idx) * cfg.N / dt, "unit": "beam-samples/s",
                           "sample": f"FP64 oracle, one block, {len(idx)} beams, {dt:.1f} s"}
        if checks is not None:
            checks.append(accuracy)
        log(f"[bench] {name}: {ms:.3f} ms per {nblk} blocks, stage 1b {s1b * 1e3:.1f} us "
            f"({ach / 1e9:.0f} GB/s), plan {plan_s:.2f} s")
        plan.close()
        del x, ws, zws, yhat, w, bo
    return out


def interp_bench(F, torch, plan, cfg, beams, *, reps=20, log=print, checks=None):
    """Off-grid beams by spline interpolation of 8 grid beams (Sec. VIII) on
    the step's own beams: one launch over 16 blocks at B directions
    drawn across the grid (seeded).  Algorithmic HBM bytes per launch: each
    grid beam read once and each interpolated beam written once,
    8 nb N (B + D); the kernel is bound by HBM."""
    # the default beam grid of a line (eq. thetab): u_b = (2b - B + 1) / B for
    # even B, (2b - B + 1) / (B - 1) for odd B, b = 0..B-1
    den = cfg.B if cfg.B % 2 == 0 else cfg.B - 1
    g = (2.0 * np.arange(cfg.B) - cfg.B + 1.0) / den
    us = np.sort(np.random.default_rng(7).uniform(g[0], g[-1], cfg.B))
    it = F.Interp(plan, us)
    D, nb = len(us), min(16, beams.shape[0])   # fixed launch size: comparable counter runs
    src = beams[:nb]
    out = torch.empty((nb, D, cfg.N), dtype=torch.complex64, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(3):
        it.execute(src, out)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        it.execute(src, out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 8 * nb * cfg.N * (cfg.B + D)
    ach = nbytes / (ms / 1e3) / 1e9
    r = {"workload": f"{cfg.name}: {D} directions drawn across the beam grid, {nb} blocks per "
                     f"launch, 8 grid beams each (not-a-knot cubic spline in u)",
         "value": nb * D * cfg.N / (ms / 1e3), "unit": "beam-samples/s", "ms_per_launch": ms,
         "roofline": {"kernel": "k_interp_beams_x2", "bound": "hbm", "achieved": ach, "peak": 8000.0,
                      "unit": "GB/s", "frac": ach / 8000.0, "bytes_per_launch": nbytes,
                      "traffic": stored_traffic("k_interp_beams_x2<1>",
                                                nb * D * ((cfg.N // 2 + 255) // 256) * 256)}}
    got = out[0].cpu().numpy().astype(np.complex128)
    b0 = src[0].cpu().numpy().astype(np.complex128)

    def accuracy():
        from oracle import interp as oi
        ref = oi.interp_beams(b0, g, us)
        r["rel_l2_vs_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    if checks is not None:
        checks.append(accuracy)
    log(f"[bench] interp: {ms * 1e3:.1f} us per {nb}-block launch ({ach:.0f} GB/s)")
    it.close()
    return r


def _oracle_problem(cfg):
    """The oracle's Problem of a perturbed synthetic array (positions from the
    input generator, beam grid of eq. (thetab))."""
    from oracle import direct as od
    px, py = cfg.array.positions()
    if cfg.kind == "ura":
        u, v = np.repeat(od.beam_grid(cfg.bu), cfg.bv), np.tile(od.beam_grid(cfg.bv), cfg.bu)
    else:
        u, v = od.beam_grid(cfg.B), None
    b = cfg.band
    return od.make_problem(N=cfg.N, L=cfg.L, eps=cfg.eps, delta=cfg.delta_noise, fc=b.fc,
                           omega=b.omega, ts=b.ts, px=px, py=py, u=u, v=v)


def serve_bench(F, torch, configs, *, seconds=2.0, loads=(0.5, 0.8, 0.95), burst=768,
                slots=16, seed=0, precision="fp32", log=print, checks=None):
    """Continuous-batching server over resident plans: saturation throughput
    from a burst, then Poisson arrivals at fractions of it (arrays chosen
    uniformly); latency = completion - submission on the server clock.  Each
    array's input is block 0 of its synthetic scene.  checks: a list that
    receives (config, plan-precision, served beams of block 0) for the first
    arrays of each distinct shape class, compared with the oracle in the CPU
    leg."""
    from concurrent.futures import ThreadPoolExecutor

    t0 = time.perf_counter()

    def mk(c):
        return F.plan_for_config(c, precision=precision)

    with ThreadPoolExecutor(4) as ex:
        plans = list(ex.map(mk, configs))
    plan_s = time.perf_counter() - t0
    rng = np.random.default_rng(seed)
    xs, outs = [], []
    for c, p in zip(configs, plans):
        x = torch.from_numpy(c.scene().block(0).astype(np.complex64)).cuda()
        xs.append(x)
        outs.append([torch.empty((c.B, c.N), dtype=torch.complex64, device="cuda") for _ in range(slots)])
    torch.cuda.synchronize()
    srv = F.Server(workspace_bytes=4 << 30, streams=4, max_batch=16)
    samples = [c.B * c.N for c in configs]
    A = len(configs)

    def run_point(arrivals_us, choice):
        free = [list(range(slots)) for _ in range(A)]
        inflight = {}
        lat, batch, done_samples = [], [], 0
        base = srv.clock_us()
        k = 0
        tag = 0

        def harvest():
            nonlocal done_samples
            for comp in srv.poll(4096):
                a, s, sub = inflight.pop(comp.tag)
                free[a].append(s)
                lat.append(comp.done_us - comp.submit_us)
                batch.append(comp.batch)
                done_samples += samples[a]

        while k < len(arrivals_us):
            now = srv.clock_us() - base
            if now < arrivals_us[k]:
                harvest()
                continue
            a = choice[k]
            if not free[a]:
                harvest()
                continue
            s = free[a].pop()
            inflight[tag] = (a, s, now)
            srv.submit(plans[a], xs[a], outs[a][s], tag, sync=False)
            tag += 1
            k += 1
        srv.drain(timeout_s=120)
        harvest()
        elapsed_s = (srv.clock_us() - base) / 1e6
        return (np.array(lat) / 1e3, done_samples / elapsed_s, len(lat) / elapsed_s,
                float(np.mean(batch)) if batch else 0.0)

    # saturation: everything submitted at once
    choice = rng.integers(0, A, burst)
    lat, sat_samples, sat_blocks, sat_batch = run_point(np.zeros(burst), choice)
    log(f"[serve {precision}] {A} arrays, plans {plan_s:.1f} s; saturation {sat_blocks:.0f} blocks/s, "
        f"{sat_samples:.3e} beam-samples/s, mean batch {sat_batch:.1f}")
    res = {"arrays": A, "precision": precision, "plan_build_s": plan_s,
           "saturation_blocks_per_s": sat_blocks, "saturation_beam_samples_per_s": sat_samples,
           "saturation_mean_batch": sat_batch, "points": []}
    for load in loads:
        rate = load * sat_blocks
        n = max(50, int(rate * seconds))
        arr = np.cumsum(rng.exponential(1e6 / rate, n))
        choice = rng.integers(0, A, n)
        lat, thr, blk, mb = run_point(arr, choice)
        pt = {"load": load, "offered_blocks_per_s": rate, "blocks": int(len(lat)),
              "beam_samples_per_s": thr, "p50_ms": float(np.percentile(lat, 50)),
              "p99_ms": float(np.percentile(lat, 99)), "mean_batch": mb}
        log(f"[serve {precision}] load {load:.2f}: {blk:.0f} blocks/s, p50 {pt['p50_ms']:.3f} ms, "
            f"p99 {pt['p99_ms']:.3f} ms, mean batch {mb:.2f}")
        res["points"].append(pt)
    srv.close()
    if checks is not None:
        # the largest array and the extreme fractional bandwidths of the mix
        pick = sorted(set([int(np.argmax([c.M * c.N for c in configs])),
                           int(np.argmin([c.fb for c in configs])),
                           int(np.argmax([c.fb for c in configs]))]))
        for a in pick:
            out = plans[a].execute(xs[a])
            torch.cuda.synchronize()
            checks.append((configs[a], precision, xs[a].cpu().numpy(), out.cpu().numpy()))
    for p in plans:
        p.close()
    return res


def serve_accuracy(checks, n_beams=6):
    """Relative L2 error of served beams against the second FP64 oracle
    (oracle.fbst64) on sampled beams, per checked array and precision."""
    from oracle import fbst64 as fb
    out = []
    for cfg, prec, y, got in checks:
        p = _oracle_problem(cfg)
        idx = np.unique(np.linspace(0, cfg.B - 1, n_beams).round().astype(int))
        ref = fb.beams(y.astype(np.complex128), p, beam_idx=idx)
        out.append({"array": cfg.name, "M": cfg.M, "N": cfg.N, "fb": round(cfg.fb, 3),
                    "precision": prec,
                    "rel_l2": float(np.linalg.norm(got[idx] - ref) / np.linalg.norm(ref))})
    return out


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--sq-summary":
        # bench.py --sq-summary PMC_DIR[,PMC_DIR...] [KERNEL_PREFIX,...]: per-wave SQ counters
        # of the hot kernels (default: the three stages of the path)
        if len(sys.argv) > 3:
            print(sq_summary(sys.argv[2].split(","), tuple(sys.argv[3].split(","))))
        else:
            print(sq_summary(sys.argv[2].split(",")))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--rocprof-summary":
        # bench.py --rocprof-summary KT_DIR PMC_DIR[,PMC_DIR] COPY_DIR[,COPY_DIR] [COUNTERS_JSON]
        text, scaled = rocprof_summary(sys.argv[2], sys.argv[3].split(","), sys.argv[4].split(","))
        print(text)
        if len(sys.argv) > 5:
            with open(sys.argv[5], "w") as fh:
                json.dump({"what": "HBM bytes per dispatch: FETCH_SIZE and WRITE_SIZE medians, scaled "
                                   "by a plain-copy calibration; keyed 'kernel | grid work-items'",
                           "source_sha256": kernel_source_digest(), "kernels": scaled}, fh, indent=1)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk", type=int, default=-1,
                    help="blocks per launch (-1: chosen by fbst_autotune, 0: all 64)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the planar array and 1024-element line throughputs")
    ap.add_argument("--no-fbst64", action="store_true",
                    help="skip timing the FP64 FBST oracle on every workload")
    ap.add_argument("--latency-reps", type=int, default=200)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-mix measurement")
    ap.add_argument("--no-n64", action="store_true",
                    help="skip the N = 64 Gohberg-Semencul vs precomputed stage-2 comparison")
    ap.add_argument("--no-variants", action="store_true", help="skip the bf16/fp16 split variants")
    ap.add_argument("--no-nu", action="store_true", help="skip the non-uniform array measurement")
    ap.add_argument("--no-interp", action="store_true",
                    help="skip the spline-interpolated off-grid beams measurement")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(blocks are independent: more GPUs would each run this same path on their own blocks)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2512_08887_amd import fbst as F

    if args.copy_calib:
        # a plain copy of known size: FETCH_SIZE / WRITE_SIZE per dispatch of
        # this kernel give the counters' scale (bytes counted per byte moved)
        n = args.copy_calib * 2**20 // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_each_way": n * 4, "dispatches": 5}))
        return

    cfg = synth.config("ula256")
    nblk = cfg.n_blocks
    sc = cfg.scene()
    t0 = time.perf_counter()
    ys = np.stack([sc.block(k) for k in range(nblk)])
    gen_s = time.perf_counter() - t0
    print(f"[bench] generated {nblk} blocks in {gen_s:.1f} s", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    plan = F.plan_for_config(cfg)
    plan_s = time.perf_counter() - t0
    info = plan.info
    print(f"[bench] plan: L={info.L} P1={info.p1} P2={info.p2x} P3={info.p3} "
          f"tables {info.device_bytes / 2**20:.1f} MiB, {plan_s:.2f} s", file=sys.stderr, flush=True)

    x = torch.from_numpy(ys).to(torch.complex64).cuda()
    beams = torch.empty((nblk, cfg.B, cfg.N), dtype=torch.complex64, device="cuda")
    tuned_chunk = tuned_ms = tuned_var = None
    untuned = None
    if args.chunk < 0:
        tune_ws = plan.workspace(min(nblk, F.MAX_LAUNCH_BLOCKS))
        # the untuned configuration for comparison: the plan's default stage-2
        # variant at 16 blocks per launch
        u_var, u_chunk = plan.variant, min(16, nblk)
        tuned_chunk, tuned_var, tuned_ms = plan.autotune_ex(x, beams=beams, workspace=tune_ws)

        def step_ms(var, ch):
            # both configurations timed alike, after the autotuner's sweep has
            # warmed the GPU: 3 untimed, 10 timed steps
            plan.variant = var
            for _ in range(3):
                plan.execute_batched(x, beams=beams, workspace=tune_ws, max_chunk=ch)
            ua, ub = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ua.record()
            for _ in range(10):
                plan.execute_batched(x, beams=beams, workspace=tune_ws, max_chunk=ch)
            ub.record()
            torch.cuda.synchronize()
            return ua.elapsed_time(ub) / 10

        untuned = {"blocks_per_launch": u_chunk, "k3_variant": u_var,
                   "ms_per_step": step_ms(u_var, u_chunk)}
        tuned_ms = step_ms(tuned_var, tuned_chunk)
        plan.variant = tuned_var
        del tune_ws
        chunk = tuned_chunk
        print(f"[bench] autotuned: {chunk} blocks per launch, stage-2 variant {tuned_var} "
              f"({tuned_ms:.3f} ms per 64 blocks; untuned {untuned['ms_per_step']:.3f} ms)",
              file=sys.stderr, flush=True)
    else:
        chunk = nblk if args.chunk == 0 else min(args.chunk, nblk)
    ws = plan.workspace(chunk)
    yhat = ws[: chunk * cfg.M * info.L * 8].view(torch.complex64).view(chunk, cfg.M, info.L)
    w = ws[chunk * cfg.M * info.L * 8: chunk * (cfg.M + cfg.B) * info.L * 8].view(torch.complex64).view(chunk, cfg.B, info.L)
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream

    ev_pairs = []

    def step(record):
        for b0 in range(0, nblk, chunk):
            nb = min(chunk, nblk - b0)
            F.fbst_execute_stage(plan.handle, 0, nb, x[b0].data_ptr(), yhat.data_ptr(), 0, sptr)
            F.fbst_execute_stage(plan.handle, 1, nb, yhat.data_ptr(), w.data_ptr(), 0, sptr)
            if record:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            F.fbst_execute_stage(plan.handle, 2, nb, w.data_ptr(), beams[b0].data_ptr(), 0, sptr)
            if record:
                e1.record(stream)
                ev_pairs.append((e0, e1))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for _ in range(args.steps):
        step(True)
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / args.steps
    k3_ms = float(np.mean([a.elapsed_time(b) for a, b in ev_pairs]))
    samples = nblk * cfg.B * cfg.N
    value = samples * args.steps / (total_ms / 1e3)
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step, stage-2 launch {k3_ms:.3f} ms",
          file=sys.stderr, flush=True)

    # whole-path cross-check of the timed output against a single-block execute
    ref0 = plan.execute(x[0].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(ref0, beams[0]), "batched output differs from single-block output"

    # latency of one block alone (execute + completion), host clock
    lat = []
    one = x[0].contiguous()
    out1 = torch.empty((cfg.B, cfg.N), dtype=torch.complex64, device="cuda")
    # single blocks on a plan of their own, its kernel instances tuned for one
    # block per launch (the step's plan keeps the ones tuned for 64)
    lplan = F.plan_for_config(cfg, precision="fp32")
    ws1 = lplan.workspace(1)
    lat_var = lplan.autotune_ex(one.unsqueeze(0), workspace=ws1)[1] if args.chunk < 0 else lplan.variant
    for i in range(args.latency_reps + 5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.fbst_execute(lplan.handle, one.data_ptr(), out1.data_ptr(), ws1.data_ptr(), sptr)
        stream.synchronize()
        if i >= 5:
            lat.append((time.perf_counter() - t0) * 1e3)
    lat = np.array(lat)
    # the same single block replayed from a captured graph (one launch call)
    g1 = lplan.graph(one.unsqueeze(0), out1.unsqueeze(0), workspace=ws1)
    glat = []
    for i in range(args.latency_reps + 5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g1.launch()
        stream.synchronize()
        if i >= 5:
            glat.append((time.perf_counter() - t0) * 1e3)
    glat = np.array(glat)
    g1.close()
    lplan.close()
    # the whole 64-block step as one graph, and the autotuned blocks per launch
    gb = torch.empty_like(beams)
    gall = plan.graph(x, gb, workspace=ws, max_chunk=chunk)
    gall.launch()
    torch.cuda.synchronize()
    ga = torch.cuda.Event(enable_timing=True)
    gz = torch.cuda.Event(enable_timing=True)
    ga.record(stream)
    for _ in range(args.steps):
        gall.launch()
    gz.record(stream)
    torch.cuda.synchronize()
    graph_ms = ga.elapsed_time(gz) / args.steps
    assert torch.equal(gb, beams), "graph replay differs from the eager step"
    gall.close()
    if tuned_chunk is None:
        tune_ws = plan.workspace(min(nblk, F.MAX_LAUNCH_BLOCKS))
        fixed_var = plan.variant
        tuned_chunk, tuned_var, tuned_ms = plan.autotune_ex(x, beams=gb, workspace=tune_ws)
        plan.variant = fixed_var       # the timed run above used the plan's own variant
        del tune_ws
    del gb
    print(f"[bench] graph step {graph_ms:.3f} ms; autotune chunk {tuned_chunk} ({tuned_ms:.3f} ms)",
          file=sys.stderr, flush=True)

    s0, s1, s2 = stage_flops(info)
    k3_flops_launch = s2 * chunk
    achieved = k3_flops_launch / (k3_ms / 1e3)
    result = {
        "metric": "beam-samples/s at M=B=256,N=1024 (FP32 vs batched/BF16) + p50/p99 block latency",
        "value": value,
        "unit": "beam-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ula256: line M=256, B=256, N=1024, L=2048, eps=1.01, FB=0.5, "
                               "8 sources over 30 dB, 10 dB SNR, delta=sigma^2 L=204.8, 64 blocks per step",
                   "blocks_per_step": nblk, "blocks_per_launch": chunk, "precision": "fp32"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "variant": lat_var,
                       "what": "one block alone: execute + stream sync, host clock; kernel "
                               "instances tuned by fbst_autotune_ex for one block per launch"},
        "graph": {"latency_ms": {"p50": float(np.percentile(glat, 50)), "p99": float(np.percentile(glat, 99))},
                  "ms_per_step": graph_ms,
                  "what": "the single block and the 64-block step replayed from captured HIP graphs"},
        "autotune": {"blocks_per_launch": tuned_chunk, "k3_variant": tuned_var,
                     "ms_per_step": tuned_ms, "untuned": untuned,
                     "gain": (untuned["ms_per_step"] / tuned_ms) if untuned else None,
                     "what": "fbst_autotune_ex over blocks per launch x stage-2 kernel variant "
                             "(bit 0 single-buffer form, bit 1 persistent grid, 4 three waves per "
                             "SIMD), then the stage-1b workgroup size (16 half, 32 twice the "
                             "frequencies per workgroup); untuned = the plan's default variant at "
                             "16 blocks per launch"},
        "stage_gflop_per_block": [s0 / 1e9, s1 / 1e9, s2 / 1e9],
        "path_tflops": (s0 + s1 + s2) * nblk / (ms_step / 1e3) / 1e12,
        "roofline": {"kernel": "k_toeplitz_fu (stage 2: Gohberg-Semencul apply + F_u chirp-z)",
                     "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                     "traffic": stored_traffic(
                         f"k_toeplitz_fu<float, float, float, 4096, 4, 0, {plan.variant & 15}>",
                         chunk * cfg.B * 256),
                     "k3_variant": plan.variant & 15,
                     "avg_launch_ms": k3_ms,
                     "flops_per_launch": k3_flops_launch},
    }
    # the matrix-core split-precision stage 1a: same 64 blocks, same launches
    variants = {}
    if not args.no_variants:
        for prec in ("bf16_split", "fp16_split", "fp32_refine"):
            if prec == "fp32_refine":   # float32 with one refinement step of the stage-2 solve
                vp = F.plan_for_config(cfg, precision="fp32", flags=F.FBST_FLAG_STAGE2_REFINE)
            else:
                vp = F.plan_for_config(cfg, precision=prec)
            vb = torch.empty_like(beams)
            vws = vp.workspace(chunk)

            def vstep():
                vp.execute_batched(x, beams=vb, workspace=vws, max_chunk=chunk)

            for _ in range(args.warmup):
                vstep()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            nst = max(1, min(args.steps, 10))
            for _ in range(nst):
                vstep()
            e1.record(stream)
            torch.cuda.synchronize()
            vms = e0.elapsed_time(e1) / nst
            # stage 1a alone, the stage this variant changes
            s0a = torch.cuda.Event(enable_timing=True)
            s0b = torch.cuda.Event(enable_timing=True)
            s0a.record(stream)
            F.fbst_execute_stage(vp.handle, 0, chunk, x[0].data_ptr(), yhat.data_ptr(), 0, sptr)
            s0b.record(stream)
            torch.cuda.synchronize()
            variants[prec] = {"value": samples / (vms / 1e3), "ms_per_step": vms,
                              "stage1a_ms_per_launch": s0a.elapsed_time(s0b),
                              "beams0": vb[0].cpu().numpy()}
            print(f"[bench] {prec}: {vms:.3f} ms/step", file=sys.stderr, flush=True)
            vp.close()
    s1a = torch.cuda.Event(enable_timing=True)
    s1b = torch.cuda.Event(enable_timing=True)
    s1a.record(stream)
    F.fbst_execute_stage(plan.handle, 0, chunk, x[0].data_ptr(), yhat.data_ptr(), 0, sptr)
    s1b.record(stream)
    torch.cuda.synchronize()
    result["stage1a_ms_per_launch"] = s1a.elapsed_time(s1b)

    oracle_checks = []          # oracle comparisons, run with the CPU baseline leg only
    if not args.no_n64:
        result["precompute_n64"] = precompute_bench(
            F, torch, steps=max(2, min(args.steps, 10)), warmup=1,
            log=lambda m: print(m, file=sys.stderr, flush=True), checks=oracle_checks)
    if not args.no_interp:
        result["interp"] = interp_bench(F, torch, plan, cfg, beams,
                                        log=lambda m: print(m, file=sys.stderr, flush=True),
                                        checks=oracle_checks)
    if not args.no_nu:
        result["nonuniform"] = nonuniform_bench(
            F, torch, log=lambda m: print(m, file=sys.stderr, flush=True), checks=oracle_checks)
    if not args.no_serve:
        print("[bench] serving mix", file=sys.stderr, flush=True)
        log = lambda m: print(m, file=sys.stderr, flush=True)
        serve_checks = []
        result["serving"] = {
            "mix": serve_bench(F, torch, synth.serving_arrays(), seconds=args.serve_seconds, log=log,
                               checks=serve_checks),
            "mix_fp16_split": serve_bench(F, torch, synth.serving_arrays(),
                                          seconds=args.serve_seconds, precision="fp16_split",
                                          log=log, checks=serve_checks),
            "ula256_stream": serve_bench(F, torch, [cfg], seconds=args.serve_seconds, loads=(0.8,),
                                         log=log),
            "what": "continuous-batching server (4 streams, up to 16 blocks of one plan per launch); "
                    "inputs: block 0 of each array's synthetic scene; latency = completion - "
                    "submission; mean_batch = blocks per launch seen by the completed requests; "
                    "mix_fp16_split: the same mix with stage 1a as float16 split products on the "
                    "matrix cores",
        }
    large_first = {}
    if not args.no_large:
        print("[bench] planar array and 1024-element line", file=sys.stderr, flush=True)
        result["large"], large_first = large_bench(F, torch, log=lambda m: print(m, file=sys.stderr,
                                                                                flush=True))
    fp32_0 = beams[0].cpu().numpy()
    if not args.no_cpu:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        y0 = x[0].cpu().numpy().astype(np.complex128)
        result["cpu_baseline"], idx, ref = cpu_baseline(cfg, y0, cfg.delta_noise)
        acc = {"fp32": float(np.linalg.norm(fp32_0[idx] - ref) / np.linalg.norm(ref))}
        for k, v in variants.items():
            acc[k] = float(np.linalg.norm(v["beams0"][idx] - ref) / np.linalg.norm(ref))
        result["accuracy_vs_oracle"] = {"rel_l2": acc, "sample": f"block 0, the {len(idx)} oracle beams"}
        print(f"[bench] oracle accuracy checks of the other measurements ({len(oracle_checks)})",
              file=sys.stderr, flush=True)
        for check in oracle_checks:
            check()
        if "serving" in result:
            result["serving"]["accuracy_vs_oracle"] = {
                "arrays": serve_accuracy(serve_checks),
                "sample": "block 0 of the largest array and of the lowest and highest fractional "
                          "bandwidth in the mix, 6 beams, against the FP64 FBST oracle"}
        if not args.no_fbst64:
            print("[bench] timing the FP64 FBST oracle on every workload", file=sys.stderr, flush=True)
            result["cpu_baseline"]["fbst64"], ref64 = fbst64_baseline()
            for key, (name, got) in large_first.items():
                ref = ref64[name]
                result["large"][key]["rel_l2_vs_oracle"] = float(
                    np.linalg.norm(got - ref) / np.linalg.norm(ref))
                result["large"][key]["per_beam_max_vs_oracle"] = float(
                    (np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)).max())
    if variants:
        result["variants"] = {k: {kk: vv for kk, vv in v.items() if kk != "beams0"}
                              for k, v in variants.items()}
    print(json.dumps(result), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
