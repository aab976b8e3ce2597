"""The merged radix-16 butterflies of the FFT core (csrc/fft_lds.h), compiled
for the host: a twiddled Stockham pass from the merged (cosine-scaled)
factors against the direct 16-point sum of x_r w^{r k} in float64, forward
and inverse, for spans NS = 16 .. 4096 (fft_core_check.cpp).  Runs without a
GPU; needs hipcc."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2512_08887_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_radix16_butterflies_match_the_direct_sum(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    exe = tmp_path / "fft_core_check"
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", CSRC,
                        os.path.join(HERE, "fft_core_check.cpp"), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
