"""Build libfbst.so (HIP for gfx950) in-tree.

    python -m paper_2512_08887_amd.build [-v]

Sources are compiled to objects in parallel under _build/ and linked into
paper_2512_08887_amd/libfbst.so.  Packed-FP32 instructions are disabled for
the device code (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfbst.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["kernels.hip", "stage2.hip", "mfma_czt.hip", "precompute.hip", "levinson.hip", "superfast.hip", "gs_spectra.hip", "plan.cpp", "api.cpp",
           "server.cpp", "noalloc.cpp"]

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}")
    # hipcc's host pass warns that it does not know the packed-fp32 feature: harmless
    noise = "not a recognized feature for this target"
    for line in (r.stdout + r.stderr).splitlines():
        if verbose and line.strip() and noise not in line:
            print(line)
    return r


def _stale(obj, src, defines_file, defines):
    """True when obj is missing, older than its source or any header, or was
    built with other definitions."""
    if not os.path.exists(obj) or not os.path.exists(defines_file):
        return True
    with open(defines_file) as f:
        if f.read() != repr(sorted(defines)):
            return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps.append(os.path.join(ROOT, "include", "fbst.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, defines=(), out: str = LIB, build_dir: str = BUILD,
          incremental: bool = False) -> str:
    """Compile every source for gfx950 and link libfbst.so; returns its path.

    defines: extra preprocessor definitions ("NAME=VALUE") for tuning builds;
    out / build_dir: where the library and objects go; incremental: recompile
    only objects older than their source or a header (a development aid; the
    default recompiles everything)."""
    os.makedirs(build_dir, exist_ok=True)
    objs = []
    cmds = []
    defines_file = os.path.join(build_dir, "defines.txt")
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        path = os.path.join(CSRC, src)
        if incremental and not _stale(obj, path, defines_file, defines):
            continue
        lang = ["-x", "hip"]
        dflags = [f"-D{d}" for d in defines]
        cmds.append([HIPCC, *lang, *CFLAGS, *dflags, "-c", path, "-o", obj])
    if cmds:
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            list(ex.map(lambda c: _run(c, verbose), cmds))
    with open(defines_file, "w") as f:
        f.write(repr(sorted(defines)))
    tmp = out + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp,
          "-Wl,-soname,libfbst.so"], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
