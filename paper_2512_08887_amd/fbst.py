"""Python binding of libfbst.so (include/fbst.h): argument marshalling only.

The functions keep the C names; they take device pointers as Python ints.
``Plan`` is a small convenience around them that takes torch tensors and the
current torch stream (PyTorch provides device memory and streams; every step
of the transformation runs in the library's HIP kernels).

The library must be built (``python -m paper_2512_08887_amd.build``); there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_size_t, c_uint, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfbst.so")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fbst.h")

FBST_OK, FBST_E_INVALID, FBST_E_UNSUPPORTED, FBST_E_NOMEM, FBST_E_DEVICE = 0, -1, -2, -3, -4
FBST_LINE, FBST_GRID, FBST_ARBITRARY = 0, 1, 2
FBST_PREC_FP32, FBST_PREC_FP64_STAGE2, FBST_PREC_FP64, FBST_PREC_BF16_SPLIT, FBST_PREC_FP16_SPLIT = range(5)
FBST_FLAG_HOST_ONLY, FBST_FLAG_KEEP_HOST_TABLES, FBST_FLAG_NO_SPLIT, FBST_FLAG_PRECOMPUTE = 1, 2, 4, 8
FBST_FLAG_NU_UNFUSED = 16
FBST_FLAG_DEVICE_GENERATORS = 32
FBST_FLAG_STAGE2_REFINE = 64
FBST_FLAG_SUPERFAST_GENERATORS = 128
FBST_VARIANT_K3_SINGLE, FBST_VARIANT_K3_PERSISTENT, FBST_VARIANT_K3_WAVES3 = 1, 2, 4
FBST_VARIANT_K2_TILE_HALF, FBST_VARIANT_K2_TILE_DOUBLE = 16, 32
FBST_TABLE_BEAM_U, FBST_TABLE_BEAM_V, FBST_TABLE_GRAM, FBST_TABLE_GENERATOR = 0, 1, 2, 3
MAX_LAUNCH_BLOCKS = 256  # FBST_MAX_LAUNCH_BLOCKS: blocks per kernel launch (pointers in the kernel arguments)

PRECISIONS = {"fp32": FBST_PREC_FP32, "fp64_stage2": FBST_PREC_FP64_STAGE2, "fp64": FBST_PREC_FP64,
              "bf16_split": FBST_PREC_BF16_SPLIT, "fp16_split": FBST_PREC_FP16_SPLIT}


class fbst_geometry(ctypes.Structure):
    _fields_ = [("kind", c_int), ("mx", c_int), ("my", c_int), ("dx", c_double), ("dy", c_double),
                ("x0", c_double), ("y0", c_double), ("px", POINTER(c_double)),
                ("py", POINTER(c_double))]


class fbst_band(ctypes.Structure):
    _fields_ = [("fc", c_double), ("omega", c_double), ("ts", c_double)]


class fbst_grid(ctypes.Structure):
    _fields_ = [("bu", c_int), ("bv", c_int), ("u0", c_double), ("du", c_double), ("v0", c_double),
                ("dv", c_double)]


class fbst_options(ctypes.Structure):
    _fields_ = [("eps", c_double), ("L", c_int), ("delta", c_double), ("precision", c_int),
                ("flags", c_uint)]


class fbst_info(ctypes.Structure):
    _fields_ = [("M", c_int), ("N", c_int), ("B", c_int), ("L", c_int), ("mx", c_int), ("my", c_int),
                ("bu", c_int), ("bv", c_int), ("p1", c_int), ("p2x", c_int), ("p2y", c_int),
                ("p3", c_int), ("precision", c_int), ("io_elem_bytes", c_size_t),
                ("device_bytes", c_size_t), ("workspace_per_block", c_size_t), ("p1_split", c_int),
                ("stage2_precomputed", c_int), ("nu_width", c_int),
                ("nu_lanes", c_int), ("cond_bound", c_double), ("generator_ms", c_double),
                ("workspace_fixed", c_size_t)]


class fbst_server_options(ctypes.Structure):
    _fields_ = [("workspace_bytes", c_size_t), ("streams", c_int), ("max_batch", c_int),
                ("device", c_int)]


class fbst_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_ulonglong), ("status", c_int), ("batch", c_int),
                ("submit_us", c_double), ("start_us", c_double), ("done_us", c_double)]


class FbstError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fbst status {status}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Open a libfbst.so and declare the C signatures of include/fbst.h."""
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2512_08887_amd.build`")
    L = ctypes.CDLL(path)
    L.fbst_plan_create.argtypes = [c_int, c_int, c_int, POINTER(fbst_geometry), POINTER(fbst_band),
                                   POINTER(fbst_grid), POINTER(fbst_options), POINTER(c_void_p)]
    L.fbst_plan_create.restype = c_int
    L.fbst_execute.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.fbst_execute.restype = c_int
    L.fbst_execute_batched.argtypes = [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p]
    L.fbst_execute_batched.restype = c_int
    L.fbst_execute_static.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_void_p]
    L.fbst_execute_static.restype = c_int
    L.fbst_static_scratch_bytes.argtypes = []
    L.fbst_static_scratch_bytes.restype = c_size_t
    L.fbst_execute_stage.argtypes = [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p]
    L.fbst_execute_stage.restype = c_int
    L.fbst_workspace_bytes.argtypes = [c_void_p, c_int]
    L.fbst_workspace_bytes.restype = c_size_t
    L.fbst_plan_device_bytes.argtypes = [c_void_p]
    L.fbst_plan_device_bytes.restype = c_size_t
    L.fbst_plan_info.argtypes = [c_void_p, POINTER(fbst_info)]
    L.fbst_plan_info.restype = c_int
    L.fbst_plan_table.argtypes = [c_void_p, c_int, c_void_p, c_size_t]
    L.fbst_plan_table.restype = c_int
    L.fbst_destroy.argtypes = [c_void_p]
    L.fbst_destroy.restype = None
    L.fbst_last_error.argtypes = []
    L.fbst_last_error.restype = c_char_p
    L.fbst_version.argtypes = []
    L.fbst_version.restype = c_char_p
    L.fbst_graph_create.argtypes = [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, POINTER(c_void_p)]
    L.fbst_graph_create.restype = c_int
    L.fbst_graph_launch.argtypes = [c_void_p, c_void_p]
    L.fbst_graph_launch.restype = c_int
    L.fbst_graph_destroy.argtypes = [c_void_p]
    L.fbst_graph_destroy.restype = None
    L.fbst_autotune.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                POINTER(c_int), POINTER(ctypes.c_float)]
    L.fbst_autotune.restype = c_int
    L.fbst_autotune_ex.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                   POINTER(c_int), POINTER(c_int), POINTER(ctypes.c_float)]
    L.fbst_autotune_ex.restype = c_int
    L.fbst_plan_set_variant.argtypes = [c_void_p, c_int]
    L.fbst_plan_set_variant.restype = c_int
    L.fbst_plan_variant.argtypes = [c_void_p]
    L.fbst_plan_variant.restype = c_int
    L.fbst_plan_steer.argtypes = [c_void_p, POINTER(fbst_grid), c_void_p]
    L.fbst_plan_steer.restype = c_int
    L.fbst_execute_stream.argtypes = [c_void_p, ctypes.c_longlong, c_int, c_void_p, c_void_p, c_void_p,
                                      c_int, c_void_p]
    L.fbst_execute_stream.restype = c_int
    L.fbst_nulls_create.argtypes = [c_void_p, c_int, POINTER(c_int), POINTER(c_void_p)]
    L.fbst_nulls_create.restype = c_int
    L.fbst_nulls_create_directions.argtypes = [c_void_p, c_int, POINTER(ctypes.c_double),
                                               POINTER(ctypes.c_double), POINTER(c_void_p)]
    L.fbst_nulls_create_directions.restype = c_int
    L.fbst_directions_create.argtypes = [c_void_p, c_int, POINTER(ctypes.c_double),
                                         POINTER(ctypes.c_double), POINTER(c_void_p)]
    L.fbst_directions_create.restype = c_int
    L.fbst_directions_create_interp.argtypes = [c_void_p, c_int, POINTER(ctypes.c_double),
                                                POINTER(ctypes.c_double), POINTER(c_void_p)]
    L.fbst_directions_create_interp.restype = c_int
    L.fbst_nulls_create_interp.argtypes = [c_void_p, c_int, POINTER(ctypes.c_double),
                                           POINTER(ctypes.c_double), POINTER(c_void_p)]
    L.fbst_nulls_create_interp.restype = c_int
    L.fbst_directions_destroy.argtypes = [c_void_p]
    L.fbst_directions_destroy.restype = None
    L.fbst_workspace_bytes_directions.argtypes = [c_void_p, c_void_p, c_int]
    L.fbst_workspace_bytes_directions.restype = c_size_t
    L.fbst_execute_directions.argtypes = [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p,
                                          c_void_p, c_void_p]
    L.fbst_execute_directions.restype = c_int
    L.fbst_interp_create.argtypes = [c_void_p, c_int, POINTER(ctypes.c_double),
                                     POINTER(ctypes.c_double), POINTER(c_void_p)]
    L.fbst_interp_create.restype = c_int
    L.fbst_interp_destroy.argtypes = [c_void_p]
    L.fbst_interp_destroy.restype = None
    L.fbst_interp_table.argtypes = [c_void_p, POINTER(c_int), POINTER(ctypes.c_double)]
    L.fbst_interp_table.restype = c_int
    L.fbst_execute_interp.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_void_p]
    L.fbst_execute_interp.restype = c_int
    L.fbst_nulls_destroy.argtypes = [c_void_p]
    L.fbst_nulls_destroy.restype = None
    L.fbst_workspace_bytes_nulled.argtypes = [c_void_p, c_void_p, c_int]
    L.fbst_workspace_bytes_nulled.restype = c_size_t
    L.fbst_execute_nulled.argtypes = [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                      c_void_p]
    L.fbst_execute_nulled.restype = c_int
    L.fbst_server_create.argtypes = [POINTER(fbst_server_options), POINTER(c_void_p)]
    L.fbst_server_create.restype = c_int
    L.fbst_server_submit.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_ulonglong]
    L.fbst_server_submit.restype = c_int
    L.fbst_server_poll.argtypes = [c_void_p, POINTER(fbst_completion), c_int]
    L.fbst_server_poll.restype = c_int
    L.fbst_server_drain.argtypes = [c_void_p, c_double]
    L.fbst_server_drain.restype = c_int
    L.fbst_server_clock_us.argtypes = [c_void_p]
    L.fbst_server_clock_us.restype = c_double
    L.fbst_server_destroy.argtypes = [c_void_p]
    L.fbst_server_destroy.restype = None
    return L


def lib():
    """The in-tree libfbst.so, loaded once (raises if it has not been built)."""
    global _lib
    if _lib is None:
        _lib = load_library(LIB_PATH)
    return _lib


def header_functions() -> list[str]:
    """Names of the functions include/fbst.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fbst_[a-z_]+)\s*\(", txt)))


def _check(st: int):
    if st != FBST_OK:
        raise FbstError(st, lib().fbst_last_error().decode())


def fbst_last_error() -> str:
    return lib().fbst_last_error().decode()


def fbst_version() -> str:
    return lib().fbst_version().decode()


def fbst_plan_create(M, N, B, geometry=None, band=None, grid=None, options=None) -> int:
    h = c_void_p()
    g = byref(geometry) if geometry is not None else None
    b = byref(band) if band is not None else None
    gr = byref(grid) if grid is not None else None
    o = byref(options) if options is not None else None
    _check(lib().fbst_plan_create(M, N, B, g, b, gr, o, byref(h)))
    return h.value


def fbst_plan_create_status(M, N, B, geometry=None, band=None, grid=None, options=None):
    """Like fbst_plan_create but returns (status, handle or None) without raising."""
    h = c_void_p()
    g = byref(geometry) if geometry is not None else None
    b = byref(band) if band is not None else None
    gr = byref(grid) if grid is not None else None
    o = byref(options) if options is not None else None
    st = lib().fbst_plan_create(M, N, B, g, b, gr, o, byref(h))
    return st, h.value


def fbst_execute(plan, x, beams, workspace=0, stream=0):
    _check(lib().fbst_execute(plan, x, beams, workspace or None, stream or None))


def fbst_execute_batched(plan, nblocks, max_chunk, x, beams, workspace=0, stream=0):
    _check(lib().fbst_execute_batched(plan, nblocks, max_chunk, x, beams, workspace or None,
                                      stream or None))


def fbst_execute_static(plan, nblocks, x, beams, stream=0):
    _check(lib().fbst_execute_static(plan, nblocks, x, beams, stream or None))


def fbst_static_scratch_bytes() -> int:
    return int(lib().fbst_static_scratch_bytes())


def fbst_execute_stage(plan, stage, nblocks, inp, out, workspace=0, stream=0):
    _check(lib().fbst_execute_stage(plan, stage, nblocks, inp, out, workspace or None, stream or None))


def fbst_workspace_bytes(plan, nblocks) -> int:
    return int(lib().fbst_workspace_bytes(plan, nblocks))


def fbst_plan_device_bytes(plan) -> int:
    return int(lib().fbst_plan_device_bytes(plan))


def fbst_plan_info(plan) -> fbst_info:
    info = fbst_info()
    _check(lib().fbst_plan_info(plan, byref(info)))
    return info


def fbst_plan_table(plan, table, out_array):
    """Copy a kept FP64 host table into a numpy array (float64 or complex128)."""
    _check(lib().fbst_plan_table(plan, table, out_array.ctypes.data, out_array.nbytes))
    return out_array


def fbst_destroy(plan):
    lib().fbst_destroy(plan)


def fbst_graph_create(plan, nblocks, max_chunk, x, beams, workspace=0) -> int:
    h = c_void_p()
    _check(lib().fbst_graph_create(plan, nblocks, max_chunk, x, beams, workspace or None, byref(h)))
    return h.value


def fbst_graph_launch(graph, stream=0):
    _check(lib().fbst_graph_launch(graph, stream or None))


def fbst_graph_destroy(graph):
    lib().fbst_graph_destroy(graph)


def fbst_autotune(plan, nblocks, x, beams, workspace, stream=0, force=False):
    """Returns (best_chunk, ms_per_batch)."""
    c = c_int()
    ms = ctypes.c_float()
    _check(lib().fbst_autotune(plan, nblocks, x, beams, workspace, stream or None, int(force),
                               byref(c), byref(ms)))
    return c.value, ms.value


def fbst_autotune_ex(plan, nblocks, x, beams, workspace, stream=0, force=False):
    chunk, var, ms = c_int(0), c_int(0), ctypes.c_float(0.0)
    _check(lib().fbst_autotune_ex(plan, nblocks, x, beams, workspace, stream or None, int(force),
                                  byref(chunk), byref(var), byref(ms)))
    return chunk.value, var.value, ms.value


def fbst_plan_set_variant(plan, variant):
    _check(lib().fbst_plan_set_variant(plan, int(variant)))


def fbst_plan_variant(plan) -> int:
    return int(lib().fbst_plan_variant(plan))


def fbst_plan_steer(plan, grid, stream=0):
    _check(lib().fbst_plan_steer(plan, byref(grid), stream or None))


def fbst_execute_stream(plan, T, hop, x, beams, workspace=0, max_chunk=0, stream=0):
    _check(lib().fbst_execute_stream(plan, T, hop, x, beams, workspace or None, max_chunk,
                                     stream or None))


def fbst_nulls_create(plan, beams) -> int:
    arr = (c_int * len(beams))(*[int(b) for b in beams])
    h = c_void_p()
    _check(lib().fbst_nulls_create(plan, len(beams), arr, byref(h)))
    return h.value


def fbst_nulls_create_directions(plan, u, v=None) -> int:
    n = len(u)
    ua = (ctypes.c_double * n)(*[float(a) for a in u])
    va = (ctypes.c_double * n)(*[float(a) for a in v]) if v is not None else None
    h = c_void_p()
    _check(lib().fbst_nulls_create_directions(plan, n, ua, va, byref(h)))
    return h.value


def fbst_nulls_create_interp(plan, u, v=None) -> int:
    n = len(u)
    ua = (ctypes.c_double * n)(*[float(a) for a in u])
    va = (ctypes.c_double * n)(*[float(a) for a in v]) if v is not None else None
    h = c_void_p()
    _check(lib().fbst_nulls_create_interp(plan, n, ua, va, byref(h)))
    return h.value


def fbst_directions_create(plan, u, v=None) -> int:
    n = len(u)
    ua = (ctypes.c_double * n)(*[float(a) for a in u])
    va = (ctypes.c_double * n)(*[float(a) for a in v]) if v is not None else None
    h = c_void_p()
    _check(lib().fbst_directions_create(plan, n, ua, va, byref(h)))
    return h.value


def fbst_directions_create_interp(plan, u, v=None) -> int:
    n = len(u)
    ua = (ctypes.c_double * n)(*[float(a) for a in u])
    va = (ctypes.c_double * n)(*[float(a) for a in v]) if v is not None else None
    h = c_void_p()
    _check(lib().fbst_directions_create_interp(plan, n, ua, va, byref(h)))
    return h.value


def fbst_directions_destroy(dirs):
    lib().fbst_directions_destroy(dirs)


def fbst_workspace_bytes_directions(plan, dirs, nblocks) -> int:
    return lib().fbst_workspace_bytes_directions(plan, dirs, nblocks)


def fbst_execute_directions(plan, dirs, nblocks, max_chunk, x, beams, workspace, stream=0):
    _check(lib().fbst_execute_directions(plan, dirs, nblocks, max_chunk, x, beams, workspace,
                                         stream or None))


def fbst_interp_create(plan, u, v=None) -> int:
    n = len(u)
    ua = (ctypes.c_double * n)(*[float(a) for a in u])
    va = (ctypes.c_double * n)(*[float(a) for a in v]) if v is not None else None
    h = c_void_p()
    _check(lib().fbst_interp_create(plan, n, ua, va, byref(h)))
    return h.value


def fbst_interp_destroy(interp):
    lib().fbst_interp_destroy(interp)


def fbst_interp_table(interp, D):
    """(first [D][2] ints (u, v windows), weights [D][2][8] float64) as lists."""
    fa = (c_int * (2 * D))()
    wa = (ctypes.c_double * (16 * D))()
    _check(lib().fbst_interp_table(interp, fa, wa))
    return ([(fa[2 * d], fa[2 * d + 1]) for d in range(D)],
            [(list(wa[16 * d:16 * d + 8]), list(wa[16 * d + 8:16 * d + 16])) for d in range(D)])


def fbst_execute_interp(interp, nblocks, beams, out, stream=0):
    _check(lib().fbst_execute_interp(interp, nblocks, beams, out, stream or None))


def fbst_nulls_destroy(nulls):
    lib().fbst_nulls_destroy(nulls)


def fbst_workspace_bytes_nulled(plan, nulls, nblocks) -> int:
    return lib().fbst_workspace_bytes_nulled(plan, nulls, nblocks)


def fbst_execute_nulled(plan, nulls, nblocks, max_chunk, x, beams, workspace, stream=0):
    _check(lib().fbst_execute_nulled(plan, nulls, nblocks, max_chunk, x, beams, workspace,
                                     stream or None))


def fbst_server_create(options=None) -> int:
    h = c_void_p()
    _check(lib().fbst_server_create(byref(options) if options is not None else None, byref(h)))
    return h.value


def fbst_server_submit(server, plan, x, beams, tag):
    _check(lib().fbst_server_submit(server, plan, x, beams, tag))


def fbst_server_poll(server, max_n=256):
    buf = (fbst_completion * max_n)()
    n = lib().fbst_server_poll(server, buf, max_n)
    if n < 0:
        raise FbstError(n, "fbst_server_poll: invalid arguments")
    return [buf[i] for i in range(n)]


def fbst_server_drain(server, timeout_s=0.0):
    _check(lib().fbst_server_drain(server, timeout_s))


def fbst_server_clock_us(server) -> float:
    return float(lib().fbst_server_clock_us(server))


def fbst_server_destroy(server):
    lib().fbst_server_destroy(server)


# ---------------------------------------------------------------------------
# Convenience layer over torch tensors.
# ---------------------------------------------------------------------------

def make_band(fc, omega, ts=1.0):
    return fbst_band(fc, omega, ts)


def make_line(M, dx=0.0, x0=0.0):
    return fbst_geometry(FBST_LINE, M, 1, dx, 0.0, x0, 0.0)


def make_grid_geometry(mx, my, dx=0.0, dy=0.0, x0=0.0, y0=0.0):
    return fbst_geometry(FBST_GRID, mx, my, dx, dy, x0, y0)


def make_arbitrary(px, py=None):
    """Non-uniform array: element coordinates px, py in seconds per unit
    direction cosine (py None: a line along x).  The returned struct keeps
    the float64 copies it points to alive."""
    import numpy as np
    x = np.ascontiguousarray(px, dtype=np.float64)
    y = None if py is None else np.ascontiguousarray(py, dtype=np.float64)
    if y is not None and y.shape != x.shape:
        raise ValueError("px and py must have the same length")
    g = fbst_geometry(FBST_ARBITRARY, len(x), 1, 0.0, 0.0, 0.0, 0.0,
                      x.ctypes.data_as(POINTER(c_double)),
                      y.ctypes.data_as(POINTER(c_double)) if y is not None else None)
    g._keep = (x, y)
    return g


def make_beam_grid(bu, bv=1, u0=0.0, du=0.0, v0=0.0, dv=0.0):
    return fbst_grid(bu, bv, u0, du, v0, dv)


def make_options(delta, eps=1.01, L=0, precision="fp32", flags=0):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return fbst_options(eps, L, delta, prec, flags)


class Plan:
    """Owns one fbst plan; executes on torch tensors on the current stream."""

    def __init__(self, M, N, B, *, band, geometry=None, grid=None, options=None):
        self.handle = fbst_plan_create(M, N, B, geometry, band, grid, options)
        self.info = fbst_plan_info(self.handle)
        self.M, self.N, self.B, self.L = M, N, B, self.info.L

    @property
    def complex_dtype(self):
        import torch
        return torch.complex128 if self.info.io_elem_bytes == 16 else torch.complex64

    @property
    def stage1_dtype(self):
        import torch
        return torch.complex128 if self.info.precision == FBST_PREC_FP64 else torch.complex64

    def workspace(self, nblocks=1):
        import torch
        nbytes = fbst_workspace_bytes(self.handle, nblocks)
        return torch.empty(nbytes, dtype=torch.uint8, device="cuda")

    @staticmethod
    def _stream():
        import torch
        return torch.cuda.current_stream().cuda_stream

    def _check_in(self, x, shape):
        if not x.is_cuda or not x.is_contiguous() or x.dtype != self.complex_dtype or tuple(x.shape[-2:]) != shape:
            raise ValueError(f"expected a contiguous {self.complex_dtype} CUDA tensor of shape [..., {shape[0]}, {shape[1]}]")

    def execute(self, x, beams=None, workspace=None):
        import torch
        self._check_in(x, (self.M, self.N))
        if beams is None:
            beams = torch.empty((self.B, self.N), dtype=self.complex_dtype, device=x.device)
        fbst_execute(self.handle, x.data_ptr(), beams.data_ptr(),
                     workspace.data_ptr() if workspace is not None else 0, self._stream())
        return beams

    def execute_batched(self, x, beams=None, workspace=None, max_chunk=0):
        import torch
        self._check_in(x, (self.M, self.N))
        nb = x.shape[0]
        chunk = nb if max_chunk <= 0 else min(max_chunk, nb)
        if beams is None:
            beams = torch.empty((nb, self.B, self.N), dtype=self.complex_dtype, device=x.device)
        if workspace is None and chunk > 1:
            workspace = self.workspace(chunk)
        fbst_execute_batched(self.handle, nb, chunk, x.data_ptr(), beams.data_ptr(),
                             workspace.data_ptr() if workspace is not None else 0, self._stream())
        return beams

    def execute_static(self, x, beams):
        """x [nb][M][N] -> beams [nb][B][N] (both preallocated) through
        fbst_execute_static: no workspace, no allocation in the library."""
        self._check_in(x, (self.M, self.N))
        self._check_in(beams, (self.B, self.N))
        nb = x.shape[0] if x.dim() == 3 else 1
        fbst_execute_static(self.handle, nb, x.data_ptr(), beams.data_ptr(), self._stream())
        return beams

    def stage(self, stage, inp, nblocks=1, out=None, workspace=None):
        import torch
        shapes = {0: (self.M, self.L), 1: (self.B, self.L), 2: (self.B, self.N)}
        odt = self.complex_dtype if stage == 2 else self.stage1_dtype
        if out is None:
            out = torch.empty((nblocks,) + shapes[stage], dtype=odt, device=inp.device)
        if workspace is None and stage == 1 and (self.info.bv > 1 or self.info.my > 1
                                                 or self.info.nu_width > 0):
            workspace = self.workspace(nblocks)
        fbst_execute_stage(self.handle, stage, nblocks, inp.data_ptr(), out.data_ptr(),
                           workspace.data_ptr() if workspace is not None else 0, self._stream())
        return out

    def execute_stream(self, x, hop, beams=None, workspace=None, max_chunk=0):
        """x [M, T] (a recording) -> beams [(T - N) // hop + 1, B, N] of windows every hop samples."""
        import torch
        if not x.is_cuda or not x.is_contiguous() or x.dtype != self.complex_dtype or x.dim() != 2 \
                or x.shape[0] != self.M:
            raise ValueError(f"expected a contiguous {self.complex_dtype} CUDA tensor [{self.M}, T]")
        T = x.shape[1]
        nb = (T - self.N) // hop + 1
        chunk = min(nb if max_chunk <= 0 else min(max_chunk, nb), MAX_LAUNCH_BLOCKS)
        if beams is None:
            beams = torch.empty((nb, self.B, self.N), dtype=self.complex_dtype, device=x.device)
        if workspace is None and chunk > 1:
            workspace = self.workspace(chunk)
        fbst_execute_stream(self.handle, T, hop, x.data_ptr(), beams.data_ptr(),
                            workspace.data_ptr() if workspace is not None else 0, chunk, self._stream())
        return beams

    def autotune(self, x, beams=None, workspace=None, force=False):
        """Fastest blocks per launch for x [nblocks, M, N]; returns (chunk, ms per batch)."""
        import torch
        self._check_in(x, (self.M, self.N))
        nb = x.shape[0]
        if beams is None:
            beams = torch.empty((nb, self.B, self.N), dtype=self.complex_dtype, device=x.device)
        if workspace is None:
            workspace = self.workspace(min(nb, MAX_LAUNCH_BLOCKS))
        return fbst_autotune(self.handle, nb, x.data_ptr(), beams.data_ptr(), workspace.data_ptr(),
                             self._stream(), force)

    def autotune_ex(self, x, beams=None, workspace=None, force=False):
        """Fastest (blocks per launch, stage-2 variant) for x [nblocks, M, N];
        leaves that variant set on the plan; returns (chunk, variant, ms)."""
        import torch
        self._check_in(x, (self.M, self.N))
        nb = x.shape[0]
        if beams is None:
            beams = torch.empty((nb, self.B, self.N), dtype=self.complex_dtype, device=x.device)
        if workspace is None:
            workspace = self.workspace(min(nb, MAX_LAUNCH_BLOCKS))
        return fbst_autotune_ex(self.handle, nb, x.data_ptr(), beams.data_ptr(),
                                workspace.data_ptr(), self._stream(), force)

    def steer(self, grid):
        """Point the plan at a new beam grid (fbst_plan_steer; same bu, bv)."""
        fbst_plan_steer(self.handle, grid, self._stream())
        self.info = fbst_plan_info(self.handle)

    @property
    def variant(self):
        return fbst_plan_variant(self.handle)

    @variant.setter
    def variant(self, v):
        fbst_plan_set_variant(self.handle, v)

    def graph(self, x, beams, workspace=None, max_chunk=0):
        """Capture execute_batched(x -> beams) as a replayable graph bound to these tensors."""
        self._check_in(x, (self.M, self.N))
        nb = x.shape[0]
        chunk = nb if max_chunk <= 0 else min(max_chunk, nb)
        if workspace is None and chunk > 1:
            workspace = self.workspace(chunk)
        return Graph(self, x, beams, workspace, nb, chunk)

    def close(self):
        if getattr(self, "handle", None):
            fbst_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Nulls:
    """Beamspace nulling of interferers at beams of a plan (fbst_nulls_*)."""

    def __init__(self, plan, beams=None, *, u=None, v=None, interp=False):
        """Interferers at beams of the plan's grid, or at directions u (and v),
        their beam vectors projected exactly or (interp=True) interpolated
        from the grid's (fbst_nulls_create_interp)."""
        self.plan = plan
        if beams is not None:
            self.beams = [int(b) for b in beams]
            self.handle = fbst_nulls_create(plan.handle, self.beams)
        else:
            self.beams = None
            make = fbst_nulls_create_interp if interp else fbst_nulls_create_directions
            self.handle = make(plan.handle, list(u), None if v is None else list(v))

    def workspace(self, nblocks=1):
        import torch
        n = fbst_workspace_bytes_nulled(self.plan.handle, self.handle, nblocks)
        return torch.empty(n, dtype=torch.uint8, device="cuda")

    def execute(self, x, beams=None, workspace=None, max_chunk=0):
        """x [nblocks, M, N] (or [M, N]) complex64 -> nulled beams of the same leading shape."""
        import torch
        p = self.plan
        single = x.dim() == 2
        xb = x.unsqueeze(0) if single else x
        p._check_in(xb, (p.M, p.N))
        nb = xb.shape[0]
        chunk = nb if max_chunk <= 0 else min(max_chunk, nb)
        chunk = min(chunk, MAX_LAUNCH_BLOCKS)
        if beams is None:
            beams = torch.empty((nb, p.B, p.N), dtype=torch.complex64, device=x.device)
        if workspace is None:
            workspace = self.workspace(chunk)
        fbst_execute_nulled(p.handle, self.handle, nb, chunk, xb.data_ptr(), beams.data_ptr(),
                            workspace.data_ptr(), torch.cuda.current_stream().cuda_stream)
        return beams[0] if single else beams

    def close(self):
        if getattr(self, "handle", None):
            fbst_nulls_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Interp:
    """Off-grid beams interpolated from grid beams with a spline (fbst_interp_*)."""

    def __init__(self, plan, u, v=None):
        self.plan = plan
        self.D = len(u)
        self.handle = fbst_interp_create(plan.handle, list(u), None if v is None else list(v))

    def table(self):
        return fbst_interp_table(self.handle, self.D)

    def execute(self, beams, out=None):
        """beams [nblocks, B, N] (or [B, N]) -> out [nblocks, D, N] (or [D, N])."""
        import torch
        p = self.plan
        single = beams.dim() == 2
        bb = beams.unsqueeze(0) if single else beams
        p._check_in(bb, (p.B, p.N))
        nb = bb.shape[0]
        if out is None:
            out = torch.empty((nb, self.D, p.N), dtype=bb.dtype, device=bb.device)
        elif (not out.is_cuda or not out.is_contiguous() or out.dtype != bb.dtype
              or out.numel() != nb * self.D * p.N):
            raise ValueError("out must be a contiguous CUDA tensor of [nblocks, D, N] elements")
        fbst_execute_interp(self.handle, nb, bb.data_ptr(), out.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
        return out.reshape(self.D, p.N) if single else out

    def close(self):
        if getattr(self, "handle", None):
            fbst_interp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Directions:
    """Beams at arbitrary directions (u, v) of a plan (fbst_directions_*)."""

    def __init__(self, plan, u, v=None, interp=False):
        """interp=True: the paper's form, beam vectors interpolated from the
        grid's (fbst_directions_create_interp); else projected exactly."""
        self.plan = plan
        self.D = len(u)
        make = fbst_directions_create_interp if interp else fbst_directions_create
        self.handle = make(plan.handle, list(u), None if v is None else list(v))

    def workspace(self, nblocks=1):
        import torch
        n = fbst_workspace_bytes_directions(self.plan.handle, self.handle, nblocks)
        return torch.empty(n, dtype=torch.uint8, device="cuda")

    def execute(self, x, beams=None, workspace=None, max_chunk=0):
        """x [nblocks, M, N] (or [M, N]) complex64 -> beams [nblocks, D, N] (or [D, N])."""
        import torch
        p = self.plan
        single = x.dim() == 2
        xb = x.unsqueeze(0) if single else x
        p._check_in(xb, (p.M, p.N))
        nb = xb.shape[0]
        chunk = min(nb if max_chunk <= 0 else min(max_chunk, nb), MAX_LAUNCH_BLOCKS)
        if beams is None:
            beams = torch.empty((nb, self.D, p.N), dtype=torch.complex64, device=x.device)
        if workspace is None:
            workspace = self.workspace(chunk)
        fbst_execute_directions(p.handle, self.handle, nb, chunk, xb.data_ptr(), beams.data_ptr(),
                                workspace.data_ptr(), torch.cuda.current_stream().cuda_stream)
        return beams[0] if single else beams

    def close(self):
        if getattr(self, "handle", None):
            fbst_directions_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """An instantiated HIP graph of one batched execution; keeps its tensors alive."""

    def __init__(self, plan, x, beams, workspace, nblocks, chunk):
        self._keep = (plan, x, beams, workspace)
        self.handle = fbst_graph_create(plan.handle, nblocks, chunk, x.data_ptr(), beams.data_ptr(),
                                        workspace.data_ptr() if workspace is not None else 0)

    def launch(self):
        import torch
        fbst_graph_launch(self.handle, torch.cuda.current_stream().cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            fbst_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A continuous-batching block server (fbst_server_*): submit blocks of any
    resident plan with torch tensors; poll completions with their times."""

    def __init__(self, workspace_bytes=1 << 30, streams=4, max_batch=16, device=-1):
        self.handle = fbst_server_create(fbst_server_options(workspace_bytes, streams, max_batch, device))

    def submit(self, plan, x, beams, tag, sync=True):
        """Queue x -> beams.  The server's streams do not wait on torch's: with
        sync (default) the current stream is synchronised first, so x holds
        what was last written to it; pass sync=False when x is known ready."""
        if sync:
            import torch
            torch.cuda.current_stream().synchronize()
        fbst_server_submit(self.handle, plan.handle, x.data_ptr(), beams.data_ptr(), tag)

    def poll(self, max_n=256):
        return fbst_server_poll(self.handle, max_n)

    def drain(self, timeout_s=0.0):
        fbst_server_drain(self.handle, timeout_s)

    def clock_us(self):
        return fbst_server_clock_us(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            fbst_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_for_config(cfg, *, delta=None, precision="fp32", eps=None, flags=0):
    """Plan for a named synthetic workload (synth.Config)."""
    band = make_band(cfg.band.fc, cfg.band.omega, cfg.band.ts)
    d = cfg.delta_noise if delta is None else delta
    opts = make_options(d, eps=cfg.eps if eps is None else eps, L=cfg.L, precision=precision, flags=flags)
    if cfg.perturb > 0.0:
        px, py = cfg.array.positions()
        geom = make_arbitrary(px, py if cfg.kind == "ura" else None)
        grid = make_beam_grid(cfg.bu, cfg.bv) if cfg.kind == "ura" else None
        return Plan(cfg.M, cfg.N, cfg.B, band=band, geometry=geom, grid=grid, options=opts)
    if cfg.kind == "ura":
        geom = make_grid_geometry(cfg.mx, cfg.my)
        grid = make_beam_grid(cfg.bu, cfg.bv)
        return Plan(cfg.M, cfg.N, cfg.B, band=band, geometry=geom, grid=grid, options=opts)
    return Plan(cfg.M, cfg.N, cfg.B, band=band, geometry=make_line(cfg.M), options=opts)
