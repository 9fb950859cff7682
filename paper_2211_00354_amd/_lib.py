"""ctypes binding of liblensfmm (include/lens.h): argument marshalling only.

Every computation runs in the HIP library; this module converts torch CUDA
tensors into device pointers and the current HIP stream, mirrors the C
structs, and turns non-OK statuses into exceptions.  It never falls back to
any CPU computation: if the library is missing it raises.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblensfmm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lens.h")

LENS_OK, LENS_EINVAL, LENS_ENOMEM, LENS_EDEVICE, LENS_EUNSUPPORTED = range(5)
LENS_FMM, LENS_DIRECT = 0, 1
LENS_FP64, LENS_MIXED = 0, 1


class LensError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[lens status {status}] {msg}")
        self.status = status


class LensField(ctypes.Structure):
    _fields_ = [("n_stars", ctypes.c_int64), ("xy", ctypes.c_void_p), ("m", ctypes.c_void_p),
                ("kappa_s", ctypes.c_double), ("gamma", ctypes.c_double)]


class LensGrid(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64)]


class LensMapDesc(ctypes.Structure):
    _fields_ = [("y1min", ctypes.c_double), ("y2min", ctypes.c_double), ("side", ctypes.c_double),
                ("npix", ctypes.c_int32), ("counts", ctypes.c_void_p)]


class LensIpmDesc(ctypes.Structure):
    _fields_ = [("y1min", ctypes.c_double), ("y2min", ctypes.c_double), ("side", ctypes.c_double),
                ("npix", ctypes.c_int32), ("mu", ctypes.c_void_p)]


class LensOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("order_p", ctypes.c_int32), ("leaf_level", ctypes.c_int32),
                ("max_rays_per_chunk", ctypes.c_int64), ("fp32_levels", ctypes.c_int32),
                ("tol", ctypes.c_double), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


_lib = None


def declared_functions() -> list[str]:
    """Names of the functions include/lens.h declares (no GPU needed)."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"LENS_API\s+[\w\s\*]+?\b(lens_\w+)\s*\(", txt)))


def load(path: str = LIB_PATH):
    """Load liblensfmm.so and declare the C signatures (no device work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, V, I64, I32, D = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.lens_opts_default.argtypes = [P(LensOpts)]
    lib.lens_opts_default.restype = None
    lib.lens_plan_create.argtypes = [P(LensField), P(D), P(LensGrid), P(LensOpts), V, P(V)]
    lib.lens_plan_create.restype = ctypes.c_int
    lib.lens_plan_destroy.argtypes = [V]
    lib.lens_plan_destroy.restype = None
    lib.lens_plan_info.argtypes = [V, P(I32), P(I32), P(D), P(D), P(D)]
    lib.lens_plan_info.restype = ctypes.c_int
    lib.lens_deflect.argtypes = [V, P(LensField), P(LensGrid), V, I64, V, V, P(LensOpts), V]
    lib.lens_deflect.restype = ctypes.c_int
    lib.lens_deflect_noalloc.argtypes = [V, P(LensField), P(LensGrid), V, P(LensOpts), V]
    lib.lens_deflect_noalloc.restype = ctypes.c_int
    lib.lens_map.argtypes = [V, P(LensField), P(LensGrid), P(LensMapDesc), P(LensOpts), V]
    lib.lens_map.restype = ctypes.c_int
    lib.lens_last_error.argtypes = []
    lib.lens_last_error.restype = ctypes.c_char_p
    lib.lens_version.argtypes = []
    lib.lens_version.restype = ctypes.c_char_p
    lib.lens_deflect_backward.argtypes = [V, P(LensField), P(LensGrid), V, I64, V, V, V, P(LensOpts),
                                          V]
    lib.lens_deflect_backward.restype = ctypes.c_int
    lib.lens_map_batched.argtypes = [I32, P(LensField), P(LensGrid), P(LensMapDesc), P(LensOpts), V]
    lib.lens_map_batched.restype = ctypes.c_int
    lib.lens_map_ipm.argtypes = [V, P(LensField), P(LensGrid), P(LensIpmDesc), P(LensOpts), V]
    lib.lens_map_ipm.restype = ctypes.c_int
    lib.lens_find_images.argtypes = [V, P(LensField), P(LensGrid), V, I32, D, I32, V, V, I64, P(I64),
                                     P(LensOpts), V]
    lib.lens_find_images.restype = ctypes.c_int
    lib.lens_critical_curves.argtypes = [V, P(LensField), P(LensGrid), V, V, I64, P(I64), P(LensOpts),
                                         V]
    lib.lens_critical_curves.restype = ctypes.c_int
    lib.lens_deflect_multiplane.argtypes = [I32, P(LensField), P(D), P(LensGrid), V, I64, V,
                                            P(LensOpts), V]
    lib.lens_deflect_multiplane.restype = ctypes.c_int
    lib.lens_autotune.argtypes = [P(LensField), P(LensGrid), P(LensMapDesc), D, P(LensOpts), V,
                                  P(LensOpts), P(D), P(D)]
    lib.lens_autotune.restype = ctypes.c_int
    lib.lens_release_cached.argtypes = []
    lib.lens_release_cached.restype = None
    lib.lens_profile_enable.argtypes = [I32]
    lib.lens_profile_enable.restype = None
    lib.lens_profile_read.argtypes = [I32, P(ctypes.c_char_p), P(D), P(I64)]
    lib.lens_profile_read.restype = I32
    _lib = lib
    return lib


def check(status: int):
    if status != LENS_OK:
        msg = load().lens_last_error()
        raise LensError(status, msg.decode() if msg else "")


def profile_enable(on: bool):
    load().lens_profile_enable(1 if on else 0)


def profile_read() -> dict:
    """{stage: (total_ms, launches)} accumulated since profile_enable(True)."""
    lib = load()
    n = lib.lens_profile_read(0, None, None, None)
    names = (ctypes.c_char_p * max(n, 1))()
    ms = (ctypes.c_double * max(n, 1))()
    cnt = (ctypes.c_int64 * max(n, 1))()
    n = lib.lens_profile_read(n, names, ms, cnt)
    return {names[i].decode(): (ms[i], cnt[i]) for i in range(n)}
