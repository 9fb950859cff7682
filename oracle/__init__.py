"""FP64 CPU oracle for the point-lens deflection -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never loads it and the
two share no code: this is the plain definition (eq. 1 of the paper, Section
1, summed directly in FP64) that the GPU's fast multipole evaluation must
reproduce, plus inverse-ray-shooting binning (Section 2.3) and the gradient
of eq. 1 with respect to the lens parameters, and the multi-plane chain of
thin lenses built on eq. 1.

Every function below but ``multiplane`` is a thin ctypes marshaller around
``lens_oracle.c``; the arithmetic lives there and is documented there.
``multiplane`` composes ``deflect`` plane by plane in numpy.

Parity status: every function here is pinned by ``tests/test_oracle_pins.py``
against closed forms (point lens, Chang-Refsdal shear lens, Gauss's law for
the deflection flux, far-field Laurent moments, exact rational arithmetic on
tiny inputs, finite differences and scaling invariants; for the chain of
planes, its reductions to one plane, to superposition and to products of
linear maps).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lens_oracle.c")
_LIB = os.path.join(_HERE, "liblensoracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liblensoracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-std=c11", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_deflect.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int64, _dp, _dp, _dp, _i64p, ctypes.c_int]
        lib.oracle_deflect.restype = ctypes.c_int
        lib.oracle_jacobian.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_int64, _dp, _dp, ctypes.c_int]
        lib.oracle_jacobian.restype = ctypes.c_int
        lib.oracle_bin.argtypes = [ctypes.c_int64, _dp, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int32, _i32p]
        lib.oracle_bin.restype = ctypes.c_int64
        lib.oracle_grad.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_int64, _dp, _dp, _dp, _dp,
                                    ctypes.c_int]
        lib.oracle_grad.restype = ctypes.c_int
        lib.oracle_ipm.argtypes = [ctypes.c_int64, ctypes.c_int64, _dp, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int32, _dp]
        lib.oracle_ipm.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(a, shape_last=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape_last is not None and a.size and a.shape[-1] != shape_last:
        raise ValueError(f"expected trailing dimension {shape_last}, got {a.shape}")
    return a


def _ptr(a):
    return a.ctypes.data_as(_dp)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def deflect(star_xy, star_m, rays_xy, kappa_s=0.0, gamma=0.0, nthreads=0):
    """Return (y[n,2], alpha[n,2], n_coincident) for explicit rays (eq. 1)."""
    lib = _load()
    sxy = _f64(star_xy, 2).reshape(-1, 2)
    sm = _f64(star_m).reshape(-1)
    rxy = _f64(rays_xy, 2).reshape(-1, 2)
    if sxy.shape[0] != sm.shape[0]:
        raise ValueError("star_xy and star_m disagree on N")
    n = rxy.shape[0]
    y = np.empty((n, 2), np.float64)
    al = np.empty((n, 2), np.float64)
    skipped = ctypes.c_int64(0)
    rc = lib.oracle_deflect(sxy.shape[0], _ptr(sxy), _ptr(sm), float(kappa_s), float(gamma), n,
                            _ptr(rxy), _ptr(y), _ptr(al), ctypes.byref(skipped), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_deflect rejected its arguments")
    return y, al, int(skipped.value)


def jacobian(star_xy, star_m, rays_xy, nthreads=0):
    """Return J[n,3] = (J11, J12, J22) of d(alpha)/dx at each ray."""
    lib = _load()
    sxy = _f64(star_xy, 2).reshape(-1, 2)
    sm = _f64(star_m).reshape(-1)
    rxy = _f64(rays_xy, 2).reshape(-1, 2)
    out = np.empty((rxy.shape[0], 3), np.float64)
    rc = lib.oracle_jacobian(sxy.shape[0], _ptr(sxy), _ptr(sm), rxy.shape[0], _ptr(rxy), _ptr(out),
                             int(nthreads))
    if rc != 0:
        raise ValueError("oracle_jacobian rejected its arguments")
    return out


def bin_rays(y, y1min, y2min, side, npix, counts=None):
    """IRS binning; returns (counts[npix,npix] int32 indexed [v,u], n_landed)."""
    lib = _load()
    yy = _f64(y, 2).reshape(-1, 2)
    if counts is None:
        counts = np.zeros((npix, npix), np.int32)
    if counts.dtype != np.int32 or not counts.flags.c_contiguous or counts.shape != (npix, npix):
        raise ValueError("counts must be a C-contiguous int32 [npix, npix] array")
    landed = lib.oracle_bin(yy.shape[0], _ptr(yy), float(y1min), float(y2min), float(side),
                            int(npix), counts.ctypes.data_as(_i32p))
    if landed == -2:
        raise OverflowError("int32 pixel count overflow")
    if landed < 0:
        raise ValueError("oracle_bin rejected its arguments")
    return counts, int(landed)


def ipm(y_grid, cell_area, y1min, y2min, side, npix, mu=None):
    """IPM magnification map (first order, Section 2.3; see lens_oracle.c) of
    the cells spanned by the mapped grid y_grid [ny, nx, 2]; returns mu
    [npix, npix] float64 indexed [v, u] (accumulated into ``mu`` if given).
    Every cell's area is apportioned exactly among the pixels its image
    covers; a folded cell's image is its two lobes."""
    lib = _load()
    yy = np.ascontiguousarray(np.asarray(y_grid, dtype=np.float64))
    if yy.ndim != 3 or yy.shape[2] != 2:
        raise ValueError("y_grid must be [ny, nx, 2]")
    if mu is None:
        mu = np.zeros((npix, npix), np.float64)
    if mu.dtype != np.float64 or not mu.flags.c_contiguous or mu.shape != (npix, npix):
        raise ValueError("mu must be a C-contiguous float64 [npix, npix] array")
    rc = lib.oracle_ipm(yy.shape[1], yy.shape[0], _ptr(yy), float(cell_area), float(y1min),
                        float(y2min), float(side), int(npix), mu.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError("oracle_ipm rejected its arguments")
    return mu


def grad(star_xy, star_m, rays_xy, grad_y, nthreads=0):
    """Return (dL/d star_xy [N,2], dL/d star_m [N]) given dL/dy [n,2]."""
    lib = _load()
    sxy = _f64(star_xy, 2).reshape(-1, 2)
    sm = _f64(star_m).reshape(-1)
    rxy = _f64(rays_xy, 2).reshape(-1, 2)
    gy = _f64(grad_y, 2).reshape(-1, 2)
    if gy.shape[0] != rxy.shape[0]:
        raise ValueError("grad_y and rays disagree on n")
    gxy = np.empty_like(sxy)
    gm = np.empty(sxy.shape[0], np.float64)
    rc = lib.oracle_grad(sxy.shape[0], _ptr(sxy), _ptr(sm), rxy.shape[0], _ptr(rxy), _ptr(gy),
                         _ptr(gxy), _ptr(gm), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_grad rejected its arguments")
    return gxy, gm


def multiplane(planes, beta, rays_xy, nthreads=0):
    """Multi-plane ray tracing by the thin-lens chain (the introduction's
    footnote: a thick lens as a collection of thin planes), written from its
    definition: plane j (0 nearest the observer) is reached at
        x_j = x_0 - sum_{i<j} beta[j][i] alpha_i(x_i)
    and the source plane at y = x_0 - sum_i alpha_i(x_i), where
    alpha_i(x) = x - y_i(x) is plane i's whole deflection, y_i the one-plane
    lens mapping of ``deflect`` with that plane's smooth terms.  ``planes``
    lists (star_xy, star_m, kappa_s, gamma).  Returns y [n, 2]."""
    x0 = _f64(rays_xy, 2).reshape(-1, 2)
    alphas = []
    for j, (sxy, sm, ks, g) in enumerate(planes):
        xj = x0.copy()
        for i in range(j):
            xj = xj - float(beta[j][i]) * alphas[i]
        yj, _, _ = deflect(sxy, sm, xj, ks, g, nthreads=nthreads)
        alphas.append(xj - yj)
    y = x0.copy()
    for a in alphas:
        y = y - a
    return y
