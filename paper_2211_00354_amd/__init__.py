"""lensfmm for MI355X: fast-multipole gravitational-lens ray deflection.

Python face of liblensfmm (include/lens.h).  Tensors must be contiguous
float64 CUDA (HIP) tensors on the current device; work is enqueued on the
current torch stream.  Every step runs in the HIP library; there is no CPU
fallback, and a missing library raises ImportError on first use.

    import torch, paper_2211_00354_amd as lf
    y = lf.deflect(xy, m, grid=lf.Grid(x0, y0, dx, dy, nx, ny),
                   kappa_s=0.2, gamma=0.35, precision="mixed", p=12)
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

from . import _lib
from ._lib import (LENS_DIRECT, LENS_FMM, LENS_FP64, LENS_MIXED, LensError, LensField, LensGrid,
                   LensIpmDesc,
                   LensMapDesc, LensOpts)

__all__ = ["Grid", "MapDesc", "Plan", "autotune", "deflect", "deflect_backward", "ipm_map",
           "irs_map", "irs_map_batched", "LensDeflect", "LensError", "release_cached", "version"]


@dataclass
class Grid:
    """Cell-centred ray grid: ray k = j*nx + i at (x0+(i+.5)dx, y0+(j+.5)dy)."""
    x0: float
    y0: float
    dx: float
    dy: float
    nx: int
    ny: int

    def c(self) -> LensGrid:
        return LensGrid(self.x0, self.y0, self.dx, self.dy, self.nx, self.ny)


@dataclass
class MapDesc:
    y1min: float
    y2min: float
    side: float
    npix: int


def version() -> str:
    return _lib.load().lens_version().decode()


def _torch():
    import torch
    return torch


def _check_tensor(t, name, shape_last=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_last is not None and t.numel() and t.shape[-1] != shape_last:
        raise ValueError(f"{name} must have a trailing dimension of {shape_last}")
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name} is not on the current device")


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _opts(method="fmm", precision="mixed", p=12, leaf_level=0, max_rays_per_chunk=0,
          fp32_levels=0, tol=0.0) -> LensOpts:
    o = LensOpts()
    _lib.load().lens_opts_default(ctypes.byref(o))
    o.method = {"fmm": LENS_FMM, "direct": LENS_DIRECT}[method]
    o.precision = {"fp64": LENS_FP64, "mixed": LENS_MIXED}[precision]
    o.order_p = int(p)
    o.leaf_level = int(leaf_level)
    o.max_rays_per_chunk = int(max_rays_per_chunk)
    o.fp32_levels = int(fp32_levels)
    o.tol = float(tol)
    return o


def _field(xy, m, kappa_s, gamma):
    _check_tensor(xy, "star_xy", 2)
    _check_tensor(m, "star_m")
    n = m.numel()
    if xy.numel() != 2 * n:
        raise ValueError("star_xy must be [N, 2] with N = star_m.numel()")
    return LensField(n, xy.data_ptr() if n else None, m.data_ptr() if n else None,
                     float(kappa_s), float(gamma))


class Plan:
    """Star quadtree + multipoles, reusable across deflect/irs_map calls.

    ``ray_box`` = (x1min, x2min, x1max, x2max) and/or ``grid`` must contain
    every ray the plan will serve; with ``grid`` the leaf boxes are aligned
    with its cells where possible.  The plan copies the stars; it fixes
    precision, p and the leaf level.
    """

    def __init__(self, star_xy, star_m, kappa_s=0.0, gamma=0.0, ray_box=None, grid=None,
                 precision="mixed", p=12, leaf_level=0, fp32_levels=0, tol=0.0):
        lib = _lib.load()
        self._f = _field(star_xy, star_m, kappa_s, gamma)
        self.n_stars = int(self._f.n_stars)
        self.precision = precision
        self.kappa_s, self.gamma = float(kappa_s), float(gamma)
        o = _opts("fmm", precision, p, leaf_level, fp32_levels=fp32_levels, tol=tol)
        box = (ctypes.c_double * 4)(*ray_box) if ray_box is not None else None
        g = ctypes.byref(grid.c()) if grid is not None else None
        h = ctypes.c_void_p()
        _lib.check(lib.lens_plan_create(ctypes.byref(self._f), box, g, ctypes.byref(o), _stream(),
                                        ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        p, L = ctypes.c_int32(), ctypes.c_int32()
        x0, y0, s = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _lib.check(_lib.load().lens_plan_info(self._h, ctypes.byref(p), ctypes.byref(L),
                                              ctypes.byref(x0), ctypes.byref(y0), ctypes.byref(s)))
        return {"p": p.value, "leaf_level": L.value, "root_x0": x0.value, "root_y0": y0.value,
                "root_side": s.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().lens_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def deflect(star_xy=None, star_m=None, grid: Optional[Grid] = None, rays=None, kappa_s=0.0,
            gamma=0.0, method="fmm", precision="mixed", p=12, leaf_level=0,
            plan: Optional[Plan] = None, out=None, fp32_levels=0, want_dfdz=False, dfdz_out=None,
            tol=0.0, workspace=None):
    """Lens-map rays: returns y [n, 2] float64 on the GPU (eq. 1 + smooth term).

    Rays come from ``grid`` or from the explicit tensor ``rays`` [n, 2].  With
    ``plan`` the plan's stars are used; ``kappa_s``/``gamma`` still apply.
    With ``want_dfdz`` (or a ``dfdz_out`` tensor) returns (y, dfdz) where
    dfdz [n, 2] holds f'(z) = -sum m/(z - z_i)^2 (real, imaginary).
    ``p=0`` with ``tol > 0`` lets the library's autotuner choose p, the leaf
    level and the FP32 levels for that per-ray deflection error (measured
    once, then cached in-process and on disk).  ``workspace`` (a contiguous
    uint8 GPU tensor, with ``plan`` and ``grid``): the call's device memory
    is carved from it, in bands of rows that fit, and nothing is allocated.
    """
    torch = _torch()
    lib = _lib.load()
    if (grid is None) == (rays is None):
        raise ValueError("give exactly one of grid and rays")
    if plan is None:
        f = _field(star_xy, star_m, kappa_s, gamma)
    else:  # the plan supplies the stars, the call the smooth terms
        f = LensField(0, None, None, float(kappa_s), float(gamma))
    if grid is not None:
        n = int(grid.nx) * int(grid.ny)
        g = grid.c()
        gp, rp = ctypes.byref(g), None
    else:
        _check_tensor(rays, "rays", 2)
        n = rays.numel() // 2
        gp, rp = None, rays.data_ptr() if n else None
    dev = torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = torch.empty((n, 2), dtype=torch.float64, device=dev)
    else:
        _check_tensor(out, "out", 2)
        if out.numel() != 2 * n:
            raise ValueError("out must be [n, 2]")
    want = want_dfdz or dfdz_out is not None
    if want:
        if dfdz_out is None:
            dfdz_out = torch.empty((n, 2), dtype=torch.float64, device=dev)
        else:
            _check_tensor(dfdz_out, "dfdz_out", 2)
            if dfdz_out.numel() != 2 * n:
                raise ValueError("dfdz_out must be [n, 2]")
    o = _opts(method, precision, p, leaf_level, fp32_levels=fp32_levels, tol=tol)
    if workspace is not None:
        if workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 GPU tensor")
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel()
    _lib.check(lib.lens_deflect(plan.handle if plan else None, ctypes.byref(f), gp, rp, n,
                                out.data_ptr() if n else None,
                                dfdz_out.data_ptr() if (want and n) else None, ctypes.byref(o),
                                _stream()))
    return (out, dfdz_out) if want else out


def irs_map(star_xy=None, star_m=None, grid: Grid = None, map: MapDesc = None, kappa_s=0.0,
            gamma=0.0, method="fmm", precision="mixed", p=12, leaf_level=0,
            max_rays_per_chunk=0, plan: Optional[Plan] = None, counts=None, fp32_levels=0,
            tol=0.0):
    """Inverse ray shooting into an int32 [npix, npix] count map (accumulated
    into ``counts`` if given, indexed [v, u]).  ``p=0`` with ``tol > 0``: the
    autotuner's setting for that expected bin-reassignment fraction."""
    torch = _torch()
    lib = _lib.load()
    if plan is None:
        f = _field(star_xy, star_m, kappa_s, gamma)
    else:  # the plan supplies the stars, the call the smooth terms
        f = LensField(0, None, None, float(kappa_s), float(gamma))
    dev = torch.device("cuda", torch.cuda.current_device())
    if counts is None:
        counts = torch.zeros((map.npix, map.npix), dtype=torch.int32, device=dev)
    elif counts.dtype != torch.int32 or not counts.is_cuda or not counts.is_contiguous() \
            or counts.shape != (map.npix, map.npix):
        raise ValueError("counts must be a contiguous int32 [npix, npix] GPU tensor")
    md = LensMapDesc(map.y1min, map.y2min, map.side, map.npix, counts.data_ptr())
    g = grid.c()
    o = _opts(method, precision, p, leaf_level, max_rays_per_chunk, fp32_levels, tol)
    _lib.check(lib.lens_map(plan.handle if plan else None, ctypes.byref(f), ctypes.byref(g),
                            ctypes.byref(md), ctypes.byref(o), _stream()))
    return counts


def ipm_map(star_xy=None, star_m=None, grid: Grid = None, map: MapDesc = None, kappa_s=0.0,
            gamma=0.0, method="fmm", precision="mixed", p=12, leaf_level=0, max_rays_per_chunk=0,
            plan: Optional[Plan] = None, mu=None, fp32_levels=0, tol=0.0):
    """Inverse polygon mapping: the grid rays are the corners of image-plane
    cells whose areas are shared among the source pixels their mapped
    quadrilaterals overlap.  Returns the float64 [npix, npix] magnification
    map (accumulated into ``mu`` if given), indexed [v, u]."""
    torch = _torch()
    lib = _lib.load()
    if plan is None:
        f = _field(star_xy, star_m, kappa_s, gamma)
    else:  # the plan supplies the stars, the call the smooth terms
        f = LensField(0, None, None, float(kappa_s), float(gamma))
    dev = torch.device("cuda", torch.cuda.current_device())
    if mu is None:
        mu = torch.zeros((map.npix, map.npix), dtype=torch.float64, device=dev)
    elif mu.dtype != torch.float64 or not mu.is_cuda or not mu.is_contiguous() \
            or mu.shape != (map.npix, map.npix):
        raise ValueError("mu must be a contiguous float64 [npix, npix] GPU tensor")
    md = LensIpmDesc(map.y1min, map.y2min, map.side, map.npix, mu.data_ptr())
    g = grid.c()
    o = _opts(method, precision, p, leaf_level, max_rays_per_chunk, fp32_levels, tol)
    _lib.check(lib.lens_map_ipm(plan.handle if plan else None, ctypes.byref(f), ctypes.byref(g),
                                ctypes.byref(md), ctypes.byref(o), _stream()))
    return mu


def find_images(star_xy=None, star_m=None, grid: Grid = None, sources=None, kappa_s=0.0,
                gamma=0.0, tol=1e-10, max_iter=40, method="fmm", precision="fp64", p=24,
                leaf_level=0, plan: Optional[Plan] = None, cap=1 << 16, fp32_levels=0,
                max_rays_per_chunk=0):
    """Images of point sources inside the grid's region (lens_find_images).
    ``sources`` is a [n_src, 2] float64 GPU tensor.  Returns (images [k, 4]
    float64 = x1, x2, signed magnification, residual; src [k] int32), both on
    the GPU, ordered by source then x1.  Raises if more than ``cap`` images
    are found."""
    torch = _torch()
    lib = _lib.load()
    _check_tensor(sources, "sources", 2)
    ns = sources.numel() // 2
    if plan is None:
        f = _field(star_xy, star_m, kappa_s, gamma)
    else:
        f = LensField(0, None, None, float(kappa_s), float(gamma))
    dev = torch.device("cuda", torch.cuda.current_device())
    images = torch.empty((cap, 4), dtype=torch.float64, device=dev)
    src = torch.empty((cap,), dtype=torch.int32, device=dev)
    n = ctypes.c_int64()
    g = grid.c()
    o = _opts(method, precision, p, leaf_level, max_rays_per_chunk, fp32_levels)
    _lib.check(lib.lens_find_images(plan.handle if plan else None, ctypes.byref(f), ctypes.byref(g),
                                    sources.data_ptr() if ns else None, ns, float(tol),
                                    int(max_iter), images.data_ptr(), src.data_ptr(), cap,
                                    ctypes.byref(n), ctypes.byref(o), _stream()))
    if n.value > cap:
        raise ValueError(f"{n.value} images found, more than cap={cap}")
    return images[: n.value], src[: n.value]


def critical_curves(star_xy=None, star_m=None, grid: Grid = None, kappa_s=0.0, gamma=0.0,
                    method="fmm", precision="fp64", p=24, leaf_level=0,
                    plan: Optional[Plan] = None, cap=1 << 20, caustics=True, fp32_levels=0,
                    max_rays_per_chunk=0):
    """Critical-curve segments over the grid's region (lens_critical_curves):
    returns seg [k, 4] float64 (x1a, x2a, x1b, x2b) and, with ``caustics``,
    their images [k, 4] (else None), on the GPU.  Raises if more than ``cap``
    segments are found."""
    torch = _torch()
    lib = _lib.load()
    if plan is None:
        f = _field(star_xy, star_m, kappa_s, gamma)
    else:
        f = LensField(0, None, None, float(kappa_s), float(gamma))
    dev = torch.device("cuda", torch.cuda.current_device())
    seg = torch.empty((cap, 4), dtype=torch.float64, device=dev)
    cau = torch.empty((cap, 4), dtype=torch.float64, device=dev) if caustics else None
    n = ctypes.c_int64()
    g = grid.c()
    o = _opts(method, precision, p, leaf_level, max_rays_per_chunk, fp32_levels)
    _lib.check(lib.lens_critical_curves(plan.handle if plan else None, ctypes.byref(f),
                                        ctypes.byref(g), seg.data_ptr(),
                                        cau.data_ptr() if caustics else None, cap, ctypes.byref(n),
                                        ctypes.byref(o), _stream()))
    if n.value > cap:
        raise ValueError(f"{n.value} segments found, more than cap={cap}")
    return seg[: n.value], (cau[: n.value] if caustics else None)


def deflect_multiplane(planes, beta=None, grid: Optional[Grid] = None, rays=None, out=None,
                       method="fmm", precision="mixed", p=12, leaf_level=0, fp32_levels=0):
    """Multi-plane ray tracing (lens_deflect_multiplane).  ``planes`` is a list
    of (star_xy, star_m, kappa_s, gamma), nearest the observer first;
    ``beta`` an [n, n] array-like of distance ratios (only i < j read).
    Returns the source-plane positions y [n_rays, 2] float64 on the GPU."""
    torch = _torch()
    lib = _lib.load()
    npl = len(planes)
    fields = (LensField * npl)()
    for j, (xy, m, ks, g) in enumerate(planes):
        fields[j] = _field(xy, m, ks, g)
    bp = None
    if beta is not None:
        b = [float(v) for row in beta for v in row]
        if len(b) != npl * npl:
            raise ValueError("beta must be [n_planes, n_planes]")
        bp = (ctypes.c_double * (npl * npl))(*b)
    if (grid is None) == (rays is None):
        raise ValueError("give exactly one of grid and rays")
    if grid is not None:
        n = int(grid.nx) * int(grid.ny)
        g = grid.c()
        gp, rp = ctypes.byref(g), None
    else:
        _check_tensor(rays, "rays", 2)
        n = rays.numel() // 2
        gp, rp = None, rays.data_ptr() if n else None
    dev = torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = torch.empty((n, 2), dtype=torch.float64, device=dev)
    o = _opts(method, precision, p, leaf_level, fp32_levels=fp32_levels)
    _lib.check(lib.lens_deflect_multiplane(npl, fields, bp, gp, rp, n,
                                           out.data_ptr() if n else None, ctypes.byref(o),
                                           _stream()))
    return out


def irs_map_batched(fields, grids, maps, counts=None, method="fmm", precision="mixed", p=12,
                    leaf_level=0, fp32_levels=0, tol=0.0):
    """Inverse ray shooting for many independent fields in one captured HIP
    graph.  ``fields`` is a list of (star_xy, star_m, kappa_s, gamma);
    ``grids``/``maps`` lists of Grid/MapDesc; returns the list of int32 count
    maps (accumulated into ``counts`` if given).  With ``p=0`` and ``tol > 0``
    each field's p, leaf level and FP32 levels come from the autotuner (bin
    reassignment target ``tol``) when the batch is first built."""
    torch = _torch()
    lib = _lib.load()
    n = len(fields)
    if not (len(grids) == len(maps) == n):
        raise ValueError("fields, grids and maps must have the same length")
    dev = torch.device("cuda", torch.cuda.current_device())
    if counts is None:
        counts = [torch.zeros((mp.npix, mp.npix), dtype=torch.int32, device=dev) for mp in maps]
    fa = (LensField * max(n, 1))()
    ga = (LensGrid * max(n, 1))()
    ma = (LensMapDesc * max(n, 1))()
    for k, ((xy, m, ks, gm), g, mp, c) in enumerate(zip(fields, grids, maps, counts)):
        fa[k] = _field(xy, m, ks, gm)
        ga[k] = g.c()
        if c.dtype != torch.int32 or not c.is_cuda or not c.is_contiguous() \
                or c.shape != (mp.npix, mp.npix):
            raise ValueError("counts must be contiguous int32 [npix, npix] GPU tensors")
        ma[k] = LensMapDesc(mp.y1min, mp.y2min, mp.side, mp.npix, c.data_ptr())
    o = _opts(method, precision, p, leaf_level, fp32_levels=fp32_levels)
    o.tol = float(tol)
    _lib.check(lib.lens_map_batched(n, fa, ga, ma, ctypes.byref(o), _stream()))
    return counts


def autotune(star_xy, star_m, grid: Grid, map: Optional[MapDesc] = None, tol=1e-5, kappa_s=0.0,
             gamma=0.0, precision="mixed", leaf_level=0) -> dict:
    """Choose p, leaf level and FP32 levels by measurement (lens_autotune):
    on up to 256^2 strided rays the error against the FP64 direct sum (the
    largest per-ray |dalpha_k| / max(|alpha_k|, 1e-3 rms alpha), or with
    ``map`` the expected bin-reassignment fraction) must be at most half of
    ``tol``, and the fastest such whole call wins.  Returns {"p",
    "leaf_level", "fp32_levels", "error", "ms"}; raises LensError if no p up
    to 40 reaches tol."""
    lib = _lib.load()
    f = _field(star_xy, star_m, kappa_s, gamma)
    g = grid.c()
    base = _opts("fmm", precision, 0, leaf_level)
    out = LensOpts()
    err, ms = ctypes.c_double(), ctypes.c_double()
    md = None
    if map is not None:
        md = ctypes.byref(LensMapDesc(map.y1min, map.y2min, map.side, map.npix, None))
    _lib.check(lib.lens_autotune(ctypes.byref(f), ctypes.byref(g), md, float(tol), ctypes.byref(base),
                                 _stream(), ctypes.byref(out), ctypes.byref(err), ctypes.byref(ms)))
    return {"p": out.order_p, "leaf_level": out.leaf_level, "fp32_levels": out.fp32_levels,
            "error": err.value, "ms": ms.value}


def release_cached():
    """Free the cached graphs (batched maps, plan-less grid calls) and their
    buffers."""
    _lib.load().lens_release_cached()


def deflect_backward(star_xy, star_m, grad_y, grid: Optional[Grid] = None, rays=None,
                     method="fmm", precision="mixed", p=12, leaf_level=0,
                     plan: Optional["Plan"] = None):
    """Gradient of a loss with respect to the lenses: given grad_y = dL/dy
    [n, 2] for the rays of ``grid`` or ``rays``, returns (dL/d star_xy [N, 2],
    dL/d star_m [N]) as float64 GPU tensors.  With ``plan`` (the forward
    call's) its star tree, order and precision are reused (star_xy/star_m
    may then be None for the FMM)."""
    torch = _torch()
    lib = _lib.load()
    if (grid is None) == (rays is None):
        raise ValueError("give exactly one of grid and rays")
    if star_xy is None and plan is not None:
        f = LensField(plan.n_stars, None, None, 0.0, 0.0)
    else:
        f = _field(star_xy, star_m, 0.0, 0.0)
    if grid is not None:
        n = int(grid.nx) * int(grid.ny)
        g = grid.c()
        gp, rp = ctypes.byref(g), None
    else:
        _check_tensor(rays, "rays", 2)
        n = rays.numel() // 2
        gp, rp = None, rays.data_ptr() if n else None
    _check_tensor(grad_y, "grad_y", 2)
    if grad_y.numel() != 2 * n:
        raise ValueError("grad_y must be [n, 2]")
    dev = torch.device("cuda", torch.cuda.current_device())
    gxy = torch.empty((f.n_stars, 2), dtype=torch.float64, device=dev)
    gm = torch.empty((f.n_stars,), dtype=torch.float64, device=dev)
    o = _opts(method, precision, p, leaf_level)
    _lib.check(lib.lens_deflect_backward(plan.handle if plan else None, ctypes.byref(f), gp, rp, n,
                                         grad_y.data_ptr() if n else None,
                                         gxy.data_ptr() if f.n_stars else None,
                                         gm.data_ptr() if f.n_stars else None, ctypes.byref(o),
                                         _stream()))
    return gxy, gm


def _autograd_function():
    torch = _torch()

    class LensDeflect(torch.autograd.Function):
        """y = lens map of the rays (eq. 1 + smooth term) as a differentiable
        function of the star positions and masses.  Rays are a Grid (pass it
        as ``grid``) or a tensor (``rays``, treated as a constant)."""

        @staticmethod
        def forward(ctx, star_xy, star_m, rays=None, grid=None, kappa_s=0.0, gamma=0.0,
                    method="fmm", precision="mixed", p=12, leaf_level=0):
            plan = None
            if method == "fmm" and star_m.numel() > 0:
                # the forward's plan (star tree) is kept for the backward
                if rays is not None and rays.numel() > 0:
                    lo, hi = rays.amin(0).tolist(), rays.amax(0).tolist()
                    box = (lo[0], lo[1], hi[0], hi[1])
                else:
                    box = None
                plan = Plan(star_xy, star_m, kappa_s=kappa_s, gamma=gamma, ray_box=box,
                            grid=grid, precision=precision, p=p, leaf_level=leaf_level)
            y = deflect(star_xy, star_m, grid=grid, rays=rays, kappa_s=kappa_s, gamma=gamma,
                        method=method, precision=precision, p=p, leaf_level=leaf_level, plan=plan)
            ctx.save_for_backward(star_xy, star_m, rays if rays is not None else star_m)
            ctx.has_rays = rays is not None
            ctx.plan = plan
            ctx.cfg = (grid, method, precision, p, leaf_level)
            return y

        @staticmethod
        def backward(ctx, grad_y):
            star_xy, star_m, rays = ctx.saved_tensors
            grid, method, precision, p, leaf_level = ctx.cfg
            gxy, gm = deflect_backward(star_xy, star_m, grad_y.contiguous(), grid=grid,
                                       rays=rays if ctx.has_rays else None, method=method,
                                       precision=precision, p=p, leaf_level=leaf_level,
                                       plan=ctx.plan)
            if ctx.plan is not None:
                ctx.plan.close()   # released behind the backward's work (no wait)
                ctx.plan = None
            return gxy, gm, None, None, None, None, None, None, None, None

    return LensDeflect


def __getattr__(name):
    if name == "LensDeflect":
        fn = _autograd_function()
        globals()["LensDeflect"] = fn
        return fn
    raise AttributeError(name)
