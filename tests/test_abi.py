"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/lens.h declares, and rejects bad arguments before it
touches the device."""
import ctypes

import pytest

from paper_2211_00354_amd import _lib


def test_library_exports_every_declared_symbol():
    names = _lib.declared_functions()
    assert {"lens_deflect", "lens_map", "lens_plan_create", "lens_plan_destroy",
            "lens_last_error"} <= set(names)
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_version_string():
    assert b"gfx950" in _lib.load().lens_version()


def _opts(**kw):
    o = _lib.LensOpts()
    _lib.load().lens_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_opts_defaults():
    o = _opts()
    assert (o.method, o.precision, o.order_p, o.leaf_level) == (_lib.LENS_FMM, _lib.LENS_MIXED, 12, 0)
    assert o.fp32_levels == 0


@pytest.mark.parametrize("field,opts,msg", [
    (dict(n_stars=-1), {}, "n_stars"),
    (dict(n_stars=5), {}, "NULL"),                       # null star pointers
    (dict(n_stars=0, kappa_s=float("nan")), {}, "finite"),
    (dict(n_stars=0), dict(order_p=41), "order_p"),
    (dict(n_stars=0), dict(order_p=-2), "order_p"),
    (dict(n_stars=0), dict(leaf_level=1), "leaf_level"),
    (dict(n_stars=0), dict(leaf_level=16), "leaf_level"),
    (dict(n_stars=0), dict(fp32_levels=-2), "fp32_levels"),
    (dict(n_stars=0), dict(fp32_levels=16), "fp32_levels"),
    (dict(n_stars=0), dict(method=7), "method"),
    (dict(n_stars=0), dict(precision=3), "precision"),
])
def test_deflect_rejects_bad_arguments(field, opts, msg):
    lib = _lib.load()
    f = _lib.LensField(**field)
    o = _opts(**opts)
    g = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 2, 2)
    st = lib.lens_deflect(None, ctypes.byref(f), ctypes.byref(g), None, 4, ctypes.c_void_p(8),
                          None, ctypes.byref(o), None)
    assert st == _lib.LENS_EINVAL
    assert msg in lib.lens_last_error().decode()


@pytest.mark.parametrize("grid,n,msg", [
    ((0.0, 0.0, 0.0, 1.0, 2, 2), 4, "dx"),
    ((0.0, 0.0, 1.0, -1.0, 2, 2), 4, "dx"),
    ((float("inf"), 0.0, 1.0, 1.0, 2, 2), 4, "finite"),
    ((0.0, 0.0, 1.0, 1.0, -1, 2), 0, "nx"),
    ((0.0, 0.0, 1.0, 1.0, 2, 2), 5, "n_rays"),
])
def test_deflect_rejects_bad_grids(grid, n, msg):
    lib = _lib.load()
    f = _lib.LensField(n_stars=0)
    g = _lib.LensGrid(*grid)
    st = lib.lens_deflect(None, ctypes.byref(f), ctypes.byref(g), None, n, ctypes.c_void_p(8),
                          None, None, None)
    assert st == _lib.LENS_EINVAL
    assert msg in lib.lens_last_error().decode()


def test_deflect_needs_exactly_one_ray_source_and_an_output():
    lib = _lib.load()
    f = _lib.LensField(n_stars=0)
    g = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 2, 2)
    assert lib.lens_deflect(None, ctypes.byref(f), ctypes.byref(g), ctypes.c_void_p(8), 4,
                            ctypes.c_void_p(8), None, None, None) == _lib.LENS_EINVAL
    assert lib.lens_deflect(None, ctypes.byref(f), ctypes.byref(g), None, 4, None, None, None,
                            None) == _lib.LENS_EINVAL
    assert b"y_out" in lib.lens_last_error()
    # zero rays is a no-op
    g0 = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 0, 3)
    assert lib.lens_deflect(None, ctypes.byref(f), ctypes.byref(g0), None, 0, None, None, None,
                            None) == _lib.LENS_OK


@pytest.mark.parametrize("npix,side,counts,msg", [
    (0, 1.0, 8, "npix"),
    (46341, 1.0, 8, "npix"),        # npix^2 > 2^31 - 1
    (4, 0.0, 8, "side"),
    (4, float("nan"), 8, "side"),
    (4, 1.0, None, "counts"),
])
def test_map_rejects_bad_maps(npix, side, counts, msg):
    lib = _lib.load()
    f = _lib.LensField(n_stars=0)
    g = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 2, 2)
    md = _lib.LensMapDesc(0.0, 0.0, side, npix, counts)
    st = lib.lens_map(None, ctypes.byref(f), ctypes.byref(g), ctypes.byref(md), None, None)
    assert st == _lib.LENS_EINVAL
    assert msg in lib.lens_last_error().decode()


def test_map_rejects_more_rays_than_int32_counts_can_hold():
    lib = _lib.load()
    f = _lib.LensField(n_stars=0)
    g = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 65536, 32769)
    md = _lib.LensMapDesc(0.0, 0.0, 1.0, 4, ctypes.c_void_p(8))
    assert lib.lens_map(None, ctypes.byref(f), ctypes.byref(g), ctypes.byref(md), None,
                        None) == _lib.LENS_EINVAL
    assert b"2^31" in lib.lens_last_error()


def test_plan_create_rejects_bad_ray_box():
    lib = _lib.load()
    f = _lib.LensField(n_stars=0)
    box = (ctypes.c_double * 4)(1.0, 0.0, 0.0, 1.0)   # x1max < x1min
    h = ctypes.c_void_p()
    assert lib.lens_plan_create(ctypes.byref(f), box, None, None, None,
                                ctypes.byref(h)) == _lib.LENS_EINVAL
    assert lib.lens_plan_create(ctypes.byref(f), None, None, None, None, None) == _lib.LENS_EINVAL
    g = _lib.LensGrid(0.0, 0.0, -1.0, 1.0, 2, 2)
    assert lib.lens_plan_create(ctypes.byref(f), None, ctypes.byref(g), None, None,
                                ctypes.byref(h)) == _lib.LENS_EINVAL


@pytest.mark.parametrize("tol,grid,out,msg", [
    (0.0, True, True, "tol"),
    (float("nan"), True, True, "tol"),
    (1e-5, False, True, "grid"),
    (1e-5, True, False, "out"),
])
def test_autotune_rejects_bad_arguments(tol, grid, out, msg):
    lib = _lib.load()
    f = _lib.LensField(0, None, None, 0.0, 0.0)
    g = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 2, 2)
    o = _lib.LensOpts()
    st = lib.lens_autotune(ctypes.byref(f), ctypes.byref(g) if grid else None, None, tol, None, None,
                           ctypes.byref(o) if out else None, None, None)
    assert st == _lib.LENS_EINVAL
    assert msg in lib.lens_last_error().decode()


def test_batched_rejects_bad_tol():
    lib = _lib.load()
    f = (_lib.LensField * 1)(_lib.LensField(0, None, None, 0.0, 0.0))
    g = (_lib.LensGrid * 1)(_lib.LensGrid(0.0, 0.0, 1.0, 1.0, 2, 2))
    m = (_lib.LensMapDesc * 1)(_lib.LensMapDesc(0.0, 0.0, 1.0, 4, ctypes.c_void_p(8)))
    o = _opts(order_p=0, tol=float("inf"))
    assert lib.lens_map_batched(1, f, g, m, ctypes.byref(o), None) == _lib.LENS_EINVAL
    assert "tol" in lib.lens_last_error().decode()


@pytest.mark.parametrize("npix,side,mu,msg", [
    (0, 1.0, 8, "npix"),
    (50000, 1.0, 8, "npix"),
    (4, 0.0, 8, "side"),
    (4, float("nan"), 8, "side"),
    (4, 1.0, 0, "mu"),
])
def test_ipm_map_rejects_bad_maps(npix, side, mu, msg):
    lib = _lib.load()
    f = _lib.LensField(0, None, None, 0.0, 0.0)
    g = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 4, 4)
    md = _lib.LensIpmDesc(0.0, 0.0, side, npix, ctypes.c_void_p(mu) if mu else None)
    o = _opts()
    st = lib.lens_map_ipm(None, ctypes.byref(f), ctypes.byref(g), ctypes.byref(md), ctypes.byref(o),
                          None)
    assert st == _lib.LENS_EINVAL
    assert msg in lib.lens_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(tol=0.0), "tol"),
    (dict(tol=float("nan")), "tol"),
    (dict(max_iter=-1), "max_iter"),
    (dict(max_iter=1001), "max_iter"),
    (dict(n_images=False), "n_images"),
    (dict(grid=False), "grid"),
    (dict(n_src=-1), "n_sources"),
    (dict(sources=False), "sources"),
    (dict(out=False), "images"),
])
def test_find_images_rejects_bad_arguments(kw, msg):
    lib = _lib.load()
    f = _lib.LensField(0, None, None, 0.0, 0.0)
    g = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 4, 4)
    n = ctypes.c_int64(-7)
    st = lib.lens_find_images(None, ctypes.byref(f), ctypes.byref(g) if kw.get("grid", True) else None,
                              ctypes.c_void_p(8) if kw.get("sources", True) else None,
                              kw.get("n_src", 1), kw.get("tol", 1e-9), kw.get("max_iter", 10),
                              ctypes.c_void_p(8) if kw.get("out", True) else None,
                              ctypes.c_void_p(8) if kw.get("out", True) else None, 16,
                              ctypes.byref(n) if kw.get("n_images", True) else None, None, None)
    assert st == _lib.LENS_EINVAL
    assert msg in lib.lens_last_error().decode()


def test_find_images_and_critical_curves_of_a_cell_free_grid_are_empty():
    lib = _lib.load()
    f = _lib.LensField(0, None, None, 0.0, 0.0)
    g = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 1, 7)   # one column: no cells
    n = ctypes.c_int64(-7)
    assert lib.lens_find_images(None, ctypes.byref(f), ctypes.byref(g), ctypes.c_void_p(8), 1, 1e-9, 10,
                                None, None, 0, ctypes.byref(n), None, None) == _lib.LENS_OK
    assert n.value == 0
    n.value = -7
    assert lib.lens_critical_curves(None, ctypes.byref(f), ctypes.byref(g), None, None, 0,
                                    ctypes.byref(n), None, None) == _lib.LENS_OK
    assert n.value == 0


@pytest.mark.parametrize("cap,seg,nseg,msg", [(-1, True, True, "cap"), (4, False, True, "seg_out"),
                                              (4, True, False, "n_seg")])
def test_critical_curves_rejects_bad_arguments(cap, seg, nseg, msg):
    lib = _lib.load()
    f = _lib.LensField(0, None, None, 0.0, 0.0)
    g = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 4, 4)
    n = ctypes.c_int64()
    st = lib.lens_critical_curves(None, ctypes.byref(f), ctypes.byref(g),
                                  ctypes.c_void_p(8) if seg else None, None, cap,
                                  ctypes.byref(n) if nseg else None, None, None)
    assert st == _lib.LENS_EINVAL
    assert msg in lib.lens_last_error().decode()


@pytest.mark.parametrize("npl,beta,grid,rays,msg", [
    (0, None, True, False, "n_planes"),
    (65, None, True, False, "n_planes"),
    (2, None, True, False, "beta"),
    (2, [0.0, 0.0, float("nan"), 0.0], True, False, "beta"),
    (1, None, True, True, "exactly one"),
    (1, None, False, False, "exactly one"),
])
def test_multiplane_rejects_bad_arguments(npl, beta, grid, rays, msg):
    lib = _lib.load()
    k = max(npl, 1)
    fields = (_lib.LensField * k)(*[_lib.LensField(0, None, None, 0.0, 0.0) for _ in range(k)])
    g = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 2, 2)
    b = (ctypes.c_double * len(beta))(*beta) if beta else None
    st = lib.lens_deflect_multiplane(npl, fields, b, ctypes.byref(g) if grid else None,
                                     ctypes.c_void_p(8) if rays else None, 4, ctypes.c_void_p(8),
                                     None, None)
    assert st == _lib.LENS_EINVAL
    assert msg in lib.lens_last_error().decode()


@pytest.mark.parametrize("addr,size", [(8, 1 << 20), (256, 0)])
def test_workspace_must_be_aligned_and_sized(addr, size):
    lib = _lib.load()
    f = _lib.LensField(n_stars=0)
    g = _lib.LensGrid(0.0, 0.0, 1.0, 1.0, 2, 2)
    o = _opts()
    o.workspace = addr
    o.workspace_bytes = size
    st = lib.lens_deflect(None, ctypes.byref(f), ctypes.byref(g), None, 4, ctypes.c_void_p(8), None,
                          ctypes.byref(o), None)
    assert st == _lib.LENS_EINVAL
    assert "workspace" in lib.lens_last_error().decode()
