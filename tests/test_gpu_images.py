"""GPU checks of the inverse lens equation, the critical curves and the
multi-plane chain against closed forms and the FP64 oracle: the point lens
(two images on the line through lens and source; the Einstein ring as the
critical curve), the Chang-Refsdal lens (images from the roots of its quartic,
the caustic's cusps), the synthetic galaxy halo (every image a root of the
oracle's lens equation, FMM against the direct sum), and chains of two and
three planes against the oracle's recursion."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _grid(lf, half, n):
    g = wl.centred_grid(2 * half, 2 * half, n, n)
    return g, lf.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)


def _mu_oracle(xy, m, x, kappa_s, gamma):
    J = oracle.jacobian(xy, m, x)
    A11 = (1 - kappa_s - gamma) - J[:, 0]
    A22 = (1 - kappa_s + gamma) - J[:, 2]
    A12 = -J[:, 1]
    return 1.0 / (A11 * A22 - A12 * A12)


def _residual_oracle(xy, m, x, beta, kappa_s, gamma):
    y, _, _ = oracle.deflect(xy, m, x, kappa_s, gamma)
    return np.hypot(*(y - beta).T)


# ------------------------------------------------------------------ images

@pytest.mark.parametrize("method,p", [("direct", 24), ("fmm", 36)])
def test_point_lens_images_closed_form(lf, method, p):
    """Unit point lens at z_L: a source at distance u has images at
    z_L + e (u +- sqrt(u^2 + 4))/2 (e the unit vector towards the source)
    with magnifications 1/2 +- (u^2 + 2)/(2 u sqrt(u^2 + 4)).  (One star in
    a box corner is the FMM's worst case, ~0.53^p relative: p = 36.)"""
    zl = np.array([[0.0312, -0.0187]])
    m = np.ones(1)
    g, grid = _grid(lf, 3.0, 1024)
    src = np.array([[0.4, 0.1], [1.2, -0.7], [0.05, 0.02], [-0.3, 0.9]])
    _say("point lens images", method)
    im, s = lf.find_images(_dev(zl), _dev(m), grid=grid, sources=_dev(src), method=method,
                           precision="fp64", p=p, tol=1e-12)
    im, s = im.cpu().numpy(), s.cpu().numpy()
    for k, b in enumerate(src):
        mine = im[s == k]
        d = b - zl[0]
        u = np.hypot(*d)
        e = d / u
        r = np.array([(u + math.sqrt(u * u + 4)) / 2, (u - math.sqrt(u * u + 4)) / 2])
        x = zl[0] + r[:, None] * e
        mu = 0.5 + np.array([1, -1]) * (u * u + 2) / (2 * u * math.sqrt(u * u + 4))
        inside = np.all(np.abs(x) < 3.0 - 2 * g.dx, axis=1)
        x, mu = x[inside], mu[inside]
        o = np.argsort(x[:, 0])
        print(f"[img] source {b}: found {len(mine)}, expected {len(x)}", flush=True)
        assert len(mine) == len(x), (b, mine, x)
        np.testing.assert_allclose(mine[:, :2], x[o], rtol=0, atol=1e-9)
        np.testing.assert_allclose(mine[:, 2], mu[o], rtol=1e-8)
        assert np.all(mine[:, 3] <= 1e-12)


def _chang_refsdal_images(w, gamma):
    """Images of source w (complex) for a unit point lens at 0 with shear
    gamma (kappa_s = 0): w = z - gamma c - 1/c with c = conj(z).  Taking the
    conjugate equation for c, c = (gamma z^2 + conj(w) z + 1)/z = N/z, and
    substituting gives the quartic N z (w - z) + gamma N^2 + z^2 = 0; its
    roots with N/z = conj(z) are the images."""
    N = np.array([gamma, np.conj(w), 1.0])            # gamma z^2 + conj(w) z + 1
    poly = np.polyadd(np.polyadd(np.polymul(np.polymul(N, [1.0, 0.0]), [-1.0, w]),
                                 gamma * np.polymul(N, N)), [1.0, 0.0, 0.0])
    roots = np.roots(poly)
    keep = [z for z in roots if abs(np.polyval(N, z) / z - np.conj(z)) < 1e-8 * max(1, abs(z))]
    return np.array([[z.real, z.imag] for z in keep])


@pytest.mark.parametrize("source,n_expect", [((0.1, 0.1), 4), ((-0.15, 0.2), 4), ((0.8, 0.9), 2),
                                             ((-0.2, 0.35), 2)])
def test_chang_refsdal_images_against_quartic(lf, source, n_expect):
    gamma = 0.3
    zl, m = np.zeros((1, 2)), np.ones(1)
    ref = _chang_refsdal_images(complex(*source), gamma)
    assert len(ref) == n_expect
    g, grid = _grid(lf, 3.0, 1024)
    _say("chang-refsdal images", source)
    im, s = lf.find_images(_dev(zl), _dev(m), grid=grid, sources=_dev(np.array([source])),
                           gamma=gamma, method="direct", tol=1e-12)
    im = im.cpu().numpy()
    ref = ref[np.argsort(ref[:, 0])]
    print(f"[img] chang-refsdal {source}: {len(im)} images, expected {len(ref)}", flush=True)
    assert len(im) == len(ref)
    np.testing.assert_allclose(im[:, :2], ref, rtol=0, atol=1e-9)
    np.testing.assert_allclose(im[:, 2], _mu_oracle(zl, m, ref, 0.0, gamma), rtol=1e-8)


def test_synthetic_halo_images(lf):
    """The galaxy halo of 1.575e7 particles (Section 2.5's case): images of
    two sources near the centre by the FP64 FMM on the 4000^2 grid over the
    central 90 x 90.  The particles are lenses too, so a macro image may come
    split into a few; every image found is a root of the oracle's lens
    equation with the oracle's magnification, each source has at least
    three images with |mu| > 0.3 (inside the tangential caustic), and on a
    9 x 9 window around one of them the FP64 direct sum finds the same
    images."""
    import torch
    f, g = wl.synthetic_halo()
    xy, m = _dev(f.xy), _dev(f.m)
    src = np.array([[0.8, 0.5], [-2.0, 1.0]])
    grid = lf.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)
    kw = dict(kappa_s=f.kappa_s, gamma=f.gamma, tol=1e-9)
    _say("halo images, FP64 FMM on 4000^2")
    im, s = lf.find_images(xy, m, grid=grid, sources=_dev(src), method="fmm", precision="fp64", p=24,
                           **kw)
    im, s = im.cpu().numpy(), s.cpu().numpy()
    for k, b in enumerate(src):
        mine = im[s == k]
        big = np.abs(mine[:, 2]) > 0.3
        macro = mine[big]
        print(f"[img] halo source {b}: {len(mine)} images, {len(macro)} with |mu| > 0.3: "
              f"{np.round(macro[:, :3], 3).tolist()}", flush=True)
        assert len(macro) >= 3
        # every macro image and up to 200 others (tiny images next to
        # particles, where y moves by 1/|mu| per unit of x): residual of the
        # oracle's lens equation within 1e-8 max(1, 1/|mu|)
        pick = np.concatenate([np.flatnonzero(big),
                               np.random.default_rng(k).permutation(np.flatnonzero(~big))[:200]])
        res = _residual_oracle(f.xy, f.m, mine[pick, :2], b, f.kappa_s, f.gamma)
        bound = 1e-8 * np.maximum(1.0, 1.0 / np.abs(mine[pick, 2]))
        assert np.all(res <= bound), (res / bound).max()
        mo = _mu_oracle(f.xy, f.m, macro[:, :2], f.kappa_s, f.gamma)
        np.testing.assert_allclose(macro[:, 2], mo, rtol=1e-6)
    # the direct sum on a window around source 0's first macro image, at the
    # same ray spacing: the same images away from the window's edge
    c = im[(s == 0) & (np.abs(im[:, 2]) > 0.3)][0, :2]
    nw = 400
    gw = wl.Grid(x0=g.x0 + (np.floor((c[0] - g.x0) / g.dx) - nw // 2) * g.dx,
                 y0=g.y0 + (np.floor((c[1] - g.y0) / g.dy) - nw // 2) * g.dy,
                 dx=g.dx, dy=g.dy, nx=nw, ny=nw)
    _say("halo images, FP64 direct on a 400^2 window at", c)
    imd, sd = lf.find_images(xy, m, grid=lf.Grid(gw.x0, gw.y0, gw.dx, gw.dy, gw.nx, gw.ny),
                             sources=_dev(src[:1]), method="direct", **kw)
    imd = imd.cpu().numpy()
    lo = np.array([gw.x0, gw.y0]) + 1.0
    hi = np.array([gw.x0 + nw * gw.dx, gw.y0 + nw * gw.dy]) - 1.0

    def interior(a):
        return a[np.all((a[:, :2] > lo) & (a[:, :2] < hi), axis=1)]
    a, d = interior(im[s == 0]), interior(imd)
    print(f"[img] window: FMM {len(a)} images, direct {len(d)}", flush=True)
    assert len(a) == len(d) and len(a) >= 1
    for x in a[:, :2]:
        assert np.min(np.hypot(*(d[:, :2] - x).T)) < 1e-7
    torch.cuda.synchronize()


# --------------------------------------------------------- critical curves

@pytest.mark.parametrize("method", ["direct", "fmm"])
def test_point_lens_critical_curve_is_the_einstein_ring(lf, method):
    """m = 1, no shear: det A = 1 - 1/r^4 vanishes on r = 1; the segments lie
    on the ring to O(dx^2), their total length is 2 pi, and the caustic is
    the point under the lens."""
    g, grid = _grid(lf, 2.0, 512)
    _say("point lens critical curve", method)
    seg, cau = lf.critical_curves(_dev(np.zeros((1, 2))), _dev(np.ones(1)), grid=grid,
                                  method=method, precision="fp64", p=24)
    seg, cau = seg.cpu().numpy(), cau.cpu().numpy()
    r = np.hypot(seg[:, 0::2], seg[:, 1::2])
    length = np.hypot(seg[:, 2] - seg[:, 0], seg[:, 3] - seg[:, 1]).sum()
    print(f"[crit] {len(seg)} segments, |r - 1| max {np.abs(r - 1).max():.2e}, length "
          f"{length:.6f}, caustic radius max {np.hypot(cau[:, 0::2], cau[:, 1::2]).max():.2e}",
          flush=True)
    assert np.abs(r - 1).max() <= 3 * g.dx ** 2
    assert abs(length / (2 * math.pi) - 1) < 1e-4
    assert np.hypot(cau[:, 0::2], cau[:, 1::2]).max() <= 8 * g.dx ** 2


def test_chang_refsdal_critical_curve_and_caustic_cusps(lf):
    """Unit point lens with shear 0.3: det A (oracle) vanishes at the segment
    ends to O(dx^2), and the caustic reaches its cusps at |y1| =
    2 gamma/sqrt(1 + gamma), |y2| = 2 gamma/sqrt(1 - gamma)."""
    gamma = 0.3
    g, grid = _grid(lf, 2.5, 1000)
    _say("chang-refsdal critical curve")
    seg, cau = lf.critical_curves(_dev(np.zeros((1, 2))), _dev(np.ones(1)), grid=grid, gamma=gamma,
                                  method="fmm", precision="fp64", p=24)
    seg, cau = seg.cpu().numpy(), cau.cpu().numpy()
    pts = seg.reshape(-1, 2)
    det = 1.0 / _mu_oracle(np.zeros((1, 2)), np.ones(1), pts, 0.0, gamma)
    ymax = np.abs(cau.reshape(-1, 2)).max(0)
    cusp = [2 * gamma / math.sqrt(1 + gamma), 2 * gamma / math.sqrt(1 - gamma)]
    print(f"[crit] chang-refsdal: {len(seg)} segments, |det A| max {np.abs(det).max():.2e}, "
          f"caustic extent {ymax}, cusps {cusp}", flush=True)
    assert np.abs(det).max() <= 40 * g.dx ** 2
    np.testing.assert_allclose(ymax, cusp, rtol=2e-3)


# ------------------------------------------------------------- multi-plane

def _planes(seed):
    out = []
    # kappa_* ~ 0.2 per plane (masses 0.3 of a mean-1 power law), disks wider
    # than the rays' reach
    for j, (n, R, ks, gm) in enumerate(((1000, 40.0, 0.1, 0.05), (800, 35.0, 0.2, -0.1),
                                        (600, 30.0, 0.05, 0.15))):
        f = wl.random_field(n, R, seed=seed + j, masses="powerlaw")
        f.m *= 0.3
        out.append((f.xy, f.m, ks, gm))
    return out


@pytest.mark.parametrize("nplanes,prec,p,tol", [(2, "fp64", 30, 1e-10), (3, "fp64", 30, 1e-10),
                                               (3, "mixed", 16, 1e-5)])
def test_multiplane_against_oracle(lf, nplanes, prec, p, tol):
    """Chains of two and three planes (power-law stars, each plane with its
    own kappa_s and gamma), grid and explicit rays, against the oracle's
    recursion; error relative to the total deflection x - y, per ray."""
    import torch
    pl = _planes(70)[:nplanes]
    beta = [[0.0, 0.0, 0.0], [0.45, 0.0, 0.0], [0.7, 0.35, 0.0]]
    beta = [row[:nplanes] for row in beta[:nplanes]]
    g = wl.centred_grid(16.0, 12.0, 384, 288)
    dpl = [(_dev(a), _dev(b), ks, gm) for a, b, ks, gm in pl]
    _say("multiplane", nplanes, prec, p)
    y = lf.deflect_multiplane(dpl, beta, grid=lf.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny),
                              precision=prec, p=p).cpu().numpy()
    idx = g.strided(7, 3)
    x0 = g.rays(idx)
    yo = oracle.multiplane(pl, beta, x0)
    dt = np.hypot(*(x0 - yo).T)
    err = np.hypot(*(y[idx] - yo).T) / np.maximum(dt, 1e-3 * np.sqrt(np.mean(dt * dt)))
    rays = np.random.default_rng(71).uniform(-8, 8, (5000, 2))
    ye = lf.deflect_multiplane(dpl, beta, rays=_dev(rays), precision=prec, p=p).cpu().numpy()
    yeo = oracle.multiplane(pl, beta, rays)
    dte = np.hypot(*(rays - yeo).T)
    erre = np.hypot(*(ye - yeo).T) / np.maximum(dte, 1e-3 * np.sqrt(np.mean(dte * dte)))
    print(f"[mp] {nplanes} planes {prec} p={p}: grid rays p99 {np.percentile(err, 99):.2e} "
          f"max {err.max():.2e}; explicit p99 {np.percentile(erre, 99):.2e} max {erre.max():.2e}",
          flush=True)
    # a ray passing close to a star of a later plane amplifies the earlier
    # planes' errors by that plane's |d alpha/dx| (~m/r^2): the bulk is held
    # to tol, the worst rays to 50 tol
    assert np.percentile(err, 99) <= tol and np.percentile(erre, 99) <= tol
    assert err.max() <= 50 * tol and erre.max() <= 50 * tol
    torch.cuda.synchronize()


def test_images_through_a_plan_and_in_mixed_precision(lf):
    """The same point-lens images with a plan built over the grid (FP64) and
    in mixed precision (tol 1e-6: the evaluation's own error); for a distant
    source only the faint image next to the lens, and nothing for no
    source at all."""
    import ctypes
    import torch
    from paper_2211_00354_amd import _lib
    zl, m = np.array([[0.0312, -0.0187]]), np.ones(1)
    g, grid = _grid(lf, 3.0, 1024)
    src = np.array([[0.4, 0.1], [1.2, -0.7]])
    plan = lf.Plan(_dev(zl), _dev(m), grid=grid, precision="fp64", p=36)
    _say("images through a plan")
    im_p, s_p = lf.find_images(grid=grid, sources=_dev(src), plan=plan, tol=1e-12)
    im_n, s_n = lf.find_images(_dev(zl), _dev(m), grid=grid, sources=_dev(src), precision="fp64",
                               p=36, tol=1e-12)
    plan.close()
    np.testing.assert_array_equal(s_p.cpu().numpy(), s_n.cpu().numpy())
    np.testing.assert_allclose(im_p.cpu().numpy()[:, :3], im_n.cpu().numpy()[:, :3], rtol=0,
                               atol=1e-12)
    _say("images mixed")
    im_m, s_m = lf.find_images(_dev(zl), _dev(m), grid=grid, sources=_dev(src), precision="mixed",
                               p=16, tol=1e-6)
    im_m, s_m = im_m.cpu().numpy(), s_m.cpu().numpy()
    assert len(im_m) == 4
    res = _residual_oracle(zl, m, im_m[:, :2], src[s_m], 0.0, 0.0)
    print(f"[img] mixed: residual against the oracle up to {res.max():.2e}", flush=True)
    assert res.max() <= 5e-6
    # a source far outside: its bright image lies outside the grid's region,
    # the faint one next to the lens (at distance ~1/u) inside it
    far = np.array([[40.0, 40.0]])
    im_f, _ = lf.find_images(_dev(zl), _dev(m), grid=grid, sources=_dev(far), method="direct",
                             tol=1e-12)
    im_f = im_f.cpu().numpy()
    d = far[0] - zl[0]
    u = np.hypot(*d)
    x_in = zl[0] + (u - math.sqrt(u * u + 4)) / 2 * d / u
    assert len(im_f) == 1
    np.testing.assert_allclose(im_f[0, :2], x_in, rtol=0, atol=1e-9)
    # no sources at all, through the C ABI
    lib = _lib.load()
    zl_d, m_d = _dev(zl), _dev(m)
    f = _lib.LensField(1, ctypes.c_void_p(zl_d.data_ptr()), ctypes.c_void_p(m_d.data_ptr()), 0.0, 0.0)
    n = ctypes.c_int64(-1)
    g_c = grid.c()
    assert lib.lens_find_images(None, ctypes.byref(f), ctypes.byref(g_c), None, 0, 1e-9, 10, None,
                                None, 0, ctypes.byref(n), None, None) == _lib.LENS_OK
    assert n.value == 0
    torch.cuda.synchronize()


def test_critical_curves_mixed_and_cap(lf):
    """Mixed precision gives the same Einstein ring to O(dx^2); a segment
    buffer smaller than the curve reports the full count and fills the
    buffer only."""
    import ctypes
    import torch
    from paper_2211_00354_amd import _lib
    g, grid = _grid(lf, 2.0, 512)
    xy, m = _dev(np.zeros((1, 2))), _dev(np.ones(1))
    seg, _ = lf.critical_curves(xy, m, grid=grid, precision="mixed", p=16, caustics=False)
    r = np.hypot(*seg.cpu().numpy().reshape(-1, 2).T)
    print(f"[crit] mixed: {len(seg)} segments, |r - 1| max {np.abs(r - 1).max():.2e}", flush=True)
    assert np.abs(r - 1).max() <= 3 * g.dx ** 2
    lib = _lib.load()
    f = _lib.LensField(1, ctypes.c_void_p(xy.data_ptr()), ctypes.c_void_p(m.data_ptr()), 0.0, 0.0)
    buf = torch.full((10, 4), float("nan"), dtype=torch.float64, device="cuda")
    n = ctypes.c_int64(-1)
    g_c = grid.c()
    o = lf._opts("direct", "fp64", 12)
    assert lib.lens_critical_curves(None, ctypes.byref(f), ctypes.byref(g_c),
                                    ctypes.c_void_p(buf.data_ptr()), None, 10, ctypes.byref(n),
                                    ctypes.byref(o), None) == _lib.LENS_OK
    assert n.value == len(seg)
    assert bool(torch.isfinite(buf).all())
    r10 = np.hypot(*buf.cpu().numpy().reshape(-1, 2).T)
    assert np.abs(r10 - 1).max() <= 3 * g.dx ** 2


def test_multiplane_single_plane_and_no_coupling_on_gpu(lf):
    """On the GPU too: one plane equals lens_deflect, and two planes with
    beta = 0 equal one plane holding both star sets with the smooth terms
    added (explicit rays, FP64 direct sums)."""
    pl = _planes(90)[:2]
    dpl = [(_dev(a), _dev(b), ks, gm) for a, b, ks, gm in pl]
    rays = np.random.default_rng(91).uniform(-8, 8, (3000, 2))
    y1 = lf.deflect_multiplane(dpl[:1], None, rays=_dev(rays), method="direct").cpu().numpy()
    yd = lf.deflect(dpl[0][0], dpl[0][1], rays=_dev(rays), kappa_s=pl[0][2], gamma=pl[0][3],
                    method="direct").cpu().numpy()
    np.testing.assert_allclose(y1, yd, rtol=0, atol=1e-12)
    y2 = lf.deflect_multiplane(dpl, [[0.0, 0.0], [0.0, 0.0]], rays=_dev(rays),
                               method="direct").cpu().numpy()
    xy = np.concatenate([pl[0][0], pl[1][0]])
    mm = np.concatenate([pl[0][1], pl[1][1]])
    yu = lf.deflect(_dev(xy), _dev(mm), rays=_dev(rays), kappa_s=pl[0][2] + pl[1][2],
                    gamma=pl[0][3] + pl[1][3], method="direct").cpu().numpy()
    np.testing.assert_allclose(y2, yu, rtol=0, atol=1e-11)
