"""Pins for the FP64 oracle: each test checks it against something other than
itself -- closed forms, exact rational arithmetic, Gauss's law, Laurent
moments, the paper's printed worked numbers, finite differences and scaling
invariants -- chosen so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ exact arithmetic

def _exact_alpha(stars, masses, ray):
    """Eq. 1 of the paper in exact rational arithmetic; also returns the sum
    of the terms' magnitudes, which bounds the effect of per-term rounding."""
    x1, x2 = Fraction(ray[0]), Fraction(ray[1])
    a1 = a2 = Fraction(0)
    mag = Fraction(0)
    for (s1, s2), m in zip(stars, masses):
        d1, d2 = x1 - Fraction(s1), x2 - Fraction(s2)
        r2 = d1 * d1 + d2 * d2
        if r2 == 0:
            continue
        a1 += Fraction(m) * d1 / r2
        a2 += Fraction(m) * d2 / r2
        mag += abs(Fraction(m) * d1 / r2) + abs(Fraction(m) * d2 / r2)
    return a1, a2, float(mag)


def test_tiny_inputs_match_exact_rationals():
    rng = np.random.default_rng(11)
    stars = rng.uniform(-3, 3, (7, 2))
    masses = rng.uniform(-0.5, 2.0, 7)          # a negative mass too: any finite value is allowed
    rays = rng.uniform(-4, 4, (9, 2))
    rays[0] = stars[3]                          # a ray exactly on a star: pair skipped and counted
    ks, g = 0.125, -0.375
    y, al, skipped = oracle.deflect(stars, masses, rays, ks, g)
    assert skipped == 1
    for k in range(len(rays)):
        e1, e2, mag = _exact_alpha(stars, masses, rays[k])
        ey1 = (1 - Fraction(ks) - Fraction(g)) * Fraction(rays[k, 0]) - e1
        ey2 = (1 - Fraction(ks) + Fraction(g)) * Fraction(rays[k, 1]) - e2
        # each term rounds ~5 times; the compensated sum adds ~1 ulp
        eps = 2.0 ** -52
        assert abs(al[k, 0] - float(e1)) <= 6 * eps * mag + eps * abs(float(e1))
        assert abs(al[k, 1] - float(e2)) <= 6 * eps * mag + eps * abs(float(e2))
        ys = mag + abs(rays[k]).sum() * 2
        assert abs(y[k, 0] - float(ey1)) <= 8 * eps * ys
        assert abs(y[k, 1] - float(ey2)) <= 8 * eps * ys


def test_empty_star_field_and_no_rays():
    rays = np.array([[1.5, -2.0], [0.0, 0.0]])
    y, al, _ = oracle.deflect(np.zeros((0, 2)), np.zeros(0), rays, 0.25, 0.5)
    assert np.all(al == 0.0)
    np.testing.assert_array_equal(y[:, 0], (1 - 0.25 - 0.5) * rays[:, 0])
    np.testing.assert_array_equal(y[:, 1], (1 - 0.25 + 0.5) * rays[:, 1])
    y, al, _ = oracle.deflect(np.ones((3, 2)), np.ones(3), np.zeros((0, 2)))
    assert y.shape == (0, 2)


# ------------------------------------------------------------------ point lens

@pytest.mark.parametrize("m", [1.0, 0.37, 4.2])
def test_point_lens_images_map_back_to_source(m):
    """A point lens of mass m at c has two images of a source at offset u along
    u's direction, at distances (|u| +- sqrt(|u|^2 + 4m))/2 from c."""
    c = np.array([0.75, -1.25])
    rng = np.random.default_rng(3)
    srcs = rng.uniform(-3, 3, (50, 2))
    imgs, want = [], []
    for s in srcs:
        u = s - c
        un = np.hypot(*u)
        e = u / un
        for sgn in (+1, -1):
            imgs.append(c + e * (un + sgn * math.sqrt(un * un + 4 * m)) / 2)
            want.append(s)
    y, _, _ = oracle.deflect(c[None, :], np.array([m]), np.array(imgs))
    np.testing.assert_allclose(y, np.array(want), rtol=0, atol=1e-13)


def test_point_lens_irs_counts_follow_magnification():
    """IRS counts in a small source pixel ~ mu(u) * pixel area / ray cell area
    with mu(u) = (u^2+2)/(u sqrt(u^2+4)) for a unit point lens."""
    g = wl.Grid(x0=-4.0, y0=-4.0, dx=2.0 ** -9, dy=2.0 ** -9, nx=4096, ny=4096)
    rays = g.rays()
    y, _, _ = oracle.deflect(np.zeros((1, 2)), np.ones(1), rays)
    # a 16x16 map of side 0.4 centred on (u0, 0): check the central pixels
    u0 = 0.8
    side, npix = 0.4, 16
    counts, _ = oracle.bin_rays(y, u0 - side / 2, -side / 2, side, npix)
    pix = side / npix
    # aggregate a 4x4 block of pixels around (u0, 0) to beat down grid noise
    block = counts[6:10, 6:10].sum()
    # integrate mu over the block numerically (fine midpoint rule)
    t = (np.arange(400) + 0.5) / 400
    uu = u0 - 2 * pix + 4 * pix * t
    vv = -2 * pix + 4 * pix * t
    U, V = np.meshgrid(uu, vv)
    r = np.hypot(U, V)
    mu = (r * r + 2) / (r * np.sqrt(r * r + 4))
    expect = mu.mean() * (4 * pix) ** 2 / (g.dx * g.dy)
    assert abs(block - expect) / expect < 0.01


def test_point_lens_annulus_preimage_area():
    """Rays landing at source radius u in [u1, u2] come from an image-plane
    area pi[u2 sqrt(u2^2+4m) - u1 sqrt(u1^2+4m)] (both images together)."""
    m = 1.0
    g = wl.Grid(x0=-3.0, y0=-3.0, dx=2.0 ** -8, dy=2.0 ** -8, nx=1536, ny=1536)
    y, _, _ = oracle.deflect(np.zeros((1, 2)), np.array([m]), g.rays())
    u = np.hypot(y[:, 0], y[:, 1])
    u1, u2 = 0.3, 0.9
    area = np.count_nonzero((u >= u1) & (u < u2)) * g.dx * g.dy
    expect = math.pi * (u2 * math.sqrt(u2 ** 2 + 4 * m) - u1 * math.sqrt(u1 ** 2 + 4 * m))
    assert abs(area - expect) / expect < 2e-3


# --------------------------------------------------------------- Chang-Refsdal

@pytest.mark.parametrize("gamma", [0.2, 0.3, 0.6])
def test_chang_refsdal_cusps(gamma):
    """Unit point lens plus shear gamma (kappa_s=0): the critical points on the
    axes, x1 = 1/sqrt(1+gamma) and x2 = 1/sqrt(1-gamma), map to the caustic
    cusps y1 = -2 gamma/sqrt(1+gamma) and y2 = 2 gamma/sqrt(1-gamma), and the
    Jacobian determinant vanishes there."""
    pts = np.array([[1 / math.sqrt(1 + gamma), 0.0], [0.0, 1 / math.sqrt(1 - gamma)]])
    y, _, _ = oracle.deflect(np.zeros((1, 2)), np.ones(1), pts, 0.0, gamma)
    np.testing.assert_allclose(y[0], [-2 * gamma / math.sqrt(1 + gamma), 0.0], atol=1e-14)
    np.testing.assert_allclose(y[1], [0.0, 2 * gamma / math.sqrt(1 - gamma)], atol=1e-14)
    J = oracle.jacobian(np.zeros((1, 2)), np.ones(1), pts)
    for k in range(2):
        A = np.diag([1 - gamma, 1 + gamma]) - np.array([[J[k, 0], J[k, 1]], [J[k, 1], J[k, 2]]])
        assert abs(np.linalg.det(A)) < 1e-13


def test_chang_refsdal_jacobian_closed_form():
    """det A = (1-kappa_s)^2 - |gamma - m / conj(z)^2|^2 for a point lens of mass m at 0."""
    rng = np.random.default_rng(5)
    pts = rng.uniform(-2, 2, (200, 2))
    m, ks, g = 0.8, 0.15, 0.4
    J = oracle.jacobian(np.zeros((1, 2)), np.array([m]), pts)
    A11 = (1 - ks - g) - J[:, 0]
    A22 = (1 - ks + g) - J[:, 2]
    A12 = -J[:, 1]
    det = A11 * A22 - A12 * A12
    z = pts[:, 0] + 1j * pts[:, 1]
    expect = (1 - ks) ** 2 - np.abs(g - m / np.conj(z) ** 2) ** 2
    np.testing.assert_allclose(det, expect, rtol=1e-12, atol=1e-12)


def test_jacobian_matches_finite_differences():
    f = wl.random_field(12, 3.0, seed=8, masses="powerlaw")
    rng = np.random.default_rng(9)
    pts = rng.uniform(-2.5, 2.5, (30, 2))
    J = oracle.jacobian(f.xy, f.m, pts)
    h = 1e-6
    for c in range(2):
        e = np.zeros(2)
        e[c] = h
        _, ap, _ = oracle.deflect(f.xy, f.m, pts + e)
        _, am, _ = oracle.deflect(f.xy, f.m, pts - e)
        fd = (ap - am) / (2 * h)
        Jc = np.stack([J[:, 0], J[:, 1]], 1) if c == 0 else np.stack([J[:, 1], J[:, 2]], 1)
        np.testing.assert_allclose(fd, Jc, rtol=1e-5, atol=1e-5)


# ----------------------------------------------------------------- Gauss's law

def test_gauss_flux_through_circle():
    """The flux of alpha through a circle is 2 pi times the enclosed mass, so
    the mean normal component over the circle is M_in/rho and the mean
    tangential component is 0 (2-D Gauss's law for eq. 1)."""
    rng = np.random.default_rng(21)
    rho = 2.0
    xy = wl.uniform_disk(rng, 400, 4.0)
    r = np.hypot(xy[:, 0], xy[:, 1])
    keep = np.abs(r - rho) > 0.25
    xy = xy[keep]
    m = rng.uniform(0.2, 1.5, xy.shape[0])
    n = 4096
    th = 2 * math.pi * np.arange(n) / n
    nrm = np.stack([np.cos(th), np.sin(th)], 1)
    _, al, _ = oracle.deflect(xy, m, rho * nrm)
    normal = (al * nrm).sum(1).mean()
    tang = (al[:, 1] * nrm[:, 0] - al[:, 0] * nrm[:, 1]).mean()
    m_in = m[np.hypot(xy[:, 0], xy[:, 1]) < rho].sum()
    assert abs(normal - m_in / rho) < 1e-10 * (m.sum() / rho)
    assert abs(tang) < 1e-10 * (m.sum() / rho)


def test_uniform_disk_mean_field():
    """Inside a uniform disk of point masses the deflection averages to
    kappa_* x with kappa_* = sum(m)/R^2 (the reading used for the workloads)."""
    f = wl.random_field(20000, 20.0, seed=13)
    rng = np.random.default_rng(14)
    # the flux identity gives the mean over a circle exactly; the disk's
    # enclosed mass fluctuates, so compare with kappa_* times radius loosely
    n = 1024
    rho = 10.0
    th = 2 * math.pi * np.arange(n) / n
    nrm = np.stack([np.cos(th), np.sin(th)], 1)
    _, al, _ = oracle.deflect(f.xy, f.m, rho * nrm)
    normal = (al * nrm).sum(1).mean()
    assert abs(normal - f.kappa_star * rho) / (f.kappa_star * rho) < 0.02
    del rng


# ------------------------------------------------------------------- far field

def test_far_field_laurent_moments():
    """Far from a compact cluster alpha = conj(sum_k M_k / z^(k+1)) with the
    exact moments M_k = sum_i m_i z_i^k (the multipole form of Appendix A)."""
    rng = np.random.default_rng(4)
    xy = rng.uniform(-1, 1, (50, 2))
    m = rng.uniform(0.1, 2.0, 50)
    zi = xy[:, 0] + 1j * xy[:, 1]
    th = rng.uniform(0, 2 * math.pi, 64)
    z = 40.0 * np.exp(1j * th)
    series = np.zeros_like(z)
    for k in range(40):
        series += np.sum(m * zi ** k) / z ** (k + 1)
    _, al, _ = oracle.deflect(xy, m, np.stack([z.real, z.imag], 1))
    got = al[:, 0] + 1j * al[:, 1]
    np.testing.assert_allclose(got, np.conj(series), rtol=1e-13, atol=0)


# ---------------------------------------------------------- macro magnification

def test_macro_magnification_printed_values():
    """With no lenses the map is linear; its Jacobian gives mu = 1/det, which
    must reproduce the paper's printed worked values."""
    cases = json.load(open(os.path.join(GOLDEN, "macro_magnification.json")))["cases"]
    pts = np.array([[0.3, -0.7], [1.9, 2.2]])
    for c in cases:
        h = 0.5
        y0, _, _ = oracle.deflect(np.zeros((0, 2)), np.zeros(0), pts, c["kappa"], c["gamma"])
        y1, _, _ = oracle.deflect(np.zeros((0, 2)), np.zeros(0), pts + [h, 0], c["kappa"], c["gamma"])
        y2, _, _ = oracle.deflect(np.zeros((0, 2)), np.zeros(0), pts + [0, h], c["kappa"], c["gamma"])
        A = np.stack([(y1 - y0) / h, (y2 - y0) / h], -1)    # [n, 2, 2]
        mu = 1.0 / np.linalg.det(A)
        tol = 0.5 * 10 ** (math.floor(math.log10(abs(c["mu"]))) - c["printed_digits"] + 1)
        assert np.all(np.abs(mu - c["mu"]) <= tol), (c, mu)


def test_macro_magnification_irs_counts():
    """IRS under the smooth field alone: counts per pixel = |mu| * pixel area /
    ray cell area, up to the grid's edge effects (kappa=gamma=0.3, mu=2.5)."""
    g = wl.Grid(x0=-8.0, y0=-8.0, dx=2.0 ** -6, dy=2.0 ** -6, nx=1024, ny=1024)
    y, _, _ = oracle.deflect(np.zeros((0, 2)), np.zeros(0), g.rays(), 0.3, 0.3)
    counts, landed = oracle.bin_rays(y, -0.5, -0.5, 1.0, 4)
    expect = 2.5 * 0.25 ** 2 / (g.dx * g.dy)
    assert abs(counts.mean() - expect) / expect < 0.02
    assert landed == counts.sum()


# --------------------------------------------------------------------- binning

def test_binning_half_open_pixels():
    pts = np.array([
        [-1.0, -1.0],          # lower-left corner: pixel (0, 0)
        [-0.5, -1.0],          # exactly on the edge between u=0 and u=1 -> u=1
        [1.0, 0.0],            # upper map edge in y1: outside (half-open)
        [0.999999, 0.999999],  # last pixel
        [-1.0000001, 0.0],     # just left of the map: dropped
        [np.nan, 0.0],         # NaN: dropped
        [0.0, -0.5],           # u = 2, v = 1
        [-0.5 - 2.0 ** -40, 0.5 - 2.0 ** -40],   # just below both edges: u = 0, v = 2
    ])
    counts, landed = oracle.bin_rays(pts, -1.0, -1.0, 2.0, 4)
    want = np.zeros((4, 4), np.int32)
    want[0, 0] = 1
    want[0, 1] = 1
    want[3, 3] = 1
    want[1, 2] = 1
    want[2, 0] = 1
    np.testing.assert_array_equal(counts, want)
    assert landed == 5
    counts2, _ = oracle.bin_rays(pts, -1.0, -1.0, 2.0, 4, counts=counts)
    np.testing.assert_array_equal(counts2, 2 * want)


def test_binning_overflow_is_reported():
    c = np.zeros((2, 2), np.int32)
    c[0, 0] = np.iinfo(np.int32).max
    with pytest.raises(OverflowError):
        oracle.bin_rays(np.array([[0.1, 0.1]]), 0.0, 0.0, 1.0, 2, counts=c)


# -------------------------------------------------------------------- gradient

def _loss(f, rays, t, xy=None, m=None):
    y, _, _ = oracle.deflect(f.xy if xy is None else xy, f.m if m is None else m, rays,
                             f.kappa_s, f.gamma)
    return float(((y - t) ** 2).sum()), y


def test_gradient_matches_central_differences():
    f = wl.random_field(6, 2.0, seed=31, masses="powerlaw", kappa_s=0.1, gamma=0.2)
    rng = np.random.default_rng(32)
    rays = rng.uniform(-2.5, 2.5, (40, 2))
    t = rng.uniform(-2, 2, (40, 2))
    L0, y = _loss(f, rays, t)
    G = 2 * (y - t)
    gxy, gm = oracle.grad(f.xy, f.m, rays, G)
    h = 1e-6
    for i in range(f.n):
        for c in range(2):
            xp = f.xy.copy()
            xp[i, c] += h
            xm = f.xy.copy()
            xm[i, c] -= h
            fd = (_loss(f, rays, t, xy=xp)[0] - _loss(f, rays, t, xy=xm)[0]) / (2 * h)
            assert abs(fd - gxy[i, c]) <= 1e-6 * max(1.0, abs(gxy[i, c]))
        mp = f.m.copy()
        mp[i] += h
        mm = f.m.copy()
        mm[i] -= h
        fd = (_loss(f, rays, t, m=mp)[0] - _loss(f, rays, t, m=mm)[0]) / (2 * h)
        assert abs(fd - gm[i]) <= 1e-6 * max(1.0, abs(gm[i]))


def test_gradient_invariants():
    """Mass homogeneity: sum_i m_i dL/dm_i = -sum_k G_k . alpha_k.
    Translation: moving every star by e equals moving every ray by -e, so
    sum_i dL/dx_i = sum_k J(x_k) G_k with J the deflection Jacobian."""
    f = wl.random_field(30, 3.0, seed=41, masses="powerlaw")
    rng = np.random.default_rng(42)
    rays = rng.uniform(-3, 3, (200, 2))
    G = rng.standard_normal((200, 2))
    gxy, gm = oracle.grad(f.xy, f.m, rays, G)
    _, al, _ = oracle.deflect(f.xy, f.m, rays)
    lhs = (f.m * gm).sum()
    rhs = -(G * al).sum()
    assert abs(lhs - rhs) <= 1e-12 * np.abs(G * al).sum()
    J = oracle.jacobian(f.xy, f.m, rays)
    t1 = (J[:, 0] * G[:, 0] + J[:, 1] * G[:, 1]).sum()
    t2 = (J[:, 1] * G[:, 0] + J[:, 2] * G[:, 1]).sum()
    scale = np.abs(J).sum() * np.abs(G).max()
    assert abs(gxy[:, 0].sum() - t1) <= 1e-12 * scale
    assert abs(gxy[:, 1].sum() - t2) <= 1e-12 * scale


# ------------------------------------------------------------------ workloads

def test_workload_readings():
    f, g, mp = wl.small_disk()
    assert f.n == 1000 and abs(f.kappa_star - 1000 / 26.6 ** 2) < 1e-12
    assert g.dx == 10 / 512 and g.rays()[0, 0] == -5 + 0.5 * 10 / 512
    f2, g2 = wl.powerlaw_disk(n_stars=20000, n_side=256)
    assert abs(f2.m.mean() - 1.0) < 1e-12
    assert 0.44 < f2.m.min() and f2.m.max() < 4.5
    assert abs(f2.kappa_star - 0.4) < 1e-12
    # dyadic grid: every coordinate is exact, so any evaluation order agrees
    r = g2.rays()
    i = np.arange(g2.n) % g2.nx
    assert np.all(r[:, 0] == g2.x0 + (i + 0.5) * g2.dx)
    assert (g2.dx * 2 ** 20) == round(g2.dx * 2 ** 20)


# ----------------------------------------------------------------------- IPM
# Inverse polygon mapping (Section 2.3, first order): each image-plane cell's
# area is shared among the source pixels its mapped quadrilateral overlaps.

def _convex_overlap_exact(poly, u, v):
    """Area of convex polygon `poly` (Fractions) inside [u,u+1]x[v,v+1], by a
    different route than clipping: the intersection of two convex polygons is
    the hull of the vertices of each inside the other and the crossings of
    their edges."""
    F = Fraction
    sq = [(F(u), F(v)), (F(u + 1), F(v)), (F(u + 1), F(v + 1)), (F(u), F(v + 1))]

    def inside(pt, pg):
        sgn = 0
        for k in range(len(pg)):
            a, b = pg[k], pg[(k + 1) % len(pg)]
            c = (b[0] - a[0]) * (pt[1] - a[1]) - (b[1] - a[1]) * (pt[0] - a[0])
            if c != 0:
                if sgn == 0:
                    sgn = 1 if c > 0 else -1
                elif (c > 0) != (sgn > 0):
                    return False
        return True

    pts = [p for p in poly if inside(p, sq)] + [p for p in sq if inside(p, poly)]
    for k in range(len(poly)):
        a, b = poly[k], poly[(k + 1) % len(poly)]
        for q in range(4):
            c, d = sq[q], sq[(q + 1) % 4]
            den = (b[0] - a[0]) * (d[1] - c[1]) - (b[1] - a[1]) * (d[0] - c[0])
            if den == 0:
                continue
            t = ((c[0] - a[0]) * (d[1] - c[1]) - (c[1] - a[1]) * (d[0] - c[0])) / den
            s = ((c[0] - a[0]) * (b[1] - a[1]) - (c[1] - a[1]) * (b[0] - a[0])) / den
            if 0 <= t <= 1 and 0 <= s <= 1:
                pts.append((a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])))
    pts = list(set(pts))
    if len(pts) < 3:
        return Fraction(0)
    # convex hull (monotone chain) and its area
    pts.sort()

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])
    lo, hi = [], []
    for p in pts:
        while len(lo) >= 2 and cross(lo[-2], lo[-1], p) <= 0:
            lo.pop()
        lo.append(p)
    for p in reversed(pts):
        while len(hi) >= 2 and cross(hi[-2], hi[-1], p) <= 0:
            hi.pop()
        hi.append(p)
    hull = lo[:-1] + hi[:-1]
    return abs(sum(hull[k][0] * hull[(k + 1) % len(hull)][1] - hull[(k + 1) % len(hull)][0] * hull[k][1]
                   for k in range(len(hull)))) / 2


def _one_cell(corners, dx=0.5, dy=0.25, npix=8, side=8.0):
    """A 2x2 grid (one cell) whose corners map to `corners` (source plane,
    map [0, side)^2 so pixel units equal source units when side == npix)."""
    y = np.array([[corners[0], corners[1]], [corners[3], corners[2]]], dtype=np.float64)
    return oracle.ipm(y, dx * dy, 0.0, 0.0, side, npix)


def _tri_area(t):
    return abs((t[1][0] - t[0][0]) * (t[2][1] - t[0][1]) - (t[1][1] - t[0][1]) * (t[2][0] - t[0][0])) / 2


@pytest.mark.parametrize("corners", [
    [(1.25, 1.5), (5.75, 2.0), (4.5, 6.625), (0.5, 3.25)],        # convex, counter-clockwise
    [(0.5, 3.25), (4.5, 6.625), (5.75, 2.0), (1.25, 1.5)],        # same, clockwise (parity flip)
    [(2.0, 2.0), (2.75, 2.125), (2.5, 2.875), (2.125, 2.5)],      # inside one pixel... and two
])
def test_ipm_convex_cell_matches_exact_overlaps(corners):
    mu = _one_cell(corners)
    F = Fraction
    poly = [(F(x), F(y)) for x, y in corners]
    area = abs(sum(poly[k][0] * poly[(k + 1) % 4][1] - poly[(k + 1) % 4][0] * poly[k][1]
                   for k in range(4))) / 2
    cell = F(1, 8)   # dx dy in pixel units (pixel side 1)
    for v in range(8):
        for u in range(8):
            want = float(cell * _convex_overlap_exact(poly, u, v) / area)
            assert abs(mu[v, u] - want) <= 1e-15 + 1e-13 * want, (u, v, mu[v, u], want)
    assert abs(mu.sum() - 0.125) <= 1e-14


def test_ipm_concave_cell_splits_into_triangles():
    # reflex vertex at index 3: the quad is the union of triangles (0,1,3), (1,2,3)
    corners = [(1.0, 1.0), (6.5, 1.5), (5.5, 6.0), (3.25, 2.75)]
    mu = _one_cell(corners)
    F = Fraction
    P = [(F(x), F(y)) for x, y in corners]
    t1, t2 = [P[0], P[1], P[3]], [P[1], P[2], P[3]]

    def tri_area(t):
        return abs((t[1][0] - t[0][0]) * (t[2][1] - t[0][1]) - (t[1][1] - t[0][1]) * (t[2][0] - t[0][0])) / 2
    area = tri_area(t1) + tri_area(t2)
    for v in range(8):
        for u in range(8):
            ov = _convex_overlap_exact(t1, u, v) + _convex_overlap_exact(t2, u, v)
            want = float(F(1, 8) * ov / area)
            assert abs(mu[v, u] - want) <= 1e-15 + 1e-13 * want


def test_ipm_wide_cell_is_apportioned_exactly():
    """A cell stretched over ~600 pixels of a 32^2 map (as next to a star) is
    still shared exactly by overlap: Section 2.3 apportions every cell."""
    corners = [(2.25, 3.5), (29.75, 6.125), (27.5, 25.625), (4.5, 21.25)]
    mu = _one_cell(corners, npix=32, side=32.0)
    F = Fraction
    poly = [(F(x), F(y)) for x, y in corners]
    area = abs(sum(poly[k][0] * poly[(k + 1) % 4][1] - poly[(k + 1) % 4][0] * poly[k][1]
                   for k in range(4))) / 2
    for v in range(32):
        for u in range(32):
            want = float(F(1, 8) * _convex_overlap_exact(poly, u, v) / area)
            assert abs(mu[v, u] - want) <= 1e-15 + 1e-12 * want, (u, v, mu[v, u], want)
    assert np.count_nonzero(mu) > 500
    assert abs(mu.sum() - 0.125) <= 1e-13


@pytest.mark.parametrize("corners", [
    [(1.5, 1.5), (5.5, 5.5), (5.5, 1.5), (1.5, 5.5)],            # edges 0-1 and 2-3 cross
    [(1.25, 2.0), (6.5, 1.5), (1.75, 6.25), (5.75, 5.5)],         # edges 1-2 and 3-0 cross
])
def test_ipm_folded_cell_spreads_over_its_lobes(corners):
    """A critical cell (its image's edges cross) is treated as if it were not
    critical (Section 2.3): the region its edges enclose, the two triangles
    on either side of the crossing point, takes the cell's area by overlap."""
    mu = _one_cell(corners)
    F = Fraction
    P = [(F(x), F(y)) for x, y in corners]

    def crossing(a, b, c, d):
        den = (b[0] - a[0]) * (d[1] - c[1]) - (b[1] - a[1]) * (d[0] - c[0])
        t = ((c[0] - a[0]) * (d[1] - c[1]) - (c[1] - a[1]) * (d[0] - c[0])) / den
        return (a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])), 0 < t < 1
    X, ok = crossing(P[0], P[1], P[2], P[3])
    if ok:
        lobes = [[X, P[1], P[2]], [P[0], X, P[3]]]
    else:
        X, ok = crossing(P[1], P[2], P[3], P[0])
        lobes = [[P[0], P[1], X], [X, P[2], P[3]]]
    assert ok
    area = sum(_tri_area(t) for t in lobes)
    for v in range(8):
        for u in range(8):
            ov = sum(_convex_overlap_exact(t, u, v) for t in lobes)
            want = float(F(1, 8) * ov / area)
            assert abs(mu[v, u] - want) <= 1e-15 + 1e-13 * want, (u, v, mu[v, u], want)
    assert abs(mu.sum() - 0.125) <= 1e-14


def test_ipm_zero_area_cell_goes_to_its_corners():
    corners = [(1.5, 1.5), (3.5, 3.5), (5.5, 5.5), (2.5, 2.5)]   # all on one line
    mu = _one_cell(corners)
    want = np.zeros((8, 8))
    for x, y in corners:
        want[int(y), int(x)] += 0.125 / 4
    np.testing.assert_allclose(mu, want, rtol=0, atol=1e-16)


def _point_lens_pixel_average(npix, side):
    """Exact pixel averages of the point lens's total magnification
    mu(u) = (u^2+2)/(u sqrt(u^2+4)) over an npix^2 map centred on the lens
    (midpoint rule, 64^2 points per pixel; 2048^2 around the caustic point,
    where mu ~ 1/u)."""
    h = side / npix
    lo = -side / 2

    def mu(x, y):
        u = np.hypot(x, y)
        return (u * u + 2) / (u * np.sqrt(u * u + 4))
    g = (np.arange(64) + 0.5) / 64 * h
    ref = np.empty((npix, npix))
    xs = (lo + np.arange(npix)[:, None] * h + g[None, :]).ravel()
    for v in range(npix):
        ys = lo + v * h + g
        ref[v] = mu(xs[None, :], ys[:, None]).reshape(64, npix, 64).mean(axis=(0, 2))
    c = npix // 2
    g2 = (np.arange(2048) + 0.5) / 2048 * h
    for v in range(c - 2, c + 2):
        for u in range(c - 2, c + 2):
            ref[v, u] = mu(lo + u * h + g2[None, :], lo + v * h + g2[:, None]).mean()
    return ref


@pytest.mark.parametrize("n,bound", [(384, 7.5e-3), (768, 3e-3)])
def test_ipm_point_lens_whole_map_against_analytic(n, bound):
    """External pin of the whole first-order IPM, folded cells included: a
    point lens shot with n^2 grid rays over [-3,3]^2 (n0 = 1 and 4 rays per
    unlensed pixel) into a 128^2 map over [-1,1]^2 that contains the caustic
    point (cells along the Einstein ring fold).  Against the analytic
    pixel-averaged magnification the relative L1 error is 6.4e-3 and 1.5e-3
    (a zeroth-order treatment of the folded cells gives 8.6e-3 at n0 = 1,
    and inverse ray shooting of the same rays 0.30 and 0.10)."""
    npix, side = 128, 2.0
    ref = _point_lens_pixel_average(npix, side)
    dx = 6.0 / n
    xs = -3.0 + (np.arange(n) + 0.5) * dx
    X, Y = np.meshgrid(xs, xs)
    r2 = X * X + Y * Y
    yg = np.stack([X - X / r2, Y - Y / r2], -1)
    mu = oracle.ipm(yg, dx * dx, -1.0, -1.0, side, npix)
    l1 = np.abs(mu - ref).sum() / ref.sum()
    counts, _ = oracle.bin_rays(yg.reshape(-1, 2), -1.0, -1.0, side, npix)
    irs = counts * dx * dx / (side / npix) ** 2
    l1_irs = np.abs(irs - ref).sum() / ref.sum()
    print(f"point lens n={n}: IPM L1 {l1:.2e}, IRS L1 {l1_irs:.2e}")
    assert l1 <= bound
    assert l1 <= l1_irs / 20


@pytest.mark.parametrize("M", [((0.7, 0.0), (0.0, 1.3)), ((0.45, -0.62), (0.81, 0.2)),
                               ((-0.5, 0.3), (0.4, 0.9))])
def test_ipm_linear_map_gives_inverse_determinant(M):
    """Under y = M x every cell is a parallelogram of area |det M| dx dy, so
    every pixel the grid's image covers has mu = 1/|det M| exactly."""
    M = np.array(M)
    n = 241
    xs = np.linspace(-12.0, 12.0, n)
    X, Y = np.meshgrid(xs, xs)
    pts = np.stack([X, Y], -1)
    yg = pts @ M.T
    dx = xs[1] - xs[0]
    mu = oracle.ipm(yg, dx * dx, -2.0, -2.0, 4.0, 32)
    np.testing.assert_allclose(mu, 1.0 / abs(np.linalg.det(M)), rtol=1e-12)


def test_ipm_conserves_area_of_a_curved_mapping():
    xs = np.linspace(0.0, 1.0, 65)
    X, Y = np.meshgrid(xs, xs)
    yg = np.stack([2.0 + 3.0 * X + 0.2 * np.sin(5 * Y), 2.0 + 2.5 * Y + 0.15 * np.cos(4 * X)], -1)
    mu = oracle.ipm(yg, (xs[1] - xs[0]) ** 2, 0.0, 0.0, 8.0, 16)
    assert abs(mu.sum() * (8.0 / 16) ** 2 - 1.0) <= 1e-12


def test_ipm_point_lens_matches_analytic_magnification():
    """Point lens: the IPM map of a fine grid approaches the pixel average of
    mu(u) = (u^2+2)/(u sqrt(u^2+4)) (sum of both images) away from the caustic."""
    n = 2048   # even: no grid point on the lens
    xs = np.linspace(-3.0, 3.0, n)
    X, Y = np.meshgrid(xs, xs)
    r2 = X * X + Y * Y
    yg = np.stack([X - X / r2, Y - Y / r2], -1)
    side, npix = 2.0, 8
    mu = oracle.ipm(yg, (xs[1] - xs[0]) ** 2, -1.0, -1.0, side, npix)
    h = side / npix
    g = (np.arange(64) + 0.5) / 64
    for v in range(npix):
        for u in range(npix):
            cx, cy = -1.0 + (u + g) * h, -1.0 + (v + g[:, None]) * h
            uu = np.hypot(cx, cy)
            if uu.min() < 0.35:
                continue   # near the caustic point
            ana = ((uu ** 2 + 2) / (uu * np.sqrt(uu ** 2 + 4))).mean()
            assert abs(mu[v, u] / ana - 1) < 2e-3, (u, v, mu[v, u], ana)


# ------------------------------------------------------------- multi-plane

def _plane(seed, n, R, ks, g):
    f = wl.random_field(n, R, seed=seed, masses="powerlaw")
    return (f.xy, f.m, ks, g)


def test_multiplane_one_plane_is_the_single_plane_map():
    pl = _plane(31, 40, 3.0, 0.2, 0.1)
    rays = np.random.default_rng(32).uniform(-4, 4, (300, 2))
    y = oracle.multiplane([pl], None, rays)
    y1, _, _ = oracle.deflect(pl[0], pl[1], rays, pl[2], pl[3])
    np.testing.assert_allclose(y, y1, rtol=0, atol=1e-13)   # x - (x - y1) rounds once


def test_multiplane_without_coupling_is_superposition():
    """beta_10 = 0: the second plane sees the unlensed ray, so the two planes
    act as one plane holding both sets of stars, with the smooth terms
    added.  The unused upper triangle of beta holds garbage on purpose."""
    a, b = _plane(33, 30, 3.0, 0.1, 0.2), _plane(34, 25, 2.0, 0.15, -0.05)
    rays = np.random.default_rng(35).uniform(-4, 4, (300, 2))
    y = oracle.multiplane([a, b], [[0.0, 0.9], [0.0, 0.0]], rays)
    yu, _, _ = oracle.deflect(np.concatenate([a[0], b[0]]), np.concatenate([a[1], b[1]]), rays,
                              a[2] + b[2], a[3] + b[3])
    np.testing.assert_allclose(y, yu, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("b10", [0.3, 0.75])
def test_multiplane_smooth_sheets_compose_as_linear_maps(b10):
    """Two planes of smooth convergence and shear only, K_j = diag(kappa_j +
    gamma_j, kappa_j - gamma_j) (alpha_j(x) = K_j x): y = (I - K0 - K1 +
    beta_10 K1 K0) x, the two-plane cross term of the recursion."""
    k0, g0, k1, g1 = 0.3, 0.12, 0.2, -0.07
    K0, K1 = np.diag([k0 + g0, k0 - g0]), np.diag([k1 + g1, k1 - g1])
    rays = np.random.default_rng(36).uniform(-5, 5, (50, 2))
    empty = (np.zeros((0, 2)), np.zeros(0))
    y = oracle.multiplane([(*empty, k0, g0), (*empty, k1, g1)], [[0.0, -3.0], [b10, 0.0]], rays)
    M = np.eye(2) - K0 - K1 + b10 * K1 @ K0
    np.testing.assert_allclose(y, rays @ M.T, rtol=1e-14, atol=1e-14)


def test_multiplane_two_point_lenses_on_the_axis():
    """Point masses m0, m1 at the origin of two planes, a ray on the x1 axis
    at r: x_1 = r - beta m0 / r and y = r - m0 / r - m1 / x_1."""
    m0, m1, b, r = 0.7, 1.3, 0.4, 1.7
    y = oracle.multiplane([(np.zeros((1, 2)), np.array([m0]), 0.0, 0.0),
                           (np.zeros((1, 2)), np.array([m1]), 0.0, 0.0)],
                          [[0.0, 0.0], [b, 0.0]], np.array([[r, 0.0]]))
    x1 = r - b * m0 / r
    np.testing.assert_allclose(y[0], [r - m0 / r - m1 / x1, 0.0], rtol=1e-15, atol=1e-15)
