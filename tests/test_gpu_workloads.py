"""GPU checks of the two large workloads of the paper's applications: a galaxy
halo of 1.575e7 particles (Section 2.5) and the anamorphic shooting region of
a magnified star behind a cluster (Section 3.3), both at full size, against
the FP64 oracle on sampled rays and through properties that hold at any
size."""
import math
import time

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


def _ray_errors(y, y_ref, alpha_ref):
    d = np.hypot(*(y - y_ref).T)
    a = np.hypot(*alpha_ref.T)
    r = d / np.maximum(a, 1e-3 * float(np.sqrt(np.mean(a * a))))
    return float(np.linalg.norm(y - y_ref) / np.linalg.norm(alpha_ref)), float(r.max())


def _lfgrid(lf, g):
    return lf.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)


def test_synthetic_halo_full_size(lf):
    """1.575e7 particles of four kinds (dark matter, gas, stars, black holes)
    with masses from 5e-4 to 0.03 and densities from a cusp to a sparse
    envelope 1500 Einstein radii out, 4000^2 rays over the central 90 x 90:
    mixed precision with the order chosen for 1e-5 and FP64 at p = 30,
    against the oracle on ~1000 strided rays, per ray."""
    import torch
    import paper_2211_00354_amd as lf
    _say("halo: generating 1.575e7 particles")
    f, g = wl.synthetic_halo()
    xy, m = _dev(f.xy), _dev(f.m)
    idx = g.strided(128, 61)
    t0 = time.perf_counter()
    yo, ao, _ = oracle.deflect(f.xy, f.m, g.rays(idx), f.kappa_s, f.gamma)
    print(f"[halo] oracle: {len(idx)} rays in {time.perf_counter() - t0:.1f} s", flush=True)
    kw = dict(grid=_lfgrid(lf, g), kappa_s=f.kappa_s, gamma=f.gamma)
    for prec, p, tol, rel_tol, ray_tol in (("mixed", 0, 1e-5, 1e-5, 1e-5),
                                          ("fp64", 30, 0.0, 1e-10, 1e-10)):
        _say("halo", prec, p, tol)
        y = lf.deflect(xy, m, precision=prec, p=p, tol=tol, **kw)   # tunes (p=0) and warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = lf.deflect(xy, m, precision=prec, p=p, tol=tol, out=y, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ys = y[torch.from_numpy(idx).cuda()].cpu().numpy()
        assert bool(torch.isfinite(y).all())
        del y
        rel, mx = _ray_errors(ys, yo, ao)
        print(f"[err] halo {prec} p={p} tol={tol}: rel_l2 {rel:.2e} ray_max {mx:.2e}; "
              f"{dt * 1e3:.1f} ms -> {g.n / dt:.3e} rays/s", flush=True)
        assert rel <= rel_tol and mx <= ray_tol, (prec, rel, mx)
    lf.release_cached()


def _arc_setup(lf):
    f, g, mp = wl.anamorphic_arc()
    xy, m = _dev(f.xy), _dev(f.m)
    # a magnification of 4200 makes y a small difference of terms ~50: a
    # 1e-4 bin-reassignment rate at 0.001 per pixel needs |dy| ~ 1e-7, so
    # every M2L level runs in FP64 (the near field stays FP32) at p = 24
    plan = lf.Plan(xy, m, grid=_lfgrid(lf, g), kappa_s=f.kappa_s, gamma=f.gamma,
                   precision="mixed", p=24, fp32_levels=-1)
    md = lf.MapDesc(mp.y1min, mp.y2min, mp.side, mp.npix)
    return f, g, mp, plan, md


def test_anamorphic_arc_full_size_streams_through_one_plan(lf):
    """The 15000 x 10 Einstein-radius region of Section 3.3, one ray per
    0.001 (1.5e11 rays), 1.8e6 deflectors, mapped by inverse polygon mapping
    onto a 4000^2 map in passes of 2^28 rays through one plan.  Checks: the
    grid path's deflections on sampled rays of three rows against the
    oracle (expected bin reassignment), a finite non-negative map whose mean
    is the macro magnification ~4200, and the map's independence of the pass
    size on a 100-row band (bit-identical: fixed-point sums)."""
    import torch
    import paper_2211_00354_amd as lf
    _say("arc: generating 1.8e6 deflectors")
    f, g, mp, plan, md = _arc_setup(lf)
    info = plan.info()
    print(f"[arc] plan {info}", flush=True)
    kw = dict(kappa_s=f.kappa_s, gamma=f.gamma, plan=plan)
    S = mp.npix / mp.side
    # deflections of three grid rows through the plan's grid path
    for j0 in (0, g.ny // 2 - 1, g.ny - 3):
        sub = wl.Grid(x0=g.x0, y0=g.y0 + j0 * g.dy, dx=g.dx, dy=g.dy, nx=g.nx, ny=3)
        _say("arc rows", j0)
        y = lf.deflect(grid=_lfgrid(lf, sub), **kw)
        assert bool(torch.isfinite(y).all())
        idx = np.random.default_rng(j0).integers(0, sub.n, 600)
        ys = y[torch.from_numpy(idx).cuda()].cpu().numpy()
        del y
        yo, ao, _ = oracle.deflect(f.xy, f.m, sub.rays(idx), f.kappa_s, f.gamma)
        d = np.abs(ys - yo).sum(1) * S
        print(f"[err] arc rows {j0}: reassignment estimate {d.mean():.2e}, max |dy| "
              f"{d.max():.2e} px, |alpha| up to {np.hypot(*ao.T).max():.1f}", flush=True)
        assert d.mean() <= 1e-4 and d.max() <= 1e-2, (j0, d.mean(), d.max())
    # the whole region
    _say("arc: full IPM map, 1.5e11 rays")
    mu = torch.zeros((mp.npix, mp.npix), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lf.ipm_map(grid=_lfgrid(lf, g), map=md, mu=mu, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mean = float(mu.mean())
    print(f"[arc] {g.n:.3e} rays in {dt:.2f} s -> {g.n / dt:.3e} rays/s; mean mu {mean:.1f} "
          f"(macro {f.meta['mu_macro']:.1f}), max {float(mu.max()):.3e}", flush=True)
    assert bool(torch.isfinite(mu).all()) and float(mu.min()) >= 0.0
    assert abs(mean / f.meta["mu_macro"] - 1.0) < 0.25, mean
    del mu
    # the pass size does not change the map (100-row band: one pass of 1.5e9
    # rays against 99 passes of two ray rows)
    band = wl.Grid(x0=g.x0, y0=g.y0 + 4000 * g.dy, dx=g.dx, dy=g.dy, nx=g.nx, ny=100)
    maps = []
    for chunk in (band.n, 1 << 25):
        _say("arc band, rays per pass", chunk)
        maps.append(lf.ipm_map(grid=_lfgrid(lf, band), map=md, max_rays_per_chunk=chunk, **kw))
        torch.cuda.synchronize()
    assert float(maps[0].sum()) > 0
    assert torch.equal(maps[0], maps[1])
    del maps
    plan.close()
    lf.release_cached()


def test_eighty_million_deflectors(lf):
    """The largest fields the paper reports handling (Section 4: up to 8e7
    microlenses, kappa = gamma = 0.3): 8e7 unit masses in a disk of
    convergence 0.3 with gamma = 0.3, 4096^2 rays over the central 2000 x
    2000 Einstein radii, mixed p = 12; 256 rays against the oracle, per ray."""
    import torch
    import paper_2211_00354_amd as lf
    n = 80_000_000
    rng = np.random.default_rng(80)
    R = math.sqrt(n / 0.3)
    _say("8e7 deflectors: generating")
    xy = torch.from_numpy(wl.uniform_disk(rng, n, R)).cuda()
    m = torch.ones(n, dtype=torch.float64, device="cuda")
    g = wl.centred_grid(2000.0, 2000.0, 4096, 4096)
    kw = dict(grid=_lfgrid(lf, g), kappa_s=0.0, gamma=0.3, precision="mixed", p=12)
    _say("8e7 deflectors: deflect")
    y = lf.deflect(xy, m, **kw)                 # builds and warms the call
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y = lf.deflect(xy, m, out=y, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    idx = np.random.default_rng(81).integers(0, g.n, 256)
    ys = y[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert bool(torch.isfinite(y).all())
    del y
    xy_h, m_h = xy.cpu().numpy(), m.cpu().numpy()
    del xy, m
    t1 = time.perf_counter()
    yo, ao, _ = oracle.deflect(xy_h, m_h, g.rays(idx), 0.0, 0.3)
    rel, mx = _ray_errors(ys, yo, ao)
    print(f"[err] 8e7 deflectors: rel_l2 {rel:.2e} ray_max {mx:.2e}; {dt * 1e3:.1f} ms -> "
          f"{g.n / dt:.3e} rays/s (oracle {time.perf_counter() - t1:.1f} s)", flush=True)
    assert rel <= 1e-5 and mx <= 1e-4, (rel, mx)
    lf.release_cached()
