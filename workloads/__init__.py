"""Seeded synthetic inputs shaped like the paper's microlensing workloads.

This module only draws inputs: star positions and masses, ray grids or ray
positions, map placements and loss targets.  It holds none of the lensing
arithmetic, imports neither the GPU package nor the oracle, and serves both
sides of every parity test and the benchmark.

The paper's star fields are its own synthetic ones (Section 4 draws point
lenses uniformly over a region with a chosen convergence; Section 2.3 asks
that the lenses fill a circle circumscribing the rectangular shooting region,
by the 2-D shell theorem), so every workload here is synthetic:

* positions uniform in a disk: ``u = rng.random((N, 2))``, ``r = R sqrt(u0)``,
  ``theta = 2 pi u1``, centred on the origin;
* the disk radius for a target convergence is ``R = sqrt(sum(m) / kappa_star)``
  (a uniform sheet of point masses of surface number density n deflects by
  ``pi n m x``, so ``kappa_star = pi n m = sum(m) / R**2`` in Einstein-radius
  units of unit mass);
* power-law masses ``dN/dm ~ m**-2.35`` on [0.1, 1] by inverse CDF, then
  rescaled so that the sample mean is exactly 1;
* ray grids are cell-centred, ray ``k = j*nx + i`` at
  ``(x0 + (i + 0.5) dx, y0 + (j + 0.5) dy)``; spacings and origins are
  snapped to multiples of 2**-20 so that every ray coordinate is exact in
  FP64 whatever the evaluation order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SNAP_BITS = 20


def snap(v: float, bits: int = SNAP_BITS) -> float:
    """Round ``v`` to the nearest multiple of 2**-bits."""
    s = float(1 << bits)
    return round(v * s) / s


@dataclass
class Grid:
    """Cell-centred ray grid: ray k = j*nx + i at (x0+(i+.5)dx, y0+(j+.5)dy)."""
    x0: float
    y0: float
    dx: float
    dy: float
    nx: int
    ny: int

    @property
    def n(self) -> int:
        return self.nx * self.ny

    def rays(self, idx: Optional[np.ndarray] = None) -> np.ndarray:
        """Explicit FP64 coordinates [n, 2] of all rays, or of the flat indices ``idx``."""
        if idx is None:
            idx = np.arange(self.n, dtype=np.int64)
        idx = np.asarray(idx, dtype=np.int64)
        i = (idx % self.nx).astype(np.float64)
        j = (idx // self.nx).astype(np.float64)
        out = np.empty((idx.size, 2), np.float64)
        out[:, 0] = self.x0 + (i + 0.5) * self.dx
        out[:, 1] = self.y0 + (j + 0.5) * self.dy
        return out

    def strided(self, stride: int, offset: int) -> np.ndarray:
        """Flat indices of the sub-grid (offset + a*stride, offset + b*stride)."""
        ii = np.arange(offset, self.nx, stride, dtype=np.int64)
        jj = np.arange(offset, self.ny, stride, dtype=np.int64)
        return (jj[:, None] * self.nx + ii[None, :]).reshape(-1)


def centred_grid(width: float, height: float, nx: int, ny: int) -> Grid:
    """Grid of nx x ny cells centred on the origin with dyadic spacing."""
    dx = snap(width / nx)
    dy = snap(height / ny)
    return Grid(x0=-0.5 * nx * dx, y0=-0.5 * ny * dy, dx=dx, dy=dy, nx=nx, ny=ny)


@dataclass
class MapDesc:
    """Source-plane map: npix x npix pixels of a square of side `side`."""
    y1min: float
    y2min: float
    side: float
    npix: int


@dataclass
class Field:
    xy: np.ndarray                  # [N, 2] float64
    m: np.ndarray                   # [N] float64
    kappa_s: float
    gamma: float
    radius: float = 0.0             # radius of the disk the stars were drawn in
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.m.shape[0])

    @property
    def kappa_star(self) -> float:
        return float(self.m.sum()) / self.radius ** 2 if self.radius > 0 else 0.0


def uniform_disk(rng: np.random.Generator, n: int, radius: float) -> np.ndarray:
    u = rng.random((n, 2))
    r = radius * np.sqrt(u[:, 0])
    th = 2.0 * math.pi * u[:, 1]
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def powerlaw_masses(rng: np.random.Generator, n: int, lo=0.1, hi=1.0, slope=2.35) -> np.ndarray:
    a = 1.0 - slope                  # -1.35
    u = rng.random(n)
    m = (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)
    return m * (n / m.sum())


# ---------------------------------------------------------------- workloads


def small_disk():
    """1000 unit-mass lenses in a disk of radius 26.6, gamma=0.3; 512^2 rays
    over [-5,5]^2; 256^2 map over [-2,2]^2.  The literal radius is kept, so the
    effective convergence is sum(m)/R^2 = 1.413."""
    rng = np.random.default_rng(0)
    n = 1000
    R = 26.6
    xy = uniform_disk(rng, n, R)
    f = Field(xy=xy, m=np.ones(n), kappa_s=0.0, gamma=0.3, radius=R)
    g = Grid(x0=-5.0, y0=-5.0, dx=10.0 / 512, dy=10.0 / 512, nx=512, ny=512)
    mp = MapDesc(y1min=-2.0, y2min=-2.0, side=4.0, npix=256)
    return f, g, mp


def powerlaw_disk(n_stars: int = 1_000_000, n_side: int = 8192, seed: int = 2):
    """N_*=1e6 power-law masses in a disk with kappa_*=0.4, kappa_s=0.2,
    gamma=0.35; an 8192^2 ray grid over the square inscribed in the disk."""
    rng = np.random.default_rng(seed)
    m = powerlaw_masses(rng, n_stars)
    R = math.sqrt(m.sum() / 0.4)
    xy = uniform_disk(rng, n_stars, R)
    f = Field(xy=xy, m=m, kappa_s=0.2, gamma=0.35, radius=R)
    side = math.sqrt(2.0) * R
    g = centred_grid(side, side, n_side, n_side)
    return f, g


def high_magnification(n_stars: int = 5_000_000, nx: int = 16384, ny: int = 16384, kappa_s: float = 0.75,
            seed: int = 3):
    """High-magnification field: kappa_*=0.1, kappa_s=0.75, gamma=0.05
    (macro magnification 50); rays over [-120,120]x[-60,60]; 2000^2 map over
    [-10,10]^2."""
    rng = np.random.default_rng(seed)
    R = math.sqrt(n_stars / 0.1)
    xy = uniform_disk(rng, n_stars, R)
    f = Field(xy=xy, m=np.ones(n_stars), kappa_s=kappa_s, gamma=0.05, radius=R)
    g = Grid(x0=-120.0, y0=-60.0, dx=240.0 / nx, dy=120.0 / ny, nx=nx, ny=ny)
    mp = MapDesc(y1min=-10.0, y2min=-10.0, side=20.0, npix=2000)
    return f, g, mp


def field_batch(n_fields: int = 64, n_side: int = 2048, npix: int = 512, seed: int = 4,
            n_range=(1e4, 2e5)):
    """Batch of independent star fields with uneven N_*, kappa_* and gamma."""
    master = np.random.default_rng(seed)
    out = []
    for r in range(n_fields):
        n = int(round(math.exp(master.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        ks = float(master.uniform(0.05, 0.6))
        gm = float(master.uniform(0.0, 0.6))
        rng = np.random.default_rng(1000 + r)
        R = math.sqrt(n / ks)
        xy = uniform_disk(rng, n, R)
        f = Field(xy=xy, m=np.ones(n), kappa_s=0.0, gamma=gm, radius=R, meta={"kappa_star": ks})
        side = math.sqrt(2.0) * R
        g = centred_grid(side, side, n_side, n_side)
        lam = min(abs(1.0 - ks - gm), abs(1.0 - ks + gm))
        L = max(0.8 * side * lam, 0.02 * side)
        mp = MapDesc(y1min=-0.5 * L, y2min=-0.5 * L, side=L, npix=npix)
        out.append((f, g, mp))
    return out


def clustered_lenses(n_clusters: int = 2000, per_cluster: int = 100, n_rays: int = 1_000_000,
            radius: float = 60.0, sigma: float = 0.5, noise: float = 0.01, seed: int = 5):
    """Clustered lenses for the gradient workload: Gaussian clusters around
    centres uniform in a disk, rays uniform in the same disk.  Returns the
    field, the rays and the target noise; the loss target is y_true + noise."""
    rng = np.random.default_rng(seed)
    centres = uniform_disk(rng, n_clusters, radius)
    xy = (np.repeat(centres, per_cluster, axis=0)
          + sigma * rng.standard_normal((n_clusters * per_cluster, 2)))
    f = Field(xy=xy, m=np.ones(n_clusters * per_cluster), kappa_s=0.0, gamma=0.0, radius=radius)
    rays = uniform_disk(rng, n_rays, radius)
    tnoise = noise * rng.standard_normal((n_rays, 2))
    return f, rays, tnoise


def random_field(n: int, radius: float, seed: int, kappa_s=0.0, gamma=0.0, masses="unit"):
    """Small seeded field for tests: uniform disk, unit or power-law masses."""
    rng = np.random.default_rng(seed)
    m = np.ones(n) if masses == "unit" else powerlaw_masses(rng, n)
    xy = uniform_disk(rng, n, radius)
    return Field(xy=xy, m=m, kappa_s=kappa_s, gamma=gamma, radius=radius)


def synthetic_halo(n_dm: int = 10_800_000, n_gas: int = 3_760_000, n_star: int = 1_190_000,
                   n_bh: int = 128, n_side: int = 4000, half_width: float = 45.0,
                   seed: int = 8):
    """A synthetic galaxy halo standing in for the cosmological-simulation
    lens of Section 2.5 (whose particle data is not available): the same
    particle counts (1.08e7 dark matter, 3.76e6 gas, 1.19e6 stars, 128 black
    holes; 1.575e7 in all), projected on the lens plane, in Einstein-radius
    units of unit mass.

    * dark matter: surface density ~ 1/r (a projected isothermal halo) out to
      R = 1500, axis ratio 0.75;
    * gas: cored, ~ 1/sqrt(r^2 + 40^2), same extent and flattening;
    * stars: exponential disk of scale 6, axis ratio 0.6;
    * black holes: Gaussian of width 1 about the centre;
    * all rotated by 30 degrees; masses 80% / 15% / 5% of a total of 13050
      (dark matter / gas / stars), black holes 0.03 each, so that the mass
      inside r = 30 is ~30^2 (a mean convergence M(<r)/r^2 of 1 there: an
      Einstein radius of ~30, inside the ray region with the critical
      curves); kappa_s = 0, external shear 0.03.

    Rays: an n_side x n_side grid over [-half_width, half_width]^2 (the inner
    region, where the caustics and the multiple images are)."""
    rng = np.random.default_rng(seed)
    R, rc, rs = 1500.0, 40.0, 6.0

    def place(r, q):
        th = 2.0 * math.pi * rng.random(r.size)
        x, y = r * np.cos(th), q * r * np.sin(th)
        c, s = math.cos(math.pi / 6), math.sin(math.pi / 6)
        return np.stack([c * x - s * y, s * x + c * y], 1)

    r_dm = R * rng.random(n_dm)
    a = math.sqrt(R * R + rc * rc) - rc
    r_gas = np.sqrt((rng.random(n_gas) * a + rc) ** 2 - rc * rc)
    r_st = -rs * np.log(rng.random(n_star) * rng.random(n_star))
    r_st = np.minimum(r_st, R)
    xy = np.concatenate([place(r_dm, 0.75), place(r_gas, 0.75), place(r_st, 0.6),
                         rng.standard_normal((n_bh, 2))])
    M = 13050.0
    m = np.concatenate([np.full(n_dm, 0.80 * M / n_dm), np.full(n_gas, 0.15 * M / n_gas),
                        np.full(n_star, 0.05 * M / n_star), np.full(n_bh, 0.03)])
    f = Field(xy=xy, m=m, kappa_s=0.0, gamma=0.03, radius=R,
              meta={"components": {"dark": n_dm, "gas": n_gas, "stars": n_star, "bh": n_bh}})
    g = centred_grid(2 * half_width, 2 * half_width, n_side, n_side)
    return f, g


def anamorphic_arc(n_stars: int = 1_800_000, mass: float = 0.2, width: float = 15000.0,
                   height: float = 10.0, nx: int = 15_000_000, ny: int = 10_000, npix: int = 4000,
                   seed: int = 9):
    """A highly anamorphic shooting region like the magnified star of
    Section 3.3: a macro model with magnification ~4200 and an axis ratio of
    ~1500 (eigenvalues 1 - kappa - gamma = 3.98e-4 and 1 - kappa + gamma =
    0.597), a 15000 x 10 Einstein-radius region of rays, and 1.8e6
    deflectors of mass 0.2 filling the circle that circumscribes it
    (diameter 15000: kappa_* = 6.4e-3, the rest of the convergence smooth).
    The map covers 4 x 4 Einstein radii of the source plane at 0.001 per
    pixel.  Rays: nx x ny over the region; the default, 1.5e7 x 1e4 = 1.5e11
    rays 0.001 apart, is one ray per unlensed pixel."""
    rng = np.random.default_rng(seed)
    lam1, lam2 = 3.98e-4, 0.597
    kappa = 1.0 - 0.5 * (lam1 + lam2)
    gamma = 0.5 * (lam2 - lam1)
    R = 0.5 * math.hypot(width, height)
    xy = uniform_disk(rng, n_stars, R)
    m = np.full(n_stars, mass)
    kappa_star = m.sum() / R ** 2
    f = Field(xy=xy, m=m, kappa_s=kappa - kappa_star, gamma=gamma, radius=R,
              meta={"kappa_star": kappa_star, "mu_macro": 1.0 / (lam1 * lam2)})
    g = centred_grid(width, height, nx, ny)
    mp = MapDesc(y1min=-2.0, y2min=-2.0, side=4.0, npix=npix)
    return f, g, mp
