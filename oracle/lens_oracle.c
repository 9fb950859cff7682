/*
 * lens_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the GPU
 * library computes, used only by tests/, by __graft_entry__.smoke() and by
 * the cpu_baseline leg of bench.py.  Nothing in the product path may link,
 * load or call it.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Jimenez-Vicente & Mediavilla 2022, "Fast Multipole
 * Method for Gravitational Lensing"):
 *
 *  - oracle_deflect: the thin-lens lens equation for N point lenses, eq. (1)
 *    of Section 1, in its real-vector form
 *        alpha(x) = sum_i m_i (x - x_i) / |x - x_i|^2,
 *    with the smooth convergence kappa_s and shear gamma that the footnote to
 *    eq. (1) and step 3 of the map driver (Section 2.4) add:
 *        y1 = (1 - kappa_s - gamma) x1 - alpha1
 *        y2 = (1 - kappa_s + gamma) x2 - alpha2
 *    (shear along the x1 axis; the paper fixes only |gamma|).  Units are
 *    Einstein radii of unit mass.  This is the plain O(N_* x N_x) definition
 *    the FMM approximates (Section 1, after eq. 1).  Sums run in star index
 *    order with Neumaier compensation.  A ray that coincides exactly with a
 *    star is singular; that pair is skipped and counted.
 *
 *  - oracle_jacobian: the deflection Jacobian d(alpha)/d(x) at each ray,
 *        J = sum_i m_i ( I/r^2 - 2 d d^T / r^4 ),   d = x - x_i,
 *    i.e. the derivative of eq. (1); the complex form of the same thing is
 *    f'(z) = -sum_i m_i/(z - z_i)^2, which Appendix A says the expansions
 *    provide without numerical derivatives.
 *
 *  - oracle_bin: inverse ray shooting (Section 2.3): each mapped ray adds one
 *    count to the source-plane pixel it lands in.  Pixel (u, v) of an
 *    npix x npix map of side `side` whose lower-left corner is (y1min, y2min)
 *    is the half-open square [y1min + u/S, y1min + (u+1)/S) x [...),
 *    S = npix/side, decided as u = floor((y1 - y1min) * S) with one rounding
 *    per operation.  Rays outside the map are dropped.
 *
 *  - oracle_ipm: inverse polygon mapping (Section 2.3, first order as used in
 *    Section 2.4).  Adjacent grid rays are the corners of image-plane cells
 *    of area dx dy; cell (i, j) with corners y(i,j), y(i+1,j), y(i+1,j+1),
 *    y(i,j+1) maps to a quadrilateral Q in the source plane and, by Green's
 *    theorem, its area is shared exactly among the pixels Q overlaps in
 *    proportion to the overlap areas: pixel P receives dx dy |Q n P| / |Q|,
 *    and mu[P] accumulates that over the pixel area, so mu is the
 *    magnification sum S_i / S_pixel of the paper.  However far Q stretches,
 *    every pixel it covers is apportioned exactly.  A critical cell (one that
 *    straddles a critical curve) maps to a quadrilateral whose edges cross;
 *    Section 2.3 treats such cells naively, as if they were not critical: the
 *    region the quadrilateral's edges enclose -- the two triangles ("lobes")
 *    on either side of the crossing point -- takes the cell's area in
 *    proportion to overlap, |Q n P| = |T1 n P| + |T2 n P| and
 *    |Q| = |T1| + |T2|.  Only a cell whose image has zero area carries no
 *    shape: each corner then takes a quarter of its area to the pixel it
 *    falls in (the zeroth-order, inverse-ray-shooting rule).  Overlaps are
 *    found by clipping each polygon against each pixel square of the cell's
 *    bounding box (Sutherland-Hodgman) and measuring the clipped polygon by
 *    the shoelace formula, in pixel units (p = (y - ymin) S).
 *
 *  - oracle_grad: the gradient of a scalar loss L(y) with respect to the star
 *    positions and masses, given G_k = dL/dy_k, from differentiating eq. (1):
 *        dL/dx_i = m_i sum_k ( G_k / r^2 - 2 d (d . G_k) / r^4 )
 *        dL/dm_i = - sum_k (d . G_k) / r^2,           d = x_k - x_i.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see build.py);
 * contraction is off so every product and sum rounds once, as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Neumaier (improved Kahan-Babuska) compensated accumulation. */
typedef struct { double s, c; } nsum;

static inline void nadd(nsum *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}

static inline double nval(const nsum *a) { return a->s + a->c; }

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

/*
 * Deflect n_rays rays (rxy[k][2]) by n_stars point lenses (sxy[i][2], sm[i]).
 * Writes y_out[k][2] (may be NULL) and alpha_out[k][2] (may be NULL).
 * *n_coincident (may be NULL) receives the number of skipped (ray == star)
 * pairs.  nthreads <= 0 keeps the OpenMP default.  Returns 0, or -1 on a
 * negative size.
 */
int oracle_deflect(int64_t n_stars, const double *sxy, const double *sm,
                   double kappa_s, double gamma, int64_t n_rays,
                   const double *rxy, double *y_out, double *alpha_out,
                   int64_t *n_coincident, int nthreads) {
  if (n_stars < 0 || n_rays < 0) return -1;
  set_threads(nthreads);
  int64_t skipped = 0;
  const double c1 = (1.0 - kappa_s) - gamma;
  const double c2 = (1.0 - kappa_s) + gamma;
#pragma omp parallel for schedule(static) reduction(+ : skipped)
  for (int64_t k = 0; k < n_rays; ++k) {
    const double x1 = rxy[2 * k], x2 = rxy[2 * k + 1];
    nsum a1 = {0.0, 0.0}, a2 = {0.0, 0.0};
    for (int64_t i = 0; i < n_stars; ++i) {
      const double d1 = x1 - sxy[2 * i];
      const double d2 = x2 - sxy[2 * i + 1];
      const double r2 = d1 * d1 + d2 * d2;
      if (r2 == 0.0) {
        ++skipped;
        continue;
      }
      const double w = sm[i] / r2;
      nadd(&a1, w * d1);
      nadd(&a2, w * d2);
    }
    const double al1 = nval(&a1), al2 = nval(&a2);
    if (alpha_out) {
      alpha_out[2 * k] = al1;
      alpha_out[2 * k + 1] = al2;
    }
    if (y_out) {
      y_out[2 * k] = c1 * x1 - al1;
      y_out[2 * k + 1] = c2 * x2 - al2;
    }
  }
  if (n_coincident) *n_coincident = skipped;
  return 0;
}

/*
 * Deflection Jacobian at each ray: jac_out[k][3] = (J11, J12, J22) of
 * d(alpha)/d(x).  Coincident pairs are skipped.  Returns 0 or -1.
 */
int oracle_jacobian(int64_t n_stars, const double *sxy, const double *sm,
                    int64_t n_rays, const double *rxy, double *jac_out,
                    int nthreads) {
  if (n_stars < 0 || n_rays < 0) return -1;
  set_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n_rays; ++k) {
    const double x1 = rxy[2 * k], x2 = rxy[2 * k + 1];
    nsum j11 = {0, 0}, j12 = {0, 0}, j22 = {0, 0};
    for (int64_t i = 0; i < n_stars; ++i) {
      const double d1 = x1 - sxy[2 * i];
      const double d2 = x2 - sxy[2 * i + 1];
      const double r2 = d1 * d1 + d2 * d2;
      if (r2 == 0.0) continue;
      const double w = sm[i] / r2;
      const double w2 = 2.0 * w / r2;
      nadd(&j11, w - w2 * d1 * d1);
      nadd(&j12, -w2 * d1 * d2);
      nadd(&j22, w - w2 * d2 * d2);
    }
    jac_out[3 * k] = nval(&j11);
    jac_out[3 * k + 1] = nval(&j12);
    jac_out[3 * k + 2] = nval(&j22);
  }
  return 0;
}

/*
 * Inverse-ray-shooting binning of n mapped rays y[k][2] into counts[v*npix+u]
 * (accumulated, +=).  Returns the number of rays that landed in the map, or
 * -1 on bad arguments, or -2 if a pixel count would exceed INT32_MAX.
 */
int64_t oracle_bin(int64_t n, const double *y, double y1min, double y2min,
                   double side, int32_t npix, int32_t *counts) {
  if (n < 0 || npix <= 0 || !(side > 0.0)) return -1;
  const double S = (double)npix / side;
  const int64_t np2 = (int64_t)npix * npix;
  int64_t *acc = (int64_t *)calloc((size_t)np2, sizeof(int64_t));
  if (!acc) return -1;
  int64_t landed = 0;
  for (int64_t k = 0; k < n; ++k) {
    const double t1 = (y[2 * k] - y1min) * S;
    const double t2 = (y[2 * k + 1] - y2min) * S;
    if (!(t1 >= 0.0) || !(t2 >= 0.0)) continue; /* also drops NaN */
    const double f1 = floor(t1), f2 = floor(t2);
    if (f1 >= (double)npix || f2 >= (double)npix) continue;
    acc[(int64_t)f2 * npix + (int64_t)f1] += 1;
    ++landed;
  }
  int rc = 0;
  for (int64_t q = 0; q < np2; ++q) {
    const int64_t v = (int64_t)counts[q] + acc[q];
    if (v > INT32_MAX) rc = -2;
    else counts[q] = (int32_t)v;
  }
  free(acc);
  return rc ? rc : landed;
}

/*
 * Gradient of a loss L with respect to star positions and masses given
 * grad_y[k][2] = dL/dy_k.  Writes grad_xy[i][2] and grad_m[i].  Coincident
 * pairs are skipped (their term is singular).  Returns 0 or -1.
 */
int oracle_grad(int64_t n_stars, const double *sxy, const double *sm,
                int64_t n_rays, const double *rxy, const double *grad_y,
                double *grad_xy, double *grad_m, int nthreads) {
  if (n_stars < 0 || n_rays < 0) return -1;
  set_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_stars; ++i) {
    const double s1 = sxy[2 * i], s2 = sxy[2 * i + 1];
    nsum gx = {0, 0}, gy = {0, 0}, gm = {0, 0};
    for (int64_t k = 0; k < n_rays; ++k) {
      const double d1 = rxy[2 * k] - s1;
      const double d2 = rxy[2 * k + 1] - s2;
      const double r2 = d1 * d1 + d2 * d2;
      if (r2 == 0.0) continue;
      const double g1 = grad_y[2 * k], g2 = grad_y[2 * k + 1];
      const double dg = d1 * g1 + d2 * g2;
      const double inv = 1.0 / r2;
      const double two = 2.0 * dg * inv * inv;
      nadd(&gx, g1 * inv - two * d1);
      nadd(&gy, g2 * inv - two * d2);
      nadd(&gm, -dg * inv);
    }
    grad_xy[2 * i] = sm[i] * nval(&gx);
    grad_xy[2 * i + 1] = sm[i] * nval(&gy);
    grad_m[i] = nval(&gm);
  }
  return 0;
}

/* ------------------------------------------------------------------ IPM */

/* signed area (twice) of the triangle a, b, c */
static double orient2(const double *a, const double *b, const double *c) {
  return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

/* proper crossing of segments ab and cd (touching does not count) */
static int segments_cross(const double *a, const double *b, const double *c, const double *d) {
  const double o1 = orient2(a, b, c), o2 = orient2(a, b, d);
  const double o3 = orient2(c, d, a), o4 = orient2(c, d, b);
  return ((o1 > 0 && o2 < 0) || (o1 < 0 && o2 > 0)) && ((o3 > 0 && o4 < 0) || (o3 < 0 && o4 > 0));
}

/* shoelace area (signed) of an n-gon, on coordinates relative to its first
 * vertex (translation-invariant, so a small polygon far from the origin
 * keeps its digits) */
static double poly_area(int n, const double (*p)[2]) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) {
    const int k1 = (k + 1) % n;
    const double x0 = p[k][0] - p[0][0], y0 = p[k][1] - p[0][1];
    const double x1 = p[k1][0] - p[0][0], y1 = p[k1][1] - p[0][1];
    s += x0 * y1 - x1 * y0;
  }
  return 0.5 * s;
}

/* clip polygon in[n] against the half-plane coordinate c (0: x, 1: y)
 * >= lo (sign = +1) or <= hi (sign = -1); returns the new vertex count */
static int clip_half(int n, const double (*in)[2], double (*out)[2], int c, double bound, int keep_ge) {
  int m = 0;
  for (int k = 0; k < n; ++k) {
    const double *S = in[(k + n - 1) % n], *E = in[k];
    const int sin_ = keep_ge ? S[c] >= bound : S[c] <= bound;
    const int ein = keep_ge ? E[c] >= bound : E[c] <= bound;
    if (ein != sin_) {
      const double t = (bound - S[c]) / (E[c] - S[c]);
      out[m][c] = bound;
      out[m][1 - c] = S[1 - c] + t * (E[1 - c] - S[1 - c]);
      ++m;
    }
    if (ein) {
      out[m][0] = E[0];
      out[m][1] = E[1];
      ++m;
    }
  }
  return m;
}


static void add_corner(double *mu, int32_t npix, const double *p, double w) {
  if (!(p[0] >= 0.0) || !(p[1] >= 0.0)) return;
  const double f1 = floor(p[0]), f2 = floor(p[1]);
  if (f1 >= (double)npix || f2 >= (double)npix) return;
  mu[(int64_t)f2 * npix + (int64_t)f1] += w;
}

/* area of polygon p[n] (pixel units) inside the unit square [u,u+1]x[v,v+1] */
static double poly_pixel_overlap(int n0, const double (*p)[2], double u, double v) {
  double a[16][2], b[16][2];
  int n = n0;
  for (int k = 0; k < n0; ++k) {
    a[k][0] = p[k][0] - u;
    a[k][1] = p[k][1] - v;
  }
  n = clip_half(n, (const double (*)[2])a, b, 0, 0.0, 1);
  n = clip_half(n, (const double (*)[2])b, a, 0, 1.0, 0);
  n = clip_half(n, (const double (*)[2])a, b, 1, 0.0, 1);
  n = clip_half(n, (const double (*)[2])b, a, 1, 1.0, 0);
  return n >= 3 ? fabs(poly_area(n, (const double (*)[2])a)) : 0.0;
}

/*
 * IPM magnification of the (nx-1) x (ny-1) cells spanned by the mapped grid
 * y[ny][nx][2] (row-major, y[(j*nx + i)*2 + c]), accumulated into
 * mu[v*npix + u] (+=).  cell_area = dx * dy.  Returns 0 or -1.
 */
int oracle_ipm(int64_t nx, int64_t ny, const double *y, double cell_area, double y1min,
               double y2min, double side, int32_t npix, double *mu) {
  if (nx < 0 || ny < 0 || npix <= 0 || !(side > 0.0) || !(cell_area >= 0.0)) return -1;
  const double S = (double)npix / side;
  const double cell_px = cell_area * S * S; /* cell area in pixel units */
  for (int64_t j = 0; j + 1 < ny; ++j)
    for (int64_t i = 0; i + 1 < nx; ++i) {
      const int64_t id[4] = {j * nx + i, j * nx + i + 1, (j + 1) * nx + i + 1, (j + 1) * nx + i};
      double q[4][2];
      int finite = 1;
      for (int k = 0; k < 4; ++k) {
        q[k][0] = (y[2 * id[k]] - y1min) * S;
        q[k][1] = (y[2 * id[k] + 1] - y2min) * S;
        finite &= isfinite(q[k][0]) && isfinite(q[k][1]);
      }
      if (!finite) continue;
      /* the polygons that carry the cell's area: Q itself, or, if two
       * opposite edges a-b and c-d cross at X, the lobes (X, b, c) and
       * (a, X, d) */
      double poly[2][4][2];
      int nv[2] = {4, 0}, npoly = 1;
      double area;
      const int c01 = segments_cross(q[0], q[1], q[2], q[3]);
      const int c12 = !c01 && segments_cross(q[1], q[2], q[3], q[0]);
      if (c01 || c12) {
        const double *a = c01 ? q[0] : q[1], *b = c01 ? q[1] : q[2];
        const double *c = c01 ? q[2] : q[3], *d = c01 ? q[3] : q[0];
        const double den = (b[0] - a[0]) * (d[1] - c[1]) - (b[1] - a[1]) * (d[0] - c[0]);
        const double t = ((c[0] - a[0]) * (d[1] - c[1]) - (c[1] - a[1]) * (d[0] - c[0])) / den;
        const double X[2] = {a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])};
        const double *t1[3] = {X, b, c}, *t2[3] = {a, X, d};
        for (int k = 0; k < 3; ++k) {
          poly[0][k][0] = t1[k][0];
          poly[0][k][1] = t1[k][1];
          poly[1][k][0] = t2[k][0];
          poly[1][k][1] = t2[k][1];
        }
        nv[0] = nv[1] = 3;
        npoly = 2;
        area = fabs(poly_area(3, (const double (*)[2])poly[0])) +
               fabs(poly_area(3, (const double (*)[2])poly[1]));
      } else {
        for (int k = 0; k < 4; ++k) {
          poly[0][k][0] = q[k][0];
          poly[0][k][1] = q[k][1];
        }
        area = fabs(poly_area(4, (const double (*)[2])q));
      }
      if (!(area > 0.0)) {
        for (int k = 0; k < 4; ++k) add_corner(mu, npix, q[k], 0.25 * cell_px);
        continue;
      }
      double lo0 = q[0][0], hi0 = q[0][0], lo1 = q[0][1], hi1 = q[0][1];
      for (int k = 1; k < 4; ++k) {
        lo0 = fmin(lo0, q[k][0]);
        hi0 = fmax(hi0, q[k][0]);
        lo1 = fmin(lo1, q[k][1]);
        hi1 = fmax(hi1, q[k][1]);
      }
      if (hi0 < 0.0 || hi1 < 0.0 || lo0 >= (double)npix || lo1 >= (double)npix) continue;
      const int64_t u0 = lo0 < 0.0 ? 0 : (int64_t)floor(lo0);
      const int64_t v0 = lo1 < 0.0 ? 0 : (int64_t)floor(lo1);
      const int64_t u1 = hi0 >= (double)npix ? npix - 1 : (int64_t)floor(hi0);
      const int64_t v1 = hi1 >= (double)npix ? npix - 1 : (int64_t)floor(hi1);
      if (u0 == u1 && v0 == v1 && lo0 >= 0.0 && lo1 >= 0.0 && hi0 < (double)npix &&
          hi1 < (double)npix) {
        /* wholly inside one pixel: the whole cell (exactly; a ratio of two
         * rounded areas would not give 1 for a sliver-thin quadrilateral) */
        mu[v0 * npix + u0] += cell_px;
        continue;
      }
      for (int64_t v = v0; v <= v1; ++v)
        for (int64_t u = u0; u <= u1; ++u) {
          double ov = 0.0;
          for (int k = 0; k < npoly; ++k)
            ov += poly_pixel_overlap(nv[k], (const double (*)[2])poly[k], (double)u, (double)v);
          if (ov > 0.0) mu[v * npix + u] += cell_px * (ov / area);
        }
    }
  return 0;
}
