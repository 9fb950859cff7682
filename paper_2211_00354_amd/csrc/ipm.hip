// Inverse polygon mapping (Section 2.3; first order, as used in Section 2.4).
// Adjacent grid rays are the corners of image-plane cells of area dx dy; cell
// (i, j) with corners y(i,j), y(i+1,j), y(i+1,j+1), y(i,j+1) maps to a
// quadrilateral Q in the source plane, and its area is shared exactly among
// the pixels Q overlaps in proportion to the overlap areas: pixel P receives
// dx dy |Q n P| / |Q|; divided by the pixel area that is the magnification
// sum S_i / S_pixel.  A critical cell (its image's edges cross: the cell
// straddles a critical curve) is treated as if it were not critical: the
// region its edges enclose, the two triangles ("lobes") either side of the
// crossing point, takes the cell's area by overlap.  Only an image of zero
// area goes to its corners, a quarter of the cell to each corner's pixel
// (the zeroth-order, inverse-ray-shooting rule).
//
// Geometry in pixel units p = (y - ymin) S, S = npix/side.  Overlaps come
// from Green's theorem as a sum of edge terms (see poly_pixel_overlap), which
// needs no clipped polygon.  Contributions are summed as fixed-point integers
// (units of 2^-40 of a pixel's magnification) with 64-bit atomics, so the map
// does not depend on the order of the additions; a final pass adds them to
// the caller's FP64 map.
//
// Two kernels share the cells of a pass:
//   * k_ipm, a thread per cell: a cell inside one pixel (the common case)
//     adds the whole cell; a cell whose bounding box spans at most
//     kPairMax pixels is apportioned pixel by pixel, its (cell, pixel) pairs
//     shared out evenly over the workgroup; a wider cell (next to a star its
//     image can stretch over much of the map) is queued;
//   * k_ipm_wide, a wave per queued cell: its image (the quadrilateral, or a
//     folded cell's two lobes) is rasterised edge by edge, so the work is
//     proportional to its perimeter in pixels: an edge adds its Green term to
//     the few pixels it crosses in each row and a constant to the row's
//     pixels right of it through a row-difference accumulator that the final
//     pass prefix-sums along the row.
#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kThreads = 256;
constexpr double kFix = 1099511627776.0;  // 2^40
// widest bounding box (in pixels) apportioned by the per-cell pair path
constexpr int32_t kPairMax = 64;

__device__ __forceinline__ double orient2(double ax, double ay, double bx, double by, double cx,
                                          double cy) {
  return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

// Strictly opposite signs (a zero is neither).
__device__ __forceinline__ bool opposite(double u, double v) {
  return (u > 0 && v < 0) || (u < 0 && v > 0);
}

__device__ __forceinline__ double clamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }

// Signed contribution of edge a -> b to the area of (polygon n unit square):
// the line integral of clamp01(x) dy over the edge's part with 0 <= y <= 1.
// On that part x(y) = lx + (y - ly) k is linear, so clamp01(x(y)) is linear
// between the heights where x crosses 0 and 1 and the trapezoid rule on those
// pieces is exact.  k = dx/dy and kinv = dy/dx (0 for a vertical edge) depend
// only on the edge's direction, not on the pixel or on where the edge ends.
__device__ __forceinline__ double edge_term(double ax, double ay, double bx, double by, double k,
                                            double kinv) {
  if (ay == by) return 0.0;
  const bool up = by > ay;
  const double lx = up ? ax : bx, ly = up ? ay : by, hy = up ? by : ay;
  const double y0 = fmax(ly, 0.0), y1 = fmin(hy, 1.0);
  if (!(y0 < y1)) return 0.0;
  // breakpoints (heights where x = 0 and x = 1); a vertical edge has kinv =
  // 0, so both fall at ly <= y0 and are ignored, as they should be
  const double ya = fma(-lx, kinv, ly), yb = ya + kinv;
  const double lo = fmin(ya, yb), hi = fmax(ya, yb);
  double s0 = (lo > y0 && lo < y1) ? lo : y1;
  double s1 = (hi > y0 && hi < y1) ? hi : y1;
  if (s0 == y1) s0 = s1, s1 = y1;
  const double x0 = clamp01(fma(y0 - ly, k, lx));
  const double xa = clamp01(fma(s0 - ly, k, lx));
  const double xb = clamp01(fma(s1 - ly, k, lx));
  const double x1 = clamp01(fma(y1 - ly, k, lx));
  const double v = 0.5 * fma(x0 + xa, s0 - y0, fma(xa + xb, s1 - s0, (xb + x1) * (y1 - s1)));
  return up ? v : -v;
}

// Edge a -> b against the unit square at (u, v).
__device__ __forceinline__ double edge_at(const double (&a)[2], const double (&b)[2], double k,
                                          double kinv, double u, double v) {
  return edge_term(a[0] - u, a[1] - v, b[0] - u, b[1] - v, k, kinv);
}

// Slopes k = dx/dy (0 for a horizontal edge) and kinv = dy/dx (0 for a
// vertical one) of the edge a -> b, through the refined hardware reciprocal
// (within an ulp or two of the quotient, a fraction of the cost of an IEEE
// division).
__device__ __forceinline__ void edge_slope(const double (&a)[2], const double (&b)[2], double &k,
                                           double &kinv) {
  const double dx = b[0] - a[0], dy = b[1] - a[1];
  k = dy != 0.0 ? dx * rcp_f64(dy) : 0.0;
  kinv = dx != 0.0 ? dy * rcp_f64(dx) : 0.0;
}

// The image of a cell as the polygons that carry its area.
//   kind 0: the quadrilateral q itself (convex or not; Green's theorem holds
//           for any simple polygon);
//   kind 1: edges 0-1 and 2-3 cross at X: lobes (X, q1, q2) and (q0, X, q3);
//   kind 2: edges 1-2 and 3-0 cross at X: lobes (X, q2, q3) and (q1, X, q0).
// area = |Q| or |T1| + |T2| (pixel units).
struct Cell {
  double q[4][2];
  double X[2];
  int kind;
  double area;
};

__device__ __forceinline__ double tri_area(const double (&a)[2], const double (&b)[2],
                                           const double (&c)[2]) {
  return fabs(0.5 * orient2(a[0], a[1], b[0], b[1], c[0], c[1]));
}

__device__ __forceinline__ void classify(Cell &c) {
  // Twice the signed areas of four corner triangles, on differences of
  // corners (a small image far from the map origin keeps its digits):
  // A = o(q0,q1,q2), B = o(q0,q1,q3), C = o(q2,q3,q0), D = o(q2,q3,q1),
  // o(a,b,c) = (b - a) x (c - a), unchanged by a cyclic shift of a, b, c.
  // Segments 0-1 and 2-3 cross iff A, B and C, D have opposite signs;
  // segments 1-2 and 3-0 iff D, A and B, C do; and A + C is twice the
  // signed area of q (its triangles q0 q1 q2 and q0 q2 q3).
  const double(&q)[4][2] = c.q;
  const double e01x = q[1][0] - q[0][0], e01y = q[1][1] - q[0][1];
  const double e23x = q[3][0] - q[2][0], e23y = q[3][1] - q[2][1];
  const double A = e01x * (q[2][1] - q[0][1]) - e01y * (q[2][0] - q[0][0]);
  const double B = e01x * (q[3][1] - q[0][1]) - e01y * (q[3][0] - q[0][0]);
  const double C = e23x * (q[0][1] - q[2][1]) - e23y * (q[0][0] - q[2][0]);
  const double D = e23x * (q[1][1] - q[2][1]) - e23y * (q[1][0] - q[2][0]);
  const bool c01 = opposite(A, B) && opposite(C, D);
  const bool c12 = !c01 && opposite(D, A) && opposite(B, C);
  if (c01 || c12) {
    const int ia = c01 ? 0 : 1;
    const double(&a)[2] = c.q[ia];
    const double(&b)[2] = c.q[ia + 1];
    const double(&cc)[2] = c.q[ia + 2];
    const double(&d)[2] = c.q[(ia + 3) & 3];
    const double den = (b[0] - a[0]) * (d[1] - cc[1]) - (b[1] - a[1]) * (d[0] - cc[0]);
    const double t = ((cc[0] - a[0]) * (d[1] - cc[1]) - (cc[1] - a[1]) * (d[0] - cc[0])) / den;
    c.X[0] = a[0] + t * (b[0] - a[0]);
    c.X[1] = a[1] + t * (b[1] - a[1]);
    c.kind = c01 ? 1 : 2;
    c.area = tri_area(c.X, b, cc) + tri_area(a, c.X, d);
  } else {
    c.X[0] = c.X[1] = 0.0;
    c.kind = 0;
    c.area = fabs(0.5 * (A + C));
  }
}

// Area of the cell's image inside the unit square at (u, v); k/kinv are the
// slopes of the four edges q[e] -> q[e+1] (sub-edges of a lobe run along
// them in the same direction).
__device__ double cell_pixel_overlap(const double (&q)[4][2], const double (&X)[2], int kind,
                                     const double (&k)[4], const double (&kinv)[4], double u,
                                     double v) {
  if (kind == 0) {
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) s += edge_at(q[e], q[(e + 1) & 3], k[e], kinv[e], u, v);
    return fabs(s);
  }
  if (kind == 1) {
    const double t1 = edge_at(X, q[1], k[0], kinv[0], u, v) + edge_at(q[1], q[2], k[1], kinv[1], u, v) +
                      edge_at(q[2], X, k[2], kinv[2], u, v);
    const double t2 = edge_at(q[0], X, k[0], kinv[0], u, v) + edge_at(X, q[3], k[2], kinv[2], u, v) +
                      edge_at(q[3], q[0], k[3], kinv[3], u, v);
    return fabs(t1) + fabs(t2);
  }
  const double t1 = edge_at(X, q[2], k[1], kinv[1], u, v) + edge_at(q[2], q[3], k[2], kinv[2], u, v) +
                    edge_at(q[3], X, k[3], kinv[3], u, v);
  const double t2 = edge_at(q[1], X, k[1], kinv[1], u, v) + edge_at(X, q[0], k[3], kinv[3], u, v) +
                    edge_at(q[0], q[1], k[0], kinv[0], u, v);
  return fabs(t1) + fabs(t2);
}

// Area of the part of the simple quadrilateral q with x < xs (across_x) or
// y < ys, for a cell whose image spans two pixels that share that line.  By
// Green's theorem the area of q n {w < 0}, w = x - xs, is |the line integral
// of min(w, 0) dy| around q (with w = y - ys and x in the place of y for the
// other split).  min(w, 0) is linear along an edge except where the edge
// crosses w = 0, at t = wa / (wa - wb) of its length, so the trapezoid rule
// on the one or two pieces is exact.
__device__ __forceinline__ double split_area(const double (&q)[4][2], bool across_x, double xs,
                                             double ys) {
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const double(&a)[2] = q[e];
    const double(&b)[2] = q[(e + 1) & 3];
    const double wa = across_x ? a[0] - xs : a[1] - ys, wb = across_x ? b[0] - xs : b[1] - ys;
    const double dz = across_x ? b[1] - a[1] : b[0] - a[0];
    const double ma = fmin(wa, 0.0), mb = fmin(wb, 0.0);
    double m = ma + mb;
    if ((wa < 0.0) != (wb < 0.0)) {
      const double t = wa * rcp_f64(wa - wb);
      m = ma * t + mb * (1.0 - t);
    }
    s += m * dz;
  }
  return fabs(0.5 * s);
}

// Orientation of a convex q (+1 counter-clockwise, -1 clockwise), or 0 if q
// is not convex.
__device__ __forceinline__ int convex_orientation(const double (&q)[4][2]) {
  int pos = 0, neg = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int e1 = (e + 1) & 3, e2 = (e + 2) & 3;
    const double c = orient2(q[e][0], q[e][1], q[e1][0], q[e1][1], q[e2][0], q[e2][1]);
    pos += c > 0.0;
    neg += c < 0.0;
  }
  return neg == 0 ? 1 : (pos == 0 ? -1 : 0);
}

// True if the pixel [u,u+1] x [v,v+1] lies (by more than a rounding margin)
// outside one of the edge lines of the convex q of orientation o, so that
// their overlap is empty: the largest value over the pixel of the edge's
// signed distance function is its value at the centre plus (|dx| + |dy|)/2.
__device__ __forceinline__ bool convex_misses(const double (&q)[4][2], int o, double u, double v) {
  const double uc = u + 0.5, vc = v + 0.5;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int e1 = (e + 1) & 3;
    const double dx = q[e1][0] - q[e][0], dy = q[e1][1] - q[e][1];
    const double f = (double)o * (dx * (vc - q[e][1]) - dy * (uc - q[e][0]));
    if (f + (0.5 + 1e-9) * (fabs(dx) + fabs(dy)) < 0.0) return true;
  }
  return false;
}

__device__ __forceinline__ int64_t pixel_of(const double (&p)[2], int32_t npix) {
  if (!(p[0] >= 0.0) || !(p[1] >= 0.0)) return -1;
  const double f1 = floor(p[0]), f2 = floor(p[1]);
  if (f1 >= (double)npix || f2 >= (double)npix) return -1;
  return (int64_t)f2 * npix + (int64_t)f1;
}

struct IpmArgs {
  const double *y;      // rows [ybase, ...) of the mapped grid, nx rays per row
  int64_t nx, ybase, j0, j1;  // cells of rows [j0, j1), all nx - 1 columns
  double cell_px, y1min, y2min, S;
  int32_t npix;
  unsigned long long *acc;   // [npix][npix]
  unsigned long long *diff;  // [npix][npix + 1] row differences (full pixels)
  uint32_t *queue;           // wide cells: index (j - j0) (nx - 1) + i
  uint32_t *qcount;
};

// Corners of cell (i, j) (pixel units); false if any is not finite.
__device__ __forceinline__ bool load_quad(const IpmArgs &a, int64_t i, int64_t j,
                                          double (&q)[4][2]) {
  const int64_t r0 = (j - a.ybase) * a.nx + i, r1 = r0 + a.nx;
  const int64_t id[4] = {r0, r0 + 1, r1 + 1, r1};
  bool finite = true;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    q[k][0] = (a.y[2 * id[k]] - a.y1min) * a.S;
    q[k][1] = (a.y[2 * id[k] + 1] - a.y2min) * a.S;
    finite = finite && isfinite(q[k][0]) && isfinite(q[k][1]);
  }
  return finite;
}

// Pixel bounding box of q clamped to the map; false if it misses the map
// (the box is then of no use).  The corners are clamped to the map before
// the conversion, so it is a 32-bit one.
__device__ __forceinline__ bool quad_bbox(const double (&q)[4][2], int32_t npix, int32_t &u0,
                                          int32_t &v0, int32_t &u1, int32_t &v1, bool &inside) {
  double lo0 = q[0][0], hi0 = q[0][0], lo1 = q[0][1], hi1 = q[0][1];
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    lo0 = fmin(lo0, q[k][0]);
    hi0 = fmax(hi0, q[k][0]);
    lo1 = fmin(lo1, q[k][1]);
    hi1 = fmax(hi1, q[k][1]);
  }
  const double top = (double)npix, last = top - 1.0;
  u0 = (int32_t)floor(fmin(fmax(lo0, 0.0), last));
  v0 = (int32_t)floor(fmin(fmax(lo1, 0.0), last));
  u1 = (int32_t)floor(fmin(fmax(hi0, 0.0), last));
  v1 = (int32_t)floor(fmin(fmax(hi1, 0.0), last));
  inside = lo0 >= 0.0 && lo1 >= 0.0 && hi0 < top && hi1 < top;
  return !(hi0 < 0.0 || hi1 < 0.0 || lo0 >= top || lo1 >= top);
}

__device__ __forceinline__ unsigned long long to_fix(double x) {
  return (unsigned long long)llrint(x * kFix);
}

// Workgroup-local sums of pixel contributions: an LDS hash table of pixels,
// flushed to the map once per workgroup, so the many cells of a patch that
// land in the same pixels (all of them, away from stars; those around a
// star's caustic, near one) cost few global atomics.  Two probes, then the
// global map: patches near a star touch more pixels than the table holds,
// and long probe chains there (a wave waits for its slowest lane) cost more
// than the atomics they save.
constexpr int kTable = 1024;
constexpr int kPatch = 32;  // a workgroup takes kPatch x kPatch cells

__device__ __forceinline__ void table_add(int32_t *tkey, unsigned long long *tval,
                                          unsigned long long *__restrict__ acc, int32_t key,
                                          unsigned long long v) {
  const uint32_t h = ((uint32_t)key * 2654435761u) >> 22;  // 10 bits
  for (int probe = 0; probe < 2; ++probe) {
    const int slot = (int)((h + (uint32_t)probe) & (kTable - 1));
    int32_t k = tkey[slot];
    if (k == -1) {
      const int32_t old = atomicCAS(&tkey[slot], -1, key);
      k = old == -1 ? key : old;
    }
    if (k == key) {
      atomicAdd(&tval[slot], v);
      return;
    }
  }
  atomicAdd(&acc[key], v);  // crowded table
}

__device__ __forceinline__ int32_t block_excl_scan(int32_t x, int32_t *wsum, int32_t *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t v = __shfl_up(inc, d);
    if (lane >= d) inc += v;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int32_t off = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < kThreads / 64; ++q) {
    if (q < w) off += wsum[q];
    tot += wsum[q];
  }
  *total = tot;
  return off + inc - x;
}

// One workgroup per kPatch x kPatch patch of cells, taken 256 cells at a
// time, one thread per cell.  The (cell, pixel) pairs of the batch's
// multi-pixel cells are numbered by a scan and shared out evenly over the
// workgroup's threads, so a few cells near a star do not hold a whole wave.
// Four waves per SIMD (at most 128 VGPRs), as many as its LDS allows.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_ipm(
    IpmArgs a) {
  __shared__ int32_t tkey[kTable];
  __shared__ unsigned long long tval[kTable];
  __shared__ double sq[kThreads][10];       // multi-pixel cells of the batch: corners, X,
  __shared__ double sinv[kThreads];         // 1 / area,
  __shared__ int32_t sshape[kThreads];      // kind | (convex orientation + 1) << 2,
  __shared__ int32_t sbox[kThreads][3];     // u0, v0, columns of the bounding box
  __shared__ int32_t sfirst[kThreads + 1];  // first pair index of each cell
  __shared__ int32_t wsum[kThreads / 64];
  const int t = threadIdx.x;
  for (int e = t; e < kTable; e += kThreads) {
    tkey[e] = -1;
    tval[e] = 0ull;
  }
  __syncthreads();
  const int64_t ncx = a.nx - 1;
  const int64_t npx_x = (ncx + kPatch - 1) / kPatch;
  const int64_t pi = blockIdx.x % npx_x, pj = blockIdx.x / npx_x;
  const int32_t npix = a.npix;
  const unsigned long long q_cell = to_fix(a.cell_px);
  const unsigned long long q_quarter = to_fix(0.25 * a.cell_px);
  for (int base = 0; base < kPatch * kPatch; base += kThreads) {
    const int k = base + t;
    const int64_t i = pi * kPatch + (k % kPatch), j = a.j0 + pj * kPatch + (k / kPatch);
    int32_t npairs = 0;
    Cell c;
    if (i < ncx && j < a.j1 && load_quad(a, i, j, c.q)) {
      classify(c);
      int32_t u0, v0, u1, v1;
      bool inside;
      const bool hits = quad_bbox(c.q, npix, u0, v0, u1, v1, inside);
      const int64_t npx = (int64_t)(u1 - u0 + 1) * (v1 - v0 + 1);
      if (!(c.area > 0.0)) {
        // no shape: a quarter of the cell to each corner's pixel
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int64_t pk = pixel_of(c.q[cc], npix);
          if (pk >= 0) table_add(tkey, tval, a.acc, (int32_t)pk, q_quarter);
        }
      } else if (hits) {
        if (u0 == u1 && v0 == v1 && inside) {
          table_add(tkey, tval, a.acc, v0 * npix + u0, q_cell);  // wholly inside
        } else if (npx == 2 && inside && c.kind == 0) {
          // across one pixel edge: the first pixel's overlap by Green's
          // theorem, the second takes the rest of the cell (in fixed point,
          // so the cell's total is exact)
          const double ov = split_area(c.q, u1 != u0, (double)(u0 + 1), (double)(v0 + 1));
          const double f = fmin(fmax(ov / c.area, 0.0), 1.0);
          const unsigned long long q0 = to_fix(a.cell_px * f);
          const unsigned long long q1 = q_cell >= q0 ? q_cell - q0 : 0ull;
          if (q0) table_add(tkey, tval, a.acc, v0 * npix + u0, q0);
          if (q1) table_add(tkey, tval, a.acc, v1 * npix + u1, q1);
        } else if (npx > kPairMax) {
          const uint32_t slot = atomicAdd(a.qcount, 1u);
          a.queue[slot] = (uint32_t)((j - a.j0) * ncx + i);
        } else {
          npairs = (int32_t)npx;
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            sq[t][2 * cc] = c.q[cc][0];
            sq[t][2 * cc + 1] = c.q[cc][1];
          }
          sq[t][8] = c.X[0];
          sq[t][9] = c.X[1];
          sinv[t] = 1.0 / c.area;
          sshape[t] = c.kind | ((c.kind == 0 ? convex_orientation(c.q) + 1 : 1) << 2);
          sbox[t][0] = u0;
          sbox[t][1] = v0;
          sbox[t][2] = u1 - u0 + 1;
        }
      }
    }
    int32_t total;
    const int32_t first = block_excl_scan(npairs, wsum, &total);
    sfirst[t] = first;
    if (t == kThreads - 1) sfirst[kThreads] = first + npairs;
    __syncthreads();
    // each thread takes a contiguous range of the batch's pairs, so its
    // owner cell changes rarely: found once by search, then walked forward,
    // with the cell's corners and edge slopes kept in registers meanwhile
    const int32_t chunk = (total + kThreads - 1) / kThreads;
    int32_t w = t * chunk;
    const int32_t wend = min(total, w + chunk);
    if (w < wend) {
      int lo = 0, hi = kThreads - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sfirst[mid] <= w) lo = mid; else hi = mid - 1;
      }
      int cur = -1;
      double cq[4][2], X[2], k[4], kinv[4], inv = 0.0;
      int kind = 0, o = 0;
      int32_t bu = 0, bv = 0, bw = 1;
      for (; w < wend; ++w) {
        // sfirst[lo] <= w < sfirst[lo + 1] (cells without pairs are skipped)
        while (w >= sfirst[lo + 1]) ++lo;
        if (lo != cur) {
          cur = lo;
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            cq[cc][0] = sq[lo][2 * cc];
            cq[cc][1] = sq[lo][2 * cc + 1];
          }
          X[0] = sq[lo][8];
          X[1] = sq[lo][9];
#pragma unroll
          for (int e = 0; e < 4; ++e) edge_slope(cq[e], cq[(e + 1) & 3], k[e], kinv[e]);
          inv = sinv[lo];
          kind = sshape[lo] & 3;
          o = (sshape[lo] >> 2) - 1;
          bu = sbox[lo][0];
          bv = sbox[lo][1];
          bw = sbox[lo][2];
        }
        const int32_t local = w - sfirst[lo];
        const int32_t u = bu + local % bw, v = bv + local / bw;
        if (kind == 0 && o != 0 && convex_misses(cq, o, (double)u, (double)v)) continue;
        const double ov = cell_pixel_overlap(cq, X, kind, k, kinv, (double)u, (double)v);
        if (ov > 0.0) table_add(tkey, tval, a.acc, v * npix + u, to_fix(a.cell_px * (ov * inv)));
      }
    }
    __syncthreads();  // the batch's shared cells are consumed
  }
  for (int e = t; e < kTable; e += kThreads)
    if (tkey[e] >= 0) atomicAdd(&a.acc[tkey[e]], tval[e]);
}

// Wide cells are apportioned edge by edge.  By Green's theorem the overlap
// of a polygon with pixel (u, v) is the sum over its edges of
// T_e(u) = +-int clamp01(x(y) - u) dy over the edge's part in the strip
// [v, v+1] (edge_term), signed by the polygon's orientation.  Along a map row
// T_e(u) is the constant C_e = +-(height of that part) for every pixel left
// of the edge, 0 for every pixel right of it, and needs the integral only
// for the pixels the edge passes through.  Since the C_e of a closed polygon
// sum to zero in every strip,
//     sum_e T_e(u) = sum_e ( -C_e [u >= ulo_e] + P_e(u) [ulo_e <= u <= uhi_e] ),
// with [ulo_e, uhi_e] the pixels the edge crosses in that row: each (edge,
// row) adds -C_e to the row-difference accumulator at ulo_e (prefix-summed
// along the row by the final pass) and P_e(u) = T_e(u) to the few pixels it
// crosses.  C_e is formed in fixed point as G(y_end) - G(y_start) with
// G(y) = fix((y - v) w), so the constants of a closed polygon cancel exactly
// in integers and pixels outside it receive exactly nothing.  Work is
// proportional to the image's perimeter in pixels, not its area.

// An edge's part in the strip [v, v+1]: heights yb < yt, the x extent
// [xl, xh] there and (signed) start/end heights in the edge's direction.
__device__ __forceinline__ bool edge_strip(double ax, double ay, double bx, double by, double k,
                                           double v, double &xl, double &xh, double &ys,
                                           double &ye) {
  const double ey0 = fmin(ay, by), ey1 = fmax(ay, by);
  const double yb = fmax(ey0, v), yt = fmin(ey1, v + 1.0);
  if (!(yb < yt)) return false;
  const double xb = yb == ay ? ax : (yb == by ? bx : ax + (yb - ay) * k);
  const double xt = yt == ay ? ax : (yt == by ? bx : ax + (yt - ay) * k);
  xl = fmin(xb, xt);
  xh = fmax(xb, xt);
  const bool up = by > ay;
  ys = up ? yb : yt;
  ye = up ? yt : yb;
  return true;
}

// One polygon edge of a queued cell, with the items the wave's lanes take:
// a steep edge (at least as many rows as columns in the map) one item per
// row (its crossed pixels and its difference entry); a flat one an item per
// column (the pixels it crosses there) plus an item per row (the difference
// entry only).
struct EdgeJob {
  double ax, ay, bx, by, k, kinv, w;
  int32_t steep, r0, nr, c0, nc, first;
};
constexpr int kMaxEdges = 8;  // two triangles, or one quadrilateral

__device__ __forceinline__ void row_item(const EdgeJob &e, int32_t v, bool pixels,
                                         const IpmArgs &a) {
  const int32_t npix = a.npix;
  double xl, xh, ys, ye;
  if (!edge_strip(e.ax, e.ay, e.bx, e.by, e.k, (double)v, xl, xh, ys, ye)) return;
  const double ulo = floor(xl), uhi = ceil(xh) - 1.0;
  if (pixels) {
    const double ua = fmax(ulo, 0.0), ub = fmin(uhi, (double)(npix - 1));
    for (int32_t u = (int32_t)ua; (double)u <= ub; ++u) {
      const double t = edge_term(e.ax - u, e.ay - v, e.bx - u, e.by - v, e.k, e.kinv);
      if (t != 0.0) atomicAdd(&a.acc[(int64_t)v * npix + u], to_fix(t * e.w));
    }
  }
  if (ulo < (double)npix) {
    const unsigned long long c = to_fix((ye - v) * e.w) - to_fix((ys - v) * e.w);
    if (c != 0ull) {
      const int32_t d = ulo < 0.0 ? 0 : (int32_t)ulo;
      atomicAdd(&a.diff[(int64_t)v * (npix + 1) + d], 0ull - c);
    }
  }
}

__device__ __forceinline__ void column_item(const EdgeJob &e, int32_t u, const IpmArgs &a) {
  const int32_t npix = a.npix;
  const double ex0 = fmin(e.ax, e.bx), ex1 = fmax(e.ax, e.bx);
  const double x0 = fmax(ex0, (double)u), x1 = fmin(ex1, (double)u + 1.0);
  if (!(x0 <= x1)) return;
  const double y0 = x0 == e.ax ? e.ay : (x0 == e.bx ? e.by : e.ay + (x0 - e.ax) * e.kinv);
  const double y1 = x1 == e.ax ? e.ay : (x1 == e.bx ? e.by : e.ay + (x1 - e.ax) * e.kinv);
  // rows this column's part may touch, one row of margin either way; a row
  // takes the pixel only if its own strip test puts u among the crossed ones
  const double vlo = fmax(floor(fmin(y0, y1)) - 1.0, (double)e.r0);
  const double vhi = fmin(ceil(fmax(y0, y1)), (double)(e.r0 + e.nr - 1));
  for (int32_t v = (int32_t)vlo; (double)v <= vhi; ++v) {
    double xl, xh, ys, ye;
    if (!edge_strip(e.ax, e.ay, e.bx, e.by, e.k, (double)v, xl, xh, ys, ye)) continue;
    if ((double)u < floor(xl) || (double)u > ceil(xh) - 1.0) continue;
    const double t = edge_term(e.ax - u, e.ay - v, e.bx - u, e.by - v, e.k, e.kinv);
    if (t != 0.0) atomicAdd(&a.acc[(int64_t)v * npix + u], to_fix(t * e.w));
  }
}

// Adds the edges of polygon P (n vertices) to the wave's job table.
__device__ __forceinline__ void add_edges(const double (*P)[2], int n, double w, int32_t npix,
                                          EdgeJob *jobs, int &ne, int32_t &items) {
  // orientation: every edge term is signed by it, so the weight carries it
  double s = 0.0;
  for (int e = 0; e < n; ++e) {
    const int e1 = e + 1 == n ? 0 : e + 1;
    s += (P[e][0] - P[0][0]) * (P[e1][1] - P[0][1]) - (P[e1][0] - P[0][0]) * (P[e][1] - P[0][1]);
  }
  const double ws = s < 0.0 ? -w : w;
  for (int e = 0; e < n; ++e) {
    const int e1 = e + 1 == n ? 0 : e + 1;
    const double ax = P[e][0], ay = P[e][1], bx = P[e1][0], by = P[e1][1];
    if (ay == by) continue;  // horizontal: no term
    const double ey0 = fmin(ay, by), ey1 = fmax(ay, by), ex0 = fmin(ax, bx), ex1 = fmax(ax, bx);
    if (!(ey1 >= 0.0) || !(ey0 < (double)npix) || !(ex0 < (double)npix)) continue;
    // an edge wholly left of the map (ex1 < 0) still shifts its rows
    const double r0 = fmax(floor(ey0), 0.0), r1 = fmin(floor(ey1), (double)(npix - 1));
    const double c0 = fmax(floor(ex0), 0.0), c1 = fmin(floor(ex1), (double)(npix - 1));
    EdgeJob &j = jobs[ne++];
    j.ax = ax, j.ay = ay, j.bx = bx, j.by = by, j.w = ws;
    edge_slope(P[e], P[e1], j.k, j.kinv);
    j.r0 = (int32_t)r0;
    j.nr = (int32_t)(r1 - r0) + 1;
    j.c0 = (int32_t)c0;
    j.nc = c1 >= c0 ? (int32_t)(c1 - c0) + 1 : 0;
    j.steep = j.nr >= j.nc;
    j.first = items;
    items += j.steep ? j.nr : j.nc + j.nr;
  }
}

// Orders the LDS accesses of a converged wave (its lanes exchange data
// through LDS without a workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wave per queued cell: its image (the quadrilateral, or a folded cell's
// two lobes) becomes a table of edge jobs in LDS, and the wave's lanes take
// the jobs' items in turn, so even a cell of a few rows keeps most lanes busy.
// Waves pull cells in a fixed stride and exit past the queue's end.
__global__ __launch_bounds__(kThreads) void k_ipm_wide(IpmArgs a) {
  __shared__ EdgeJob jobs_all[kThreads / 64][kMaxEdges];
  __shared__ int32_t counts_all[kThreads / 64][2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  EdgeJob *jobs = jobs_all[wv];
  const uint32_t nq = *a.qcount;
  const int64_t ncx = a.nx - 1;
  const uint32_t waves = gridDim.x * (kThreads / 64);
  for (uint32_t q = blockIdx.x * (kThreads / 64) + wv; q < nq; q += waves) {
    const uint32_t id = a.queue[q];
    const int64_t i = (int64_t)(id % (uint64_t)ncx), j = a.j0 + (int64_t)(id / (uint64_t)ncx);
    Cell c;
    load_quad(a, i, j, c.q);  // finite: it was queued
    classify(c);
    const double w = a.cell_px / c.area;
    wave_sync();  // the previous cell's items have read the table
    if (lane == 0) {
      // lane 0 writes the table to LDS; the others read it after the sync
      int ne = 0;
      int32_t items = 0;
      if (c.kind == 0) {
        add_edges(c.q, 4, w, a.npix, jobs, ne, items);
      } else {
        const int ia = c.kind == 1 ? 0 : 1;
        double T[3][2];
        T[0][0] = c.X[0], T[0][1] = c.X[1];
        T[1][0] = c.q[ia + 1][0], T[1][1] = c.q[ia + 1][1];
        T[2][0] = c.q[ia + 2][0], T[2][1] = c.q[ia + 2][1];
        add_edges(T, 3, w, a.npix, jobs, ne, items);
        T[0][0] = c.q[ia][0], T[0][1] = c.q[ia][1];
        T[1][0] = c.X[0], T[1][1] = c.X[1];
        T[2][0] = c.q[(ia + 3) & 3][0], T[2][1] = c.q[(ia + 3) & 3][1];
        add_edges(T, 3, w, a.npix, jobs, ne, items);
      }
      counts_all[wv][0] = ne;
      counts_all[wv][1] = items;
    }
    wave_sync();
    const int ne = counts_all[wv][0];
    const int32_t items = counts_all[wv][1];
    for (int32_t t = lane; t < items; t += 64) {
      int e = 0;
      while (e + 1 < ne && jobs[e + 1].first <= t) ++e;
      const EdgeJob &jb = jobs[e];
      const int32_t r = t - jb.first;
      if (jb.steep) {
        row_item(jb, jb.r0 + r, true, a);
      } else if (r < jb.nc) {
        column_item(jb, jb.c0 + r, a);
      } else {
        row_item(jb, jb.r0 + (r - jb.nc), false, a);
      }
    }
  }
}

// mu[v][u] += (acc[v][u] + sum_{u' <= u} diff[v][u']) 2^-40: a workgroup per
// map row, the row's differences prefix-summed 256 at a time (integers, so
// the result does not depend on the order).
__global__ __launch_bounds__(kThreads) void k_ipm_finish(const unsigned long long *__restrict__ acc,
                                                         const unsigned long long *__restrict__ diff,
                                                         int32_t npix, double *__restrict__ mu) {
  __shared__ unsigned long long wsum[kThreads / 64];
  const int64_t v = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long *drow = diff + v * (int64_t)(npix + 1);
  unsigned long long carry = 0;
  for (int32_t base = 0; base < npix; base += kThreads) {
    const int32_t u = base + (int32_t)threadIdx.x;
    unsigned long long x = u < npix ? drow[u] : 0ull;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const unsigned long long y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    unsigned long long off = carry, tot = carry;
#pragma unroll
    for (int q = 0; q < kThreads / 64; ++q) {
      if (q < w) off += wsum[q];
      tot += wsum[q];
    }
    if (u < npix) {
      const int64_t idx = v * npix + u;
      mu[idx] += (double)(long long)(acc[idx] + off + x) * (1.0 / kFix);
    }
    carry = tot;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void k_zero_u64(unsigned long long *__restrict__ p, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads)
    p[k] = 0ull;
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

// workgroups of the wide-cell kernel
constexpr unsigned kWideBlocks = 1536;  // six waves per SIMD (its register limit)

}  // namespace

void launch_ipm_zero(unsigned long long *acc, int64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n)), dim3(kThreads), 0, stream, acc, n);
  LENS_HIP(hipGetLastError());
}

void launch_ipm_cells(const IpmPass &p, hipStream_t stream) {
  const int64_t ncx = p.nx - 1, nrows = p.j1 - p.j0;
  if (ncx <= 0 || nrows <= 0) return;
  const int64_t patches = ((ncx + kPatch - 1) / kPatch) * ((nrows + kPatch - 1) / kPatch);
  if (patches > 0x7fffffff) fail(LENS_EUNSUPPORTED, "IPM pass too large");
  if (ncx * nrows > (int64_t)0xffffffffu) fail(LENS_EUNSUPPORTED, "IPM pass too large");
  IpmArgs a{p.y, p.nx, p.ybase, p.j0, p.j1, p.cell_px, p.y1min, p.y2min, p.S, p.npix,
            p.acc, p.diff, p.queue, p.qcount};
  launch_fill_u32(p.qcount, 1, 0u, stream);
  hipLaunchKernelGGL(k_ipm, dim3((unsigned)patches), dim3(kThreads), 0, stream, a);
  LENS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_ipm_wide, dim3(kWideBlocks), dim3(kThreads), 0, stream, a);
  LENS_HIP(hipGetLastError());
}

void launch_ipm_finish(const unsigned long long *acc, const unsigned long long *diff, int32_t npix,
                       double *mu, hipStream_t stream) {
  hipLaunchKernelGGL(k_ipm_finish, dim3((unsigned)npix), dim3(kThreads), 0, stream, acc, diff, npix,
                     mu);
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
