// Inverse polygon mapping (Section 2.3; first order, as used in Section 2.4).
// Adjacent grid rays are the corners of image-plane cells of area dx dy; cell
// (i, j) with corners y(i,j), y(i+1,j), y(i+1,j+1), y(i,j+1) maps to a
// quadrilateral Q in the source plane, and its area is shared among the
// pixels Q overlaps in proportion to the overlap areas: pixel P receives
// dx dy |Q n P| / |Q|; divided by the pixel area that is the magnification
// sum S_i / S_pixel.  A quadrilateral whose edges cross (a cell on a critical
// curve), whose area is zero or whose bounding box covers more than
// max_pixels map pixels goes to its corners: a quarter of the cell to each
// corner's pixel (the zeroth-order, inverse-ray-shooting rule).
//
// Geometry in pixel units p = (y - ymin) S, S = npix/side.  Overlaps come
// from Green's theorem as a sum of four edge terms (see quad_pixel_overlap),
// which needs no per-thread polygon storage.  Contributions are summed as fixed-point
// integers (units of 2^-40 of a pixel's magnification) with 64-bit atomics,
// so the map does not depend on the order of the additions; a final pass adds
// them to the caller's FP64 map.  One thread per cell; a cell inside one
// pixel (the common case) adds the whole cell; sums go through an LDS table
// of pixels per workgroup (one global atomic per distinct pixel).  For a
// convex quadrilateral, pixels of its bounding box that lie outside one of
// its edge lines are skipped before the overlap sum.
#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kThreads = 256;
constexpr double kFix = 1099511627776.0;  // 2^40

__device__ __forceinline__ double orient2(double ax, double ay, double bx, double by, double cx,
                                          double cy) {
  return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

__device__ __forceinline__ bool segments_cross(const double (&a)[2], const double (&b)[2],
                                               const double (&c)[2], const double (&d)[2]) {
  const double o1 = orient2(a[0], a[1], b[0], b[1], c[0], c[1]);
  const double o2 = orient2(a[0], a[1], b[0], b[1], d[0], d[1]);
  const double o3 = orient2(c[0], c[1], d[0], d[1], a[0], a[1]);
  const double o4 = orient2(c[0], c[1], d[0], d[1], b[0], b[1]);
  return ((o1 > 0 && o2 < 0) || (o1 < 0 && o2 > 0)) && ((o3 > 0 && o4 < 0) || (o3 < 0 && o4 > 0));
}

// Twice the signed area of a quadrilateral (shoelace, vertex order).
__device__ __forceinline__ double shoelace4(const double (&q)[4][2]) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int k1 = (k + 1) & 3;
    s += q[k][0] * q[k1][1] - q[k1][0] * q[k][1];
  }
  return s;
}

__device__ __forceinline__ double clamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }

// Signed contribution of edge a -> b to the area of (polygon n unit square):
// the line integral of clamp01(x) dy over the edge's part with 0 <= y <= 1.
// On that part x(y) = lx + (y - ly) k is linear, so clamp01(x(y)) is linear
// between the heights where x crosses 0 and 1 and the trapezoid rule on those
// pieces is exact.  k = dx/dy and kinv = dy/dx (0 for a vertical edge) depend
// only on the edge's direction, not on the pixel.
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

// Area of quadrilateral q (pixel units) inside the square [u,u+1] x [v,v+1].
// By Green's theorem the area of (Q n B) for the unit square B is the line
// integral of clamp01(x) dy over the boundary of Q restricted to 0 <= y <= 1
// (d/dx clamp01 is the indicator of 0 < x < 1): a sum of four edge terms,
// with no clipped polygon to store.  Signed by Q's orientation; |.| taken.
__device__ double quad_pixel_overlap(const double (&q)[4][2], const double (&k)[4],
                                    const double (&kinv)[4], double u, double v) {
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int e1 = (e + 1) & 3;
    s += edge_term(q[e][0] - u, q[e][1] - v, q[e1][0] - u, q[e1][1] - v, k[e], kinv[e]);
  }
  return fabs(s);
}

// Per-edge slopes of q for edge_term: k = dx/dy (0 for a horizontal edge),
// kinv = dy/dx (0 for a vertical one).  They depend only on the cell.
__device__ __forceinline__ void edge_slopes(const double (&q)[4][2], double (&k)[4],
                                            double (&kinv)[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int e1 = (e + 1) & 3;
    const double dx = q[e1][0] - q[e][0], dy = q[e1][1] - q[e][1];
    k[e] = dy != 0.0 ? dx * rcp_f64(dy) : 0.0;
    kinv[e] = dx == 0.0 ? 0.0 : dy * rcp_f64(dx);
  }
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
  int32_t npix, max_pixels;
  unsigned long long *acc;
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

__device__ __forceinline__ double quad_area(const double (&q)[4][2]) {
  return fabs(0.5 * shoelace4(q));
}

// Pixel bounding box of q clamped to the map; false if it misses the map.
__device__ __forceinline__ bool quad_bbox(const double (&q)[4][2], int32_t npix, int64_t &u0,
                                          int64_t &v0, int64_t &u1, int64_t &v1, bool &inside) {
  double lo0 = q[0][0], hi0 = q[0][0], lo1 = q[0][1], hi1 = q[0][1];
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    lo0 = fmin(lo0, q[k][0]);
    hi0 = fmax(hi0, q[k][0]);
    lo1 = fmin(lo1, q[k][1]);
    hi1 = fmax(hi1, q[k][1]);
  }
  u0 = lo0 < 0.0 ? 0 : (int64_t)floor(lo0);
  v0 = lo1 < 0.0 ? 0 : (int64_t)floor(lo1);
  u1 = hi0 >= (double)npix ? npix - 1 : (int64_t)floor(hi0);
  v1 = hi1 >= (double)npix ? npix - 1 : (int64_t)floor(hi1);
  inside = lo0 >= 0.0 && lo1 >= 0.0 && hi0 < (double)npix && hi1 < (double)npix;
  return !(hi0 < 0.0 || hi1 < 0.0 || lo0 >= (double)npix || lo1 >= (double)npix);
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

// One workgroup per kPatch x kPatch patch of cells, taken 256 cells at a
// time, one thread per cell.  A cell inside one pixel adds the whole cell; a
// folded, degenerate or too wide cell goes to its corners.  A cell over
// several pixels (at most max_pixels) is apportioned by its overlaps; those
// (cell, pixel) pairs of the 256 cells are numbered by a scan and shared out
// evenly over the workgroup's threads, so a few wide cells near a star do
// not hold a whole wave.
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

__global__ __launch_bounds__(kThreads) void k_ipm(IpmArgs a) {
  __shared__ int32_t tkey[kTable];
  __shared__ unsigned long long tval[kTable];
  __shared__ double sq[kThreads][8];  // wide cells of the batch: corners,
  __shared__ double sk[kThreads][8];   // edge slopes (k, kinv),
  __shared__ double sinv[kThreads];    // 1 / area,
  __shared__ int32_t sorient[kThreads];  // orientation if convex, else 0,
  __shared__ int32_t sbox[kThreads][3];  // u0, v0, columns of the bounding box
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
  const unsigned long long q_cell = (unsigned long long)llrint(a.cell_px * kFix);
  const unsigned long long q_quarter = (unsigned long long)llrint(0.25 * a.cell_px * kFix);
  for (int base = 0; base < kPatch * kPatch; base += kThreads) {
    const int k = base + t;
    const int64_t i = pi * kPatch + (k % kPatch), j = a.j0 + pj * kPatch + (k / kPatch);
    int32_t npairs = 0;
    double q[4][2];
    if (i < ncx && j < a.j1 && load_quad(a, i, j, q)) {
      const double area = quad_area(q);
      const bool folded = segments_cross(q[0], q[1], q[2], q[3]) || segments_cross(q[1], q[2], q[3], q[0]);
      int64_t u0, v0, u1, v1;
      bool inside;
      const bool outside = !quad_bbox(q, npix, u0, v0, u1, v1, inside);
      const int64_t npx = (u1 - u0 + 1) * (v1 - v0 + 1);
      if (folded || !(area > 0.0) || (!outside && npx > a.max_pixels)) {
        // zeroth order: a quarter of the cell to each corner's pixel
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t pk = pixel_of(q[c], npix);
          if (pk >= 0) table_add(tkey, tval, a.acc, (int32_t)pk, q_quarter);
        }
      } else if (!outside) {
        if (u0 == u1 && v0 == v1 && inside) {
          table_add(tkey, tval, a.acc, (int32_t)(v0 * npix + u0), q_cell);  // wholly inside
        } else {
          npairs = (int32_t)npx;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            sq[t][2 * c] = q[c][0];
            sq[t][2 * c + 1] = q[c][1];
          }
          double k[4], kinv[4];
          edge_slopes(q, k, kinv);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            sk[t][e] = k[e];
            sk[t][4 + e] = kinv[e];
          }
          sinv[t] = 1.0 / area;
          sorient[t] = convex_orientation(q);
          sbox[t][0] = (int32_t)u0;
          sbox[t][1] = (int32_t)v0;
          sbox[t][2] = (int32_t)(u1 - u0 + 1);
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
    // with the cell's corners and slopes kept in registers meanwhile
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
      double cq[4][2], k[4], kinv[4], inv = 0.0;
      int o = 0;
      int32_t bu = 0, bv = 0, bw = 1;
      for (; w < wend; ++w) {
        // sfirst[lo] <= w < sfirst[lo + 1] (cells without pairs are skipped)
        while (w >= sfirst[lo + 1]) ++lo;
        if (lo != cur) {
          cur = lo;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            cq[c][0] = sq[lo][2 * c];
            cq[c][1] = sq[lo][2 * c + 1];
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            k[e] = sk[lo][e];
            kinv[e] = sk[lo][4 + e];
          }
          inv = sinv[lo];
          o = sorient[lo];
          bu = sbox[lo][0];
          bv = sbox[lo][1];
          bw = sbox[lo][2];
        }
        const int32_t local = w - sfirst[lo];
        const int32_t u = bu + local % bw, v = bv + local / bw;
        if (o != 0 && convex_misses(cq, o, (double)u, (double)v)) continue;
        const double ov = quad_pixel_overlap(cq, k, kinv, (double)u, (double)v);
        if (ov > 0.0)
          table_add(tkey, tval, a.acc, v * npix + u,
                    (unsigned long long)llrint(a.cell_px * (ov * inv) * kFix));
      }
    }
    __syncthreads();  // the batch's shared cells are consumed
  }
  for (int e = t; e < kTable; e += kThreads)
    if (tkey[e] >= 0) atomicAdd(&a.acc[tkey[e]], tval[e]);
}

__global__ __launch_bounds__(kThreads) void k_ipm_finish(const unsigned long long *__restrict__ acc,
                                                         int64_t n, double *__restrict__ mu) {
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kThreads)
    mu[k] += (double)(long long)acc[k] * (1.0 / kFix);
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

}  // namespace

void launch_ipm_zero(unsigned long long *acc, int64_t n, hipStream_t stream) {
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n)), dim3(kThreads), 0, stream, acc, n);
  LENS_HIP(hipGetLastError());
}

void launch_ipm_cells(const double *y, int64_t nx, int64_t ybase, int64_t j0, int64_t j1,
                      double cell_px, double y1min, double y2min, double S, int32_t npix,
                      int32_t max_pixels, unsigned long long *acc, hipStream_t stream) {
  const int64_t ncx = nx - 1, nrows = j1 - j0;
  if (ncx <= 0 || nrows <= 0) return;
  const int64_t patches = ((ncx + kPatch - 1) / kPatch) * ((nrows + kPatch - 1) / kPatch);
  if (patches > 0x7fffffff) fail(LENS_EUNSUPPORTED, "IPM pass too large");
  IpmArgs a{y, nx, ybase, j0, j1, cell_px, y1min, y2min, S, npix, max_pixels, acc};
  hipLaunchKernelGGL(k_ipm, dim3((unsigned)patches), dim3(kThreads), 0, stream, a);
  LENS_HIP(hipGetLastError());
}

void launch_ipm_finish(const unsigned long long *acc, int64_t n, double *mu, hipStream_t stream) {
  hipLaunchKernelGGL(k_ipm_finish, dim3(grid_for(n)), dim3(kThreads), 0, stream, acc, n, mu);
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
