// Inverse polygon mapping (Section 2.3; first order, as used in Section 2.4).
// Adjacent grid rays are the corners of image-plane cells of area dx dy; cell
// (i, j) with corners y(i,j), y(i+1,j), y(i+1,j+1), y(i,j+1) maps to a
// quadrilateral Q in the source plane, and its area is shared among the
// pixels Q overlaps in proportion to the overlap areas: pixel P receives
// dx dy |Q n P| / |Q|; divided by the pixel area that is the magnification
// sum S_i / S_pixel.  A quadrilateral whose edges cross (a cell on a critical
// curve) or whose area is zero goes to its corners: a quarter of the cell to
// each corner's pixel (the zeroth-order, inverse-ray-shooting rule).
//
// Geometry in pixel units p = (y - ymin) S, S = npix/side.  Overlaps come
// from clipping Q against the pixel square (Sutherland-Hodgman) and the
// shoelace area of the result.  Contributions are summed as fixed-point
// integers (units of 2^-40 of a pixel's magnification) with 64-bit atomics,
// so the map does not depend on the order of the additions; a final pass adds
// them to the caller's FP64 map.  One thread per cell; a cell inside one
// pixel (the common case) adds the same amount, so those are aggregated per
// wave with a ballot loop (one atomic per distinct pixel).
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

// Twice the signed area of the first n vertices, summed in vertex order.
template <int N>
__device__ __forceinline__ double shoelace2(int n, const double (&x)[N], const double (&y)[N]) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) {
    const int k1 = k + 1 < n ? k + 1 : 0;
    s += x[k] * y[k1] - x[k1] * y[k];
  }
  return s;
}

// Keep the part of polygon (ix, iy)[n] with coordinate c >= bound (ge) or
// <= bound (!ge); writes (ox, oy), returns the new vertex count.
__device__ __forceinline__ int clip_half(int n, const double (&ix)[12], const double (&iy)[12],
                                         double (&ox)[12], double (&oy)[12], int c, double bound,
                                         bool ge) {
  int m = 0;
  for (int k = 0; k < n; ++k) {
    const int ks = k > 0 ? k - 1 : n - 1;
    const double sx = ix[ks], sy = iy[ks], ex = ix[k], ey = iy[k];
    const double sc = c == 0 ? sx : sy, ec = c == 0 ? ex : ey;
    const bool sin_ = ge ? sc >= bound : sc <= bound;
    const bool ein = ge ? ec >= bound : ec <= bound;
    if (ein != sin_) {
      const double t = (bound - sc) / (ec - sc);
      if (c == 0) {
        ox[m] = bound;
        oy[m] = sy + t * (ey - sy);
      } else {
        ox[m] = sx + t * (ex - sx);
        oy[m] = bound;
      }
      ++m;
    }
    if (ein) {
      ox[m] = ex;
      oy[m] = ey;
      ++m;
    }
  }
  return m;
}

// Area of quadrilateral q (pixel units) inside the square [u,u+1] x [v,v+1].
__device__ double quad_pixel_overlap(const double (&q)[4][2], double u, double v) {
  double ax[12], ay[12], bx[12], by[12];
  for (int k = 0; k < 4; ++k) {
    ax[k] = q[k][0] - u;
    ay[k] = q[k][1] - v;
  }
  int n = 4;
  n = clip_half(n, ax, ay, bx, by, 0, 0.0, true);
  n = clip_half(n, bx, by, ax, ay, 0, 1.0, false);
  n = clip_half(n, ax, ay, bx, by, 1, 0.0, true);
  n = clip_half(n, bx, by, ax, ay, 1, 1.0, false);
  return n >= 3 ? fabs(0.5 * shoelace2(n, ax, ay)) : 0.0;
}

__device__ __forceinline__ void add_fixed(unsigned long long *acc, int64_t k, double value) {
  atomicAdd(&acc[k], (unsigned long long)llrint(value * kFix));
}

__device__ __forceinline__ int64_t pixel_of(const double (&p)[2], int32_t npix) {
  if (!(p[0] >= 0.0) || !(p[1] >= 0.0)) return -1;
  const double f1 = floor(p[0]), f2 = floor(p[1]);
  if (f1 >= (double)npix || f2 >= (double)npix) return -1;
  return (int64_t)f2 * npix + (int64_t)f1;
}

// One thread per cell of rows [j0, j1) (all nx - 1 columns); y holds rows
// [ybase, ...) of the mapped grid, row-major with nx rays per row.
__global__ __launch_bounds__(kThreads) void k_ipm(const double *__restrict__ y, int64_t nx,
                                                  int64_t ybase, int64_t j0, int64_t j1,
                                                  double cell_px, double y1min, double y2min,
                                                  double S, int32_t npix, int32_t max_pixels,
                                                  unsigned long long *__restrict__ acc) {
  const int64_t ncell = (nx - 1) * (j1 - j0);
  const int lane = threadIdx.x & 63;
  const unsigned long long q_cell = (unsigned long long)llrint(cell_px * kFix);
  for (int64_t base = (int64_t)blockIdx.x * kThreads; base < ncell;
       base += (int64_t)gridDim.x * kThreads) {  // uniform per wave
    const int64_t c = base + threadIdx.x;
    int64_t fast_key = -1;
    if (c < ncell) {
      const int64_t j = j0 + c / (nx - 1), i = c % (nx - 1);
      const int64_t r0 = (j - ybase) * nx + i, r1 = r0 + nx;
      const int64_t id[4] = {r0, r0 + 1, r1 + 1, r1};
      double q[4][2];
      bool finite = true;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        q[k][0] = (y[2 * id[k]] - y1min) * S;
        q[k][1] = (y[2 * id[k] + 1] - y2min) * S;
        finite = finite && isfinite(q[k][0]) && isfinite(q[k][1]);
      }
      if (finite) {
        double xs[4], ys[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          xs[k] = q[k][0];
          ys[k] = q[k][1];
        }
        const double area = fabs(0.5 * shoelace2(4, xs, ys));
        const bool folded = segments_cross(q[0], q[1], q[2], q[3]) || segments_cross(q[1], q[2], q[3], q[0]);
        double lo0 = q[0][0], hi0 = q[0][0], lo1 = q[0][1], hi1 = q[0][1];
#pragma unroll
        for (int k = 1; k < 4; ++k) {
          lo0 = fmin(lo0, q[k][0]);
          hi0 = fmax(hi0, q[k][0]);
          lo1 = fmin(lo1, q[k][1]);
          hi1 = fmax(hi1, q[k][1]);
        }
        const int64_t u0 = lo0 < 0.0 ? 0 : (int64_t)floor(lo0);
        const int64_t v0 = lo1 < 0.0 ? 0 : (int64_t)floor(lo1);
        const int64_t u1 = hi0 >= (double)npix ? npix - 1 : (int64_t)floor(hi0);
        const int64_t v1 = hi1 >= (double)npix ? npix - 1 : (int64_t)floor(hi1);
        const bool outside = hi0 < 0.0 || hi1 < 0.0 || lo0 >= (double)npix || lo1 >= (double)npix;
        const int64_t npx = (u1 - u0 + 1) * (v1 - v0 + 1);
        if (folded || !(area > 0.0) || (!outside && npx > max_pixels)) {
          // zeroth order: a quarter of the cell to each corner's pixel (also
          // for a cell stretched over more than max_pixels pixels)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int64_t pk = pixel_of(q[k], npix);
            if (pk >= 0) add_fixed(acc, pk, 0.25 * cell_px);
          }
        } else if (!outside) {
          if (u0 == u1 && v0 == v1 && lo0 >= 0.0 && lo1 >= 0.0 && hi0 < (double)npix &&
              hi1 < (double)npix) {
            fast_key = v0 * npix + u0;  // wholly inside one pixel
          } else {
            for (int64_t v = v0; v <= v1; ++v)
              for (int64_t u = u0; u <= u1; ++u) {
                const double ov = quad_pixel_overlap(q, (double)u, (double)v);
                if (ov > 0.0) add_fixed(acc, v * npix + u, cell_px * (ov / area));
              }
          }
        }
      }
    }
    // cells wholly inside one pixel all add cell_px: one atomic per pixel
    uint64_t pending = __ballot(fast_key >= 0);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const int64_t k = __shfl(fast_key, leader);
      const uint64_t same = __ballot(fast_key == k);
      if (lane == leader) atomicAdd(&acc[k], q_cell * (unsigned long long)__popcll(same));
      pending &= ~same;
    }
  }
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
  const int64_t ncell = (nx - 1) * (j1 - j0);
  if (ncell <= 0) return;
  hipLaunchKernelGGL(k_ipm, dim3(grid_for(ncell)), dim3(kThreads), 0, stream, y, nx, ybase, j0, j1,
                     cell_px, y1min, y2min, S, npix, max_pixels, acc);
  LENS_HIP(hipGetLastError());
}

void launch_ipm_finish(const unsigned long long *acc, int64_t n, double *mu, hipStream_t stream) {
  hipLaunchKernelGGL(k_ipm_finish, dim3(grid_for(n)), dim3(kThreads), 0, stream, acc, n, mu);
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
