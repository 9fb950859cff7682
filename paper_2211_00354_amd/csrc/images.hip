// Inverse lens equation, critical curves and multi-plane chaining, built on
// the deflection of a ray grid (Section 2.5 finds the images of a source
// behind a particle halo; Appendix A notes that the expansions give the
// derivatives of the field in closed form; the introduction's footnote
// extends the thin lens to a chain of planes).
//
// Images.  The grid rays are the corners of cells, each split along its
// (i, j)-(i+1, j+1) diagonal into two triangles.  A triangle whose mapped
// corners contain a source (inclusive barycentric test, so a source on a
// shared edge is seen by both sides) seeds a candidate at the preimage of the
// source under the triangle's linear map.  Candidates are then refined by
// Newton steps on y(x) = beta with the Jacobian
//     A = [[c1 - Re f', Im f'], [Im f', c2 + Re f']],   f' = -sum m/(z - z_i)^2,
// (alpha = conj f, f holomorphic), steps clamped in length and to the ray
// region.
//
// Critical curves.  det A at every grid ray, then marching squares on the
// cells: a cell edge whose end values differ in sign is cut where the linear
// interpolant vanishes; a cell cut on four edges is split by the sign of the
// mean of its corners.
#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double cross2(double ax, double ay, double bx, double by) {
  return ax * by - ay * bx;
}

__global__ __launch_bounds__(kThreads) void k_image_cells(ImageCellArgs a) {
  const int64_t ncx = a.nx - 1;
  const int64_t ncell = ncx * (a.j1 - a.j0);
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= ncell) return;
  const int64_t i = k % ncx, j = a.j0 + k / ncx;
  const int64_t r0 = (j - a.ybase) * a.nx + i, r1 = r0 + a.nx;
  const int64_t id[4] = {r0, r0 + 1, r1 + 1, r1};
  // image-plane corners (grid rays) and their images
  const double X[4] = {grid_coord(a.grid.x0, a.grid.dx, i), grid_coord(a.grid.x0, a.grid.dx, i + 1),
                       grid_coord(a.grid.x0, a.grid.dx, i + 1), grid_coord(a.grid.x0, a.grid.dx, i)};
  const double Y[4] = {grid_coord(a.grid.y0, a.grid.dy, j), grid_coord(a.grid.y0, a.grid.dy, j),
                       grid_coord(a.grid.y0, a.grid.dy, j + 1), grid_coord(a.grid.y0, a.grid.dy, j + 1)};
  double q[4][2];
  bool finite = true;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    q[c][0] = a.y[2 * id[c]];
    q[c][1] = a.y[2 * id[c] + 1];
    finite = finite && isfinite(q[c][0]) && isfinite(q[c][1]);
  }
  if (!finite) return;
  double lo0 = q[0][0], hi0 = q[0][0], lo1 = q[0][1], hi1 = q[0][1];
#pragma unroll
  for (int c = 1; c < 4; ++c) {
    lo0 = fmin(lo0, q[c][0]);
    hi0 = fmax(hi0, q[c][0]);
    lo1 = fmin(lo1, q[c][1]);
    hi1 = fmax(hi1, q[c][1]);
  }
  for (int32_t s = 0; s < a.n_src; ++s) {
    const double b0 = a.src[2 * s], b1 = a.src[2 * s + 1];
    if (b0 < lo0 || b0 > hi0 || b1 < lo1 || b1 > hi1) continue;
    // triangles (0, 1, 2) and (0, 2, 3)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int cb = t == 0 ? 1 : 2, cc = t == 0 ? 2 : 3;
      const double ux = q[cb][0] - q[0][0], uy = q[cb][1] - q[0][1];
      const double vx = q[cc][0] - q[0][0], vy = q[cc][1] - q[0][1];
      const double px = b0 - q[0][0], py = b1 - q[0][1];
      const double d = cross2(ux, uy, vx, vy);
      if (!(d != 0.0)) continue;
      const double lb = cross2(px, py, vx, vy) / d, lc = cross2(ux, uy, px, py) / d;
      if (!(lb >= 0.0 && lc >= 0.0 && lb + lc <= 1.0)) continue;
      const unsigned long long slot = atomicAdd(a.count, 1ull);
      if ((int64_t)slot >= a.cap) continue;
      a.cand_x[2 * slot] = X[0] + lb * (X[cb] - X[0]) + lc * (X[cc] - X[0]);
      a.cand_x[2 * slot + 1] = Y[0] + lb * (Y[cb] - Y[0]) + lc * (Y[cc] - Y[0]);
      a.cand_s[slot] = s;
    }
  }
}

// One Newton step per candidate from y(x) and f'(x): x <- x + A^-1 (beta - y),
// the step's length clamped to max_step and x to the box.  res receives
// |beta - y| at the x the step started from; *unconverged counts those above
// tol.
__global__ __launch_bounds__(kThreads) void k_newton(NewtonArgs a) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= a.n) return;
  const int32_t s = a.cand_s[k];
  const double r0 = a.src[2 * s] - a.y[2 * k], r1 = a.src[2 * s + 1] - a.y[2 * k + 1];
  const double res = sqrt(r0 * r0 + r1 * r1);
  const double fr = a.dfdz[2 * k], fi = a.dfdz[2 * k + 1];
  const double A11 = a.c1 - fr, A22 = a.c2 + fr, A12 = fi;
  const double det = A11 * A22 - A12 * A12;
  a.res[k] = res;
  a.det[k] = det;
  if (!(res <= a.tol)) atomicAdd(a.unconverged, 1u);
  if (!a.step) return;
  if (!(res > 0.0) || !(det != 0.0) || !isfinite(det)) return;
  double d0 = (A22 * r0 - A12 * r1) / det, d1 = (A11 * r1 - A12 * r0) / det;
  const double len = sqrt(d0 * d0 + d1 * d1);
  if (!(len <= a.max_step)) {
    const double f = isfinite(len) ? a.max_step / len : 0.0;
    d0 *= f;
    d1 *= f;
  }
  a.cand_x[2 * k] = fmin(fmax(a.cand_x[2 * k] + d0, a.box[0]), a.box[2]);
  a.cand_x[2 * k + 1] = fmin(fmax(a.cand_x[2 * k + 1] + d1, a.box[1]), a.box[3]);
}

// det A at the four corners of a cell: zero crossings on its edges.
__global__ __launch_bounds__(kThreads) void k_crit_cells(CritArgs a) {
  const int64_t ncx = a.nx - 1;
  const int64_t ncell = ncx * (a.j1 - a.j0);
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= ncell) return;
  const int64_t i = k % ncx, j = a.j0 + k / ncx;
  const int64_t r0 = (j - a.ybase) * a.nx + i, r1 = r0 + a.nx;
  const int64_t id[4] = {r0, r0 + 1, r1 + 1, r1};
  const double X[4] = {grid_coord(a.grid.x0, a.grid.dx, i), grid_coord(a.grid.x0, a.grid.dx, i + 1),
                       grid_coord(a.grid.x0, a.grid.dx, i + 1), grid_coord(a.grid.x0, a.grid.dx, i)};
  const double Y[4] = {grid_coord(a.grid.y0, a.grid.dy, j), grid_coord(a.grid.y0, a.grid.dy, j),
                       grid_coord(a.grid.y0, a.grid.dy, j + 1), grid_coord(a.grid.y0, a.grid.dy, j + 1)};
  double d[4];
  int npos = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double fr = a.dfdz[2 * id[c]], fi = a.dfdz[2 * id[c] + 1];
    d[c] = (a.c1 - fr) * (a.c2 + fr) - fi * fi;
    if (!isfinite(d[c])) return;
    npos += d[c] > 0.0;
  }
  if (npos == 0 || npos == 4) return;
  // crossing points on edges c -> c+1, in order round the cell
  double px[4], py[4];
  int ncut = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int e = (c + 1) & 3;
    if ((d[c] > 0.0) == (d[e] > 0.0)) continue;
    const double t = d[c] / (d[c] - d[e]);
    px[ncut] = X[c] + t * (X[e] - X[c]);
    py[ncut] = Y[c] + t * (Y[e] - Y[c]);
    ++ncut;
  }
  int pairs[2][2] = {{0, 1}, {2, 3}};
  int nseg = 1;
  if (ncut == 4) {
    nseg = 2;
    // corners 0 and 2 share a sign, 1 and 3 the other; if the centre takes
    // corner 0's sign the curve separates corners 1 and 3 from it: the cut
    // on edge 0-1 joins the cut on edge 1-2, and 2-3 joins 3-0
    const bool centre_pos = 0.25 * (d[0] + d[1] + d[2] + d[3]) > 0.0;
    if (centre_pos == (d[0] > 0.0)) {
      pairs[0][0] = 0; pairs[0][1] = 1; pairs[1][0] = 2; pairs[1][1] = 3;
    } else {
      pairs[0][0] = 0; pairs[0][1] = 3; pairs[1][0] = 1; pairs[1][1] = 2;
    }
  } else if (ncut != 2) {
    return;
  }
  for (int sg = 0; sg < nseg; ++sg) {
    const unsigned long long slot = atomicAdd(a.count, 1ull);
    if ((int64_t)slot >= a.cap) continue;
    double4 v;
    v.x = px[pairs[sg][0]];
    v.y = py[pairs[sg][0]];
    v.z = px[pairs[sg][1]];
    v.w = py[pairs[sg][1]];
    reinterpret_cast<double4 *>(a.seg)[slot] = v;
  }
}

// Multi-plane: x_j = x_0 - sum_{i<j} beta_ij alpha_i (alpha_i = x_i - y_i of
// plane i), for grid or explicit x_0.
__global__ __launch_bounds__(kThreads) void k_mp_positions(MultiPlaneArgs a) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= a.n) return;
  double x0, x1;
  if (a.grid_mode) {
    x0 = grid_coord(a.grid.x0, a.grid.dx, k % a.grid.nx);
    x1 = grid_coord(a.grid.y0, a.grid.dy, k / a.grid.nx);
  } else {
    x0 = a.rays[2 * k];
    x1 = a.rays[2 * k + 1];
  }
  for (int32_t i = 0; i < a.j; ++i) {
    const double b = a.beta[i];
    const double *al = a.alpha + (size_t)i * 2 * a.n;
    x0 -= b * al[2 * k];
    x1 -= b * al[2 * k + 1];
  }
  a.x_out[2 * k] = x0;
  a.x_out[2 * k + 1] = x1;
}

// alpha_j = x_j - y_j, kept for the later planes.
__global__ __launch_bounds__(kThreads) void k_mp_alpha(const double *__restrict__ x,
                                                       const double *__restrict__ y,
                                                       double *__restrict__ alpha, int64_t n2) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k < n2) alpha[k] = x[k] - y[k];
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

void launch_image_cells(const ImageCellArgs &a, hipStream_t stream) {
  const int64_t ncell = (a.nx - 1) * (a.j1 - a.j0);
  if (ncell <= 0) return;
  if ((ncell + kThreads - 1) / kThreads > 0x7fffffff) fail(LENS_EUNSUPPORTED, "image pass too large");
  hipLaunchKernelGGL(k_image_cells, dim3(blocks_for(ncell)), dim3(kThreads), 0, stream, a);
  LENS_HIP(hipGetLastError());
}

void launch_newton(const NewtonArgs &a, hipStream_t stream) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(k_newton, dim3(blocks_for(a.n)), dim3(kThreads), 0, stream, a);
  LENS_HIP(hipGetLastError());
}

void launch_crit_cells(const CritArgs &a, hipStream_t stream) {
  const int64_t ncell = (a.nx - 1) * (a.j1 - a.j0);
  if (ncell <= 0) return;
  if ((ncell + kThreads - 1) / kThreads > 0x7fffffff) fail(LENS_EUNSUPPORTED, "critical-curve pass too large");
  hipLaunchKernelGGL(k_crit_cells, dim3(blocks_for(ncell)), dim3(kThreads), 0, stream, a);
  LENS_HIP(hipGetLastError());
}

void launch_mp_positions(const MultiPlaneArgs &a, hipStream_t stream) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(k_mp_positions, dim3(blocks_for(a.n)), dim3(kThreads), 0, stream, a);
  LENS_HIP(hipGetLastError());
}

void launch_mp_alpha(const double *x, const double *y, double *alpha, int64_t n, hipStream_t stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mp_alpha, dim3(blocks_for(2 * n)), dim3(kThreads), 0, stream, x, y, alpha,
                     2 * n);
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
