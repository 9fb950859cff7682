// Plain FP64 direct sum of the lens equation (Section 1, eq. 1): every ray
// against every star, O(N_* x N_x).  This is the method the FMM replaces and
// the FP64 comparator it is measured against.
//
// Each workgroup holds kThreads*R rays in registers (R per thread) and
// streams the stars through LDS in tiles; every star is read back as a
// wave-uniform broadcast and applied to the R rays of each thread.  Pairs
// with |x - x_i| = 0 contribute exactly zero.  The reciprocal is the hardware estimate
// refined by two Newton-Raphson steps.
#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 1024;

// DERIV also sums f'(z) = -sum m / (z - z_i)^2 (see the evaluation kernel).
template <int R, bool MAP, bool GRID, bool DERIV>
__global__ __launch_bounds__(kThreads) void k_direct(DirectArgs a) {
  __shared__ double tx[kTile], ty[kTile], tm[kTile];
  const int tid = threadIdx.x;
  double rx[R], ry[R], ax[R], ay[R], dre[R], dim[R];
  int64_t rid[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t local = (int64_t)blockIdx.x * kThreads * R + (int64_t)r * kThreads + tid;
    rid[r] = a.ray_offset + local;
    const bool act = local < a.n_rays;
    const int64_t k = act ? rid[r] : a.ray_offset;
    if (GRID) {
      rx[r] = grid_coord(a.grid.x0, a.grid.dx, k % a.grid.nx);
      ry[r] = grid_coord(a.grid.y0, a.grid.dy, k / a.grid.nx);
    } else {
      rx[r] = a.rxy[2 * k];
      ry[r] = a.rxy[2 * k + 1];
    }
    if (!act) rid[r] = -1;
    ax[r] = 0.0;
    ay[r] = 0.0;
    dre[r] = 0.0;
    dim[r] = 0.0;
  }
  for (int64_t base = 0; base < a.n_stars; base += kTile) {
    const int cnt = (int)(a.n_stars - base < kTile ? a.n_stars - base : kTile);
    __syncthreads();
    for (int t = tid; t < cnt; t += kThreads) {
      tx[t] = a.sxy[2 * (base + t)];
      ty[t] = a.sxy[2 * (base + t) + 1];
      tm[t] = a.sm[base + t];
    }
    __syncthreads();
    for (int k = 0; k < cnt; ++k) {
      const double sx = tx[k], sy = ty[k], m = tm[k];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // a coincident pair has dx = dy = 0: the tiny term keeps its weight
        // finite, so it adds exactly zero (no other pair closer than ~1e-92
        // is affected)
        const double dx = rx[r] - sx;
        const double dy = ry[r] - sy;
        const double r2 = fma(dx, dx, fma(dy, dy, 0x1p-664));
        const double inv = rcp_f64(r2);
        const double w = m * inv;
        ax[r] = fma(w, dx, ax[r]);
        ay[r] = fma(w, dy, ay[r]);
        if (DERIV) {
          const double t = r2 > 0x1p-664 ? w * inv : 0.0;
          dre[r] = fma(-t, (dx - dy) * (dx + dy), dre[r]);
          dim[r] = fma(t + t, dx * dy, dim[r]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (rid[r] < 0) continue;
    const double y1 = a.c1 * rx[r] - ax[r];
    const double y2 = a.c2 * ry[r] - ay[r];
    if (MAP) {
      const double t1 = (y1 - a.y1min) * a.S;
      const double t2 = (y2 - a.y2min) * a.S;
      if (t1 >= 0.0 && t2 >= 0.0) {
        const double f1 = floor(t1), f2 = floor(t2);
        if (f1 < (double)a.npix && f2 < (double)a.npix)
          atomicAdd(&a.counts[(int64_t)f2 * a.npix + (int64_t)f1], 1);
      }
    } else {
      a.y_out[2 * rid[r]] = y1;
      a.y_out[2 * rid[r] + 1] = y2;
      if (DERIV) {
        a.dfdz_out[2 * rid[r]] = dre[r];
        a.dfdz_out[2 * rid[r] + 1] = dim[r];
      }
    }
  }
}

}  // namespace

void launch_direct(const DirectArgs &a, hipStream_t stream) {
  if (a.n_rays == 0) return;
  constexpr int R = 2;
  const int64_t nblk = (a.n_rays + kThreads * R - 1) / (kThreads * R);
  const bool map = a.counts != nullptr;
  const bool deriv = !map && a.dfdz_out != nullptr;
  if (a.grid_mode) {
    if (map)
      hipLaunchKernelGGL((k_direct<R, true, true, false>), dim3((unsigned)nblk), dim3(kThreads), 0, stream, a);
    else if (deriv)
      hipLaunchKernelGGL((k_direct<R, false, true, true>), dim3((unsigned)nblk), dim3(kThreads), 0, stream, a);
    else
      hipLaunchKernelGGL((k_direct<R, false, true, false>), dim3((unsigned)nblk), dim3(kThreads), 0, stream, a);
  } else {
    if (map)
      hipLaunchKernelGGL((k_direct<R, true, false, false>), dim3((unsigned)nblk), dim3(kThreads), 0, stream, a);
    else if (deriv)
      hipLaunchKernelGGL((k_direct<R, false, false, true>), dim3((unsigned)nblk), dim3(kThreads), 0, stream, a);
    else
      hipLaunchKernelGGL((k_direct<R, false, false, false>), dim3((unsigned)nblk), dim3(kThreads), 0, stream, a);
  }
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
