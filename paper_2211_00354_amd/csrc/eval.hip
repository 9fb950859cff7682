// Evaluation at the rays (Appendix A, steps 6 and 7) fused with the smooth
// field (Section 2.4, step 3) and, for maps, inverse-ray-shooting binning
// (Section 2.3).
//
// One workgroup serves one chunk of the rays of one leaf box of the target
// window:
//   * the stars of the box's 3x3 neighbourhood (three contiguous row ranges of
//     the sorted star array) are staged once in LDS and read back as
//     wave-uniform broadcasts by every ray of the workgroup;
//   * near field: alpha_near = sum m (x - x_i)/|x - x_i|^2 over those stars,
//     pair differences formed in FP64, then (LENS_MIXED) rounded to FP32 for
//     the square, reciprocal and accumulation;
//   * far field: the box's local expansion f(z) = sum_l b~_l w^l,
//     w = (z - c)/s, by Horner in FP64, alpha_far = conj(f);
//   * y = (1-kappa_s-gamma, 1-kappa_s+gamma) * x - alpha in FP64, written as
//     [n][2] or binned into the map with an integer atomic.
#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kThreads = 256;
constexpr int kStarTile = 768;

template <bool MIXED>
struct StarTile {
  double x[kStarTile], y[kStarTile];
  typename std::conditional<MIXED, float, double>::type m[kStarTile];
};

template <int PMAX, bool MIXED, bool MAP, bool GRID, int R>
__global__ __launch_bounds__(kThreads) void k_eval(EvalArgs a) {
  using real = typename std::conditional<MIXED, float, double>::type;
  __shared__ StarTile<MIXED> st;
  __shared__ cplx sloc[PMAX];

  const int tid = threadIdx.x;
  const int64_t CH = a.chunks_per_box;
  const int64_t b = (int64_t)blockIdx.x / CH;
  const int64_t c0 = (int64_t)blockIdx.x % CH;
  const int64_t bxw = b % a.win.nbx, byw = b / a.win.nbx;
  const int64_t gx = a.win.bx0 + bxw, gy = a.win.by0 + byw;

  // rays of this box
  int64_t nr, i0 = 0, j0 = 0, W = 1, r0 = 0;
  if (GRID) {
    i0 = a.col_start[bxw];
    W = a.col_start[bxw + 1] - i0;
    j0 = a.row_start[byw];
    nr = W * (a.row_start[byw + 1] - j0);
  } else {
    r0 = a.ray_start[b];
    nr = a.ray_start[b + 1] - r0;
  }
  constexpr int64_t RPC = (int64_t)kThreads * R;  // rays per chunk
  if (nr == 0 || c0 * RPC >= nr) return;          // uniform over the workgroup

  // 3x3 neighbourhood: up to three row ranges of the sorted stars
  const int64_t nL = int64_t(1) << a.g.L;
  int32_t rs[3], rn[3];
  int32_t nn = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t row = gy - 1 + d;
    rs[d] = 0;
    rn[d] = 0;
    if (row >= 0 && row < nL) {
      const int64_t cx0 = gx > 0 ? gx - 1 : 0;
      const int64_t cx1 = gx + 1 < nL ? gx + 1 : nL - 1;
      rs[d] = a.leaf_start[row * nL + cx0];
      rn[d] = a.leaf_start[row * nL + cx1 + 1] - rs[d];
    }
    nn += rn[d];
  }

  const double s = ldexp(a.g.side, -a.g.L);
  const double inv_s = 1.0 / s;
  const double cx = a.g.x0 + ((double)gx + 0.5) * s;
  const double cy = a.g.y0 + ((double)gy + 0.5) * s;
  const int p = a.p;
  if (tid < p) {
    const double *lb = a.loc + 2 * b * p;
    sloc[tid] = {lb[2 * tid], lb[2 * tid + 1]};
  }

  auto stage = [&](int32_t base, int32_t cnt) {
    for (int32_t t = tid; t < cnt; t += kThreads) {
      int32_t k = base + t;
      int32_t gi;
      if (k < rn[0]) {
        gi = rs[0] + k;
      } else if (k < rn[0] + rn[1]) {
        gi = rs[1] + (k - rn[0]);
      } else {
        gi = rs[2] + (k - rn[0] - rn[1]);
      }
      st.x[t] = a.sxy[2 * (int64_t)gi];
      st.y[t] = a.sxy[2 * (int64_t)gi + 1];
      st.m[t] = (real)a.sm[gi];
    }
  };

  const bool single = nn <= kStarTile;
  if (single) stage(0, nn);
  __syncthreads();

  for (int64_t c = c0; c * RPC < nr; c += CH) {
    double rx[R], ry[R];
    real ax[R], ay[R];
    bool act[R];
    int64_t oidx[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t idx = c * RPC + (int64_t)r * kThreads + tid;
      act[r] = idx < nr;
      const int64_t id = act[r] ? idx : 0;
      if (GRID) {
        const int64_t i = i0 + id % W, j = j0 + id / W;
        rx[r] = grid_coord(a.grid.x0, a.grid.dx, i);
        ry[r] = grid_coord(a.grid.y0, a.grid.dy, j);
        oidx[r] = j * a.grid.nx + i;
      } else {
        rx[r] = a.rxy[2 * (r0 + id)];
        ry[r] = a.rxy[2 * (r0 + id) + 1];
        oidx[r] = a.rperm ? (int64_t)a.rperm[r0 + id] : r0 + id;
      }
      ax[r] = 0;
      ay[r] = 0;
    }

    auto accumulate = [&](int32_t cnt) {
      for (int32_t k = 0; k < cnt; ++k) {
        const double sx = st.x[k], sy = st.y[k];
        const real m = st.m[k];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (MIXED) {
            const float dx = (float)(rx[r] - sx);
            const float dy = (float)(ry[r] - sy);
            const float r2 = fmaf(dx, dx, dy * dy);
            const float w = r2 > 0.f ? (float)m * rcp_f32(r2) : 0.f;
            ax[r] = fmaf(w, dx, (float)ax[r]);
            ay[r] = fmaf(w, dy, (float)ay[r]);
          } else {
            const double dx = rx[r] - sx;
            const double dy = ry[r] - sy;
            const double r2 = fma(dx, dx, dy * dy);
            const double w = r2 > 0.0 ? (double)m * rcp_f64(r2) : 0.0;
            ax[r] = fma(w, dx, (double)ax[r]);
            ay[r] = fma(w, dy, (double)ay[r]);
          }
        }
      }
    };

    if (single) {
      accumulate(nn);
    } else {
      for (int32_t base = 0; base < nn; base += kStarTile) {
        const int32_t cnt = nn - base < kStarTile ? nn - base : kStarTile;
        __syncthreads();
        stage(base, cnt);
        __syncthreads();
        accumulate(cnt);
      }
    }

#pragma unroll
    for (int r = 0; r < R; ++r) {
      // far field by Horner on the rescaled local expansion
      const cplx w = {(rx[r] - cx) * inv_s, (ry[r] - cy) * inv_s};
      cplx f = {0.0, 0.0};
#pragma unroll
      for (int l = PMAX - 1; l >= 0; --l)
        if (l < p) f = cmad(f, w, sloc[l]);
      const double al1 = f.re + (double)ax[r];
      const double al2 = (double)ay[r] - f.im;
      const double y1 = a.c1 * rx[r] - al1;
      const double y2 = a.c2 * ry[r] - al2;
      if (!act[r]) continue;
      if (MAP) {
        const double t1 = (y1 - a.y1min) * a.S;
        const double t2 = (y2 - a.y2min) * a.S;
        if (t1 >= 0.0 && t2 >= 0.0) {
          const double f1 = floor(t1), f2 = floor(t2);
          if (f1 < (double)a.npix && f2 < (double)a.npix)
            atomicAdd(&a.counts[(int64_t)f2 * a.npix + (int64_t)f1], 1);
        }
      } else {
        a.y_out[2 * oidx[r]] = y1;
        a.y_out[2 * oidx[r] + 1] = y2;
      }
    }
  }
}

// first ray column (row) of every box column (row) of the window
__global__ __launch_bounds__(kThreads) void k_grid_ranges(double x0, double dx, int64_t lo_i,
                                                          int64_t hi_i, double origin, double s,
                                                          int64_t nL, int64_t b0, int64_t nb,
                                                          int32_t *__restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c > nb) return;
  const int64_t B = b0 + c;
  int64_t lo = lo_i, hi = hi_i;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (box_coord(grid_coord(x0, dx, mid), origin, s, nL) < B)
      lo = mid + 1;
    else
      hi = mid;
  }
  out[c] = (int32_t)lo;
}

__global__ __launch_bounds__(kThreads) void k_ray_keys(const double *__restrict__ rxy, int64_t n,
                                                       Geometry g, Window win,
                                                       uint32_t *__restrict__ keys,
                                                       uint32_t *__restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t nL = int64_t(1) << g.L;
  const double s = ldexp(g.side, -g.L);
  int64_t ix = box_coord(rxy[2 * i], g.x0, s, nL) - win.bx0;
  int64_t iy = box_coord(rxy[2 * i + 1], g.y0, s, nL) - win.by0;
  ix = ix < 0 ? 0 : (ix >= win.nbx ? win.nbx - 1 : ix);
  iy = iy < 0 ? 0 : (iy >= win.nby ? win.nby - 1 : iy);
  keys[i] = (uint32_t)(iy * win.nbx + ix);
  vals[i] = (uint32_t)i;
}

template <int PM, bool MIXED, bool MAP, bool GRID>
void eval_launch(const EvalArgs &a, hipStream_t stream) {
  constexpr int R = 2;
  const int64_t nblk = a.win.count() * a.chunks_per_box;
  hipLaunchKernelGGL((k_eval<PM, MIXED, MAP, GRID, R>), dim3((unsigned)nblk), dim3(kThreads), 0,
                     stream, a);
}

template <int PM>
void eval_dispatch(const EvalArgs &a, int precision, hipStream_t stream) {
  const bool mixed = precision == LENS_MIXED, map = a.counts != nullptr;
  if (a.grid_mode) {
    if (mixed) {
      if (map) eval_launch<PM, true, true, true>(a, stream);
      else eval_launch<PM, true, false, true>(a, stream);
    } else {
      if (map) eval_launch<PM, false, true, true>(a, stream);
      else eval_launch<PM, false, false, true>(a, stream);
    }
  } else {
    if (mixed) eval_launch<PM, true, false, false>(a, stream);
    else eval_launch<PM, false, false, false>(a, stream);
  }
}

}  // namespace

int64_t eval_rays_per_chunk() { return (int64_t)kThreads * 2; }

void launch_eval(const EvalArgs &a, int precision, hipStream_t stream) {
  if (a.win.count() == 0) return;
  LENS_PMAX_DISPATCH(a.p, eval_dispatch<PM>(a, precision, stream));
  LENS_HIP(hipGetLastError());
}

void launch_grid_ranges(const lens_grid &grid, Geometry g, Window win, int64_t j_begin,
                        int64_t j_end, int32_t *col_start, int32_t *row_start,
                        hipStream_t stream) {
  const int64_t nL = int64_t(1) << g.L;
  const double s = ldexp(g.side, -g.L);
  hipLaunchKernelGGL(k_grid_ranges, dim3((unsigned)((win.nbx + 1 + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, stream, grid.x0, grid.dx, (int64_t)0, grid.nx, g.x0, s, nL,
                     win.bx0, win.nbx, col_start);
  hipLaunchKernelGGL(k_grid_ranges, dim3((unsigned)((win.nby + 1 + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, stream, grid.y0, grid.dy, j_begin, j_end, g.y0, s, nL,
                     win.by0, win.nby, row_start);
  LENS_HIP(hipGetLastError());
}

void launch_ray_keys(const double *rxy, int64_t n, Geometry g, Window win, uint32_t *keys,
                     uint32_t *vals, hipStream_t stream) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_ray_keys, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     stream, rxy, n, g, win, keys, vals);
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
