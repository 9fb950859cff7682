// Adjoint of the lens map with respect to the lenses (the gradient of a loss
// L(y) with respect to star positions and masses), derived from eq. 1 of
// Section 1.  With g_k = dL/dy1_k + i dL/dy2_k per ray and
//
//     h(z) = sum_k g_k / (z - z_k)          (a Cauchy sum: rays are the
//                                            sources, with complex charges)
//
// the gradients at star i are
//
//     dL/dm_i              = Re h(z_i)
//     dL/dx_i + i dL/dy_i  = m_i conj(h'(z_i)),   h'(z) = -sum_k g_k/(z - z_k)^2
//
// (from y = x - conj(sum m_i / (z - z_i)) and dL = Re sum_k conj(g_k) dy_k).
// The FMM evaluates h and h' with the same tree, expansions and downward pass
// as the forward problem, sources and targets exchanged: P2M over rays with
// complex charges, then at the stars the local expansion and its derivative
// (Horner) plus the near field over the rays of the 3x3 leaf neighbourhood.
// A ray exactly on a star is skipped, as in the forward map.
#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kWave = 64;
constexpr int kThreads = 256;
constexpr int32_t kFlushSources = 128;  // LENS_MIXED near-field partials per FP64 flush

// One source (position, complex charge) against the R targets of a lane:
// h += q/d, hp -= q/d^2 with d = z_target - z_source.  A coincident pair has
// d = 0 and adds exactly zero (the tiny term keeps 1/|d|^2 finite).
template <bool MIXED, int R, typename A>
__device__ __forceinline__ void adj_pair(const double (&tx)[R], const double (&ty)[R], double sx,
                                         double sy, double qr, double qi, A (&hr)[R], A (&hi)[R],
                                         A (&pr)[R], A (&pi)[R]) {
  using T = A;
  constexpr T tiny = MIXED ? (T)0x1p-66f : (T)0x1p-664;
  const T q_re = (T)qr, q_im = (T)qi;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const T dx = (T)(tx[r] - sx), dy = (T)(ty[r] - sy);
    const T r2 = fma(dx, dx, fma(dy, dy, tiny));
    const T w = MIXED ? (T)rcp_f32((float)r2) : (T)rcp_f64((double)r2);
    // 1/d = (dx - i dy) w
    const T ir = dx * w, ii = -dy * w;
    // q/d
    const T ar = fma(q_re, ir, -q_im * ii), ai = fma(q_re, ii, q_im * ir);
    hr[r] += ar;
    hi[r] += ai;
    // q/d^2 = (q/d)(1/d)
    pr[r] -= fma(ar, ir, -ai * ii);
    pi[r] -= fma(ar, ii, ai * ir);
  }
}

template <int PMAX, bool MIXED, int R>
__global__ __launch_bounds__(kWave) void k_eval_adj(
    EvalArgs a, const double *__restrict__ loc, const double *__restrict__ sxy,
    const double *__restrict__ sq, const int32_t *__restrict__ leaf_start,
    const double *__restrict__ txy, const double *__restrict__ tm, const uint32_t *__restrict__ tperm,
    const int32_t *__restrict__ tstart, int32_t tglobal, double *__restrict__ grad_xy,
    double *__restrict__ grad_m) {
  const int lane = threadIdx.x;
  const uint32_t CH = (uint32_t)a.chunks_per_box;
  const uint32_t nbx = (uint32_t)a.win.nbx;
  const uint32_t nunits = (uint32_t)(a.win.count() * CH);
  const int64_t nL = int64_t(1) << a.g.L;
  const double s = ldexp(a.g.side, -a.g.L);
  const double inv_s = 1.0 / s;
  const int p = a.p;
  constexpr int RPC = kWave * R;
  using acc_t = typename std::conditional<MIXED, float, double>::type;

  for (uint32_t u = blockIdx.x; u < nunits; u += gridDim.x) {
    const uint32_t b = u / CH, c0 = u - b * CH;
    const uint32_t byw = b / nbx, bxw = b - byw * nbx;
    const int64_t gx = a.win.bx0 + bxw, gy = a.win.by0 + byw;
    // target starts per window box, or (tglobal) per box of the whole leaf
    // level, row-major (a forward plan's leaf starts)
    const int64_t tb = tglobal ? gy * nL + gx : (int64_t)b;
    const int32_t t0 = tstart[tb], nt = tstart[tb + 1] - t0;
    if (nt == 0 || (int64_t)c0 * RPC >= nt) continue;  // uniform

    int32_t rs[3], re[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t row = gy - 1 + d;
      rs[d] = 0;
      re[d] = 0;
      if (row >= 0 && row < nL) {
        const int64_t cx0 = gx > 0 ? gx - 1 : 0;
        const int64_t cx1 = gx + 1 < nL ? gx + 1 : nL - 1;
        rs[d] = leaf_start[row * nL + cx0];
        re[d] = leaf_start[row * nL + cx1 + 1];
      }
    }
    const double cx = a.g.x0 + ((double)gx + 0.5) * s;
    const double cy = a.g.y0 + ((double)gy + 0.5) * s;

    for (int32_t base = (int32_t)c0 * RPC; base < nt; base += (int32_t)CH * RPC) {
      double tx[R], ty[R];
      acc_t hr[R], hi[R], pr[R], pi[R];
      bool act[R];
      int32_t id[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int32_t idx = base + r * kWave + lane;
        act[r] = idx < nt;
        id[r] = t0 + (act[r] ? idx : 0);
        tx[r] = txy[2 * (int64_t)id[r]];
        ty[r] = txy[2 * (int64_t)id[r] + 1];
        hr[r] = hi[r] = pr[r] = pi[r] = 0;
      }
      // LENS_MIXED: the FP32 partial sums move into FP64 ones every
      // kFlushSources sources, so a neighbourhood of thousands of rays does
      // not accumulate thousands of FP32 roundings
      double Sr[R], Si[R], Tr[R], Ti[R];
#pragma unroll
      for (int r = 0; r < R; ++r) Sr[r] = Si[r] = Tr[r] = Ti[r] = 0.0;
      int32_t since = 0;
#pragma unroll
      for (int d = 0; d < 3; ++d)
        for (int32_t i = rs[d]; i < re[d]; ++i) {
          adj_pair<MIXED, R>(tx, ty, sxy[2 * (int64_t)i], sxy[2 * (int64_t)i + 1],
                             sq[2 * (int64_t)i], sq[2 * (int64_t)i + 1], hr, hi, pr, pi);
          if (MIXED && ++since == kFlushSources) {
            since = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              Sr[r] += (double)hr[r];
              Si[r] += (double)hi[r];
              Tr[r] += (double)pr[r];
              Ti[r] += (double)pi[r];
              hr[r] = hi[r] = pr[r] = pi[r] = 0;
            }
          }
        }

      const double *lb = loc + 2 * (int64_t)b * p;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // far field: h = sum b_l w^l and dh/dw by one Horner recurrence
        const cplx w = {(tx[r] - cx) * inv_s, (ty[r] - cy) * inv_s};
        cplx f = {0.0, 0.0}, df = {0.0, 0.0};
#pragma unroll
        for (int l = PMAX - 1; l >= 0; --l)
          if (l < p) {
            df = cmad(df, w, f);
            f = cmad(f, w, cplx{lb[2 * l], lb[2 * l + 1]});
          }
        const double Hr = f.re + (Sr[r] + (double)hr[r]), Hi = f.im + (Si[r] + (double)hi[r]);
        const double Pr = df.re * inv_s + (Tr[r] + (double)pr[r]);
        const double Pi = df.im * inv_s + (Ti[r] + (double)pi[r]);
        (void)Hi;
        if (!act[r]) continue;
        const uint32_t o = tperm[id[r]];
        const double m = tm[id[r]];
        grad_m[o] = Hr;
        grad_xy[2 * (int64_t)o] = m * Pr;
        grad_xy[2 * (int64_t)o + 1] = -(m * Pi);
      }
    }
  }
}

// Direct FP64 gradient: every star against every ray, rays streamed through
// LDS as (x, y, Re g, Im g) tiles.  The comparator of the adjoint FMM.
constexpr int kAdjTile = 512;

template <int R>
__global__ __launch_bounds__(kThreads) void k_direct_adj(int64_t n_stars,
                                                         const double *__restrict__ star_xy,
                                                         const double *__restrict__ star_m,
                                                         int64_t n_rays,
                                                         const double *__restrict__ rays_xy,
                                                         const double *__restrict__ grad_y,
                                                         double *__restrict__ grad_xy,
                                                         double *__restrict__ grad_m) {
  __shared__ double rx[kAdjTile], ry[kAdjTile], gr[kAdjTile], gi[kAdjTile];
  const int tid = threadIdx.x;
  double tx[R], ty[R], hr[R], hi[R], pr[R], pi[R];
  int64_t sid[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    sid[r] = (int64_t)blockIdx.x * kThreads * R + (int64_t)r * kThreads + tid;
    const int64_t k = sid[r] < n_stars ? sid[r] : 0;
    tx[r] = n_stars ? star_xy[2 * k] : 0.0;
    ty[r] = n_stars ? star_xy[2 * k + 1] : 0.0;
    hr[r] = hi[r] = pr[r] = pi[r] = 0.0;
  }
  for (int64_t base = 0; base < n_rays; base += kAdjTile) {
    const int cnt = (int)(n_rays - base < kAdjTile ? n_rays - base : kAdjTile);
    __syncthreads();
    for (int t = tid; t < cnt; t += kThreads) {
      rx[t] = rays_xy[2 * (base + t)];
      ry[t] = rays_xy[2 * (base + t) + 1];
      gr[t] = grad_y[2 * (base + t)];
      gi[t] = grad_y[2 * (base + t) + 1];
    }
    __syncthreads();
    for (int k = 0; k < cnt; ++k)
      adj_pair<false, R>(tx, ty, rx[k], ry[k], gr[k], gi[k], hr, hi, pr, pi);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (sid[r] >= n_stars) continue;
    const double m = star_m[sid[r]];
    grad_m[sid[r]] = hr[r];
    grad_xy[2 * sid[r]] = m * pr[r];
    grad_xy[2 * sid[r] + 1] = -(m * pi[r]);
  }
}

__global__ __launch_bounds__(kThreads) void k_grid_rays(lens_grid g, double *__restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= g.nx * g.ny) return;
  out[2 * k] = grid_coord(g.x0, g.dx, k % g.nx);
  out[2 * k + 1] = grid_coord(g.y0, g.dy, k / g.nx);
}

template <int PM, bool MIXED>
void adj_launch(const EvalArgs &a, const AdjArgs &d, hipStream_t stream) {
  constexpr int R = 1;
  const int64_t units = a.win.count() * a.chunks_per_box;
  const int64_t nblk = units < 65536 ? units : 65536;
  hipLaunchKernelGGL((k_eval_adj<PM, MIXED, R>), dim3((unsigned)nblk), dim3(kWave), 0, stream, a,
                     a.loc, a.sxy, d.sq, a.leaf_start, d.txy, d.tm, d.tperm, d.tstart,
                     (int32_t)d.tglobal, d.grad_xy, d.grad_m);
}

}  // namespace

int64_t adj_targets_per_unit() { return kWave; }

void launch_eval_adj(const EvalArgs &a, const AdjArgs &d, int precision, hipStream_t stream) {
  if (a.win.count() == 0) return;
  if (precision == LENS_MIXED)
    LENS_PMAX_DISPATCH(a.p, (adj_launch<PM, true>(a, d, stream)));
  else
    LENS_PMAX_DISPATCH(a.p, (adj_launch<PM, false>(a, d, stream)));
  LENS_HIP(hipGetLastError());
}

void launch_direct_adj(int64_t n_stars, const double *star_xy, const double *star_m, int64_t n_rays,
                       const double *rays_xy, const double *grad_y, double *grad_xy,
                       double *grad_m, hipStream_t stream) {
  if (n_stars == 0) return;
  constexpr int R = 2;
  const int64_t nblk = (n_stars + kThreads * R - 1) / (kThreads * R);
  hipLaunchKernelGGL((k_direct_adj<R>), dim3((unsigned)nblk), dim3(kThreads), 0, stream, n_stars,
                     star_xy, star_m, n_rays, rays_xy, grad_y, grad_xy, grad_m);
  LENS_HIP(hipGetLastError());
}

void launch_grid_rays(const lens_grid &g, double *out, hipStream_t stream) {
  const int64_t n = g.nx * g.ny;
  if (n == 0) return;
  hipLaunchKernelGGL(k_grid_rays, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     stream, g, out);
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
