// Downward pass (Appendix A, downward passes 1 and 2), one launch per level
// l = 2..L over the target window (the boxes that hold rays):
//
//   local(t) = L2L(local(parent(t)))                      (l >= 3, FP64)
//            + (1/s_l) sum_{tau in IL(t)} T_tau a~(t + tau)   (M2L)
//
// IL(t) is the interaction list: the children of the parent's neighbours
// that are not neighbours of t.  For a target that is child (qx, qy) of its
// parent, tau = (c_src - c_tgt)/s ranges over [-2-qx, 3-qx] x [-2-qy, 3-qy]
// minus the 3x3 neighbourhood: 27 offsets out of 40 distinct ones, the same
// operators at every level on rescaled coefficients.  Source boxes outside the
// root are empty and skipped.
//
// Launch shape: blockIdx.y is the quadrant (qx, qy), so every wave applies
// the same 27 operators in the same order and the operator table is read
// through uniform (scalar) loads; threads enumerate parent boxes of the window.
// The FP32 variant (fine levels of LENS_MIXED) runs M2L on FP32 multipoles
// and tables, accumulated in FP32, and adds the result to the FP64 L2L part.
#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kThreads = 256;

struct Target {
  int64_t tx, ty;
  bool ok;
};

__device__ __forceinline__ Target target_of(const DownArgs &a) {
  const int q = blockIdx.y, qx = q & 1, qy = q >> 1;
  const int64_t px0 = a.win.bx0 >> 1, py0 = a.win.by0 >> 1;
  const int64_t pnx = ((a.win.bx0 + a.win.nbx - 1) >> 1) - px0 + 1;
  const int64_t pny = ((a.win.by0 + a.win.nby - 1) >> 1) - py0 + 1;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  Target t;
  t.tx = 2 * (px0 + idx % pnx) + qx;
  t.ty = 2 * (py0 + idx / pnx) + qy;
  t.ok = idx < pnx * pny && t.tx >= a.win.bx0 && t.tx < a.win.bx0 + a.win.nbx &&
         t.ty >= a.win.by0 && t.ty < a.win.by0 + a.win.nby;
  return t;
}

template <int PMAX>
__device__ __forceinline__ void l2l_into(const DownArgs &a, const double *__restrict__ l2l,
                                         int64_t tx, int64_t ty, cplx (&acc)[PMAX]) {
  const int p = a.p;
  const int q = blockIdx.y;
  const int64_t pb = ((ty >> 1) - a.pwin.by0) * a.pwin.nbx + ((tx >> 1) - a.pwin.bx0);
  const double *par = a.ploc + 2 * pb * p;
  const double *t = l2l + (size_t)q * p * p * 2;
#pragma unroll
  for (int l = 0; l < PMAX; ++l) {
    if (l < p) {
      const cplx b = {par[2 * l], par[2 * l + 1]};
#pragma unroll
      for (int j = 0; j <= l; ++j) {
        const cplx m = {t[((size_t)l * p + j) * 2], t[((size_t)l * p + j) * 2 + 1]};
        acc[j] = cmad(m, b, acc[j]);
      }
    }
  }
}

template <int PMAX>
__global__ __launch_bounds__(kThreads) void k_down_f64(DownArgs a, const double *__restrict__ l2l,
                                                       const double *__restrict__ m2l) {
  const Target tg = target_of(a);
  if (!tg.ok) return;
  const int p = a.p;
  const int q = blockIdx.y, qx = q & 1, qy = q >> 1;
  cplx acc[PMAX];
#pragma unroll
  for (int l = 0; l < PMAX; ++l) acc[l] = {0.0, 0.0};
  if (a.ploc) l2l_into<PMAX>(a, l2l, tg.tx, tg.ty, acc);
  const int64_t nb = int64_t(1) << a.level;
  const double inv_s = 1.0 / a.s;
  for (int ty = -2 - qy; ty <= 3 - qy; ++ty) {
    for (int tx = -2 - qx; tx <= 3 - qx; ++tx) {
      if (tx >= -1 && tx <= 1 && ty >= -1 && ty <= 1) continue;
      const int64_t sx = tg.tx + tx, sy = tg.ty + ty;
      if (sx < 0 || sy < 0 || sx >= nb || sy >= nb) continue;
      const double *src = a.mp + 2 * (sy * nb + sx) * p;
      const double *t = m2l + (size_t)((ty + 3) * 7 + (tx + 3)) * p * p * 2;
#pragma unroll
      for (int k = 0; k < PMAX; ++k) {
        if (k < p) {
          const cplx s = {src[2 * k] * inv_s, src[2 * k + 1] * inv_s};
#pragma unroll
          for (int l = 0; l < PMAX; ++l)
            if (l < p) {
              const cplx m = {t[((size_t)k * p + l) * 2], t[((size_t)k * p + l) * 2 + 1]};
              acc[l] = cmad(m, s, acc[l]);
            }
        }
      }
    }
  }
  const int64_t ob = (tg.ty - a.win.by0) * a.win.nbx + (tg.tx - a.win.bx0);
  double *out = a.loc + 2 * ob * p;
#pragma unroll
  for (int l = 0; l < PMAX; ++l)
    if (l < p) {
      out[2 * l] = acc[l].re;
      out[2 * l + 1] = acc[l].im;
    }
}

template <int PMAX>
__global__ __launch_bounds__(kThreads) void k_down_f32(DownArgs a, const double *__restrict__ l2l,
                                                       const float *__restrict__ m2l) {
  const Target tg = target_of(a);
  if (!tg.ok) return;
  const int p = a.p;
  const int q = blockIdx.y, qx = q & 1, qy = q >> 1;
  cplx acc[PMAX];
#pragma unroll
  for (int l = 0; l < PMAX; ++l) acc[l] = {0.0, 0.0};
  if (a.ploc) l2l_into<PMAX>(a, l2l, tg.tx, tg.ty, acc);
  cplxf acc32[PMAX];
#pragma unroll
  for (int l = 0; l < PMAX; ++l) acc32[l] = {0.f, 0.f};
  const int64_t nb = int64_t(1) << a.level;
  for (int ty = -2 - qy; ty <= 3 - qy; ++ty) {
    for (int tx = -2 - qx; tx <= 3 - qx; ++tx) {
      if (tx >= -1 && tx <= 1 && ty >= -1 && ty <= 1) continue;
      const int64_t sx = tg.tx + tx, sy = tg.ty + ty;
      if (sx < 0 || sy < 0 || sx >= nb || sy >= nb) continue;
      const float *src = a.mp32 + 2 * (sy * nb + sx) * p;
      const float *t = m2l + (size_t)((ty + 3) * 7 + (tx + 3)) * p * p * 2;
#pragma unroll
      for (int k = 0; k < PMAX; ++k) {
        if (k < p) {
          const cplxf s = {src[2 * k], src[2 * k + 1]};
#pragma unroll
          for (int l = 0; l < PMAX; ++l)
            if (l < p) {
              const cplxf m = {t[((size_t)k * p + l) * 2], t[((size_t)k * p + l) * 2 + 1]};
              acc32[l] = cmadf(m, s, acc32[l]);
            }
        }
      }
    }
  }
  const double inv_s = 1.0 / a.s;
  const int64_t ob = (tg.ty - a.win.by0) * a.win.nbx + (tg.tx - a.win.bx0);
  double *out = a.loc + 2 * ob * p;
#pragma unroll
  for (int l = 0; l < PMAX; ++l)
    if (l < p) {
      out[2 * l] = fma((double)acc32[l].re, inv_s, acc[l].re);
      out[2 * l + 1] = fma((double)acc32[l].im, inv_s, acc[l].im);
    }
}

__global__ __launch_bounds__(kThreads) void k_to_f32(const double *__restrict__ src,
                                                     float *__restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

dim3 down_grid(const DownArgs &a) {
  const int64_t px0 = a.win.bx0 >> 1, py0 = a.win.by0 >> 1;
  const int64_t pnx = ((a.win.bx0 + a.win.nbx - 1) >> 1) - px0 + 1;
  const int64_t pny = ((a.win.by0 + a.win.nby - 1) >> 1) - py0 + 1;
  return dim3((unsigned)((pnx * pny + kThreads - 1) / kThreads), 4);
}

}  // namespace

void launch_down_f64(const DownArgs &a, const OpTables &t, hipStream_t stream) {
  if (a.win.count() == 0) return;
  LENS_PMAX_DISPATCH(a.p, hipLaunchKernelGGL(k_down_f64<PM>, down_grid(a), dim3(kThreads), 0,
                                             stream, a, t.l2l, t.m2l));
  LENS_HIP(hipGetLastError());
}

void launch_down_f32(const DownArgs &a, const OpTables &t, hipStream_t stream) {
  if (a.win.count() == 0) return;
  LENS_PMAX_DISPATCH(a.p, hipLaunchKernelGGL(k_down_f32<PM>, down_grid(a), dim3(kThreads), 0,
                                             stream, a, t.l2l, t.m2l32));
  LENS_HIP(hipGetLastError());
}

void launch_to_f32(const double *src, float *dst, size_t n, hipStream_t stream) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     stream, src, dst, n);
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
