// Upward pass (Appendix A, upward passes 1 and 2): P2M forms the order-p
// multipole of every leaf box from its stars; M2M shifts the four children's
// multipoles to their parent's centre, level by level toward the root.
// Both run in FP64 (they touch each star once and each box once).
//
// Coefficients are box-size rescaled: a~_k = sum_{i in box} m_i w_i^k,
// w_i = (z_i - c)/s, stored box-major as [box][p] complex (re, im).
#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kThreads = 256;

template <int PMAX>
__global__ __launch_bounds__(kThreads) void k_p2m(Geometry g, const double *__restrict__ sxy,
                                                  const double *__restrict__ sm,
                                                  const int32_t *__restrict__ leaf_start, int p,
                                                  double *__restrict__ mp) {
  const int64_t nb = int64_t(1) << g.L;
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b >= nb * nb) return;
  const int64_t ix = b % nb, iy = b / nb;
  const double s = ldexp(g.side, -g.L);
  const double inv_s = 1.0 / s;
  const double cx = g.x0 + ((double)ix + 0.5) * s;
  const double cy = g.y0 + ((double)iy + 0.5) * s;
  cplx acc[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) acc[k] = {0.0, 0.0};
  const int32_t i0 = leaf_start[b], i1 = leaf_start[b + 1];
  for (int32_t i = i0; i < i1; ++i) {
    const cplx w = {(sxy[2 * (int64_t)i] - cx) * inv_s, (sxy[2 * (int64_t)i + 1] - cy) * inv_s};
    cplx pw = {sm[i], 0.0};
#pragma unroll
    for (int k = 0; k < PMAX; ++k) {
      acc[k].re += pw.re;
      acc[k].im += pw.im;
      pw = cmul(pw, w);
    }
  }
  double *out = mp + 2 * b * p;
#pragma unroll
  for (int k = 0; k < PMAX; ++k)
    if (k < p) {
      out[2 * k] = acc[k].re;
      out[2 * k + 1] = acc[k].im;
    }
}

// parent box (ix, iy) at `level`; child quadrant q = a + 2c is the child
// (2ix + a, 2iy + c) at level + 1.  Table layout M[q][k][l] (complex).
template <int PMAX>
__global__ __launch_bounds__(kThreads) void k_m2m(int level, int p,
                                                  const double *__restrict__ child,
                                                  double *__restrict__ parent,
                                                  const double *__restrict__ tab) {
  const int64_t nb = int64_t(1) << level;
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b >= nb * nb) return;
  const int64_t ix = b % nb, iy = b / nb;
  const int64_t ncb = nb * 2;
  cplx acc[PMAX];
#pragma unroll
  for (int l = 0; l < PMAX; ++l) acc[l] = {0.0, 0.0};
  for (int q = 0; q < 4; ++q) {
    const int64_t cb = (2 * iy + (q >> 1)) * ncb + (2 * ix + (q & 1));
    const double *src = child + 2 * cb * p;
    const double *t = tab + (size_t)q * p * p * 2;
#pragma unroll
    for (int k = 0; k < PMAX; ++k) {
      if (k < p) {
        const cplx a = {src[2 * k], src[2 * k + 1]};
#pragma unroll
        for (int l = k; l < PMAX; ++l)
          if (l < p) {
            const cplx m = {t[((size_t)k * p + l) * 2], t[((size_t)k * p + l) * 2 + 1]};
            acc[l] = cmad(m, a, acc[l]);
          }
      }
    }
  }
  double *out = parent + 2 * b * p;
#pragma unroll
  for (int l = 0; l < PMAX; ++l)
    if (l < p) {
      out[2 * l] = acc[l].re;
      out[2 * l + 1] = acc[l].im;
    }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace


void launch_p2m(Geometry g, const double *sxy, const double *sm, const int32_t *leaf_start, int p,
                double *mp_leaf, hipStream_t stream) {
  const int64_t nb = int64_t(1) << g.L;
  LENS_PMAX_DISPATCH(p, hipLaunchKernelGGL(k_p2m<PM>, dim3(blocks_for(nb * nb)), dim3(kThreads), 0,
                                           stream, g, sxy, sm, leaf_start, p, mp_leaf));
  LENS_HIP(hipGetLastError());
}

void launch_m2m(int level, int p, const double *child, double *parent, const double *m2m,
                hipStream_t stream) {
  const int64_t nb = int64_t(1) << level;
  LENS_PMAX_DISPATCH(p, hipLaunchKernelGGL(k_m2m<PM>, dim3(blocks_for(nb * nb)), dim3(kThreads), 0,
                                           stream, level, p, child, parent, m2m));
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
