// Device helpers shared by the kernels: box geometry, grid ray positions,
// reciprocals and complex arithmetic.  Everything here is compiled with
// contraction off; fused multiply-adds are written out where wanted.
#pragma once

#include <hip/hip_runtime.h>

#include "lens_internal.h"

namespace lensfmm {

// Box coordinate of x along one axis: floor((x - origin) / s), clamped to
// [0, nbox-1].  The division is correctly rounded, so every kernel that asks
// agrees on the box of a point.
__device__ __forceinline__ int64_t box_coord(double x, double origin, double s, int64_t nbox) {
  double t = (x - origin) / s;
  t = fmin(fmax(t, 0.0), (double)(nbox - 1));  // NaN -> 0
  return (int64_t)floor(t);
}

// Ray i of a cell-centred grid axis: origin + (i + 0.5) * step, the product
// and the sum each rounded once.
__device__ __forceinline__ double grid_coord(double origin, double step, int64_t i) {
  return origin + ((double)i + 0.5) * step;
}

// FP64 reciprocal: hardware estimate refined by two Newton-Raphson steps
// x <- x (2 - a x), written as x + x (1 - a x).
__device__ __forceinline__ double rcp_f64(double a) {
  double x = __builtin_amdgcn_rcp(a);
  double e = fma(-a, x, 1.0);
  x = fma(x, e, x);
  e = fma(-a, x, 1.0);
  return fma(x, e, x);
}

__device__ __forceinline__ float rcp_f32(float a) { return __builtin_amdgcn_rcpf(a); }

// Complex numbers as (re, im) pairs.
struct cplx {
  double re, im;
};

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}

// acc + a * b
__device__ __forceinline__ cplx cmad(cplx a, cplx b, cplx acc) {
  return {fma(a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(a.im, b.re, acc.im))};
}

struct cplxf {
  float re, im;
};

__device__ __forceinline__ cplxf cmadf(cplxf a, cplxf b, cplxf acc) {
  return {fmaf(a.re, b.re, fmaf(-a.im, b.im, acc.re)), fmaf(a.re, b.im, fmaf(a.im, b.re, acc.im))};
}

// Expansion orders are compiled in buckets; a kernel for bucket PM serves
// every runtime order p <= PM (terms past p are skipped).
#define LENS_PMAX_DISPATCH(p, KERNEL_LAUNCH) \
  do {                                       \
    if ((p) <= 8) {                          \
      constexpr int PM = 8;                  \
      KERNEL_LAUNCH;                         \
    } else if ((p) <= 12) {                  \
      constexpr int PM = 12;                 \
      KERNEL_LAUNCH;                         \
    } else if ((p) <= 16) {                  \
      constexpr int PM = 16;                 \
      KERNEL_LAUNCH;                         \
    } else if ((p) <= 24) {                  \
      constexpr int PM = 24;                 \
      KERNEL_LAUNCH;                         \
    } else if ((p) <= 32) {                  \
      constexpr int PM = 32;                 \
      KERNEL_LAUNCH;                         \
    } else {                                 \
      constexpr int PM = 40;                 \
      KERNEL_LAUNCH;                         \
    }                                        \
  } while (0)

}  // namespace lensfmm
