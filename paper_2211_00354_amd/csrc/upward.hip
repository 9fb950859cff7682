// Upward pass (Appendix A, upward passes 1 and 2): P2M forms the order-p
// multipole of every leaf box from its sources (stars with real masses, or
// rays with complex charges for the adjoint); M2M shifts the four children's
// multipoles to their parent's centre, level by level toward the root.  The
// two levels above the leaves are also formed straight from the stars (a
// star then enters three expansions), which replaces the two largest M2M
// sweeps with passes over the stars.  Everything runs in FP64.
//
// Coefficients are box-size rescaled: a~_k = sum_{i in box} m_i w_i^k,
// w_i = (z_i - c)/s, stored box-major as [box][p] complex (re, im).
#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kThreads = 256;
constexpr int kWave = 64;

// P2M at `level` (<= L) straight from the stars, for the boxes of `win`:
// one thread per (box, coefficient k), so consecutive threads write
// consecutive coefficients; output [win][p], row-major in the window.  A box
// at `level` covers 2^(L-level) rows of leaf boxes, each a contiguous range
// of the sorted stars.  w^k by binary powering.
template <int QDIM>
__global__ __launch_bounds__(kThreads) void k_p2m(Geometry g, int level, Window win,
                                                  const double *__restrict__ sxy,
                                                  const double *__restrict__ sq,
                                                  const int32_t *__restrict__ leaf_start, int p,
                                                  double *__restrict__ mp, float *__restrict__ mp32) {
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= win.count() * p) return;
  const int64_t b = idx / p;
  const int k = (int)(idx - b * p);
  const int64_t ix = win.bx0 + b % win.nbx, iy = win.by0 + b / win.nbx;
  const double s = ldexp(g.side, -level);
  const double inv_s = 1.0 / s;
  const double cx = g.x0 + ((double)ix + 0.5) * s;
  const double cy = g.y0 + ((double)iy + 0.5) * s;
  const int sh = g.L - level;
  const int64_t nL = int64_t(1) << g.L;
  const int64_t span = int64_t(1) << sh;
  cplx acc = {0.0, 0.0};
  for (int64_t r = 0; r < span; ++r) {
    const int64_t row = (iy << sh) + r;
    const int32_t i0 = leaf_start[row * nL + (ix << sh)];
    const int32_t i1 = leaf_start[row * nL + (ix << sh) + span];
    for (int32_t i = i0; i < i1; ++i) {
      const cplx w = {(sxy[2 * (int64_t)i] - cx) * inv_s, (sxy[2 * (int64_t)i + 1] - cy) * inv_s};
      cplx pw = {1.0, 0.0}, base = w;
      for (int e = k; e; e >>= 1) {
        if (e & 1) pw = cmul(pw, base);
        base = cmul(base, base);
      }
      if (QDIM == 1) {
        const double m = sq[i];
        acc.re = fma(m, pw.re, acc.re);
        acc.im = fma(m, pw.im, acc.im);
      } else {
        acc = cmad(cplx{sq[2 * (int64_t)i], sq[2 * (int64_t)i + 1]}, pw, acc);
      }
    }
  }
  mp[2 * idx] = acc.re;
  mp[2 * idx + 1] = acc.im;
  if (mp32) {
    mp32[2 * idx] = (float)acc.re;
    mp32[2 * idx + 1] = (float)acc.im;
  }
}

// P2M for boxes holding few sources: one thread per box of `win` with all p
// coefficients in registers (running powers m w^k); the wave's 64 boxes are
// staged in LDS so that the [64][p] block is written with coalesced stores.
template <int PMAX, int QDIM>
__global__ __launch_bounds__(kWave) void k_p2m_box(Geometry g, int level, Window win,
                                                   const double *__restrict__ sxy,
                                                   const double *__restrict__ sq,
                                                   const int32_t *__restrict__ leaf_start, int p,
                                                   double *__restrict__ mp, float *__restrict__ mp32) {
  constexpr int STR = 2 * PMAX + 1;
  __shared__ double stage[kWave * STR];
  const int lane = threadIdx.x;
  const int64_t nbox = win.count();
  const int64_t b0 = (int64_t)blockIdx.x * kWave;
  const int64_t b = b0 + lane;
  cplx acc[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) acc[k] = cplx{0.0, 0.0};
  if (b < nbox) {
    const int64_t ix = win.bx0 + b % win.nbx, iy = win.by0 + b / win.nbx;
    const double s = ldexp(g.side, -level);
    const double inv_s = 1.0 / s;
    const double cx = g.x0 + ((double)ix + 0.5) * s;
    const double cy = g.y0 + ((double)iy + 0.5) * s;
    const int sh = g.L - level;
    const int64_t nL = int64_t(1) << g.L;
    const int64_t span = int64_t(1) << sh;
    for (int64_t r = 0; r < span; ++r) {
      const int64_t row = (iy << sh) + r;
      const int32_t i0 = leaf_start[row * nL + (ix << sh)];
      const int32_t i1 = leaf_start[row * nL + (ix << sh) + span];
      for (int32_t i = i0; i < i1; ++i) {
        const cplx w = {(sxy[2 * (int64_t)i] - cx) * inv_s, (sxy[2 * (int64_t)i + 1] - cy) * inv_s};
        cplx pw = QDIM == 1 ? cplx{sq[i], 0.0} : cplx{sq[2 * (int64_t)i], sq[2 * (int64_t)i + 1]};
#pragma unroll
        for (int k = 0; k < PMAX; ++k)
          if (k < p) {
            acc[k].re += pw.re;
            acc[k].im += pw.im;
            pw = cmul(pw, w);
          }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < PMAX; ++k)
    if (k < p) {
      stage[lane * STR + 2 * k] = acc[k].re;
      stage[lane * STR + 2 * k + 1] = acc[k].im;
    }
  __syncthreads();
  const int twop = 2 * p;
  const int64_t nb = nbox - b0 < kWave ? nbox - b0 : kWave;
  for (int e = lane; e < nb * twop; e += kWave) {
    const int bl = e / twop, c = e - bl * twop;
    const double v = stage[bl * STR + c];
    mp[b0 * twop + e] = v;
    if (mp32) mp32[b0 * twop + e] = (float)v;
  }
}

// P2M for boxes holding many sources: one wave per box of `win`.  The box's
// leaf rows are taken 64 at a time; their source counts are scanned across
// the wave so that the lanes share the rows' sources evenly (lane t takes
// sources t, t+64, ... of the concatenated rows), each lane accumulating all
// p coefficients with running powers m w^k.  The 64 partial expansions are
// then summed through LDS in lane order, so the result is deterministic.
template <int PMAX, int QDIM>
__global__ __launch_bounds__(kWave) void k_p2m_wave(Geometry g, int level, Window win,
                                                    const double *__restrict__ sxy,
                                                    const double *__restrict__ sq,
                                                    const int32_t *__restrict__ leaf_start, int p,
                                                    double *__restrict__ mp, float *__restrict__ mp32) {
  constexpr int STR = 2 * PMAX + 1;  // odd stride: the column sums hit distinct banks
  __shared__ double part[kWave * STR];
  __shared__ int32_t row_first[kWave], row_pre[kWave];
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int64_t ix = win.bx0 + b % win.nbx, iy = win.by0 + b / win.nbx;
  const double s = ldexp(g.side, -level);
  const double inv_s = 1.0 / s;
  const double cx = g.x0 + ((double)ix + 0.5) * s;
  const double cy = g.y0 + ((double)iy + 0.5) * s;
  const int sh = g.L - level;
  const int64_t nL = int64_t(1) << g.L;
  const int64_t span = int64_t(1) << sh;
  cplx acc[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) acc[k] = cplx{0.0, 0.0};

  for (int64_t rb = 0; rb < span; rb += kWave) {
    int32_t first = 0, cnt = 0;
    if (rb + lane < span) {
      const int64_t row = (iy << sh) + rb + lane;
      first = leaf_start[row * nL + (ix << sh)];
      cnt = leaf_start[row * nL + (ix << sh) + span] - first;
    }
    // inclusive scan of the row counts across the wave
    int32_t inc = cnt;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int32_t v = __shfl_up(inc, d);
      if (lane >= d) inc += v;
    }
    const int32_t total = __shfl(inc, kWave - 1);
    __syncthreads();  // the previous batch's reads are done
    row_first[lane] = first;
    row_pre[lane] = inc - cnt;
    __syncthreads();
    for (int32_t t = lane; t < total; t += kWave) {
      // the row holding source t: the last row whose prefix is <= t
      int lo = 0, hi = kWave - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_pre[mid] <= t) lo = mid; else hi = mid - 1;
      }
      // rows past the batch have prefix == total > t, so lo is a real row
      const int64_t i = (int64_t)row_first[lo] + (t - row_pre[lo]);
      const cplx w = {(sxy[2 * i] - cx) * inv_s, (sxy[2 * i + 1] - cy) * inv_s};
      cplx pw = QDIM == 1 ? cplx{sq[i], 0.0} : cplx{sq[2 * i], sq[2 * i + 1]};
#pragma unroll
      for (int k = 0; k < PMAX; ++k)
        if (k < p) {
          acc[k].re += pw.re;
          acc[k].im += pw.im;
          pw = cmul(pw, w);
        }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PMAX; ++k)
    if (k < p) {
      part[lane * STR + 2 * k] = acc[k].re;
      part[lane * STR + 2 * k + 1] = acc[k].im;
    }
  __syncthreads();
  if (lane < 2 * p) {
    double t = 0.0;
    for (int j = 0; j < kWave; ++j) t += part[j * STR + lane];
    mp[b * 2 * p + lane] = t;
    if (mp32) mp32[b * 2 * p + lane] = (float)t;
  }
}

// One thread per (parent box at `level`, output coefficient l); child
// quadrant q = a + 2c is the child (2ix + a, 2iy + c) at level + 1.  Table
// layout M[q][k][l] (complex, zero for k > l).
__global__ __launch_bounds__(kThreads) void k_m2m(int level, int p,
                                                  const double *__restrict__ child,
                                                  double *__restrict__ parent,
                                                  float *__restrict__ parent32,
                                                  const double *__restrict__ tab) {
  const int64_t nb = int64_t(1) << level;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= nb * nb * p) return;
  const int64_t b = idx / p;
  const int l = (int)(idx - b * p);
  const int64_t ix = b % nb, iy = b / nb;
  const int64_t ncb = nb * 2;
  cplx acc = {0.0, 0.0};
  for (int q = 0; q < 4; ++q) {
    const int64_t cb = (2 * iy + (q >> 1)) * ncb + (2 * ix + (q & 1));
    const double *src = child + 2 * cb * p;
    const double *t = tab + (size_t)q * p * p * 2;
    for (int k = 0; k <= l; ++k) {
      const cplx a = {src[2 * k], src[2 * k + 1]};
      const cplx m = {t[((size_t)k * p + l) * 2], t[((size_t)k * p + l) * 2 + 1]};
      acc = cmad(m, a, acc);
    }
  }
  parent[2 * idx] = acc.re;
  parent[2 * idx + 1] = acc.im;
  if (parent32) {
    parent32[2 * idx] = (float)acc.re;
    parent32[2 * idx + 1] = (float)acc.im;
  }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace


void launch_p2m(Geometry g, int level, Window win, const double *sxy, const double *sq, int qdim,
                const int32_t *leaf_start, int p, double *mp, float *mp32, int64_t n_sources,
                hipStream_t stream) {
  const int64_t n = win.count() * p;
  if (n == 0) return;
  // boxes of ~16 sources or more (on average over the level): a wave per box
  if ((double)n_sources > 16.0 * (double)(int64_t(1) << (2 * level))) {
    const unsigned nb = (unsigned)win.count();
    if (qdim == 2)
      LENS_PMAX_DISPATCH(p, hipLaunchKernelGGL((k_p2m_wave<PM, 2>), dim3(nb), dim3(kWave), 0, stream,
                                               g, level, win, sxy, sq, leaf_start, p, mp, mp32));
    else
      LENS_PMAX_DISPATCH(p, hipLaunchKernelGGL((k_p2m_wave<PM, 1>), dim3(nb), dim3(kWave), 0, stream,
                                               g, level, win, sxy, sq, leaf_start, p, mp, mp32));
    LENS_HIP(hipGetLastError());
    return;
  }
  // otherwise a thread per box (all coefficients), unless p exceeds the
  // register budget of that kernel's largest instance
  if (p <= 24) {
    const unsigned nb = (unsigned)((win.count() + kWave - 1) / kWave);
    if (qdim == 2)
      LENS_PMAX_DISPATCH(p, hipLaunchKernelGGL((k_p2m_box<PM, 2>), dim3(nb), dim3(kWave), 0, stream,
                                               g, level, win, sxy, sq, leaf_start, p, mp, mp32));
    else
      LENS_PMAX_DISPATCH(p, hipLaunchKernelGGL((k_p2m_box<PM, 1>), dim3(nb), dim3(kWave), 0, stream,
                                               g, level, win, sxy, sq, leaf_start, p, mp, mp32));
    LENS_HIP(hipGetLastError());
    return;
  }
  if (qdim == 2)
    hipLaunchKernelGGL(k_p2m<2>, dim3(blocks_for(n)), dim3(kThreads), 0, stream, g, level, win,
                       sxy, sq, leaf_start, p, mp, mp32);
  else
    hipLaunchKernelGGL(k_p2m<1>, dim3(blocks_for(n)), dim3(kThreads), 0, stream, g, level, win,
                       sxy, sq, leaf_start, p, mp, mp32);
  LENS_HIP(hipGetLastError());
}

void launch_m2m(int level, int p, const double *child, double *parent, float *parent32,
                const double *m2m, hipStream_t stream) {
  const int64_t nb = int64_t(1) << level;
  hipLaunchKernelGGL(k_m2m, dim3(blocks_for(nb * nb * p)), dim3(kThreads), 0, stream, level, p,
                     child, parent, parent32, m2m);
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
