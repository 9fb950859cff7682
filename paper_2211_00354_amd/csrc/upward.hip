// Upward pass (Appendix A, upward passes 1 and 2): P2M forms the order-p
// multipole of every leaf box from its sources (stars with real masses, or
// rays with complex charges for the adjoint); M2M shifts the four children's
// multipoles to their parent's centre toward the root.  Levels whose boxes
// hold a few sources on average, and the windowed fine levels, are formed
// straight from the stars (a star then enters several expansions), which
// replaces the largest M2M sweeps with passes over the stars; the coarser
// dense levels come from M2M, up to four levels per launch.  Everything runs
// in FP64.
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

// Wave-cooperative P2M of one box (wave-uniform ix, iy): the box's leaf rows
// are taken 64 at a time, their source counts scanned across the wave so
// that the lanes share the rows' sources evenly (lane t takes sources t,
// t+64, ... of the concatenated rows), each lane accumulating all p
// coefficients with running powers m w^k into acc; the 64 partial
// expansions are then summed by a fixed cross-lane butterfly (every lane
// ends with the total, in the same order on every run).
template <int PMAX, int QDIM>
__device__ __forceinline__ void p2m_wave_box(const Geometry &g, int level, int64_t ix, int64_t iy,
                                             const double *__restrict__ sxy,
                                             const double *__restrict__ sq,
                                             const int32_t *__restrict__ leaf_start, int p,
                                             int32_t *row_first, int32_t *row_pre,
                                             cplx (&acc)[PMAX]) {
  const int lane = threadIdx.x;
  const double s = ldexp(g.side, -level);
  const double inv_s = 1.0 / s;
  const double cx = g.x0 + ((double)ix + 0.5) * s;
  const double cy = g.y0 + ((double)iy + 0.5) * s;
  const int sh = g.L - level;
  const int64_t nL = int64_t(1) << g.L;
  const int64_t span = int64_t(1) << sh;
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
#pragma unroll
  for (int k = 0; k < PMAX; ++k)
    if (k < p) {
      double re = acc[k].re, im = acc[k].im;
#pragma unroll
      for (int d = kWave / 2; d >= 1; d >>= 1) {
        re += __shfl_xor(re, d);
        im += __shfl_xor(im, d);
      }
      acc[k] = cplx{re, im};
    }
}

// The level below a P2M level, when it is already formed: its window (in its
// own box coordinates) and its [window][p] FP64 multipoles.  A crowded box
// whose four children are all in that window is formed from them by M2M
// (4 p(p-1)/2 shift updates) instead of from its stars.
struct ChildLevel {
  Window win;
  const double *mp;  // nullptr: no child level
};

__device__ __forceinline__ bool children_ready(const ChildLevel &c, int64_t ix, int64_t iy) {
  return c.mp != nullptr && 2 * ix >= c.win.bx0 && 2 * ix + 1 < c.win.bx0 + c.win.nbx &&
         2 * iy >= c.win.by0 && 2 * iy + 1 < c.win.by0 + c.win.nby;
}

// Coefficient l of a parent's rescaled multipole from its four children
// (M2M; one lane per coefficient): in child-size units child q's centre sits
// at d = (qa - 1/2) + i (qc - 1/2) from the parent's, and
//     a_l = 2^-l sum_q sum_{j<=l} C(l, j) d^j a_(l-j)(q),
// summed by Horner in d with the binomials of row l formed on the way
// (C(l, j-1) = C(l, j) j / (l - j + 1): integers below 2^53, so exact).
__device__ __forceinline__ cplx m2m_coeff(const ChildLevel &c, int64_t ix, int64_t iy, int p, int l) {
  cplx sum = {0.0, 0.0};
  for (int q = 0; q < 4; ++q) {
    const int qa = q & 1, qc = q >> 1;
    const double dr = qa - 0.5, di = qc - 0.5;
    const int64_t cb = (2 * iy + qc - c.win.by0) * c.win.nbx + (2 * ix + qa - c.win.bx0);
    const double2 *src = reinterpret_cast<const double2 *>(c.mp) + cb * p;
    double bin = 1.0;  // C(l, l)
    double2 v = src[0];
    cplx acc = {v.x, v.y};  // C(l, l) a_0
    for (int jj = l; jj >= 1; --jj) {
      // acc <- acc d + C(l, jj - 1) a_(l - jj + 1)
      bin = bin * (double)jj / (double)(l - jj + 1);
      v = src[l - jj + 1];
      const double re = fma(acc.re, dr, fma(-acc.im, di, bin * v.x));
      const double im = fma(acc.re, di, fma(acc.im, dr, bin * v.y));
      acc = cplx{re, im};
    }
    sum.re += acc.re;
    sum.im += acc.im;
  }
  return cplx{ldexp(sum.re, -l), ldexp(sum.im, -l)};
}

// A box holding more than kCrowdedBox sources is formed by M2M from its
// four children when the level below has them; one holding more than
// kWaveBox sources (and no formed children) is formed by the whole wave
// (p2m_wave_box) rather than by its own lane.
constexpr int64_t kCrowdedBox = 32;
constexpr int64_t kWaveBox = 256;

// The rescaled multipole of a box from its four formed children, in one
// lane: each child's coefficients are shifted to the parent's centre by the
// synthetic division of k_m2m_tile below (p(p-1)/2 updates
// a_j += d a_(j-1), d = (+-1/2, +-1/2) in child-size units) and the four
// are summed, then scaled by 2^-l.
template <int PMAX>
__device__ __forceinline__ void m2m_lane(const ChildLevel &c, int64_t ix, int64_t iy, int p,
                                         cplx (&acc)[PMAX]) {
#pragma unroll
  for (int k = 0; k < PMAX; ++k) acc[k] = cplx{0.0, 0.0};
  for (int q = 0; q < 4; ++q) {
    const int qa = q & 1, qc = q >> 1;
    const double dr = qa - 0.5, di = qc - 0.5;
    const int64_t cb = (2 * iy + qc - c.win.by0) * c.win.nbx + (2 * ix + qa - c.win.bx0);
    const double2 *src = reinterpret_cast<const double2 *>(c.mp) + cb * p;
    cplx a[PMAX];
#pragma unroll
    for (int k = 0; k < PMAX; ++k)
      if (k < p) {
        const double2 v = src[k];
        a[k] = cplx{v.x, v.y};
      }
#pragma unroll
    for (int k = 0; k + 1 < PMAX; ++k)
      if (k + 1 < p) {
#pragma unroll
        for (int j = PMAX - 1; j > k; --j)
          if (j < p) {
            a[j].re = fma(dr, a[j - 1].re, fma(-di, a[j - 1].im, a[j].re));
            a[j].im = fma(dr, a[j - 1].im, fma(di, a[j - 1].re, a[j].im));
          }
      }
#pragma unroll
    for (int k = 0; k < PMAX; ++k)
      if (k < p) {
        acc[k].re += a[k].re;
        acc[k].im += a[k].im;
      }
  }
#pragma unroll
  for (int k = 0; k < PMAX; ++k)
    if (k < p) acc[k] = cplx{ldexp(acc[k].re, -k), ldexp(acc[k].im, -k)};
}

// P2M for levels whose boxes hold few sources on average: one thread per box
// of `win` with all p coefficients in registers (running powers m w^k).
// Occupancy is heavy-tailed in clustered fields (a galaxy's centre, a
// cluster of lenses): a lane whose box holds more than kCrowdedBox sources
// forms it by M2M from its children when the level below has them all (in
// its own lane, so a wave of crowded boxes shifts them side by side), and a
// box of more than kWaveBox sources without them is left to the whole wave,
// which forms such boxes one after another -- or, with `defer`, to a second
// pass of k_p2m_wave (a wave per box), this pass storing zeros for them.
// The kernel is bound by memory
// latency (a few sources per lane): a box of one or two leaf rows keeps its
// source ranges in registers and the next source's loads are issued before
// the current one's powers are summed.  The wave's 64 boxes are staged in
// LDS so that the [64][p] block is written with coalesced stores.
template <int PMAX, int QDIM>
__global__ __launch_bounds__(kWave) void k_p2m_box(Geometry g, int level, Window win,
                                                   const double *__restrict__ sxy,
                                                   const double *__restrict__ sq,
                                                   const int32_t *__restrict__ leaf_start, int p,
                                                   double *__restrict__ mp, float *__restrict__ mp32,
                                                   ChildLevel child, int defer) {
  constexpr int STR = 2 * PMAX + 1;
  __shared__ double stage[kWave * STR];
  __shared__ int32_t row_first[kWave], row_pre[kWave];
  const int lane = threadIdx.x;
  const int64_t nbox = win.count();
  const int64_t b0 = (int64_t)blockIdx.x * kWave;
  const int64_t b = b0 + lane;
  const int sh = g.L - level;
  const int64_t nL = int64_t(1) << g.L;
  const int64_t span = int64_t(1) << sh;
  const int64_t ix = b < nbox ? win.bx0 + b % win.nbx : 0;
  const int64_t iy = b < nbox ? win.by0 + b / win.nbx : 0;
  // source ranges of the box's (first two) leaf rows, and its source count
  int32_t a0 = 0, e0 = 0, a1 = 0, e1 = 0;
  int64_t count = 0;
  if (b < nbox) {
    const int64_t c0 = (iy << sh) * nL + (ix << sh);
    a0 = leaf_start[c0];
    e0 = leaf_start[c0 + span];
    if (span >= 2) {
      a1 = leaf_start[c0 + nL];
      e1 = leaf_start[c0 + nL + span];
    }
    count = (int64_t)(e0 - a0) + (e1 - a1);
    for (int64_t r = 2; r < span; ++r) {
      const int64_t row = (iy << sh) + r;
      count += leaf_start[row * nL + (ix << sh) + span] - leaf_start[row * nL + (ix << sh)];
    }
  }
  const bool by_m2m = count > kCrowdedBox && b < nbox && children_ready(child, ix, iy);
  const bool by_wave = count > kWaveBox && !by_m2m;
  cplx acc[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) acc[k] = cplx{0.0, 0.0};
  auto add_source = [&](double x, double y, cplx pw, const cplx &c, double inv_s) {
    const cplx w = {(x - c.re) * inv_s, (y - c.im) * inv_s};
#pragma unroll
    for (int k = 0; k < PMAX; ++k)
      if (k < p) {
        acc[k].re += pw.re;
        acc[k].im += pw.im;
        pw = cmul(pw, w);
      }
  };
  auto charge = [&](int64_t i) {
    return QDIM == 1 ? cplx{sq[i], 0.0} : cplx{sq[2 * i], sq[2 * i + 1]};
  };
  if (by_m2m) m2m_lane<PMAX>(child, ix, iy, p, acc);
  if (b < nbox && !by_m2m && !by_wave) {
    const double s = ldexp(g.side, -level);
    const double inv_s = 1.0 / s;
    const cplx c = {g.x0 + ((double)ix + 0.5) * s, g.y0 + ((double)iy + 0.5) * s};
    // the first two rows as one run of n0 + n1 sources, software-pipelined
    const int32_t n0 = e0 - a0, n = n0 + (e1 - a1);
    auto src = [&](int32_t t) { return (int64_t)(t < n0 ? a0 + t : a1 + (t - n0)); };
    double nx = 0.0, ny = 0.0;
    cplx nq = {0.0, 0.0};
    if (n > 0) {
      const int64_t i = src(0);
      nx = sxy[2 * i];
      ny = sxy[2 * i + 1];
      nq = charge(i);
    }
    for (int32_t t = 0; t < n; ++t) {
      const double x = nx, y = ny;
      const cplx q = nq;
      if (t + 1 < n) {
        const int64_t i = src(t + 1);
        nx = sxy[2 * i];
        ny = sxy[2 * i + 1];
        nq = charge(i);
      }
      add_source(x, y, q, c, inv_s);
    }
    for (int64_t r = 2; r < span; ++r) {
      const int64_t row = (iy << sh) + r;
      const int32_t i0 = leaf_start[row * nL + (ix << sh)];
      const int32_t i1 = leaf_start[row * nL + (ix << sh) + span];
      for (int32_t i = i0; i < i1; ++i) add_source(sxy[2 * (int64_t)i], sxy[2 * (int64_t)i + 1], charge(i), c, inv_s);
    }
  }
#pragma unroll
  for (int k = 0; k < PMAX; ++k)
    if (k < p) {
      stage[lane * STR + 2 * k] = acc[k].re;
      stage[lane * STR + 2 * k + 1] = acc[k].im;
    }
  // the boxes left to the whole wave, one at a time (a wave-uniform loop),
  // unless a second pass (k_p2m_wave) forms them, a wave each, afterwards
  uint64_t todo = defer ? 0ull : __ballot(b < nbox && by_wave);
  while (todo) {
    const int owner = __builtin_ctzll(todo);
    todo &= todo - 1;
    const int64_t ob = b0 + owner;
    p2m_wave_box<PMAX, QDIM>(g, level, win.bx0 + ob % win.nbx, win.by0 + ob / win.nbx, sxy, sq,
                             leaf_start, p, row_first, row_pre, acc);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < PMAX; ++k)
        if (k < p) {
          stage[owner * STR + 2 * k] = acc[k].re;
          stage[owner * STR + 2 * k + 1] = acc[k].im;
        }
    }
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

// P2M for levels whose boxes hold many sources on average: one wave per box
// of `win` (p2m_wave_box; deterministic, and no LDS buffer limits the waves
// per CU beyond the 512-byte row table).
template <int PMAX, int QDIM>
__global__ __launch_bounds__(kWave) void k_p2m_wave(Geometry g, int level, Window win,
                                                    const double *__restrict__ sxy,
                                                    const double *__restrict__ sq,
                                                    const int32_t *__restrict__ leaf_start, int p,
                                                    double *__restrict__ mp, float *__restrict__ mp32,
                                                    ChildLevel child, int64_t only_above) {
  __shared__ int32_t row_first[kWave], row_pre[kWave];
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int64_t ix = win.bx0 + b % win.nbx, iy = win.by0 + b / win.nbx;
  cplx acc[PMAX];
  bool by_m2m = false;
  const bool ready = children_ready(child, ix, iy);
  // only_above >= 0: the second pass behind k_p2m_box, which left this
  // kernel its boxes of more than only_above sources without formed children
  if (only_above >= 0 && ready) return;
  if (ready || only_above >= 0) {
    // the box's source count, its leaf rows spread over the wave
    const int sh = g.L - level;
    const int64_t nL = int64_t(1) << g.L;
    const int64_t span = int64_t(1) << sh;
    int64_t cnt = 0;
    for (int64_t r = lane; r < span; r += kWave) {
      const int64_t row = (iy << sh) + r;
      cnt += leaf_start[row * nL + (ix << sh) + span] - leaf_start[row * nL + (ix << sh)];
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d);
    if (cnt <= only_above) return;  // wave-uniform
    by_m2m = ready && cnt > kCrowdedBox;
  }
  if (by_m2m) {  // from the children, one coefficient per lane
    if (lane < p) {
      const cplx a = m2m_coeff(child, ix, iy, p, lane);
      mp[b * 2 * p + 2 * lane] = a.re;
      mp[b * 2 * p + 2 * lane + 1] = a.im;
      if (mp32) {
        mp32[b * 2 * p + 2 * lane] = (float)a.re;
        mp32[b * 2 * p + 2 * lane + 1] = (float)a.im;
      }
    }
    return;
  }
  p2m_wave_box<PMAX, QDIM>(g, level, ix, iy, sxy, sq, leaf_start, p, row_first, row_pre, acc);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < PMAX; ++k)
      if (k < p) {
        mp[b * 2 * p + 2 * k] = acc[k].re;
        mp[b * 2 * p + 2 * k + 1] = acc[k].im;
        if (mp32) {
          mp32[b * 2 * p + 2 * k] = (float)acc[k].re;
          mp32[b * 2 * p + 2 * k + 1] = (float)acc[k].im;
        }
      }
  }
}

// M2M for up to four consecutive levels in one launch.  A 256-thread
// workgroup owns a T x T tile of parent boxes at the finest level of the
// launch (T = min(8, boxes per side)); four neighbouring lanes take the four
// children of one parent, each shifting its child's p coefficients (held in
// registers) to the parent's centre, and the four shifted expansions are
// summed across the lanes.  The tile's parents are kept in LDS and the next
// coarser level's (T/2)^2 parents formed from them, and so on, so a tile of
// 8 x 8 boxes yields its 4 x 4, 2 x 2 and 1 x 1 ancestors in the same launch.
//
// The shift needs no table: in child-size units the child centre sits at
// d = (a - 1/2) + i(c - 1/2) from the parent's (quadrant q = a + 2c, child
// (2x + a, 2y + c)), and the parent's rescaled coefficients are
// a_l = 2^-l sum_q sum_{k<=l} C(l,k) d^(l-k) a_k(child q).  The binomial sums
// are formed by repeated synthetic division (p(p-1)/2 updates
// a_j += d a_(j-1)); d's parts are +-1/2, so every product in them is exact.
template <int PMAX>
__global__ __launch_bounds__(kThreads) void k_m2m_tile(M2MChain c) {
  __shared__ double2 bufA[64 * PMAX];  // stage 0 and 2 results
  __shared__ double2 bufB[16 * PMAX];  // stage 1 results
  const int tid = threadIdx.x;
  const int q = tid & 3, par = tid >> 2;  // child quadrant, parent in the tile
  const int p = c.p;
  const int64_t n = int64_t(1) << c.level;
  const int T = n < 8 ? (int)n : 8;
  const int64_t tiles = n / T;
  const int64_t tbx = blockIdx.x % tiles, tby = blockIdx.x / tiles;
  const double dr = (q & 1) - 0.5, di = (q >> 1) - 0.5;
  for (int st = 0; st < c.nlev; ++st) {
    const int Ts = T >> st;      // parents per tile side at this stage
    const int64_t ns = n >> st;  // boxes per side at this level
    // whole waves stay in step for the cross-lane sums below
    if ((tid & ~63) < 4 * Ts * Ts) {
      const bool on = par < Ts * Ts;
      const int tx = on ? par % Ts : 0, ty = on ? par / Ts : 0;
      cplx a[PMAX];
      if (st == 0) {
        const int64_t cb = (2 * (tby * T + ty) + (q >> 1)) * (2 * n) + 2 * (tbx * T + tx) + (q & 1);
        const double2 *src = reinterpret_cast<const double2 *>(c.child) + cb * p;
#pragma unroll
        for (int k = 0; k < PMAX; ++k)
          if (k < p) {
            const double2 v = on ? src[k] : make_double2(0.0, 0.0);
            a[k] = cplx{v.x, v.y};
          }
      } else {
        const double2 *src = (st == 2 ? bufB : bufA) + ((2 * ty + (q >> 1)) * (2 * Ts) + 2 * tx + (q & 1)) * PMAX;
#pragma unroll
        for (int k = 0; k < PMAX; ++k)
          if (k < p) {
            const double2 v = on ? src[k] : make_double2(0.0, 0.0);
            a[k] = cplx{v.x, v.y};
          }
      }
#pragma unroll
      for (int k = 0; k + 1 < PMAX; ++k)
        if (k + 1 < p) {
#pragma unroll
          for (int j = PMAX - 1; j > k; --j)
            if (j < p) {
              a[j].re = fma(dr, a[j - 1].re, fma(-di, a[j - 1].im, a[j].re));
              a[j].im = fma(dr, a[j - 1].im, fma(di, a[j - 1].re, a[j].im));
            }
        }
      // sum over the four children (lanes 4i .. 4i+3), in a fixed order
#pragma unroll
      for (int l = 0; l < PMAX; ++l)
        if (l < p) {
          double re = a[l].re + __shfl_xor(a[l].re, 1);
          double im = a[l].im + __shfl_xor(a[l].im, 1);
          re += __shfl_xor(re, 2);
          im += __shfl_xor(im, 2);
          a[l] = cplx{ldexp(re, -l), ldexp(im, -l)};
        }
      if (on && q == 0) {
        const int64_t box = (tby * Ts + ty) * ns + tbx * Ts + tx;
        double2 *gout = reinterpret_cast<double2 *>(c.out[st]) + box * p;
        float2 *gout32 = c.out32[st] ? reinterpret_cast<float2 *>(c.out32[st]) + box * p : nullptr;
        double2 *keep = st == 1 ? bufB : bufA;
#pragma unroll
        for (int l = 0; l < PMAX; ++l)
          if (l < p) {
            gout[l] = make_double2(a[l].re, a[l].im);
            if (gout32) gout32[l] = make_float2((float)a[l].re, (float)a[l].im);
            if (st + 1 < c.nlev) keep[par * PMAX + l] = make_double2(a[l].re, a[l].im);
          }
      }
    }
    __syncthreads();
  }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace


void launch_p2m(Geometry g, int level, Window win, const double *sxy, const double *sq, int qdim,
                const int32_t *leaf_start, int p, double *mp, float *mp32, double win_sources,
                bool clustered, Window child_win, const double *child_mp, hipStream_t stream) {
  const ChildLevel child{child_win, child_mp};
  const int64_t n = win.count() * p;
  if (n == 0) return;
  // boxes of ~128 sources or more (on average over the window): a wave per
  // box (below that a thread per box, crowded boxes by M2M in their lanes,
  // measured faster on a galaxy halo's levels of 24 and 91 stars per box)
  auto wave_per_box = [&](int64_t only_above) {
    const unsigned nb = (unsigned)win.count();
    if (qdim == 2)
      LENS_PMAX_DISPATCH(p, hipLaunchKernelGGL((k_p2m_wave<PM, 2>), dim3(nb), dim3(kWave), 0, stream,
                                               g, level, win, sxy, sq, leaf_start, p, mp, mp32,
                                               child, only_above));
    else
      LENS_PMAX_DISPATCH(p, hipLaunchKernelGGL((k_p2m_wave<PM, 1>), dim3(nb), dim3(kWave), 0, stream,
                                               g, level, win, sxy, sq, leaf_start, p, mp, mp32,
                                               child, only_above));
    LENS_HIP(hipGetLastError());
  };
  const double mean = win_sources / (double)win.count();
  if (mean > 128.0) {
    wave_per_box(-1);
    return;
  }
  // otherwise a thread per box (all coefficients), unless p exceeds the
  // register budget of that kernel's largest instance.  In a clustered
  // field whose leaf boxes hold a few sources on average, those of more
  // than kWaveBox sources get a wave each in a second pass rather than their
  // lane's wave one after another (above the leaf level such boxes are
  // formed from their children).
  if (p <= 24) {
    const int defer = (clustered && mean > 2.0 && child_mp == nullptr) ? 1 : 0;
    const unsigned nb = (unsigned)((win.count() + kWave - 1) / kWave);
    if (qdim == 2)
      LENS_PMAX_DISPATCH(p, hipLaunchKernelGGL((k_p2m_box<PM, 2>), dim3(nb), dim3(kWave), 0, stream,
                                               g, level, win, sxy, sq, leaf_start, p, mp, mp32,
                                               child, defer));
    else
      LENS_PMAX_DISPATCH(p, hipLaunchKernelGGL((k_p2m_box<PM, 1>), dim3(nb), dim3(kWave), 0, stream,
                                               g, level, win, sxy, sq, leaf_start, p, mp, mp32,
                                               child, defer));
    LENS_HIP(hipGetLastError());
    if (defer) wave_per_box(kWaveBox);
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

int m2m_chain_levels(int level) {
  // T = min(8, 2^level) parents per tile side; T halves per fused level
  int T = level >= 3 ? 8 : (1 << level), k = 1;
  while (T > 1 && k < kMaxM2MChain) {
    T >>= 1;
    ++k;
  }
  return k;
}

void launch_m2m_chain(const M2MChain &c, hipStream_t stream) {
  if (c.nlev < 1 || c.nlev > m2m_chain_levels(c.level))
    fail(LENS_EINVAL, "M2M chain: bad level count");
  const int64_t n = int64_t(1) << c.level;
  const int64_t T = n < 8 ? n : 8;
  const unsigned blocks = (unsigned)((n / T) * (n / T));
  LENS_PMAX_DISPATCH(c.p, hipLaunchKernelGGL((k_m2m_tile<PM>), dim3(blocks), dim3(kThreads), 0, stream, c));
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
