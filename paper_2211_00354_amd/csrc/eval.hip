// Evaluation at the rays (Appendix A, steps 6 and 7) fused with the smooth
// field (Section 2.4, step 3) and, for maps, inverse-ray-shooting binning
// (Section 2.3).
//
// Work unit = one chunk of up to 64*R rays of one leaf box of the target
// window, handled by one wave (a 64-thread workgroup):
//   * the stars of the box's 3x3 neighbourhood (three contiguous row ranges
//     of the sorted star array) and the box's local expansion are the same
//     for every lane, so they are read with wave-uniform scalar loads into
//     SGPRs and used directly as VALU operands -- every star is fetched once
//     per wave and shared by all 64*R rays;
//   * near field: alpha_near = sum m (x - x_i)/|x - x_i|^2 over those stars;
//     LENS_MIXED takes ray and star coordinates relative to the box centre
//     (FP64, rounded to FP32) and does the pair arithmetic in FP32;
//   * far field: f(z) = sum_l b~_l w^l, w = (z - c)/s, by Horner in FP64,
//     alpha_far = conj(f);
//   * y = (1-kappa_s-gamma, 1-kappa_s+gamma) * x - alpha in FP64, written as
//     [n][2] or binned into the map: counts are summed per unit in an LDS
//     table and added to the map with one integer atomic per distinct pixel.
// Units are spread over a bounded grid; consecutive units (neighbouring
// boxes, which share stars) go to the same XCD so that they share its L2.
#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kWave = 64;
constexpr int kXcd = 8;
constexpr int32_t kFlushStars = 128;  // LENS_MIXED near-field partials per FP64 flush
constexpr int kThreads = 256;  // helper kernels


// One star against the R rays of a lane.  The pair difference x - x_i is
// formed in FP64 from absolute coordinates (the star's are wave-uniform
// scalars), so it is exact to ~1e-16 of the coordinates however close the
// pair; LENS_MIXED rounds it once to FP32 and does the rest of the pair
// arithmetic in FP32, so every pair carries only a few FP32 roundings
// relative to its own size.  A coincident pair (dx = dy = 0) contributes
// exactly zero: the tiny term keeps its weight finite (for |m| below ~1e8 in
// FP32, ~1e108 in FP64) and it multiplies dx = dy = 0, so no branch or
// select is needed; it changes no pair farther apart than ~1e-13 (FP32).
//
// DERIV also accumulates f'(z) = -sum m / (z - z_i)^2: with dz = dx + i dy,
// 1/dz^2 = (dx^2 - dy^2 - 2i dx dy) / r^4, so f' gains -t (dx - dy)(dx + dy)
// (real) and 2 t dx dy (imaginary), t = m / r^4; a coincident pair has
// r2 = tiny exactly and gets t = 0.
template <bool MIXED, bool DERIV, int R, typename A, typename M>
__device__ __forceinline__ void pair_update(const double (&rx)[R], const double (&ry)[R], double sx,
                                            double sy, M mm, A (&ax)[R], A (&ay)[R],
                                            A (&dre)[R], A (&dim)[R]) {
  if constexpr (MIXED) {
    const float m = mm;  // the mass, rounded to FP32 when the stars were sorted
    constexpr float tiny = 0x1p-100f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float dx = (float)(rx[r] - sx);
      const float dy = (float)(ry[r] - sy);
      const float r2 = fmaf(dx, dx, fmaf(dy, dy, tiny));
      const float inv = rcp_f32(r2);
      const float w = m * inv;
      ax[r] = fmaf(w, dx, ax[r]);
      ay[r] = fmaf(w, dy, ay[r]);
      if constexpr (DERIV) {
        const float t = r2 > tiny ? w * inv : 0.0f;
        dre[r] = fmaf(-t, (dx - dy) * (dx + dy), dre[r]);
        dim[r] = fmaf(t + t, dx * dy, dim[r]);
      }
    }
  } else {
    constexpr double tiny = 0x1p-664;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double dx = rx[r] - sx;
      const double dy = ry[r] - sy;
      const double r2 = fma(dx, dx, fma(dy, dy, tiny));
      const double inv = rcp_f64(r2);
      const double w = mm * inv;
      ax[r] = fma(w, dx, ax[r]);
      ay[r] = fma(w, dy, ay[r]);
      if constexpr (DERIV) {
        const double t = r2 > tiny ? w * inv : 0.0;
        dre[r] = fma(-t, (dx - dy) * (dx + dy), dre[r]);
        dim[r] = fma(t + t, dx * dy, dim[r]);
      }
    }
  }
}

// Map counts of a work unit are first summed in a small per-wave table in
// LDS (pixel key -> count, open addressing with four linear probes; a ray
// whose pixel finds all probed slots taken by other pixels goes straight to
// the global map), then added to the map with one atomic per distinct pixel.
// A unit's rays land on a compact patch of pixels, so 256 entries suffice.
constexpr int kMapTableBits = 8;
constexpr int kMapTable = 1 << kMapTableBits;

__device__ __forceinline__ void map_table_add(int32_t *hkey, uint32_t *hval, int32_t key,
                                              int32_t *__restrict__ counts) {
  uint32_t slot = ((uint32_t)key * 2654435761u) >> (32 - kMapTableBits);
#pragma unroll
  for (int probe = 0; probe < 4; ++probe) {
    const int32_t prev = atomicCAS(&hkey[slot], -1, key);
    if (prev == -1 || prev == key) {
      atomicAdd(&hval[slot], 1u);
      return;
    }
    slot = (slot + 1) & (kMapTable - 1);
  }
  atomicAdd(&counts[key], 1);
}

__device__ __forceinline__ void map_table_flush(int32_t *hkey, uint32_t *hval,
                                                int32_t *__restrict__ counts, int lane) {
  __syncthreads();
#pragma unroll
  for (int e = lane; e < kMapTable; e += 64) {
    const int32_t k = hkey[e];
    if (k >= 0) {
      atomicAdd(&counts[k], (int32_t)hval[e]);
      hkey[e] = -1;
      hval[e] = 0;
    }
  }
  __syncthreads();
}

// The mixed kernels are compiled for five waves per SIMD (at most 96 VGPRs;
// the R = 4 instances spill a few bytes of per-lane scratch outside the pair
// loop), which measured faster than four waves without spills.
template <int PMAX, bool MIXED, bool MAP, bool GRID, int R, bool DERIV>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(MIXED && !DERIV ? 5 : 1))) void k_eval(EvalArgs a, const double *__restrict__ loc,
                                                const double *__restrict__ sxy,
                                                const double *__restrict__ sm,
                                                const float *__restrict__ sm32,
                                                const int32_t *__restrict__ leaf_start,
                                                const int32_t *__restrict__ col_start,
                                                const int32_t *__restrict__ row_start,
                                                const double *__restrict__ rxy,
                                                const uint32_t *__restrict__ rperm,
                                                const int32_t *__restrict__ ray_start,
                                                double *__restrict__ y_out,
                                                int32_t *__restrict__ counts) {
  // the box's local expansion, read by every lane (LDS broadcast)
  __shared__ double2 lds_loc[PMAX];
  // LENS_MIXED: FP64 sums of the lanes' FP32 near-field partials, flushed
  // every kFlushStars stars (alpha; f' with DERIV)
  __shared__ double2 lds_acc[MIXED ? kWave * R * (DERIV ? 2 : 1) : 1];
  __shared__ int32_t hkey[MAP ? kMapTable : 1];
  __shared__ uint32_t hval[MAP ? kMapTable : 1];
  const int lane = threadIdx.x;
  if (MAP) {
    for (int e = lane; e < kMapTable; e += 64) {
      hkey[e] = -1;
      hval[e] = 0;
    }
  }
  // unit counts fit in 31 bits (checked at launch)
  const uint32_t CH = (uint32_t)a.chunks_per_box;
  const uint32_t nbx = (uint32_t)a.win.nbx;
  const uint32_t nunits = (uint32_t)(a.win.count() * CH);
  // XCD-aware virtual block id: blocks dispatched to one XCD (blockIdx % 8)
  // take a contiguous range of units in each sweep of the grid.
  const uint32_t G = gridDim.x;
  const uint32_t per_xcd = G / kXcd;
  const uint32_t vb = (G % kXcd == 0) ? (blockIdx.x % kXcd) * per_xcd + blockIdx.x / kXcd : blockIdx.x;
  const int64_t nL = int64_t(1) << a.g.L;
  const double s = ldexp(a.g.side, -a.g.L);
  const double inv_s = 1.0 / s;
  const int p = a.p;
  constexpr int RPC = kWave * R;
  // grid rays: a wave's R slots are R tiles of TX x TY rays (TX * TY = 64)
  const int tsh = a.tile_shift;
  const int TX = 1 << tsh, TY = kWave >> tsh;
  const int lx = lane & (TX - 1), ly = lane >> tsh;

  for (uint32_t u = vb; u < nunits; u += G) {
    const uint32_t b = CH == 1 ? u : u / CH;
    const uint32_t c0 = u - b * CH;
    const uint32_t byw = b / nbx, bxw = b - byw * nbx;
    const int64_t gx = a.win.bx0 + bxw, gy = a.win.by0 + byw;

    // grid: the box's rays are columns [i0, i0+W) x rows [j0, j0+H), cut into
    // nt = TW x TH tiles, tpc consecutive tiles per unit; explicit: rays
    // [r0, r0+nr) of the sorted array in chunks of RPC
    int32_t nr = 0, r0 = 0, i0 = 0, j0 = 0, W = 0, H = 0, TW = 1, nt = 0, tpc = 0;
    if (GRID) {
      i0 = col_start[bxw];
      W = col_start[bxw + 1] - i0;
      j0 = row_start[byw];
      H = row_start[byw + 1] - j0;
      TW = (W + TX - 1) >> tsh;
      nt = TW * ((H + TY - 1) / TY);
      tpc = (nt + (int32_t)CH - 1) / (int32_t)CH;
      if (nt == 0 || (int64_t)c0 * tpc >= nt) continue;  // uniform
    } else {
      r0 = ray_start[b];
      nr = ray_start[b + 1] - r0;
      if (nr == 0 || (int64_t)c0 * RPC >= nr) continue;  // uniform
    }

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
    __syncthreads();  // the previous unit's reads of lds_loc are done
    if (lane < p) lds_loc[lane] = reinterpret_cast<const double2 *>(loc + 2 * (int64_t)b * p)[lane];
    __syncthreads();

    // passes of R tiles (grid) or RPC rays (explicit); explicit rays beyond
    // CH chunks are looped over by the box's units
    int32_t pos, pend, pstep;
    if (GRID) {
      pos = (int32_t)c0 * tpc;
      pend = min(nt, pos + tpc);
      pstep = R;
    } else {
      pos = (int32_t)c0 * RPC;
      pend = nr;
      pstep = (int32_t)CH * RPC;
    }
    for (; pos < pend; pos += pstep) {
      double rx[R], ry[R];
      using acc_t = typename std::conditional<MIXED, float, double>::type;
      acc_t ax[R], ay[R], dre[R], dim[R];
      int64_t oidx[R];
      bool act[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (GRID) {
          // slot r's ray (an inactive slot takes the box's first ray); its
          // output index is formed after the pair loop
          const int32_t t = pos + r;  // wave-uniform tile index
          const int32_t ty = t / TW, tx = t - ty * TW;
          const int32_t ci = tx * TX + lx, cj = ty * TY + ly;
          const bool on = t < pend && ci < W && cj < H;
          rx[r] = grid_coord(a.grid.x0, a.grid.dx, i0 + (on ? ci : 0));
          ry[r] = grid_coord(a.grid.y0, a.grid.dy, j0 + (on ? cj : 0));
        } else {
          const int32_t idx = pos + r * kWave + lane;
          act[r] = idx < min(nr, pos + RPC);
          const int32_t id = act[r] ? idx : 0;
          rx[r] = rxy[2 * ((int64_t)r0 + id)];
          ry[r] = rxy[2 * ((int64_t)r0 + id) + 1];
          oidx[r] = rperm ? (int64_t)rperm[r0 + id] : (int64_t)r0 + id;
        }
        ax[r] = 0;
        ay[r] = 0;
        dre[r] = 0;
        dim[r] = 0;
      }

      // LENS_MIXED reads the masses' FP32 copies (no conversion per star)
      using mass_t = typename std::conditional<MIXED, float, double>::type;
      auto mass = [&](int32_t i) -> mass_t {
        if constexpr (MIXED) return sm32[i]; else return sm[i];
      };
      auto star = [&](double x, double y, mass_t m) {
        pair_update<MIXED, DERIV, R>(rx, ry, x, y, m, ax, ay, dre, dim);
      };
      // LENS_MIXED: every kFlushStars stars the FP32 partial sums move into
      // FP64 ones in LDS (a wave-uniform count), so a ray with thousands
      // of near stars (a cluster's core) does not accumulate thousands of
      // FP32 roundings; a box of fewer stars never flushes
      int32_t since = 0;
      bool flushed = false;
      auto flush = [&]() {
        if constexpr (MIXED) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            double2 &acc = lds_acc[r * kWave + lane];
            const double2 old = flushed ? acc : make_double2(0.0, 0.0);
            acc = make_double2(old.x + (double)ax[r], old.y + (double)ay[r]);
            ax[r] = 0;
            ay[r] = 0;
            if (DERIV) {
              double2 &acd = lds_acc[(R + r) * kWave + lane];
              const double2 od = flushed ? acd : make_double2(0.0, 0.0);
              acd = make_double2(od.x + (double)dre[r], od.y + (double)dim[r]);
              dre[r] = 0;
              dim[r] = 0;
            }
          }
          flushed = true;
          since = 0;
        }
      };
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int32_t i = rs[d];
        // four stars per step: their scalar loads issue together
        for (; i + 4 <= re[d]; i += 4) {
          double sx[4], sy[4];
          mass_t mm[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            sx[q] = sxy[2 * (int64_t)(i + q)];
            sy[q] = sxy[2 * (int64_t)(i + q) + 1];
            mm[q] = mass(i + q);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) star(sx[q], sy[q], mm[q]);
          if (MIXED) {
            since += 4;
            if (since >= kFlushStars) flush();
          }
        }
        for (; i < re[d]; ++i) star(sxy[2 * (int64_t)i], sxy[2 * (int64_t)i + 1], mass(i));
      }

      // ray offsets from the box centre (FP64) for the far field; grid rays'
      // output indices and activity recomputed from the lane's tile position
      // (integers) rather than kept live through the pair loop
      double dxr[R], dyr[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        dxr[r] = rx[r] - cx;
        dyr[r] = ry[r] - cy;
      }
      if (GRID) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int32_t t = pos + r;
          const int32_t ty = t / TW, tx = t - ty * TW;
          const int32_t ci = tx * TX + lx, cj = ty * TY + ly;
          act[r] = t < pend && ci < W && cj < H;
          const int32_t cc = act[r] ? ci : 0, rr = act[r] ? cj : 0;
          oidx[r] = (int64_t)(j0 + rr) * a.grid.nx + (i0 + cc);
        }
      }
      // far field: Horner over the R rays from the top coefficient down, one
      // LDS read per coefficient
      // (DERIV: the derivative sum g = sum l b_l w^(l-1) in the same sweep,
      // g <- g w + f before f <- f w + b_l; f' = g / s)
      cplx w[R], f[R], gd[R];
      {
        const double2 top = lds_loc[p - 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          w[r] = cplx{dxr[r] * inv_s, dyr[r] * inv_s};
          f[r] = cplx{top.x, top.y};
          gd[r] = cplx{0.0, 0.0};
        }
      }
      // a runtime trip count (the order-guarded unrolled form keeps one
      // spilled branch mask per level)
#pragma unroll 2
      for (int l = p - 2; l >= 0; --l) {
        const double2 c = lds_loc[l];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (DERIV) gd[r] = cmad(gd[r], w[r], f[r]);
          f[r] = cmad(f[r], w[r], cplx{c.x, c.y});
        }
      }

      int32_t key[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // the FP64 near-field sum: the FP32 partial plus, where a flush
        // happened, the flushed ones
        double nx = (double)ax[r], ny = (double)ay[r];
        if (MIXED && flushed) {
          const double2 acc = lds_acc[r * kWave + lane];
          nx += acc.x;
          ny += acc.y;
        }
        const double al1 = f[r].re + nx;
        const double al2 = ny - f[r].im;
        const double y1 = a.c1 * rx[r] - al1;
        const double y2 = a.c2 * ry[r] - al2;
        if (MAP) {
          key[r] = -1;
          const double t1 = (y1 - a.y1min) * a.S;
          const double t2 = (y2 - a.y2min) * a.S;
          if (act[r] && t1 >= 0.0 && t2 >= 0.0) {
            const double f1 = floor(t1), f2 = floor(t2);
            if (f1 < (double)a.npix && f2 < (double)a.npix)
              key[r] = (int32_t)f2 * a.npix + (int32_t)f1;
          }
        } else if (act[r]) {
          *reinterpret_cast<double2 *>(y_out + 2 * oidx[r]) = make_double2(y1, y2);
          if (DERIV) {
            double nre = (double)dre[r], nim = (double)dim[r];
            if (MIXED && flushed) {
              const double2 acd = lds_acc[(R + r) * kWave + lane];
              nre += acd.x;
              nim += acd.y;
            }
            *reinterpret_cast<double2 *>(a.dfdz_out + 2 * oidx[r]) =
                make_double2(fma(gd[r].re, inv_s, nre), fma(gd[r].im, inv_s, nim));
          }
        }
      }
      if (MAP) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (key[r] >= 0) map_table_add(hkey, hval, key[r], counts);
      }
    }
    if (MAP) map_table_flush(hkey, hval, counts, lane);
  }
}

// first ray column (row) of every box column (row) of the window: columns in
// blockIdx.y = 0, rows in blockIdx.y = 1 (one launch)
struct GridAxis {
  double x0, dx;       // grid origin and step along the axis
  int64_t lo_i, hi_i;  // ray index range searched
  double origin;       // root square origin along the axis
  int64_t b0, nb;      // first window box and window size along the axis
  int32_t *out;        // [nb + 1]
};

__global__ __launch_bounds__(kThreads) void k_grid_ranges(GridAxis ax, GridAxis ay, double s,
                                                          int64_t nL) {
  const GridAxis &a = blockIdx.y == 0 ? ax : ay;
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c > a.nb) return;
  const int64_t B = a.b0 + c;
  int64_t lo = a.lo_i, hi = a.hi_i;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (box_coord(grid_coord(a.x0, a.dx, mid), a.origin, s, nL) < B)
      lo = mid + 1;
    else
      hi = mid;
  }
  a.out[c] = (int32_t)lo;
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

constexpr int64_t kMaxEvalBlocks = 256 * 32 * 4;  // CUs x waves per CU x sweeps in flight

template <int PM, bool MIXED, bool MAP, bool GRID, int R, bool DERIV = false>
void eval_launch_r(const EvalArgs &a, hipStream_t stream) {
  const int64_t units = a.win.count() * a.chunks_per_box;
  int64_t nblk = units < kMaxEvalBlocks ? units : kMaxEvalBlocks;
  if (nblk > kXcd) nblk = nblk / kXcd * kXcd;
  hipLaunchKernelGGL((k_eval<PM, MIXED, MAP, GRID, R, DERIV>), dim3((unsigned)nblk), dim3(kWave), 0, stream,
                     a, a.loc, a.sxy, a.sm, a.sm32, a.leaf_start, a.col_start, a.row_start, a.rxy, a.rperm,
                     a.ray_start, a.y_out, a.counts);
}

template <int PM, bool MIXED, bool MAP, bool GRID>
void eval_launch(const EvalArgs &a, hipStream_t stream) {
  if constexpr (!MAP) {
    // f' wanted: one instance per order bucket, two rays per lane (the
    // launch shape is chosen for R = 2 in that case)
    if (a.dfdz_out) {
      eval_launch_r<PM, MIXED, MAP, GRID, 2, true>(a, stream);
      return;
    }
  }
  switch (a.rays_per_lane) {
    case 1: eval_launch_r<PM, MIXED, MAP, GRID, 1>(a, stream); break;
    case 2: eval_launch_r<PM, MIXED, MAP, GRID, 2>(a, stream); break;
    case 3: eval_launch_r<PM, MIXED, MAP, GRID, 3>(a, stream); break;
    default: eval_launch_r<PM, MIXED, MAP, GRID, 4>(a, stream); break;
  }
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

// Rays per lane R and units per box CH for boxes of at most max_rays rays:
// the fewest lane slots 64*R*passes*CH, ties going to the larger R, with up
// to kPassesPerUnit passes of 64*R rays per unit.  A unit starts by loading
// its box's local expansion with a vector load, which waits for every
// earlier vector memory operation of the wave (the previous unit's stores or
// map atomics); several passes per unit spread that wait.
constexpr int64_t kPassesPerUnit = 8;

void eval_shape(int64_t max_rays, int *R, int64_t *CH) {
  int best_r = 1;
  int64_t best_ch = 1, best_slots = -1;
  for (int r = 1; r <= 4; ++r) {
    const int64_t passes = (max_rays + kWave * r - 1) / (kWave * r);
    const int64_t ch = (passes + kPassesPerUnit - 1) / kPassesPerUnit;
    const int64_t per = (passes + ch - 1) / ch;
    const int64_t slots = ch * per * kWave * r;
    if (best_slots < 0 || slots <= best_slots) {
      best_slots = slots;
      best_r = r;
      best_ch = ch < 1 ? 1 : ch;
    }
  }
  *R = best_r;
  *CH = best_ch;
}

// Tile shape for grid rays in boxes of at most W x H rays: TX = 2^shift
// columns by 64/TX rows, the fewest tiles per box, ties going to the
// squarest tile (rays of a square tile land close together in a map).
void grid_tile_shape(int64_t W, int64_t H, int *shift, int64_t *tiles) {
  int best = 3;
  int64_t best_t = -1;
  for (int sh : {3, 2, 4, 1, 5, 0, 6}) {
    const int64_t tx = int64_t(1) << sh, ty = kWave / tx;
    const int64_t t = ((W + tx - 1) / tx) * ((H + ty - 1) / ty);
    if (best_t < 0 || t < best_t) {
      best_t = t;
      best = sh;
    }
  }
  *shift = best;
  *tiles = best_t;
}

void launch_eval(const EvalArgs &a, int precision, hipStream_t stream) {
  if (a.win.count() == 0) return;
  if (precision == LENS_MIXED && !a.sm32)
    fail(LENS_EINVAL, "mixed-precision evaluation needs the plan's FP32 masses");
  LENS_PMAX_DISPATCH(a.p, eval_dispatch<PM>(a, precision, stream));
  LENS_HIP(hipGetLastError());
}

void launch_grid_ranges(const lens_grid &grid, Geometry g, Window win, int64_t j_begin,
                        int64_t j_end, int32_t *col_start, int32_t *row_start,
                        hipStream_t stream) {
  const int64_t nL = int64_t(1) << g.L;
  const double s = ldexp(g.side, -g.L);
  const GridAxis ax{grid.x0, grid.dx, 0, grid.nx, g.x0, win.bx0, win.nbx, col_start};
  const GridAxis ay{grid.y0, grid.dy, j_begin, j_end, g.y0, win.by0, win.nby, row_start};
  const int64_t nmax = std::max(win.nbx, win.nby) + 1;
  hipLaunchKernelGGL(k_grid_ranges, dim3((unsigned)((nmax + kThreads - 1) / kThreads), 2),
                     dim3(kThreads), 0, stream, ax, ay, s, nL);
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
