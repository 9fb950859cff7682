// Downward pass (Appendix A, downward passes 1 and 2), for each level
// l = 2..L over the target window (the boxes that hold rays):
//
//   M2L:  local(t)  = (1/s_l) sum_{tau in IL(t)} T_tau a~(t + tau)
//   L2L:  local(t) += L2L(local(parent(t)))        (l >= 3), FP64
//
// M2L of every level runs first (one batched launch per arithmetic type, as
// levels are independent there), then L2L sweeps the levels coarse to fine.
//
// IL(t) is the interaction list: the children of the parent's neighbours
// that are not neighbours of t.  For a target that is child (qx, qy) of its
// parent, tau = (c_src - c_tgt)/s ranges over [-2-qx, 3-qx] x [-2-qy, 3-qy]
// minus the 3x3 neighbourhood: 27 offsets out of 40 distinct ones, the same
// operators at every level on rescaled coefficients.  Source boxes outside the
// root are empty.
//
// M2L on MFMA (k_m2l_mfma): a workgroup takes a TILE x TILE block of target
// boxes; its four waves take the four quadrant classes, so every wave applies
// the same 27 operators.  The (TILE+4)^2 source multipoles the block needs are
// staged once in LDS (coalesced row loads of box-major coefficients).  For one
// offset the wave's 16-target M-tiles form a real GEMM
//   C[16 targets][2p] += A[16][2p] B_tau[2p][2p]
// over interleaved (re, im) coefficients, done with 16x16x4 MFMAs: A rows are
// read from the LDS tile at the target + tau, B fragments come pre-swizzled
// in lane order from global memory (L1/L2 resident, shared by every wave).
// FP32 (fine levels of LENS_MIXED) uses v_mfma_f32_16x16x4f32, FP64 uses
// v_mfma_f64_16x16x4f64; B fragments of the next offset are loaded while the
// current one computes.  The result, scaled by 1/s, is stored as the FP64
// locals.  Orders whose tile does not fit the LDS budget use the VALU kernel.
#include <type_traits>

#include <mutex>
#include <vector>

#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kThreads = 256;
constexpr size_t kLdsBudget = 64 * 1024;

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------- L2L

// loc += L2L(parent locals); one thread per (target box, output coefficient j).
__global__ __launch_bounds__(kThreads) void k_l2l(DownArgs a, const double *__restrict__ l2l) {
  const int p = a.p;
  const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= a.win.count() * p) return;
  const int64_t ob = idx / p;
  const int j = (int)(idx - ob * p);
  const int64_t tx = a.win.bx0 + ob % a.win.nbx, ty = a.win.by0 + ob / a.win.nbx;
  cplx acc = {a.loc[2 * idx], a.loc[2 * idx + 1]};
  {
    const int q = (int)((tx & 1) + 2 * (ty & 1));
    const int64_t pb = ((ty >> 1) - a.pwin.by0) * a.pwin.nbx + ((tx >> 1) - a.pwin.bx0);
    const double *par = a.ploc + 2 * pb * p;
    const double *t = l2l + (size_t)q * p * p * 2;
    for (int l = j; l < p; ++l) {
      const cplx b = {par[2 * l], par[2 * l + 1]};
      const cplx m = {t[((size_t)l * p + j) * 2], t[((size_t)l * p + j) * 2 + 1]};
      acc = cmad(m, b, acc);
    }
  }
  a.loc[2 * idx] = acc.re;
  a.loc[2 * idx + 1] = acc.im;
}

// L2L down up to three levels in one launch: a 64-thread workgroup owns one
// box of the chain's top level (its locals final) and its descendants: at
// depth j, thread t < 4^j takes descendant (t mod 2^j, t div 2^j) of the
// 2^j x 2^j block, adds the shifted locals of its parent (the previous
// depth's result, kept in LDS) to its own M2L locals and stores them.  A box
// outside its level's window is skipped; its children lie outside theirs.
//
// The shift needs no table: with the child centre at d = (a - 1/2) +
// i(c - 1/2) parent half-sides from the parent's (child (2x + a, 2y + c)),
// the child gets c_j += sum_{l>=j} C(l,j) d^(l-j) 2^-l b_l, the coefficients
// of B(w + d) for B(w) = sum_l 2^-l b_l w^l, formed by Horner-style synthetic
// division (p(p-1)/2 updates b_j += d b_(j+1), exact products).
template <int PMAX>
__global__ __launch_bounds__(64) void k_l2l_tile(L2LChain c) {
  __shared__ double2 bufA[16 * PMAX];  // depth-2 results
  __shared__ double2 bufB[4 * PMAX];   // depth-1 results
  const int lane = threadIdx.x;
  const int p = c.p;
  const int64_t rb = blockIdx.x;
  const int64_t RX = c.win[0].bx0 + rb % c.win[0].nbx, RY = c.win[0].by0 + rb / c.win[0].nbx;
  for (int j = 1; j <= c.nlev; ++j) {
    const int side = 1 << j;
    if (lane < side * side) {
      const int dx = lane % side, dy = lane / side;
      const int64_t X = RX * side + dx, Y = RY * side + dy;
      const Window &w = c.win[j];
      if (X >= w.bx0 && X < w.bx0 + w.nbx && Y >= w.by0 && Y < w.by0 + w.nby) {
        double2 *dst = reinterpret_cast<double2 *>(c.loc[j]) + ((Y - w.by0) * w.nbx + (X - w.bx0)) * p;
        const double dr = (double)(X & 1) - 0.5, di = (double)(Y & 1) - 0.5;
        cplx b[PMAX];
        // parent from global memory (depth 1) or LDS, through separate loads
        // so that no pointer mixes the two address spaces
        auto load = [&](auto parent_coef) {
#pragma unroll
          for (int l = 0; l < PMAX; ++l)
            if (l < p) {
              const double2 v = parent_coef(l);
              b[l] = cplx{ldexp(v.x, -l), ldexp(v.y, -l)};
            }
        };
        if (j == 1) {
          const double2 *root = reinterpret_cast<const double2 *>(c.loc[0]) + rb * p;
          load([&](int l) { return root[l]; });
        } else {
          const double2 *lp = (j == 2 ? bufB : bufA) + ((dy >> 1) * (side >> 1) + (dx >> 1)) * PMAX;
          load([&](int l) { return lp[l]; });
        }
#pragma unroll
        for (int k = 0; k + 1 < PMAX; ++k)
          if (k + 1 < p) {
#pragma unroll
            for (int i = PMAX - 2; i >= k; --i)
              if (i + 1 < p) {
                b[i].re = fma(dr, b[i + 1].re, fma(-di, b[i + 1].im, b[i].re));
                b[i].im = fma(dr, b[i + 1].im, fma(di, b[i + 1].re, b[i].im));
              }
          }
        double2 *keep = j == 1 ? bufB : bufA;
#pragma unroll
        for (int i = 0; i < PMAX; ++i)
          if (i < p) {
            const double2 v = dst[i];
            const double2 r = make_double2(v.x + b[i].re, v.y + b[i].im);
            dst[i] = r;
            if (j < c.nlev) keep[lane * PMAX + i] = r;
          }
      }
    }
    __syncthreads();
  }
}

// --------------------------------------------------------- M2L on MFMA

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  using acc = f4v;
  __device__ static acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of output register r in lane `lane` (16x16 f32 result layout)
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct Mfma<double> {
  using acc = d4v;
  __device__ static acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// Interaction list of a quadrant class as 27 (tau_x, tau_y) offsets.
struct IList {
  int8_t t[4][27][2];
};
constexpr IList make_ilist() {
  IList il{};
  for (int q = 0; q < 4; ++q) {
    const int qx = q & 1, qy = q >> 1;
    int j = 0;
    for (int ty = -2 - qy; ty <= 3 - qy; ++ty)
      for (int tx = -2 - qx; tx <= 3 - qx; ++tx) {
        if (tx >= -1 && tx <= 1 && ty >= -1 && ty <= 1) continue;
        il.t[q][j][0] = (int8_t)tx;
        il.t[q][j][1] = (int8_t)ty;
        ++j;
      }
  }
  return il;
}
__constant__ IList kIL = make_ilist();

// TILE x TILE targets per workgroup; the 4 waves own the quadrant classes;
// each quadrant class holds (TILE/2)^2 targets = MT M-tiles of 16.  KS
// K-steps of 4 cover the 2p interleaved input coefficients, NT N-tiles of 16
// the 2p outputs.  One launch serves several levels (M2L of different levels
// is independent): blockIdx.x indexes the concatenated tile lists.  Up to
// moderate orders the register budget is set for three or more waves per
// SIMD (the accumulators then live in VGPRs, not AGPRs), which keeps several
// workgroups per CU in flight; larger orders keep the compiler's choice.
template <typename T, int TILE, int KS>
constexpr int m2l_min_waves() {
  return KS <= (sizeof(T) == 4 ? 8 : 6) ? 3 : 1;
}
template <typename T, int TILE, int KS, bool FUSE>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(m2l_min_waves<T, TILE, KS>()))) void k_m2l_mfma(
    M2LBatch bt, const T *__restrict__ bfrag, const double *__restrict__ l2l_frag) {
  constexpr int S = TILE + 4;            // source tile side
  constexpr int H = TILE / 2;            // targets per quadrant class per side
  constexpr int MT = H * H / 16;         // M-tiles per wave
  constexpr int NT = (KS + 3) / 4;       // N-tiles: 2p <= 4 KS outputs
  constexpr int REC = 4 * KS + 1;        // LDS record stride (odd: spreads banks)
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T *lds = reinterpret_cast<T *>(lds_raw);

  int li = 0;
  while (li + 1 < bt.count && (int64_t)blockIdx.x >= bt.tile_begin[li + 1]) ++li;
  const M2LLevel &a = bt.lv[li];
  const T *__restrict__ mp = static_cast<const T *>(a.mp);
  const int p = bt.p, twop = 2 * p;
  const int64_t ex0 = a.win.bx0 & ~int64_t(1), ey0 = a.win.by0 & ~int64_t(1);
  const int64_t ntx = (a.win.bx0 + a.win.nbx - ex0 + TILE - 1) / TILE;
  const int64_t tile = (int64_t)blockIdx.x - bt.tile_begin[li];
  const int64_t tx0 = ex0 + TILE * (tile % ntx);
  const int64_t ty0 = ey0 + TILE * (tile / ntx);

  // stage the source multipoles of boxes [tx0-2, tx0+TILE+2) x [ty0-2, ...)
  // (zero outside the stored window swin, which holds every source of the
  // level's targets): all of a thread's loads are issued before its LDS stores
  constexpr int KP = 4 * KS;
  if ((twop & 3) == 0) {
    // 16-byte loads (2p a multiple of 4: every box record is 16-byte aligned)
    constexpr int K4 = KS;  // float4 chunks per padded record
    constexpr int NE4 = S * S * K4, NIT4 = (NE4 + kThreads - 1) / kThreads;
    const int k4n = twop >> 2;
    using V4 = typename std::conditional<std::is_same<T, float>::value, float4, double4>::type;
    V4 v[NIT4];
#pragma unroll
    for (int it = 0; it < NIT4; ++it) {
      const int e = it * kThreads + threadIdx.x;
      const int k4 = e % K4, bl = e / K4;
      const int bx = bl % S, by = bl / S;
      const int64_t gx = tx0 - 2 + bx - a.swin.bx0, gy = ty0 - 2 + by - a.swin.by0;
      v[it] = V4{0, 0, 0, 0};
      if (e < NE4 && k4 < k4n && gx >= 0 && gy >= 0 && gx < a.swin.nbx && gy < a.swin.nby)
        v[it] = reinterpret_cast<const V4 *>(mp + (gy * a.swin.nbx + gx) * twop)[k4];
    }
#pragma unroll
    for (int it = 0; it < NIT4; ++it) {
      const int e = it * kThreads + threadIdx.x;
      if (e < NE4) {
        T *d = lds + (e / K4) * REC + 4 * (e % K4);
        d[0] = v[it].x;
        d[1] = v[it].y;
        d[2] = v[it].z;
        d[3] = v[it].w;
      }
    }
  } else {
    constexpr int NE = S * S * KP, NIT = (NE + kThreads - 1) / kThreads;
    T v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = it * kThreads + threadIdx.x;
      const int k = e % KP, bl = e / KP;
      const int bx = bl % S, by = bl / S;
      const int64_t gx = tx0 - 2 + bx - a.swin.bx0, gy = ty0 - 2 + by - a.swin.by0;
      v[it] = 0;
      if (e < NE && k < twop && gx >= 0 && gy >= 0 && gx < a.swin.nbx && gy < a.swin.nby)
        v[it] = mp[(gy * a.swin.nbx + gx) * twop + k];
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = it * kThreads + threadIdx.x;
      if (e < NE) lds[(e / KP) * REC + e % KP] = v[it];
    }
  }
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int qx = wave & 1, qy = wave >> 1;
  using M = Mfma<T>;
  typename M::acc acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = typename M::acc{0, 0, 0, 0};

  // A operand: lane holds row i = lane % 16 of the M-tile, column lane / 16
  const int i = lane & 15, kq = lane >> 4;
  int base[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int t = mt * 16 + i;           // target index within the quadrant class
    const int ta = t % H, tb = t / H;
    base[mt] = ((2 * tb + qy + 2) * S + (2 * ta + qx + 2)) * REC + kq;
  }

  // B fragments of the current offset, and of the next one in flight
  constexpr int NB = KS * NT;
  T bcur[NB], bnxt[NB];
  auto load_b = [&](int j, T (&dst)[NB]) {
    const int tx = kIL.t[wave][j][0], ty = kIL.t[wave][j][1];
    const T *src = bfrag + (size_t)((ty + 3) * 7 + (tx + 3)) * NB * 64 + lane;
#pragma unroll
    for (int q = 0; q < NB; ++q) dst[q] = src[q * 64];
  };
  load_b(0, bcur);
  for (int j = 0; j < 27; ++j) {
    load_b(j + 1 < 27 ? j + 1 : j, bnxt);
    const int tx = kIL.t[wave][j][0], ty = kIL.t[wave][j][1];
    const int toff = (ty * S + tx) * REC;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const T av = lds[base[mt] + toff + 4 * ks];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = M::op(av, bcur[ks * NT + nt], acc[mt][nt]);
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) bcur[q] = bnxt[q];
  }

  const double inv_s = 1.0 / a.s;
  double *__restrict__ loc = a.loc;
  auto target_xy = [&](int t, int64_t &gx, int64_t &gy) {
    gx = tx0 + 2 * (t % H) + qx;
    gy = ty0 + 2 * (t / H) + qy;
    return gx >= a.win.bx0 && gy >= a.win.by0 && gx < a.win.bx0 + a.win.nbx &&
           gy < a.win.by0 + a.win.nby;
  };

  if constexpr (!FUSE) {
    // epilogue: loc[target][n] = acc / s
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t gx, gy;
        if (!target_xy(mt * 16 + M::row(lane, r), gx, gy)) continue;
        double *out = loc + ((gy - a.win.by0) * a.win.nbx + (gx - a.win.bx0)) * twop;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int n = nt * 16 + (lane & 15);
          if (n < twop) out[n] = (double)acc[mt][nt][r] * inv_s;
        }
      }
    }
  } else {
    // FP32 M2L part first to LDS (in the FP64 result layout), so that its
    // accumulators are free before the L2L ones are live
    float *xch = reinterpret_cast<float *>(lds_raw) + (size_t)wave * MT * 16 * NT * 16;
    if constexpr (std::is_same<T, float>::value) {
      __syncthreads();  // the source tile is no longer read
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            xch[(mt * 16 + M::row(lane, r)) * (NT * 16) + nt * 16 + (lane & 15)] = acc[mt][nt][r];
      __syncthreads();
    }
    // L2L on FP64 MFMA: A = the targets' parent locals, B = L2L fragments of
    // this wave's quadrant; accumulated apart from the M2L part.
    using M64 = Mfma<double>;
    d4v acc2[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc2[mt][nt] = d4v{0, 0, 0, 0};
    int64_t pidx[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      int64_t gx, gy;
      pidx[mt] = -1;
      if (target_xy(mt * 16 + i, gx, gy))
        pidx[mt] = ((gy >> 1) - a.pwin.by0) * a.pwin.nbx + ((gx >> 1) - a.pwin.bx0);
    }
    const double *lf = l2l_frag + (size_t)wave * KS * NT * 64 + lane;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      double b2[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) b2[nt] = lf[(ks * NT + nt) * 64];
      const int k = 4 * ks + kq;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const double av = (pidx[mt] >= 0 && k < twop) ? a.ploc[pidx[mt] * twop + k] : 0.0;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc2[mt][nt] = M64::op(av, b2[nt], acc2[mt][nt]);
      }
    }
    // bring the M2L part into the FP64 result layout (same for FP64 M2L)
    if constexpr (std::is_same<T, float>::value) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int t = mt * 16 + M64::row(lane, r);
          int64_t gx, gy;
          if (!target_xy(t, gx, gy)) continue;
          double *out = loc + ((gy - a.win.by0) * a.win.nbx + (gx - a.win.bx0)) * twop;
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int n = nt * 16 + (lane & 15);
            if (n < twop) out[n] = fma((double)xch[t * (NT * 16) + n], inv_s, acc2[mt][nt][r]);
          }
        }
    } else {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int64_t gx, gy;
          if (!target_xy(mt * 16 + M::row(lane, r), gx, gy)) continue;
          double *out = loc + ((gy - a.win.by0) * a.win.nbx + (gx - a.win.bx0)) * twop;
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int n = nt * 16 + (lane & 15);
            if (n < twop) out[n] = fma((double)acc[mt][nt][r], inv_s, acc2[mt][nt][r]);
          }
        }
    }
  }
}

// ------------------------------------------------------------ M2L on VALU
// Fallback for orders whose MFMA tile does not fit in LDS: one thread per
// target box, blockIdx.y = quadrant so operator reads are wave-uniform.

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

template <int PMAX, typename T>
__global__ __launch_bounds__(kThreads) void k_m2l_valu(DownArgs a, const T *__restrict__ mp,
                                                       const T *__restrict__ m2l) {
  const Target tg = target_of(a);
  if (!tg.ok) return;
  const int p = a.p;
  const int q = blockIdx.y, qx = q & 1, qy = q >> 1;
  T ar[PMAX], ai[PMAX];
#pragma unroll
  for (int l = 0; l < PMAX; ++l) ar[l] = ai[l] = 0;
  for (int ty = -2 - qy; ty <= 3 - qy; ++ty) {
    for (int tx = -2 - qx; tx <= 3 - qx; ++tx) {
      if (tx >= -1 && tx <= 1 && ty >= -1 && ty <= 1) continue;
      const int64_t sx = tg.tx + tx - a.swin.bx0, sy = tg.ty + ty - a.swin.by0;
      if (sx < 0 || sy < 0 || sx >= a.swin.nbx || sy >= a.swin.nby) continue;
      const T *src = mp + 2 * (sy * a.swin.nbx + sx) * p;
      const T *t = m2l + (size_t)((ty + 3) * 7 + (tx + 3)) * p * p * 2;
#pragma unroll
      for (int k = 0; k < PMAX; ++k) {
        if (k < p) {
          const T sr = src[2 * k], si = src[2 * k + 1];
#pragma unroll
          for (int l = 0; l < PMAX; ++l)
            if (l < p) {
              const T mr = t[((size_t)k * p + l) * 2], mi = t[((size_t)k * p + l) * 2 + 1];
              ar[l] = fma(mr, sr, fma(-mi, si, ar[l]));
              ai[l] = fma(mr, si, fma(mi, sr, ai[l]));
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
      out[2 * l] = (double)ar[l] * inv_s;
      out[2 * l + 1] = (double)ai[l] * inv_s;
    }
}

__global__ __launch_bounds__(kThreads) void k_to_f32(const double *__restrict__ src,
                                                     float *__restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

dim3 valu_grid(const DownArgs &a) {
  const int64_t px0 = a.win.bx0 >> 1, py0 = a.win.by0 >> 1;
  const int64_t pnx = ((a.win.bx0 + a.win.nbx - 1) >> 1) - px0 + 1;
  const int64_t pny = ((a.win.by0 + a.win.nby - 1) >> 1) - py0 + 1;
  return dim3((unsigned)((pnx * pny + kThreads - 1) / kThreads), 4);
}

template <typename T, int TILE, int KS, bool FUSE>
void mfma_batch(const M2LBatch &b, const T *bfrag, const double *l2l_frag, hipStream_t stream) {
  constexpr int S = TILE + 4;
  constexpr int MT = (TILE / 2) * (TILE / 2) / 16, NT = (KS + 3) / 4;
  size_t lds = (size_t)S * S * (4 * KS + 1) * sizeof(T);
  const size_t xch = (size_t)4 * MT * 16 * NT * 16 * sizeof(float);
  if (FUSE && std::is_same<T, float>::value && xch > lds) lds = xch;
  hipLaunchKernelGGL((k_m2l_mfma<T, TILE, KS, FUSE>), dim3((unsigned)b.tile_begin[b.count]),
                     dim3(kThreads), lds, stream, b, bfrag, l2l_frag);
}

template <typename T, int KS, bool FUSE>
void mfma_dispatch_tile(M2LBatch &b, const T *bfrag, const double *l2l_frag, hipStream_t stream) {
  const size_t rec = 4 * KS + 1;
  const int tile = ((size_t)20 * 20 * rec * sizeof(T) <= kLdsBudget) ? 16 : 8;
  // tile lists of every level
  int64_t acc = 0;
  for (int i = 0; i < b.count; ++i) {
    const Window &w = b.lv[i].win;
    const int64_t ex0 = w.bx0 & ~int64_t(1), ey0 = w.by0 & ~int64_t(1);
    const int64_t ntx = (w.bx0 + w.nbx - ex0 + tile - 1) / tile;
    const int64_t nty = (w.by0 + w.nby - ey0 + tile - 1) / tile;
    b.tile_begin[i] = acc;
    acc += ntx * nty;
  }
  b.tile_begin[b.count] = acc;
  if (acc == 0) return;
  if (tile == 16)
    mfma_batch<T, 16, KS, FUSE>(b, bfrag, l2l_frag, stream);
  else
    mfma_batch<T, 8, KS, FUSE>(b, bfrag, l2l_frag, stream);
}

// The device's LDS per workgroup (160 KB on gfx950), read once per device.
size_t lds_per_block() {
  static std::mutex mu;
  static std::vector<size_t> known;
  int dev = 0;
  LENS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if ((size_t)dev >= known.size()) known.resize(dev + 1, 0);
  if (!known[dev]) {
    int v = 0;
    LENS_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    known[dev] = v > 0 ? (size_t)v : kLdsBudget;
  }
  return known[dev];
}

template <typename T, bool FUSE>
bool mfma_dispatch(M2LBatch &b, const T *bfrag, const double *l2l_frag, int ks,
                   hipStream_t stream) {
  // the tile must fit the workgroup's LDS at TILE = 8 (the larger tile is
  // taken only within kLdsBudget, which keeps two or more workgroups per CU)
  if ((size_t)12 * 12 * (4 * ks + 1) * sizeof(T) > lds_per_block()) return false;
  switch (ks) {
    case 2: mfma_dispatch_tile<T, 2, FUSE>(b, bfrag, l2l_frag, stream); return true;
    case 4: mfma_dispatch_tile<T, 4, FUSE>(b, bfrag, l2l_frag, stream); return true;
    case 6: mfma_dispatch_tile<T, 6, FUSE>(b, bfrag, l2l_frag, stream); return true;
    case 8: mfma_dispatch_tile<T, 8, FUSE>(b, bfrag, l2l_frag, stream); return true;
    case 10: mfma_dispatch_tile<T, 10, FUSE>(b, bfrag, l2l_frag, stream); return true;
    case 12: mfma_dispatch_tile<T, 12, FUSE>(b, bfrag, l2l_frag, stream); return true;
    case 16: mfma_dispatch_tile<T, 16, FUSE>(b, bfrag, l2l_frag, stream); return true;
    case 20: mfma_dispatch_tile<T, 20, FUSE>(b, bfrag, l2l_frag, stream); return true;
    default: return false;
  }
}

}  // namespace

void launch_l2l(const DownArgs &a, const OpTables &t, hipStream_t stream) {
  const int64_t n = a.win.count() * a.p;
  if (n == 0) return;
  hipLaunchKernelGGL(k_l2l, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     stream, a, t.l2l);
  LENS_HIP(hipGetLastError());
}

void launch_l2l_chain(const L2LChain &c, const OpTables &t, hipStream_t stream) {
  if (c.nlev < 1 || c.nlev > kMaxL2LChain) fail(LENS_EINVAL, "L2L chain: bad level count");
  const int64_t n = c.win[0].count();
  if (n == 0) return;
  LENS_PMAX_DISPATCH(c.p, hipLaunchKernelGGL((k_l2l_tile<PM>), dim3((unsigned)n), dim3(64), 0,
                                             stream, c));
  (void)t;
  LENS_HIP(hipGetLastError());
}

void launch_m2l_batch(M2LBatch &b, const OpTables &t, bool fp32, hipStream_t stream) {
  if (b.count == 0) return;
  bool done;
  if (fp32)
    done = mfma_dispatch<float, false>(b, t.bfrag32, nullptr, t.ks, stream);
  else
    done = mfma_dispatch<double, false>(b, t.bfrag64, nullptr, t.ks, stream);
  if (!done) {
    for (int i = 0; i < b.count; ++i) {
      DownArgs a{};
      a.level = b.lv[i].level;
      a.p = b.p;
      a.s = b.lv[i].s;
      a.win = b.lv[i].win;
      a.swin = b.lv[i].swin;
      a.loc = b.lv[i].loc;
      if (a.win.count() == 0) continue;
      if (fp32) {
        a.mp32 = static_cast<const float *>(b.lv[i].mp);
        LENS_PMAX_DISPATCH(a.p, hipLaunchKernelGGL((k_m2l_valu<PM, float>), valu_grid(a),
                                                   dim3(kThreads), 0, stream, a, a.mp32, t.m2l32));
      } else {
        a.mp = static_cast<const double *>(b.lv[i].mp);
        LENS_PMAX_DISPATCH(a.p, hipLaunchKernelGGL((k_m2l_valu<PM, double>), valu_grid(a),
                                                   dim3(kThreads), 0, stream, a, a.mp, t.m2l));
      }
    }
  }
  LENS_HIP(hipGetLastError());
}

bool launch_m2l_l2l(M2LBatch &b, const OpTables &t, bool fp32, hipStream_t stream) {
  if (b.count != 1 || !b.lv[0].ploc) return false;
  if (b.lv[0].win.count() == 0) return true;
  bool done;
  if (fp32)
    done = mfma_dispatch<float, true>(b, t.bfrag32, t.l2l_frag, t.ks, stream);
  else
    done = mfma_dispatch<double, true>(b, t.bfrag64, t.l2l_frag, t.ks, stream);
  if (done) LENS_HIP(hipGetLastError());
  return done;
}

void launch_to_f32(const double *src, float *dst, size_t n, hipStream_t stream) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     stream, src, dst, n);
  LENS_HIP(hipGetLastError());
}

}  // namespace lensfmm
