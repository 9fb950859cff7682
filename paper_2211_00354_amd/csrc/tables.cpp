// Translation operators of the complex-variable FMM (Appendix A: M2M, M2L,
// L2L), built on the host in FP64 and uploaded once per expansion order.
//
// Expansions use box-size-rescaled coefficients.  For a box with centre c
// and side s:
//   multipole  f(z) = sum_k a_k / (z - c)^(k+1),  a~_k = a_k / s^k
//              = sum_{i in box} m_i w_i^k,        w_i = (z_i - c) / s
//   local      f(z) = sum_l b_l (z - c)^l,        b~_l = b_l s^l
//              = sum_l b~_l w^l,                  w = (z - c) / s
// With this scaling every operator below depends only on the geometry in
// units of the box side, so one table serves every level.
//
// * M2M (child -> parent, delta = (c_child - c_parent)/s_child in {+-1/2 +- i/2}):
//     a~'_l = 2^-l sum_{k<=l} C(l,k) a~_k delta^(l-k)            (exact)
// * L2L (parent -> child, same delta):
//     b~'_j = sum_{l>=j} C(l,j) 2^-l delta^(l-j) b~_l            (exact)
// * M2L (source box -> target box at the same level,
//        tau = (c_src - c_tgt)/s, an integer offset with max(|Re|,|Im|) in {2,3}):
//     b~_l += (1/s) sum_k (-1)^(k+1) C(k+l,l) tau^-(k+l+1) a~_k
//   from expanding 1/(z - c_src)^(k+1) about c_tgt.
#include <cmath>
#include <complex>
#include <map>
#include <mutex>

#include "lens_internal.h"

namespace lensfmm {

namespace {

using cd = std::complex<double>;

std::vector<std::vector<double>> binomials(int n) {
  std::vector<std::vector<double>> C(n + 1, std::vector<double>(n + 1, 0.0));
  for (int i = 0; i <= n; ++i) {
    C[i][0] = 1.0;
    for (int j = 1; j <= i; ++j) C[i][j] = C[i - 1][j - 1] + (j < i ? C[i - 1][j] : 0.0);
  }
  return C;
}

cd quadrant_delta(int q) {
  const int a = q & 1, c = q >> 1;
  return cd(a - 0.5, c - 0.5);
}

cd cpow_int(cd z, int n) {
  cd r(1.0, 0.0), b = z;
  bool neg = n < 0;
  unsigned e = (unsigned)(neg ? -n : n);
  while (e) {
    if (e & 1) r *= b;
    b *= b;
    e >>= 1;
  }
  return neg ? 1.0 / r : r;
}

}  // namespace

// out[((q*p + k)*p + l)*2 + {0,1}] = M[q][l][k]  (input index k major)
void build_m2m_table(int p, std::vector<double> &out) {
  auto C = binomials(2 * p);
  out.assign((size_t)4 * p * p * 2, 0.0);
  for (int q = 0; q < 4; ++q) {
    const cd d = quadrant_delta(q);
    for (int k = 0; k < p; ++k)
      for (int l = k; l < p; ++l) {
        const cd v = std::ldexp(1.0, -l) * C[l][k] * cpow_int(d, l - k);
        const size_t o = (((size_t)q * p + k) * p + l) * 2;
        out[o] = v.real();
        out[o + 1] = v.imag();
      }
  }
}

// out[((q*p + l)*p + j)*2 + {0,1}] = L[q][j][l]  (input index l major)
void build_l2l_table(int p, std::vector<double> &out) {
  auto C = binomials(2 * p);
  out.assign((size_t)4 * p * p * 2, 0.0);
  for (int q = 0; q < 4; ++q) {
    const cd d = quadrant_delta(q);
    for (int l = 0; l < p; ++l)
      for (int j = 0; j <= l; ++j) {
        const cd v = std::ldexp(1.0, -l) * C[l][j] * cpow_int(d, l - j);
        const size_t o = (((size_t)q * p + l) * p + j) * 2;
        out[o] = v.real();
        out[o + 1] = v.imag();
      }
  }
}

// out[((t*p + k)*p + l)*2 + {0,1}] = T_tau[l][k], t = (ty+3)*7 + (tx+3);
// entries with max(|tx|,|ty|) <= 1 (near neighbours) stay zero.
void build_m2l_table(int p, std::vector<double> &out) {
  auto C = binomials(2 * p);
  out.assign((size_t)49 * p * p * 2, 0.0);
  for (int ty = -3; ty <= 3; ++ty)
    for (int tx = -3; tx <= 3; ++tx) {
      if (std::abs(tx) <= 1 && std::abs(ty) <= 1) continue;
      const int t = (ty + 3) * 7 + (tx + 3);
      const cd tau((double)tx, (double)ty);
      for (int k = 0; k < p; ++k)
        for (int l = 0; l < p; ++l) {
          const double sgn = ((k + 1) & 1) ? -1.0 : 1.0;
          const cd v = sgn * C[k + l][l] * cpow_int(tau, -(k + l + 1));
          const size_t o = (((size_t)t * p + k) * p + l) * 2;
          out[o] = v.real();
          out[o + 1] = v.imag();
        }
    }
}

// M2L operators as MFMA B fragments.  The complex product b~_l += T[l][c] a~_c
// is written as a real GEMM over interleaved (re, im) coefficients,
// b[2l+o] += sum_{2c+i} B[2c+i][2l+o] a[2c+i], with
//   B[2c][2l] = Re T,  B[2c+1][2l] = -Im T,  B[2c][2l+1] = Im T,  B[2c+1][2l+1] = Re T,
// zero-padded to ks_count*4 rows and nt_count*16 columns.  For each offset t,
// K-step ks and N-tile nt, the 64 values are stored in lane order of the
// 16x16x4 MFMA B operand (lane l holds B[4 ks + l/16][16 nt + l%16]).
// K-steps compiled for order p: the smallest of {2,4,6,8,10,12,16,20} >= p/2.
int m2l_ksteps(int p) {
  const int need = (p + 1) / 2;
  for (int k : {2, 4, 6, 8, 10, 12, 16, 20})
    if (k >= need) return k;
  return 20;
}

void build_m2l_bfrag(int p, std::vector<double> &out, int &ks_count, int &nt_count) {
  std::vector<double> T;
  build_m2l_table(p, T);
  ks_count = m2l_ksteps(p);
  nt_count = (ks_count + 3) / 4;
  out.assign((size_t)49 * ks_count * nt_count * 64, 0.0);
  for (int t = 0; t < 49; ++t)
    for (int ks = 0; ks < ks_count; ++ks)
      for (int nt = 0; nt < nt_count; ++nt)
        for (int lane = 0; lane < 64; ++lane) {
          const int k = 4 * ks + lane / 16, n = 16 * nt + lane % 16;
          const int c = k / 2, pin = k % 2, l = n / 2, pout = n % 2;
          if (c >= p || l >= p) continue;
          const size_t o = (((size_t)t * p + c) * p + l) * 2;
          const double tr = T[o], ti = T[o + 1];
          const double v = pin == 0 ? (pout == 0 ? tr : ti) : (pout == 0 ? -ti : tr);
          out[(((size_t)t * ks_count + ks) * nt_count + nt) * 64 + lane] = v;
        }
}

// L2L operators as MFMA B fragments, one per child quadrant q, same layout
// and padding as the M2L fragments: b'[2j+o] += sum_{2l+i} B[2l+i][2j+o] b[2l+i]
// with the complex L[q][j][l] (zero for l < j) in real form.
void build_l2l_bfrag(int p, int ks_count, int nt_count, std::vector<double> &out) {
  std::vector<double> Lt;
  build_l2l_table(p, Lt);
  out.assign((size_t)4 * ks_count * nt_count * 64, 0.0);
  for (int q = 0; q < 4; ++q)
    for (int ks = 0; ks < ks_count; ++ks)
      for (int nt = 0; nt < nt_count; ++nt)
        for (int lane = 0; lane < 64; ++lane) {
          const int k = 4 * ks + lane / 16, n = 16 * nt + lane % 16;
          const int l = k / 2, pin = k % 2, j = n / 2, pout = n % 2;
          if (l >= p || j >= p || l < j) continue;
          const size_t o = (((size_t)q * p + l) * p + j) * 2;
          const double tr = Lt[o], ti = Lt[o + 1];
          const double v = pin == 0 ? (pout == 0 ? tr : ti) : (pout == 0 ? -ti : tr);
          out[(((size_t)q * ks_count + ks) * nt_count + nt) * 64 + lane] = v;
        }
}

namespace {
std::mutex g_tab_mu;
std::map<std::pair<int, int>, OpTables> g_tabs;

template <typename T>
T *upload(const std::vector<T> &h) {
  void *d = nullptr;
  LENS_HIP(hipMalloc(&d, h.size() * sizeof(T)));
  LENS_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return static_cast<T *>(d);
}
}  // namespace

const OpTables *op_tables_if_built(int p) {
  int dev = 0;
  LENS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto it = g_tabs.find(std::make_pair(dev, p));
  return it == g_tabs.end() ? nullptr : &it->second;
}

const OpTables &op_tables(int p, hipStream_t stream) {
  (void)stream;
  int dev = 0;
  LENS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto key = std::make_pair(dev, p);
  auto it = g_tabs.find(key);
  if (it != g_tabs.end()) return it->second;
  OpTables t;
  t.p = p;
  std::vector<double> h;
  build_m2m_table(p, h);
  t.m2m = upload(h);
  build_l2l_table(p, h);
  t.l2l = upload(h);
  build_m2l_table(p, h);
  t.m2l = upload(h);
  std::vector<float> hf(h.begin(), h.end());
  t.m2l32 = upload(hf);
  std::vector<double> bf;
  build_m2l_bfrag(p, bf, t.ks, t.nt);
  t.bfrag64 = upload(bf);
  std::vector<float> bf32(bf.begin(), bf.end());
  t.bfrag32 = upload(bf32);
  build_l2l_bfrag(p, t.ks, t.nt, bf);
  t.l2l_frag = upload(bf);
  return g_tabs.emplace(key, t).first->second;  // device tables live until exit
}

}  // namespace lensfmm
