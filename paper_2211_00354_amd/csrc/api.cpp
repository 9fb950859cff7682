// C ABI of liblensfmm: argument checks, plans (star quadtree + multipoles),
// target windows, ray chunking and the launch sequence of every entry point.
//
// Call sequence of lens_deflect with LENS_FMM (Appendix A):
//   plan (stars):  bbox -> leaf keys -> radix sort -> gather -> leaf starts
//                  -> P2M at level L -> M2M for L-1 .. 2
//   per call:      target windows per level from the rays' bounding box
//                  -> for l = 2..L: L2L + M2L into the window (FP64, or FP32
//                     M2L on the finest levels in LENS_MIXED)
//                  -> fused L2P + P2P + smooth term per leaf box of the window
// All device work goes to the caller's stream; plan creation and explicit-ray
// calls read one bounding box back from the device.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <limits>
#include <memory>
#include <mutex>

#include <sys/stat.h>

#include "lens_internal.h"

using namespace lensfmm;

struct lens_plan {
  int device = 0;
  int p = 12;
  int precision = LENS_MIXED;
  int fine_levels = 0;  // LENS_MIXED: levels L-fine_levels+1 .. L run M2L in FP32
  int qdim = 1;         // charge components per source: 1 (masses) or 2 (complex)
  Geometry g{};
  int64_t n_stars = 0;
  double kappa_s = 0, gamma = 0;
  double domain[4] = {0, 0, 0, 0};
  double target[4] = {0, 0, 0, 0};  // every ray evaluated with the plan lies in this box
  double star_bb[4] = {0, 0, 0, 0};  // the sources' bounding box (n_stars > 0)
  const uint32_t *perm = nullptr;    // sorted position -> caller's source index
  // Levels 2..dense_top hold the multipoles of every box; a finer level only
  // those of its source window swin[l] (the boxes that can be M2L sources
  // for targets in the box above), each formed straight from the stars.
  int dense_top = 0;
  double rho_local = -1.0;   // sources per unit area where the rays are (< 0: unknown)
  std::vector<Window> swin;  // index = level
  std::vector<char> direct;  // index = level: multipoles formed from the stars (else M2M)
  DevBuf sxy, sm, leaf_start;
  DevBuf sm32;               // FP32 copies of real masses (mixed-precision near field)
  std::vector<DevBuf> mp;    // index = level, FP64 multipoles
  std::vector<DevBuf> mp32;  // index = level, FP32 copies (fine levels, mixed)
  DevBuf keys, vals, keys_tmp, vals_tmp, cnt, scan_tmp, box_coarse;  // tree-build scratch
  hipStream_t last_stream = nullptr;

  const double *mp_at(int l) const { return static_cast<const double *>(mp[l].ptr); }
  const float *mp32_at(int l) const {
    return mp32.size() > (size_t)l ? static_cast<const float *>(mp32[l].ptr) : nullptr;
  }
  // return every buffer to the pool, ordered after the work on `st`
  void put_all(hipStream_t st) {
    std::vector<DevBuf *> ps = {&sxy, &sm, &sm32, &leaf_start, &keys, &vals, &keys_tmp, &vals_tmp,
                                &cnt, &scan_tmp, &box_coarse};
    for (auto &b : mp) ps.push_back(&b);
    for (auto &b : mp32) ps.push_back(&b);
    pool_put_batch(ps.data(), ps.size(), st);
  }
  void release() {
    if (last_stream) (void)hipStreamSynchronize(last_stream);
    put_all(nullptr);
  }
};

namespace {

// lens_map rays per pass by default: all of them (the paper's bounded passes,
// Section 2.4, are kept as an option; a map needs no per-ray memory)
constexpr int64_t kDefaultChunk = std::numeric_limits<int64_t>::max();
// Inverse polygon mapping: default rays per pass (16 bytes of deflected
// corners each), and the most cells one pass may hold.
constexpr int64_t kIpmPassRays = int64_t(1) << 28;
constexpr int64_t kIpmPassCellsMax = (int64_t)std::numeric_limits<uint32_t>::max() - 1;
constexpr int kDefaultFp32Levels = 2;

bool is_finite(double v) { return std::isfinite(v); }

void check_opts(const lens_opts &o) {
  if (o.method != LENS_FMM && o.method != LENS_DIRECT) fail(LENS_EINVAL, "opts.method must be LENS_FMM or LENS_DIRECT");
  if (o.precision != LENS_FP64 && o.precision != LENS_MIXED)
    fail(LENS_EINVAL, "opts.precision must be LENS_FP64 or LENS_MIXED");
  if (o.order_p < 0 || o.order_p > LENS_MAX_ORDER)
    fail(LENS_EINVAL, "opts.order_p must be in [1, " + std::to_string(LENS_MAX_ORDER) + "] or 0");
  if (o.leaf_level != 0 && (o.leaf_level < 2 || o.leaf_level > LENS_MAX_LEVEL))
    fail(LENS_EINVAL, "opts.leaf_level must be in [2, " + std::to_string(LENS_MAX_LEVEL) + "] or 0");
  if (o.max_rays_per_chunk < 0) fail(LENS_EINVAL, "opts.max_rays_per_chunk must be >= 0");
  if (o.fp32_levels < -1 || o.fp32_levels > LENS_MAX_LEVEL)
    fail(LENS_EINVAL, "opts.fp32_levels must be in [-1, " + std::to_string(LENS_MAX_LEVEL) + "]");
  if (o.workspace && (reinterpret_cast<uintptr_t>(o.workspace) % 256 != 0 || o.workspace_bytes == 0))
    fail(LENS_EINVAL, "opts.workspace must be 256-byte aligned with workspace_bytes > 0");
}

lens_opts resolve_opts(const lens_opts *o) {
  lens_opts r;
  lens_opts_default(&r);
  if (o) r = *o;
  check_opts(r);
  if (r.order_p == 0) r.order_p = 12;
  if (r.max_rays_per_chunk == 0) r.max_rays_per_chunk = kDefaultChunk;
  r.fp32_levels = r.fp32_levels == 0 ? kDefaultFp32Levels : (r.fp32_levels < 0 ? 0 : r.fp32_levels);
  return r;
}

void check_field(const lens_field *f) {
  if (!f) fail(LENS_EINVAL, "field is NULL");
  if (f->n_stars < 0) fail(LENS_EINVAL, "field.n_stars < 0");
  if (f->n_stars > (int64_t)std::numeric_limits<int32_t>::max())
    fail(LENS_EINVAL, "field.n_stars exceeds 2^31-1");
  if (f->n_stars > 0 && (!f->xy || !f->m)) fail(LENS_EINVAL, "field.xy / field.m is NULL");
  if (!is_finite(f->kappa_s) || !is_finite(f->gamma)) fail(LENS_EINVAL, "kappa_s and gamma must be finite");
}

void check_grid(const lens_grid *g) {
  if (g->nx < 0 || g->ny < 0) fail(LENS_EINVAL, "grid.nx / grid.ny < 0");
  if (!is_finite(g->x0) || !is_finite(g->y0) || !is_finite(g->dx) || !is_finite(g->dy))
    fail(LENS_EINVAL, "grid origin and spacing must be finite");
  if (!(g->dx > 0) || !(g->dy > 0)) fail(LENS_EINVAL, "grid.dx and grid.dy must be > 0");
  if (g->nx > (int64_t)std::numeric_limits<int32_t>::max() ||
      g->ny > (int64_t)std::numeric_limits<int32_t>::max())
    fail(LENS_EINVAL, "grid side exceeds 2^31-1 rays");
}

double grid_x(const lens_grid &g, int64_t i) { return g.x0 + ((double)i + 0.5) * g.dx; }
double grid_y(const lens_grid &g, int64_t j) { return g.y0 + ((double)j + 0.5) * g.dy; }

int64_t box_coord_host(double x, double origin, double s, int64_t nbox) {
  double t = (x - origin) / s;
  t = std::fmin(std::fmax(t, 0.0), (double)(nbox - 1));
  return (int64_t)std::floor(t);
}

// Pinned, coherent host landing buffer for the bounding-box read-back (one
// per host thread, kept for the process): the final reduction kernel writes
// it directly, so the one wait of a plan-less call needs no copy.
struct Landing {
  double *host = nullptr;
  double *dev = nullptr;  // the same memory as the device addresses it
};

const Landing &bbox_landing() {
  thread_local Landing l;
  if (!l.host) {
    LENS_HIP(hipHostMalloc(reinterpret_cast<void **>(&l.host), 8 * sizeof(double),
                           hipHostMallocCoherent));
    LENS_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&l.dev), l.host, 0));
  }
  return l;
}

// Bounding box of the points (one read-back); with count_box, also the
// number of points inside that rectangle (same read-back).  In two halves:
// bbox_enqueue puts the reductions, the last of which writes the calling
// thread's landing buffer, on the stream and records an event; bbox_finish
// waits for that event only (not for work enqueued after it).
struct BBoxRead {
  hipEvent_t ev = nullptr;
  bool with_count = false;
};

hipEvent_t bbox_event() {
  thread_local std::vector<hipEvent_t> evs;
  int dev = 0;
  LENS_HIP(hipGetDevice(&dev));
  if ((size_t)dev >= evs.size()) evs.resize(dev + 1, nullptr);
  if (!evs[dev]) LENS_HIP(hipEventCreateWithFlags(&evs[dev], hipEventDisableTiming));
  return evs[dev];
}

BBoxRead bbox_enqueue(const double *xy, int64_t n, hipStream_t st, const double *count_box = nullptr) {
  Scratch sc(st);
  const int parts = bbox_parts(n);
  double *partial = sc.get<double>((size_t)parts * 5);
  launch_bbox(xy, n, partial, parts, count_box, bbox_landing().dev, st);
  BBoxRead r;
  r.ev = bbox_event();
  r.with_count = count_box != nullptr;
  LENS_HIP(hipEventRecord(r.ev, st));
  return r;
}

void bbox_finish(const BBoxRead &r, double out[4], int64_t *count = nullptr) {
  LENS_HIP(hipEventSynchronize(r.ev));
  const double *landing = bbox_landing().host;
  std::copy(landing, landing + 4, out);
  if (r.with_count && count) {
    uint64_t c;
    std::memcpy(&c, landing + 4, 8);
    *count = (int64_t)c;
  }
  for (int c = 0; c < 4; ++c)
    if (!is_finite(out[c])) fail(LENS_EINVAL, "non-finite coordinates in the input positions");
}

void device_bbox(const double *xy, int64_t n, hipStream_t st, double out[4],
                 const double *count_box = nullptr, int64_t *count = nullptr) {
  bbox_finish(bbox_enqueue(xy, n, st, count_box), out, count);
}

// Cost model of the evaluation per ray, in VALU lane-instructions: 9 q near
// pairs at ~12 each (q = stars per leaf) plus the leaf-level M2L, 27 p^2
// complex MACs per target box at ~6 each (MFMA), shared by the box's rays.
constexpr double kCostPair = 12.0, kCostM2L = 6.0;

double eval_cost(double rho, double s, double rays_per_box, int p) {
  return kCostPair * 9.0 * rho * s * s + kCostM2L * 27.0 * p * p / std::max(rays_per_box, 1.0);
}

// Leaf side minimising eval_cost for a ray density rho_ray (no alignment):
// s^4 = 27 p^2 c_m2l / (9 rho rho_ray c_pair).  Without rays, ~8 stars per leaf.
double preferred_leaf_side(double rho, double rays_density, double side, int p) {
  double s;
  if (rho <= 0) {
    s = side / 4;
  } else if (rays_density > 0) {
    s = std::sqrt(std::sqrt(27.0 * p * p * kCostM2L / (9.0 * rho * rays_density * kCostPair)));
    s = std::max(s, std::sqrt(0.5 / rho));   // at least ~0.5 stars per leaf
    s = std::min(s, std::sqrt(64.0 / rho));  // at most ~64
  } else {
    s = std::sqrt(8.0 / rho);
  }
  return s;
}

// Device bytes of a plan with leaf level L: the leaf starts (4^L + 1),
// dense multipole levels down to where boxes hold ~512 sources, and below
// them windows around the rays' box rb (w x h) grown by 4 boxes a side,
// FP64 plus FP32 copies; the evaluation's locals take about as much again
// as the windows.
double plan_bytes(int L, int p, int64_t n_sources, double side, double w, double h) {
  double bytes = 4.0 * (double)(int64_t(1) << (2 * L));
  int D = 2;
  while (D < L && (double)n_sources / (double)(int64_t(1) << (2 * D)) > 512.0) ++D;
  for (int l = 2; l <= L; ++l) {
    const double nb = (double)(int64_t(1) << l), s = side / nb;
    const double win = std::min(nb, w / s + 9.0) * std::min(nb, h / s + 9.0);
    const double boxes = l <= D ? nb * nb : win;
    bytes += (boxes * 2.0 + win) * p * 16.0 * 1.5;
  }
  return bytes;
}
constexpr double kPlanBytesMax = 16e9;

int level_for_side(double side, double s, int p, int64_t n_sources, double w, double h) {
  int L = (int)std::ceil(std::log2(side / s) - 1e-9);
  L = std::max(2, std::min(L, LENS_MAX_LEVEL));
  while (L > 2 && plan_bytes(L, p, n_sources, side, w, h) > kPlanBytesMax) --L;
  return L;
}

// Stars per unit area inside the rays' box, from a count of them (or -1 when
// the count is too small to say: the mean density is used then).
double local_density(int64_t count, const double rb[4]) {
  const double area = (rb[2] - rb[0]) * (rb[3] - rb[1]);
  if (!(area > 0) || count < 32) return -1.0;
  return (double)count / area;
}

double star_density(int64_t n_stars, const double sb[4]) {
  const double area = std::max((sb[2] - sb[0]) * (sb[3] - sb[1]), 1e-300);
  return n_stars > 0 ? (double)n_stars / area : 0.0;
}

// Root placement with leaf boxes aligned to a ray grid: a leaf box spans kx
// grid columns and ky rows (kx dx == ky dy exactly) and kx*ky is a multiple of
// 64, so every interior box holds whole waves of rays.  With leaf_level given,
// the smallest such box that lets 2^L boxes cover the domain; otherwise the
// candidate with the lowest eval_cost.  Returns false if no candidate fits.
bool aligned_geometry(const lens_grid &g, const double dom[4], int leaf_level, double rho, int p,
                      int64_t n_sources, Geometry *out) {
  struct Cand {
    double s;
    int kx, ky;
  };
  std::vector<Cand> cands;
  for (int kx = 1; kx <= 64; ++kx) {
    const long ky = std::lround((double)kx * g.dx / g.dy);
    if (ky < 1 || ky > 64 || (double)ky * g.dy != (double)kx * g.dx) continue;
    if ((kx * ky) % 64 != 0 || kx * ky > 1024) continue;
    cands.push_back({(double)kx * g.dx, kx, (int)ky});
  }
  std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.s < b.s; });
  const double w = dom[2] - dom[0], h = dom[3] - dom[1];
  bool found = false;
  double best_cost = 0;
  for (const Cand &c : cands) {
    // boxes to the left of / below the grid origin needed to reach the domain,
    // rounded up to a multiple of 4 so that the rays' boxes start at an index
    // divisible by 4 (the M2L tiles of the two finest levels start at even
    // box indices; an odd start would cost one more row and column of tiles)
    const double mx = 4.0 * std::ceil(std::max(0.0, std::ceil((g.x0 - dom[0]) / c.s)) / 4.0);
    const double my = 4.0 * std::ceil(std::max(0.0, std::ceil((g.y0 - dom[1]) / c.s)) / 4.0);
    const double x0 = g.x0 - mx * c.s, y0 = g.y0 - my * c.s;
    const double need = std::max(dom[2] - x0, dom[3] - y0) * (1.0 + 1e-12);
    int L = 2;
    while (L < LENS_MAX_LEVEL && std::ldexp(c.s, L) <= need) ++L;
    if (std::ldexp(c.s, L) <= need) continue;
    if (leaf_level > 0) {
      if (L > leaf_level) continue;  // box too small for this depth
      L = leaf_level;
      *out = Geometry{x0, y0, std::ldexp(c.s, L), L};
      return true;  // smallest fitting box
    }
    const double gw = (double)g.nx * g.dx, gh = (double)g.ny * g.dy;
    if (plan_bytes(L, p, n_sources, std::ldexp(c.s, L), gw, gh) > kPlanBytesMax) continue;
    const double cost = eval_cost(rho, c.s, (double)c.kx * c.ky, p);
    if (!found || cost < best_cost) {
      found = true;
      best_cost = cost;
      *out = Geometry{x0, y0, std::ldexp(c.s, L), L};
    }
  }
  (void)w;
  (void)h;
  return found;
}

// Boxes of `level` that hold points of bb: the host and the kernels place a
// point with the same correctly rounded division, which is monotone in the
// coordinate, so the boxes of bb's corners bound those of every point in it
// (and a box in a level's window has its parent in the window above).
Window window_for(const lens_plan &P, int level, const double bb[4]) {
  const int64_t n = int64_t(1) << level;
  const double s = std::ldexp(P.g.side, -level);
  int64_t x0 = box_coord_host(bb[0], P.g.x0, s, n), x1 = box_coord_host(bb[2], P.g.x0, s, n);
  int64_t y0 = box_coord_host(bb[1], P.g.y0, s, n), y1 = box_coord_host(bb[3], P.g.y0, s, n);
  x0 = std::max<int64_t>(x0, 0);
  y0 = std::max<int64_t>(y0, 0);
  x1 = std::min<int64_t>(x1, n - 1);
  y1 = std::min<int64_t>(y1, n - 1);
  return Window{x0, y0, x1 - x0 + 1, y1 - y0 + 1};
}

// Multipole storage per level.  M2L sources of a target box lie within 3
// boxes of it, so level l needs the multipoles of the target window (the
// rays' boxes) grown by 3 boxes (4 are kept, see below).  Where that covers under a quarter of the
// level, and at every finer level, only that window is stored and formed
// from the stars ("windowed" levels); the coarser ("dense") levels reach down
// at least to where boxes hold ~512 sources, so that forming the finest of
// them from the stars stays short, and are formed by M2M above that.  A
// dense level formed from the stars whose parent level is too also stores
// only its window.  When the rays cover the sources (the common case) every
// level is dense.
void source_windows(lens_plan *P) {
  const int L = P->g.L;
  P->swin.assign(L + 1, Window{0, 0, 0, 0});
  int lw = L + 1;
  for (int l = L; l >= 2; --l) {
    const int64_t n = int64_t(1) << l;
    Window w = window_for(*P, l, P->target);
    // 3 boxes of M2L sources, plus one for rays that check_inside admits
    // just outside the target (within its tolerance)
    const int64_t x0 = std::max<int64_t>(w.bx0 - 4, 0), y0 = std::max<int64_t>(w.by0 - 4, 0);
    const int64_t x1 = std::min<int64_t>(w.bx0 + w.nbx + 4, n), y1 = std::min<int64_t>(w.by0 + w.nby + 4, n);
    P->swin[l] = Window{x0, y0, x1 - x0, y1 - y0};
    if (P->swin[l].count() * 4 <= n * n && lw == l + 1) lw = l;
  }
  int dmin = 2;
  while (dmin < L && (double)P->n_stars / (double)(int64_t(1) << (2 * dmin)) > 512.0) ++dmin;
  int D = std::max(lw - 1, dmin);
  if (D >= L) D = L;
  P->dense_top = std::max(D, 2);
  // formed from the stars: the windowed levels, the finest dense level, and
  // dense levels whose boxes hold ~8 sources or fewer on average (a thread
  // per box then beats M2M from the children); the others by M2M
  P->direct.assign(L + 1, 0);
  for (int l = 2; l <= L; ++l)
    P->direct[l] = l >= P->dense_top ||
                   (double)P->n_stars <= 8.0 * (double)(int64_t(1) << (2 * l));
  // a dense level keeps every box only if the level above is formed from it
  for (int l = 2; l <= P->dense_top; ++l) {
    const int64_t n = int64_t(1) << l;
    const bool m2m_child = l > 2 && !P->direct[l - 1];
    if (m2m_child || !P->direct[l]) P->swin[l] = Window{0, 0, n, n};
  }
}

// Plan phase 1 (host): domain = star bounding box sb (if any) united with
// ray_box, root square and leaf level (aligned with `align` if possible).
// rho_local >= 0: the stars' density where the rays are (else the mean
// density over the stars' bounding box is used for the leaf choice).
void plan_geometry(lens_plan *P, int64_t n_sources, const double *sb, const double *ray_box,
                   const lens_grid *align, double rays_density, const lens_opts &o,
                   double rho_local = -1.0) {
  P->p = o.order_p;
  P->precision = o.precision;
  P->fine_levels = o.fp32_levels;
  P->n_stars = n_sources;
  bool have = sb != nullptr;
  double dom[4];
  if (have) std::copy(sb, sb + 4, dom);
  if (ray_box) {
    if (!have) std::copy(ray_box, ray_box + 4, dom);
    dom[0] = std::min(dom[0], ray_box[0]);
    dom[1] = std::min(dom[1], ray_box[1]);
    dom[2] = std::max(dom[2], ray_box[2]);
    dom[3] = std::max(dom[3], ray_box[3]);
    have = true;
  }
  if (!have) dom[0] = dom[1] = 0, dom[2] = dom[3] = 1;
  std::copy(dom, dom + 4, P->domain);
  double side = std::max(dom[2] - dom[0], dom[3] - dom[1]);
  if (!(side > 0)) side = 1.0;
  side *= 1.0 + 1.0 / 1024;
  const double rho = rho_local >= 0.0 ? rho_local : star_density(n_sources, sb ? sb : dom);
  P->rho_local = rho_local;
  bool aligned = false;
  if (align && align->nx > 0 && align->ny > 0 && n_sources > 0)
    aligned = aligned_geometry(*align, dom, o.leaf_level, rho, P->p, n_sources, &P->g);
  if (!aligned) {
    const double cxm = 0.5 * (dom[0] + dom[2]), cym = 0.5 * (dom[1] + dom[3]);
    P->g.side = side;
    P->g.x0 = cxm - 0.5 * side;
    P->g.y0 = cym - 0.5 * side;
    const double rw = ray_box ? ray_box[2] - ray_box[0] : side;
    const double rh = ray_box ? ray_box[3] - ray_box[1] : side;
    P->g.L = o.leaf_level > 0
                 ? o.leaf_level
                 : level_for_side(side, preferred_leaf_side(rho, rays_density, side, P->p), P->p,
                                  n_sources, rw, rh);
  }
  if (ray_box)
    std::copy(ray_box, ray_box + 4, P->target);
  else
    std::copy(dom, dom + 4, P->target);
  source_windows(P);
}

// Plan phase 2: every device buffer the tree build and the upward pass use.
void plan_alloc(lens_plan *P, hipStream_t st) {
  const int L = P->g.L;
  const int64_t nbox = int64_t(1) << (2 * L);
  const int64_t N = std::max<int64_t>(P->n_stars, 1);
  P->mp.resize(L + 1);
  P->mp32.resize(L + 1);
  P->leaf_start = pool_get((size_t)(nbox + 1) * sizeof(int32_t), st);
  P->sxy = pool_get((size_t)N * 16, st);
  P->sm = pool_get((size_t)N * 8 * P->qdim, st);
  if (P->qdim == 1) P->sm32 = pool_get((size_t)N * 4, st);
  for (DevBuf *b : {&P->keys, &P->vals, &P->keys_tmp, &P->vals_tmp})
    *b = pool_get((size_t)N * sizeof(uint32_t), st);
  const size_t ncnt = radix_counts_len(N);
  P->cnt = pool_get(ncnt * sizeof(uint32_t), st);
  P->scan_tmp = pool_get(scan_tmp_len(ncnt) * sizeof(uint32_t), st);
  P->box_coarse = pool_get((size_t)box_starts_coarse_len(nbox) * sizeof(int32_t), st);
  for (int l = 2; l <= L; ++l) {
    const size_t n = (size_t)P->swin[l].count() * P->p * 2;
    P->mp[l] = pool_get(n * sizeof(double), st);
    // LENS_MIXED: the fine levels also get FP32 copies for their M2L
    if (P->precision == LENS_MIXED && l > L - P->fine_levels)
      P->mp32[l] = pool_get(n * sizeof(float), st);
  }
}

// Plan phase 3: kernels only (no allocation, no copy, no memset) -- sort the
// sources by leaf box (plan_tree), then P2M / M2M (plan_upward).
void plan_upward(lens_plan *P, hipStream_t st);

void plan_tree(lens_plan *P, const double *xy, const double *q, hipStream_t st) {
  const int L = P->g.L;
  const int64_t nbox = int64_t(1) << (2 * L);
  const int64_t N = P->n_stars;
  StageTimer tm("tree", st);
  auto *k = static_cast<uint32_t *>(P->keys.ptr), *v = static_cast<uint32_t *>(P->vals.ptr);
  auto *kt = static_cast<uint32_t *>(P->keys_tmp.ptr), *vt = static_cast<uint32_t *>(P->vals_tmp.ptr);
  launch_leaf_keys(xy, N, P->g, k, v, nullptr, st);
  const bool in_tmp = radix_sort_pairs(k, v, kt, vt, N, 2 * L, static_cast<uint32_t *>(P->cnt.ptr),
                                       static_cast<uint32_t *>(P->scan_tmp.ptr), st);
  const uint32_t *ks = in_tmp ? kt : k, *vs = in_tmp ? vt : v;
  P->perm = vs;
  launch_gather_stars(vs, xy, q, P->qdim, N, static_cast<double *>(P->sxy.ptr),
                      static_cast<double *>(P->sm.ptr), static_cast<float *>(P->sm32.ptr), st);
  // all zero when N = 0
  launch_box_starts(ks, N, nbox, static_cast<int32_t *>(P->leaf_start.ptr),
                    static_cast<int32_t *>(P->box_coarse.ptr), st);
}

void plan_enqueue(lens_plan *P, const double *xy, const double *q, hipStream_t st) {
  plan_tree(P, xy, q, st);
  plan_upward(P, st);
}

void plan_upward(lens_plan *P, hipStream_t st) {
  const int L = P->g.L;
  const int64_t N = P->n_stars;
  auto *leaf_start = static_cast<int32_t *>(P->leaf_start.ptr);
  auto *sxy = static_cast<double *>(P->sxy.ptr);
  auto *sm = static_cast<double *>(P->sm.ptr);
  const OpTables &T = op_tables(P->p, st);
  // clustered: the sources are much denser where the rays are than over
  // their bounding box (a galaxy's centre), so some leaf boxes may hold
  // hundreds of them
  const double bb_area = std::max((P->star_bb[2] - P->star_bb[0]) * (P->star_bb[3] - P->star_bb[1]), 1e-300);
  const bool clustered = P->rho_local > 4.0 * (double)N / bb_area;
  {
    StageTimer tm("upward", st);
    // from the stars or by M2M, as source_windows decided; runs of M2M
    // levels go up to four levels per launch
    for (int l = L; l >= 2;) {
      if (P->direct[l]) {
        // sources expected in the level's window: from the density where
        // the rays are for a window that is not the whole level
        const int64_t nl = int64_t(1) << l;
        const Window &w = P->swin[l];
        double n_win = (double)N;
        if (P->rho_local >= 0.0 && w.count() < nl * nl) {
          const double s = std::ldexp(P->g.side, -l);
          n_win = std::min((double)N, P->rho_local * s * s * (double)w.count());
        }
        launch_p2m(P->g, l, w, sxy, sm, P->qdim, leaf_start, P->p,
                   static_cast<double *>(P->mp[l].ptr), static_cast<float *>(P->mp32[l].ptr), n_win,
                   clustered, l < L ? P->swin[l + 1] : Window{0, 0, 0, 0},
                   l < L ? P->mp_at(l + 1) : nullptr, st);
        --l;
        continue;
      }
      M2MChain c{};
      c.level = l;
      c.p = P->p;
      c.child = P->mp_at(l + 1);
      const int kmax = m2m_chain_levels(l);
      c.nlev = 0;
      while (c.nlev < kmax && l - c.nlev >= 2 && !P->direct[l - c.nlev]) {
        c.out[c.nlev] = static_cast<double *>(P->mp[l - c.nlev].ptr);
        c.out32[c.nlev] = static_cast<float *>(P->mp32[l - c.nlev].ptr);
        ++c.nlev;
      }
      launch_m2m_chain(c, st);
      l -= c.nlev;
    }
  }
  P->last_stream = st;
}

// Sources are f.xy with charges f.m (real), or, if qc is given, the complex
// charges qc[n][2] (the adjoint's rays).  sb_known: the sources' bounding box
// if already known (else it is read back from the device).
lens_plan *build_plan(const lens_field &f, const double *ray_box, const lens_grid *align,
                      double rays_density, const lens_opts &o, hipStream_t st,
                      const double *qc = nullptr, const double *sb_known = nullptr,
                      double rho_known = -1.0) {
  auto *P = new lens_plan();
  P->qdim = qc ? 2 : 1;
  try {
    LENS_HIP(hipGetDevice(&P->device));
    P->kappa_s = f.kappa_s;
    P->gamma = f.gamma;
    double sb[4];
    const double *sbp = nullptr;
    double rho_local = -1.0;
    if (f.n_stars > 0) {
      if (sb_known) {
        std::copy(sb_known, sb_known + 4, sb);
        rho_local = rho_known;
      } else if (ray_box) {
        int64_t cnt = 0;
        device_bbox(f.xy, f.n_stars, st, sb, ray_box, &cnt);
        rho_local = local_density(cnt, ray_box);
      } else {
        device_bbox(f.xy, f.n_stars, st, sb);
      }
      sbp = sb;
      std::copy(sb, sb + 4, P->star_bb);
    }
    plan_geometry(P, f.n_stars, sbp, ray_box, align, rays_density, o, rho_local);
    (void)op_tables(o.order_p, st);
    plan_alloc(P, st);
    plan_enqueue(P, f.xy, qc ? qc : f.m, st);
  } catch (...) {
    P->release();
    delete P;
    throw;
  }
  return P;
}

void check_inside(const lens_plan &P, const double bb[4]) {
  const double tol = 1e-12 * P.g.side;
  if (bb[0] < P.target[0] - tol || bb[1] < P.target[1] - tol || bb[2] > P.target[2] + tol ||
      bb[3] > P.target[3] + tol)
    fail(LENS_EINVAL, "rays lie outside the region the plan was built for (pass ray_box to lens_plan_create)");
}

// Windows and local-expansion buffers of every level for rays in `bb`.
struct LocalSet {
  std::vector<Window> win;
  std::vector<DevBuf> loc;
  double *at(int l) const { return static_cast<double *>(loc[l].ptr); }
  void put_all(hipStream_t st) {
    std::vector<DevBuf *> ps;
    for (auto &b : loc) ps.push_back(&b);
    pool_put_batch(ps.data(), ps.size(), st);
  }
};

void locals_alloc(const lens_plan &P, const double bb[4], LocalSet &ls, hipStream_t st) {
  const int L = P.g.L;
  ls.win.assign(L + 1, Window{0, 0, 0, 0});
  ls.loc.assign(L + 1, DevBuf{});
  for (int l = 2; l <= L; ++l) {
    ls.win[l] = window_for(P, l, bb);
    ls.loc[l] = pool_get((size_t)ls.win[l].count() * P.p * 16, st);
  }
}

// Downward pass (kernels only): locals of every level 2..L.  Levels >= 3
// among the two finest run M2L and L2L in one fused kernel, in order; the
// coarser ones run M2L batched, then the L2L sweep.
void downward_enqueue(const lens_plan &P, const LocalSet &ls, hipStream_t st) {
  const int L = P.g.L;
  const OpTables &T = op_tables(P.p, st);
  StageTimer tm("downward", st);
  auto is_f32 = [&](int l) {
    return P.precision == LENS_MIXED && l > L - P.fine_levels && P.mp32_at(l) != nullptr;
  };
  auto level_of = [&](int l) {
    return M2LLevel{l, std::ldexp(P.g.side, -l), ls.win[l],
                    is_f32(l) ? (const void *)P.mp32_at(l) : (const void *)P.mp_at(l), ls.at(l),
                    nullptr, Window{0, 0, 0, 0}, P.swin[l]};
  };
  const int first_fused = std::max(3, L - 1);
  M2LBatch coarse, fine;
  coarse.p = fine.p = P.p;
  for (int l = 2; l < first_fused && l <= L; ++l) {
    M2LBatch &b = is_f32(l) ? fine : coarse;
    b.lv[b.count++] = level_of(l);
  }
  launch_m2l_batch(coarse, T, false, st);
  launch_m2l_batch(fine, T, true, st);
  auto l2l = [&](int l) {
    DownArgs d{};
    d.level = l;
    d.p = P.p;
    d.s = std::ldexp(P.g.side, -l);
    d.win = ls.win[l];
    d.pwin = ls.win[l - 1];
    d.ploc = ls.at(l - 1);
    d.loc = ls.at(l);
    launch_l2l(d, T, st);
  };
  // coarse L2L sweep, up to three levels per launch
  for (int l = 3; l < first_fused && l <= L;) {
    L2LChain c{};
    c.level = l - 1;
    c.p = P.p;
    c.nlev = std::min(kMaxL2LChain, std::min(first_fused, L + 1) - l);
    for (int j = 0; j <= c.nlev; ++j) {
      c.win[j] = ls.win[l - 1 + j];
      c.loc[j] = ls.at(l - 1 + j);
    }
    launch_l2l_chain(c, T, st);
    l += c.nlev;
  }
  for (int l = first_fused; l <= L; ++l) {
    M2LBatch one;
    one.p = P.p;
    one.count = 1;
    one.lv[0] = level_of(l);
    one.lv[0].ploc = ls.at(l - 1);
    one.lv[0].pwin = ls.win[l - 1];
    if (!launch_m2l_l2l(one, T, is_f32(l), st)) {
      one.lv[0].ploc = nullptr;
      launch_m2l_batch(one, T, is_f32(l), st);
      l2l(l);
    }
  }
}

// Convenience: allocate (released behind the stream's work by `sc`) and run.
Window downward(lens_plan &P, const double bb[4], Scratch &sc, hipStream_t st, double **leaf_loc) {
  LocalSet ls;
  locals_alloc(P, bb, ls, st);
  downward_enqueue(P, ls, st);
  for (auto &b : ls.loc)
    if (b.ptr) sc.bufs.push_back(b);
  *leaf_loc = ls.at(P.g.L);
  return ls.win[P.g.L];
}

void fill_star_side(const lens_plan &P, Window wl, double *loc, EvalArgs &ea) {
  ea.g = P.g;
  ea.p = P.p;
  ea.win = wl;
  ea.loc = loc;
  ea.sxy = static_cast<const double *>(P.sxy.ptr);
  ea.sm = static_cast<const double *>(P.sm.ptr);
  ea.sm32 = static_cast<const float *>(P.sm32.ptr);
  ea.leaf_start = static_cast<const int32_t *>(P.leaf_start.ptr);
}

void launch_eval_checked(EvalArgs &ea, int precision, hipStream_t st) {
  while (ea.win.count() * ea.chunks_per_box > (int64_t)0x7fffffff && ea.chunks_per_box > 1)
    ea.chunks_per_box = (ea.chunks_per_box + 1) / 2;
  if (ea.win.count() > (int64_t)0x7fffffff) fail(LENS_EUNSUPPORTED, "leaf window too large");
  StageTimer tm(ea.counts ? "eval_map" : "eval", st);
  launch_eval(ea, precision, st);
}

template <typename F>
lens_status guarded(F &&fn) {
  try {
    fn();
    return LENS_OK;
  } catch (const LensError &e) {
    set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return LENS_ENOMEM;
  } catch (...) {
    set_error("unexpected internal error");
    return LENS_EDEVICE;
  }
}

void grid_bbox(const lens_grid &g, int64_t j0, int64_t j1, double bb[4]) {
  bb[0] = grid_x(g, 0);
  bb[2] = grid_x(g, g.nx - 1);
  bb[1] = grid_y(g, j0);
  bb[3] = grid_y(g, j1 - 1);
}

// Evaluation of grid rows [j0, j1): its locals, ray ranges and launch shape.
struct GridExec {
  int64_t j0 = 0, j1 = 0;
  double bb[4];
  LocalSet ls;
  DevBuf col_start, row_start;
  EvalArgs ea{};
  void put_all(hipStream_t st) {
    std::vector<DevBuf *> ps = {&col_start, &row_start};
    for (auto &b : ls.loc) ps.push_back(&b);
    pool_put_batch(ps.data(), ps.size(), st);
  }
};

// Bytes of per-call device memory the evaluation of grid rows [j0, j1)
// needs: the locals of every level over the rows' windows and the ray
// ranges of the leaf window (each piece aligned to 256 bytes).
constexpr size_t kAlign = 256;
size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

size_t gridexec_bytes(const lens_plan &P, const lens_grid &grid, int64_t j0, int64_t j1) {
  double bb[4];
  grid_bbox(grid, j0, j1, bb);
  size_t total = 0;
  for (int l = 2; l <= P.g.L; ++l) total += align_up((size_t)window_for(P, l, bb).count() * P.p * 16);
  const Window wl = window_for(P, P.g.L, bb);
  total += align_up((size_t)(wl.nbx + 1) * sizeof(int32_t));
  total += align_up((size_t)(wl.nby + 1) * sizeof(int32_t));
  return total;
}

// Windows, buffers and launch shape of grid rows [j0, j1).  Buffers come
// from the pool, or, if `region` is given, are carved from it in order
// (gridexec_bytes of them; the GridExec then owns nothing).
void gridexec_alloc(const lens_plan &P, const lens_grid &grid, int64_t j0, int64_t j1, GridExec &ge,
                    hipStream_t st, char *region = nullptr) {
  ge.j0 = j0;
  ge.j1 = j1;
  grid_bbox(grid, j0, j1, ge.bb);
  check_inside(P, ge.bb);
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    DevBuf b;
    b.ptr = region + off;
    b.bytes = bytes;
    off += align_up(bytes);
    return b;
  };
  if (region) {
    const int L = P.g.L;
    ge.ls.win.assign(L + 1, Window{0, 0, 0, 0});
    ge.ls.loc.assign(L + 1, DevBuf{});
    for (int l = 2; l <= L; ++l) {
      ge.ls.win[l] = window_for(P, l, ge.bb);
      ge.ls.loc[l] = carve((size_t)ge.ls.win[l].count() * P.p * 16);
    }
  } else {
    locals_alloc(P, ge.bb, ge.ls, st);
  }
  const Window wl = ge.ls.win[P.g.L];
  ge.col_start = region ? carve((size_t)(wl.nbx + 1) * sizeof(int32_t))
                        : pool_get((size_t)(wl.nbx + 1) * sizeof(int32_t), st);
  ge.row_start = region ? carve((size_t)(wl.nby + 1) * sizeof(int32_t))
                        : pool_get((size_t)(wl.nby + 1) * sizeof(int32_t), st);
  EvalArgs &ea = ge.ea;
  fill_star_side(P, wl, ge.ls.at(P.g.L), ea);
  ea.grid_mode = 1;
  ea.grid = grid;
  ea.col_start = static_cast<int32_t *>(ge.col_start.ptr);
  ea.row_start = static_cast<int32_t *>(ge.row_start.ptr);
  // a leaf box of side s holds k grid columns when s = k dx, else at most
  // floor(s/dx) + 1 (rows likewise); a longer box chunk is still processed
  // whole by the kernel, only less efficiently
  const double s = std::ldexp(P.g.side, -P.g.L);
  auto per_box = [&](double step, int64_t cap) {
    const double r = s / step;
    const double k = std::round(r);
    const int64_t n = std::fabs(r - k) < 1e-9 * r ? (int64_t)k : (int64_t)std::floor(r) + 1;
    return std::max<int64_t>(1, std::min(n, cap));
  };
  int64_t tiles = 0;
  grid_tile_shape(per_box(grid.dx, grid.nx), per_box(grid.dy, j1 - j0), &ea.tile_shift, &tiles);
  eval_shape(tiles * 64, &ea.rays_per_lane, &ea.chunks_per_box);
  while (wl.count() * ea.chunks_per_box > (int64_t)0x7fffffff && ea.chunks_per_box > 1)
    ea.chunks_per_box = (ea.chunks_per_box + 1) / 2;
  if (wl.count() > (int64_t)0x7fffffff) fail(LENS_EUNSUPPORTED, "leaf window too large");
}

// Kernels only: downward pass, ray ranges, evaluation (y_out or map).
void gridexec_enqueue(const lens_plan &P, GridExec &ge, double c1, double c2, double *y_out,
                      const lens_map_desc *map, hipStream_t st, double *dfdz = nullptr) {
  downward_enqueue(P, ge.ls, st);
  EvalArgs ea = ge.ea;
  ea.c1 = c1;
  ea.c2 = c2;
  ea.y_out = y_out;
  ea.dfdz_out = dfdz;
  if (map) {
    ea.counts = map->counts;
    ea.y1min = map->y1min;
    ea.y2min = map->y2min;
    ea.S = (double)map->npix / map->side;
    ea.npix = map->npix;
  }
  launch_grid_ranges(ea.grid, P.g, ea.win, ge.j0, ge.j1, const_cast<int32_t *>(ea.col_start),
                     const_cast<int32_t *>(ea.row_start), st);
  StageTimer tm(ea.counts ? "eval_map" : "eval", st);
  launch_eval(ea, P.precision, st);
}

// Grid rows [j0, j1) through the FMM path (deflect: y_out; map: binning).
void fmm_grid_rows(lens_plan &P, const lens_grid &grid, int64_t j0, int64_t j1, double c1, double c2,
                   double *y_out, const lens_map_desc *map, double S, hipStream_t st,
                   double *dfdz = nullptr) {
  (void)S;
  GridExec ge;
  try {
    gridexec_alloc(P, grid, j0, j1, ge, st);
    gridexec_enqueue(P, ge, c1, c2, y_out, map, st, dfdz);
  } catch (...) {
    ge.put_all(st);
    throw;
  }
  ge.put_all(st);
  P.last_stream = st;
}

// Explicit rays: sorted by leaf box of the window, evaluated box by box,
// written back in the caller's order.  The downward pass over the window of
// bb is separate, so that repeated evaluations at moving points inside bb
// (Newton steps) share it.
struct ExplicitLocals {
  Window wl;
  double *loc = nullptr;
};

ExplicitLocals explicit_locals(lens_plan &P, const double bb[4], Scratch &sc, hipStream_t st) {
  check_inside(P, bb);
  ExplicitLocals e;
  e.wl = downward(P, bb, sc, st, &e.loc);
  return e;
}

void fmm_explicit_eval(lens_plan &P, const ExplicitLocals &e, const double *rays, int64_t n,
                       double c1, double c2, double *y_out, hipStream_t st, double *dfdz = nullptr) {
  Scratch sc(st);
  const Window wl = e.wl;
  uint32_t *k = sc.get<uint32_t>(n), *v = sc.get<uint32_t>(n);
  uint32_t *kt = sc.get<uint32_t>(n), *vt = sc.get<uint32_t>(n);
  const size_t ncnt = radix_counts_len(n);
  uint32_t *cnt = sc.get<uint32_t>(ncnt);
  uint32_t *stmp = sc.get<uint32_t>(scan_tmp_len(ncnt));
  launch_ray_keys(rays, n, P.g, wl, k, v, st);
  int bits = 1;
  while ((int64_t(1) << bits) < wl.count()) ++bits;
  const bool in_tmp = radix_sort_pairs(k, v, kt, vt, n, bits, cnt, stmp, st);
  const uint32_t *ks = in_tmp ? kt : k, *vs = in_tmp ? vt : v;
  double *srays = sc.get<double>((size_t)n * 2);
  launch_gather_rays(vs, rays, n, srays, st);
  int32_t *rstart = sc.get<int32_t>(wl.count() + 1);
  launch_box_starts(ks, n, wl.count(), rstart, sc.get<int32_t>(box_starts_coarse_len(wl.count())), st);
  EvalArgs ea{};
  fill_star_side(P, wl, e.loc, ea);
  ea.grid_mode = 0;
  ea.rxy = srays;
  ea.rperm = vs;
  ea.ray_start = rstart;
  ea.c1 = c1;
  ea.c2 = c2;
  ea.y_out = y_out;
  ea.dfdz_out = dfdz;
  // explicit rays: shape for the mean box occupancy; fuller boxes loop
  const int64_t per = (n + wl.count() - 1) / std::max<int64_t>(wl.count(), 1);
  eval_shape(std::max<int64_t>(per, 1), &ea.rays_per_lane, &ea.chunks_per_box);
  launch_eval_checked(ea, P.precision, st);
  P.last_stream = st;
}

void fmm_explicit(lens_plan &P, const double *rays, int64_t n, const double bb[4], double c1, double c2,
                  double *y_out, hipStream_t st,
                  double *dfdz = nullptr) {
  Scratch sc(st);
  const ExplicitLocals e = explicit_locals(P, bb, sc, st);
  fmm_explicit_eval(P, e, rays, n, c1, c2, y_out, st, dfdz);
}

void release_owned(lens_plan *owned, hipStream_t st) {
  // stream-ordered release: the buffers go back to the pool behind the work
  owned->put_all(st);
  delete owned;
}

struct FieldView {
  lens_field f;
  bool from_plan;
};

FieldView field_for(const lens_plan *plan, const lens_field *field) {
  if (!plan) {
    check_field(field);
    return {*field, false};
  }
  // a plan supplies the stars; a field given with it supplies kappa_s and gamma
  lens_field f{plan->n_stars, static_cast<const double *>(plan->sxy.ptr),
               static_cast<const double *>(plan->sm.ptr), plan->kappa_s, plan->gamma};
  if (field) {
    if (!is_finite(field->kappa_s) || !is_finite(field->gamma))
      fail(LENS_EINVAL, "kappa_s and gamma must be finite");
    f.kappa_s = field->kappa_s;
    f.gamma = field->gamma;
  }
  return {f, true};
}

void check_plan_device(const lens_plan *plan) {
  int dev = 0;
  LENS_HIP(hipGetDevice(&dev));
  if (dev != plan->device) fail(LENS_EINVAL, "plan was created on another device");
}

}  // namespace

namespace {

// ------------------------------------------------------------- autotuner
// Accuracy is measured, not modelled: a strided sample of at most 256 x 256
// rays of the grid is deflected by the FP64 direct sum and by the FMM (a
// plan over the whole grid, as a real call builds it) at increasing p.  The
// error is the largest per-ray relative deflection error, or for a map the
// expected fraction of rays binned into another pixel,
// mean(|dy1| + |dy2|) * npix / side.  Among
// the settings that reach the target the fastest whole call is kept.

struct TuneOut {
  lens_opts o;
  double err = 0, ms = 0;
  bool met = false;
};

struct TuneSample {
  int64_t n = 0;
  std::vector<double> rays, yref;
  double *d_rays = nullptr, *d_y = nullptr;
  double bb[4];
};

double tune_error(const TuneSample &ts, const std::vector<double> &y, double c1, double c2,
                  const lens_map_desc *map) {
  if (map) {
    double acc = 0;
    for (int64_t k = 0; k < ts.n; ++k)
      acc += std::fabs(y[2 * k] - ts.yref[2 * k]) + std::fabs(y[2 * k + 1] - ts.yref[2 * k + 1]);
    return acc / (double)std::max<int64_t>(ts.n, 1) * (double)map->npix / map->side;
  }
  // deflection: the largest per-ray relative error |dalpha_k| /
  // max(|alpha_k|, 1e-3 rms alpha) over the sample
  double ms = 0;
  for (int64_t k = 0; k < ts.n; ++k) {
    const double a1 = c1 * ts.rays[2 * k] - ts.yref[2 * k];
    const double a2 = c2 * ts.rays[2 * k + 1] - ts.yref[2 * k + 1];
    ms += a1 * a1 + a2 * a2;
  }
  const double floor_a = 1e-3 * std::sqrt(ms / (double)std::max<int64_t>(ts.n, 1));
  double worst = 0;
  for (int64_t k = 0; k < ts.n; ++k) {
    const double d1 = y[2 * k] - ts.yref[2 * k], d2 = y[2 * k + 1] - ts.yref[2 * k + 1];
    const double a1 = c1 * ts.rays[2 * k] - ts.yref[2 * k];
    const double a2 = c2 * ts.rays[2 * k + 1] - ts.yref[2 * k + 1];
    const double den = std::max(std::hypot(a1, a2), floor_a);
    const double d = std::hypot(d1, d2);
    worst = std::max(worst, den > 0 ? d / den : d);
  }
  return worst;
}

// Time of one whole call (lens_map into a scratch map, or lens_deflect into
// a scratch output), after one untimed call.
double tune_time(const lens_field &f, const lens_grid &g, const lens_map_desc *map,
                 const lens_opts &o, void *scratch, hipStream_t st) {
  lens_map_desc md{};
  if (map) {
    md = *map;
    md.counts = static_cast<int32_t *>(scratch);
  }
  auto call = [&] {
    const lens_status r = map ? lens_map(nullptr, &f, &g, &md, &o, st)
                              : lens_deflect(nullptr, &f, &g, nullptr, g.nx * g.ny,
                                             static_cast<double *>(scratch), nullptr, &o, st);
    if (r != LENS_OK) fail(r, last_error());
  };
  call();
  hipEvent_t e0, e1;
  LENS_HIP(hipEventCreate(&e0));
  LENS_HIP(hipEventCreate(&e1));
  float ms = 0;
  try {
    LENS_HIP(hipEventRecord(e0, st));
    call();
    LENS_HIP(hipEventRecord(e1, st));
    LENS_HIP(hipEventSynchronize(e1));
    LENS_HIP(hipEventElapsedTime(&ms, e0, e1));
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

// A setting qualifies when its sampled error is below this fraction of the
// target: the margin covers the rays outside the sample (the errors are
// heavy-tailed -- a few rays near stars dominate the mean -- so the sampled
// error of one setting can differ by ~2x between disjoint samples).
constexpr double kTuneMargin = 0.5;

TuneOut autotune_field(const lens_field &f, const lens_grid &g, const lens_map_desc *map,
                       double tol, const lens_opts &base, hipStream_t st) {
  TuneOut best;
  best.o = base;
  if (base.method == LENS_DIRECT || f.n_stars == 0 || g.nx == 0 || g.ny == 0) {
    best.met = true;
    return best;
  }
  Scratch sc(st);
  TuneSample ts;
  const int64_t sx = std::max<int64_t>(1, g.nx / 256), sy = std::max<int64_t>(1, g.ny / 256);
  for (int64_t j = sy / 2; j < g.ny; j += sy)
    for (int64_t i = sx / 2; i < g.nx; i += sx) {
      ts.rays.push_back(grid_x(g, i));
      ts.rays.push_back(g.y0 + ((double)j + 0.5) * g.dy);
    }
  ts.n = (int64_t)ts.rays.size() / 2;
  ts.d_rays = sc.get<double>(ts.rays.size());
  ts.d_y = sc.get<double>(ts.rays.size());
  LENS_HIP(hipMemcpyAsync(ts.d_rays, ts.rays.data(), ts.rays.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
  const double c1 = (1.0 - f.kappa_s) - f.gamma, c2 = (1.0 - f.kappa_s) + f.gamma;
  {
    DirectArgs d{};
    d.n_stars = f.n_stars;
    d.sxy = f.xy;
    d.sm = f.m;
    d.rxy = ts.d_rays;
    d.n_rays = ts.n;
    d.c1 = c1;
    d.c2 = c2;
    d.y_out = ts.d_y;
    launch_direct(d, st);
  }
  ts.yref.resize(ts.rays.size());
  LENS_HIP(hipMemcpyAsync(ts.yref.data(), ts.d_y, ts.rays.size() * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  LENS_HIP(hipStreamSynchronize(st));
  double gb[4];
  grid_bbox(g, 0, g.ny, gb);
  const double area = std::max((gb[2] - gb[0]) * (gb[3] - gb[1]), 1e-300);
  const double density = (double)(g.nx * g.ny) / area;
  // sampled error of one setting
  auto measure = [&](lens_opts o) {
    const lens_opts r = resolve_opts(&o);
    lens_plan *P = build_plan(f, gb, &g, density, r, st);
    std::vector<double> y(ts.rays.size());
    try {
      fmm_explicit(*P, ts.d_rays, ts.n, gb, c1, c2, ts.d_y, st);
      LENS_HIP(hipMemcpyAsync(y.data(), ts.d_y, y.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      LENS_HIP(hipStreamSynchronize(st));
    } catch (...) {
      lens_plan_destroy(P);
      throw;
    }
    lens_plan_destroy(P);
    return tune_error(ts, y, c1, c2, map);
  };
  // per FP32-level family, the smallest p that reaches tol.  The error falls
  // in steps rather than smoothly (for near-uniform boxes the moments a_k
  // with k a multiple of 4 dominate, so p = 14 and p = 16 can tie), so every
  // p is tried; a family stops after six orders without a 30% gain (its
  // rounding floor).
  std::vector<int> families = {0};
  if (base.precision == LENS_MIXED) families = {2, -1};
  std::vector<TuneOut> met;
  TuneOut most{};
  most.err = std::numeric_limits<double>::infinity();
  for (int fl : families) {
    double best_e = std::numeric_limits<double>::infinity();
    int stall = 0;
    for (int p = 6; p <= LENS_MAX_ORDER; ++p) {
      lens_opts o = base;
      o.order_p = p;
      o.fp32_levels = fl;
      const double e = measure(o);
      if (e < most.err) {
        most.o = o;
        most.err = e;
      }
      if (e <= kTuneMargin * tol) {
        TuneOut t;
        t.o = o;
        t.err = e;
        t.met = true;
        met.push_back(t);
        break;
      }
      if (e < 0.7 * best_e) {
        best_e = e;
        stall = 0;
      } else if (++stall >= 6) {
        break;
      }
    }
  }
  if (met.empty()) {
    most.met = false;
    return most;
  }
  // the fastest of the families' settings, then the leaf level around the
  // library's choice
  void *scratch = map ? (void *)sc.get<int32_t>((size_t)map->npix * map->npix)
                      : (void *)sc.get<double>((size_t)g.nx * g.ny * 2);
  for (auto &t : met) t.ms = tune_time(f, g, map, t.o, scratch, st);
  best = *std::min_element(met.begin(), met.end(),
                           [](const TuneOut &a, const TuneOut &b) { return a.ms < b.ms; });
  if (base.leaf_level == 0) {
    lens_plan *P = build_plan(f, gb, &g, density, resolve_opts(&best.o), st);
    const int L0 = P->g.L;
    lens_plan_destroy(P);
    best.o.leaf_level = L0;
    for (int L : {L0 - 1, L0 + 1}) {
      if (L < 2 || L > 13) continue;
      lens_opts o = best.o;
      o.leaf_level = L;
      const double ms = tune_time(f, g, map, o, scratch, st);
      if (ms < best.ms) {
        const double e = measure(o);
        if (e <= kTuneMargin * tol) {
          best.o = o;
          best.ms = ms;
          best.err = e;
        }
      }
    }
  }
  return best;
}

// cache keys: words of the call's arguments
void key_push(std::vector<uint64_t> &k, double v) {
  uint64_t w;
  std::memcpy(&w, &v, 8);
  k.push_back(w);
}
void key_push(std::vector<uint64_t> &k, int64_t v) { k.push_back((uint64_t)v); }
void key_push(std::vector<uint64_t> &k, const void *p) { k.push_back((uint64_t)(uintptr_t)p); }

// ------------------------------------------------- automatic order (tol)
// order_p = 0 with tol > 0 asks for the autotuner's setting.  Results are
// kept in-process (by the call's arrays, sizes and parameters) and on disk
// (by a coarse description of the problem: precision, target, tol, N_*,
// rays per star, smooth terms and pixel scale, rounded), so a later process
// with a similar field reuses the measured order without measuring.  The
// file is $LENS_TUNE_CACHE (empty or "off": no disk cache), else
// $XDG_CACHE_HOME/lensfmm/autotune.txt, else ~/.cache/lensfmm/autotune.txt.

std::mutex g_tune_mu;
std::vector<std::pair<std::vector<uint64_t>, TuneOut>> g_tuned;  // most recent last
bool g_disk_loaded = false;
std::map<std::string, lens_opts> g_disk;

std::string tune_cache_path() {
  const char *e = std::getenv("LENS_TUNE_CACHE");
  if (e) return (std::string(e) == "off") ? std::string() : std::string(e);
  const char *x = std::getenv("XDG_CACHE_HOME");
  if (x && *x) return std::string(x) + "/lensfmm/autotune.txt";
  const char *h = std::getenv("HOME");
  if (h && *h) return std::string(h) + "/.cache/lensfmm/autotune.txt";
  return std::string();
}

// coarse description of a tuning problem (the on-disk key)
std::string tune_disk_key(int device, const lens_field &f, const lens_grid &g,
                          const lens_map_desc *map, const lens_opts &o) {
  hipDeviceProp_t prop{};
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
  (void)hipGetLastError();
  auto r2 = [](double v) { return std::lround(2.0 * std::log2(std::max(v, 1e-300))); };
  auto r100 = [](double v) { return std::lround(100.0 * v); };
  const double rays = (double)(g.nx * g.ny);
  std::string k = arch.substr(0, arch.find(':')) + (o.precision == LENS_MIXED ? " mixed" : " fp64") +
                  (map ? " map" : " deflect") + " tol " + std::to_string(std::lround(8.0 * std::log2(o.tol))) +
                  " n " + std::to_string(r2((double)f.n_stars)) +
                  " rps " + std::to_string(r2(rays / std::max<double>((double)f.n_stars, 1.0))) +
                  " ks " + std::to_string(r100(f.kappa_s)) + " g " + std::to_string(r100(f.gamma)) +
                  " leaf " + std::to_string(o.leaf_level);
  if (map) k += " px " + std::to_string(r2(map->side / map->npix / std::sqrt(g.dx * g.dy)));
  return k;
}

void load_disk_locked() {
  if (g_disk_loaded) return;
  g_disk_loaded = true;
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  FILE *fp = std::fopen(path.c_str(), "r");
  if (!fp) return;
  char line[512];
  while (std::fgets(line, sizeof line, fp)) {
    // key | p fp32_levels leaf_level
    char *bar = std::strchr(line, '|');
    if (!bar) continue;
    *bar = 0;
    int p = 0, fl = 0, L = 0;
    if (std::sscanf(bar + 1, "%d %d %d", &p, &fl, &L) != 3) continue;
    if (p < 1 || p > LENS_MAX_ORDER || L < 0 || L > LENS_MAX_LEVEL) continue;
    lens_opts o;
    lens_opts_default(&o);
    o.order_p = p;
    o.fp32_levels = fl;
    o.leaf_level = L;
    g_disk[std::string(line)] = o;
  }
  std::fclose(fp);
}

void save_disk_locked(const std::string &key, const lens_opts &o) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    // create the directory chain (best effort; failures only skip caching)
    std::string dir = path.substr(0, slash);
    for (size_t i = 1; i <= dir.size(); ++i)
      if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
  }
  FILE *fp = std::fopen(path.c_str(), "a");
  if (!fp) return;
  std::fprintf(fp, "%s|%d %d %d\n", key.c_str(), o.order_p, o.fp32_levels, o.leaf_level);
  std::fclose(fp);
}

// The autotuner's choice for a problem, measured once per process (and
// once per machine, through the disk cache; a disk hit carries no measured
// error or time: NaN).  opts: the caller's method, precision, leaf level and
// fp32_levels unless tuned.
TuneOut tuned_cached(const lens_field &f, const lens_grid &g, const lens_map_desc *map,
                     const lens_opts &user, hipStream_t st) {
  lens_opts base = user;
  base.order_p = 0;
  int dev = 0;
  LENS_HIP(hipGetDevice(&dev));
  std::vector<uint64_t> key;
  key_push(key, (int64_t)dev);
  key_push(key, (const void *)f.xy);
  key_push(key, (const void *)f.m);
  key_push(key, f.n_stars);
  key_push(key, f.kappa_s);
  key_push(key, f.gamma);
  key_push(key, g.x0);
  key_push(key, g.y0);
  key_push(key, g.dx);
  key_push(key, g.dy);
  key_push(key, g.nx);
  key_push(key, g.ny);
  key_push(key, (int64_t)(map != nullptr));
  if (map) {
    key_push(key, map->y1min);
    key_push(key, map->y2min);
    key_push(key, map->side);
    key_push(key, (int64_t)map->npix);
  }
  key_push(key, user.tol);
  key_push(key, (int64_t)user.method);
  key_push(key, (int64_t)user.precision);
  key_push(key, (int64_t)user.leaf_level);
  key_push(key, (int64_t)user.fp32_levels);
  const std::string dkey = tune_disk_key(dev, f, g, map, user);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (size_t i = 0; i < g_tuned.size(); ++i)
      if (g_tuned[i].first == key) {
        auto e = g_tuned[i];
        g_tuned.erase(g_tuned.begin() + (long)i);
        g_tuned.push_back(e);
        return e.second;
      }
    load_disk_locked();
    auto it = g_disk.find(dkey);
    if (it != g_disk.end()) {
      TuneOut t;
      t.o = base;
      t.o.order_p = it->second.order_p;
      t.o.fp32_levels = it->second.fp32_levels;
      t.o.leaf_level = it->second.leaf_level;
      t.err = t.ms = std::numeric_limits<double>::quiet_NaN();
      t.met = true;
      g_tuned.emplace_back(key, t);
      if (g_tuned.size() > 32) g_tuned.erase(g_tuned.begin());
      return t;
    }
  }
  const TuneOut t = autotune_field(f, g, map, user.tol, base, st);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.emplace_back(key, t);
  if (g_tuned.size() > 32) g_tuned.erase(g_tuned.begin());
  if (t.met && user.method == LENS_FMM) {
    g_disk[dkey] = t.o;
    save_disk_locked(dkey, t.o);
  }
  return t;
}

// The options a call with order_p = 0 and tol > 0 runs with (the most
// accurate setting tried if none reached tol).
lens_opts auto_opts(const lens_field &f, const lens_grid &g, const lens_map_desc *map,
                    const lens_opts &user, hipStream_t st) {
  const TuneOut t = tuned_cached(f, g, map, user, st);
  return resolve_opts(&t.o);
}

bool wants_auto(const lens_opts *o) {
  return o && o->order_p == 0 && o->tol > 0 && std::isfinite(o->tol) && o->method == LENS_FMM;
}

// A 128 x 128 grid over the box bb, standing in for explicit rays when tuning.
lens_grid tuning_grid(const double bb[4]) {
  lens_grid g{};
  g.nx = g.ny = 128;
  const double w = std::max(bb[2] - bb[0], 1e-12), h = std::max(bb[3] - bb[1], 1e-12);
  g.dx = w / 128.0;
  g.dy = h / 128.0;
  g.x0 = bb[0];
  g.y0 = bb[1];
  return g;
}

// ------------------------------------------------------- batched fields
// lens_map_batched: every field's tree build, upward pass, downward pass and
// binned evaluation, allocated up front and captured as one HIP graph whose
// branches (fields spread over kSideStreams forked streams) run
// concurrently; the graph is cached by the batch's arrays and parameters and
// replayed while every field's stars stay inside its captured tree.  With
// the default four hardware queues, 16 branches measured ~10% faster than 4
// (more queues per process measured slower).

constexpr int kSideStreams = 16;
constexpr size_t kBatchCache = 4;

struct BatchExec {
  std::vector<uint64_t> key;
  int device = 0;
  std::vector<lens_plan *> plans;  // nullptr for fields without stars
  std::vector<std::unique_ptr<GridExec>> ge;
  // the fields' trees sorted together: job table and combined sort arrays
  std::vector<DevBuf> tree;
  hipStream_t origin = nullptr;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last = nullptr;

  ~BatchExec() {
    if (last) (void)hipStreamSynchronize(last);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto *P : plans)
      if (P) {
        P->put_all(nullptr);
        delete P;
      }
    for (auto &g : ge)
      if (g) g->put_all(nullptr);
    std::vector<DevBuf *> tb;
    for (auto &b : tree) tb.push_back(&b);
    pool_put_batch(tb.data(), tb.size(), nullptr);
    for (auto e : ev) (void)hipEventDestroy(e);
    for (auto s : side) (void)hipStreamDestroy(s);
    if (origin) (void)hipStreamDestroy(origin);
  }
};

std::mutex g_batch_mu;
std::vector<std::unique_ptr<BatchExec>> g_batches;


std::vector<uint64_t> batch_key(int dev, int n, const lens_field *f, const lens_grid *g,
                                const lens_map_desc *m, const lens_opts &o) {
  std::vector<uint64_t> k;
  key_push(k, (int64_t)dev);
  key_push(k, (int64_t)n);
  key_push(k, (int64_t)o.method);
  key_push(k, (int64_t)o.precision);
  key_push(k, (int64_t)o.order_p);
  key_push(k, (int64_t)o.fp32_levels);
  key_push(k, o.tol);
  key_push(k, (int64_t)o.leaf_level);
  for (int i = 0; i < n; ++i) {
    key_push(k, f[i].n_stars);
    key_push(k, (const void *)f[i].xy);
    key_push(k, (const void *)f[i].m);
    key_push(k, f[i].kappa_s);
    key_push(k, f[i].gamma);
    key_push(k, g[i].x0);
    key_push(k, g[i].y0);
    key_push(k, g[i].dx);
    key_push(k, g[i].dy);
    key_push(k, g[i].nx);
    key_push(k, g[i].ny);
    key_push(k, m[i].y1min);
    key_push(k, m[i].y2min);
    key_push(k, m[i].side);
    key_push(k, (int64_t)m[i].npix);
    key_push(k, (const void *)m[i].counts);
  }
  return k;
}

bool inside(const double dom[4], const double bb[4]) {
  return bb[0] >= dom[0] && bb[1] >= dom[1] && bb[2] <= dom[2] && bb[3] <= dom[3];
}

// tune: each field's options come from the autotuner (target tune_base.tol,
// method and precision of tune_base); otherwise every field uses o.
std::unique_ptr<BatchExec> batch_build(int n, const lens_field *f, const lens_grid *g,
                                       const lens_map_desc *m, const lens_opts &o,
                                       const std::vector<double> &bbox, bool tune,
                                       const lens_opts &tune_base, hipStream_t st) {
  auto B = std::make_unique<BatchExec>();
  LENS_HIP(hipGetDevice(&B->device));
  (void)op_tables(o.order_p, st);
  B->plans.assign(n, nullptr);
  B->ge.resize(n);
  for (int i = 0; i < n; ++i) {
    if (f[i].n_stars == 0 || o.method == LENS_DIRECT) continue;
    lens_opts oi = o;
    if (tune) {
      oi = auto_opts(f[i], g[i], &m[i], tune_base, st);
      (void)op_tables(oi.order_p, st);
    }
    auto *P = new lens_plan();
    B->plans[i] = P;
    P->device = B->device;
    P->kappa_s = f[i].kappa_s;
    P->gamma = f[i].gamma;
    double gb[4];
    grid_bbox(g[i], 0, g[i].ny, gb);
    const double area = std::max((gb[2] - gb[0]) * (gb[3] - gb[1]), 1e-300);
    plan_geometry(P, f[i].n_stars, &bbox[4 * i], gb, &g[i], (double)(g[i].nx * g[i].ny) / area, oi);
    std::copy(&bbox[4 * i], &bbox[4 * i] + 4, P->star_bb);
    plan_alloc(P, st);
    B->ge[i] = std::make_unique<GridExec>();
    gridexec_alloc(*P, g[i], 0, g[i].ny, *B->ge[i], st);
  }
  // one sort for every field's tree: keys (field << shift) | leaf key, when
  // they fit 32 bits
  std::vector<TreeJob> jobs;
  std::vector<int> job_field;
  int shift = 0;
  int64_t total = 0;
  for (int i = 0; i < n; ++i) {
    lens_plan *P = B->plans[i];
    if (!P) continue;
    TreeJob t{};
    t.xy = f[i].xy;
    t.q = f[i].m;
    t.sxy = static_cast<double *>(P->sxy.ptr);
    t.sq = static_cast<double *>(P->sm.ptr);
    t.sq32 = static_cast<float *>(P->sm32.ptr);
    t.g = P->g;
    t.off = total;
    t.n = P->n_stars;
    total += P->n_stars;
    shift = std::max(shift, 2 * P->g.L);
    jobs.push_back(t);
    job_field.push_back(i);
  }
  int fbits = 0;
  while ((size_t(1) << fbits) < jobs.size()) ++fbits;
  const bool multi = jobs.size() >= 2 && shift + fbits <= 32 &&
                     total < (int64_t)std::numeric_limits<int32_t>::max();
  uint32_t *mk = nullptr, *mv = nullptr, *mkt = nullptr, *mvt = nullptr, *mcnt = nullptr, *mscan = nullptr;
  TreeJob *jobs_dev = nullptr;
  if (multi) {
    auto grab = [&](size_t bytes) {
      B->tree.push_back(pool_get(bytes, st));
      return B->tree.back().ptr;
    };
    jobs_dev = static_cast<TreeJob *>(grab(jobs.size() * sizeof(TreeJob)));
    mk = static_cast<uint32_t *>(grab((size_t)total * 4));
    mv = static_cast<uint32_t *>(grab((size_t)total * 4));
    mkt = static_cast<uint32_t *>(grab((size_t)total * 4));
    mvt = static_cast<uint32_t *>(grab((size_t)total * 4));
    const size_t ncnt = radix_counts_len(total);
    mcnt = static_cast<uint32_t *>(grab(ncnt * 4));
    mscan = static_cast<uint32_t *>(grab(scan_tmp_len(ncnt) * 4));
    LENS_HIP(hipMemcpyAsync(jobs_dev, jobs.data(), jobs.size() * sizeof(TreeJob), hipMemcpyHostToDevice, st));
  }
  LENS_HIP(hipStreamCreateWithFlags(&B->origin, hipStreamNonBlocking));
  B->side.assign(kSideStreams, nullptr);
  for (auto &s : B->side) LENS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  B->ev.assign(kSideStreams + 1, nullptr);
  for (auto &e : B->ev) LENS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  // the buffers above were handed out on `st`; the graph runs after it
  LENS_HIP(hipStreamSynchronize(st));

  set_capturing(true);
  hipError_t began = hipStreamBeginCapture(B->origin, hipStreamCaptureModeThreadLocal);
  if (began != hipSuccess) {
    set_capturing(false);
    LENS_HIP(began);
  }
  try {
    const uint32_t *msk = nullptr, *msv = nullptr;
    if (multi) {
      launch_leaf_keys_multi(jobs_dev, (int)jobs.size(), total, shift, mk, mv, B->origin);
      const bool in_tmp = radix_sort_pairs(mk, mv, mkt, mvt, total, shift + fbits, mcnt, mscan, B->origin);
      uint32_t *ks = in_tmp ? mkt : mk;
      msv = in_tmp ? mvt : mv;
      launch_gather_multi(jobs_dev, (int)jobs.size(), total, (uint32_t)((uint64_t(1) << shift) - 1), ks,
                          msv, B->origin);
      msk = ks;
    }
    LENS_HIP(hipEventRecord(B->ev[0], B->origin));
    for (auto s : B->side) LENS_HIP(hipStreamWaitEvent(s, B->ev[0], 0));
    size_t job = 0;
    for (int i = 0; i < n; ++i) {
      hipStream_t s = B->side[i % kSideStreams];
      const double c1 = (1.0 - f[i].kappa_s) - f[i].gamma;
      const double c2 = (1.0 - f[i].kappa_s) + f[i].gamma;
      if (!B->plans[i]) {
        DirectArgs d{};
        d.n_stars = f[i].n_stars;
        d.sxy = f[i].xy;
        d.sm = f[i].m;
        d.grid_mode = 1;
        d.grid = g[i];
        d.n_rays = g[i].nx * g[i].ny;
        d.c1 = c1;
        d.c2 = c2;
        d.counts = m[i].counts;
        d.y1min = m[i].y1min;
        d.y2min = m[i].y2min;
        d.S = (double)m[i].npix / m[i].side;
        d.npix = m[i].npix;
        launch_direct(d, s);
        continue;
      }
      lens_plan *P = B->plans[i];
      if (multi) {
        // the field's segment of the combined sort: its leaf starts, then P2M / M2M
        const TreeJob &t = jobs[job++];
        P->perm = msv + t.off;
        launch_box_starts(msk + t.off, t.n, int64_t(1) << (2 * P->g.L),
                          static_cast<int32_t *>(P->leaf_start.ptr),
                          static_cast<int32_t *>(P->box_coarse.ptr), s);
        plan_upward(P, s);
      } else {
        plan_enqueue(P, f[i].xy, f[i].m, s);
      }
      gridexec_enqueue(*P, *B->ge[i], c1, c2, nullptr, &m[i], s);
    }
    for (int j = 0; j < kSideStreams; ++j) {
      LENS_HIP(hipEventRecord(B->ev[j + 1], B->side[j]));
      LENS_HIP(hipStreamWaitEvent(B->origin, B->ev[j + 1], 0));
    }
  } catch (...) {
    hipGraph_t tmp = nullptr;
    (void)hipStreamEndCapture(B->origin, &tmp);
    if (tmp) (void)hipGraphDestroy(tmp);
    set_capturing(false);
    (void)hipGetLastError();
    throw;
  }
  const hipError_t ended = hipStreamEndCapture(B->origin, &B->graph);
  set_capturing(false);
  LENS_HIP(ended);
  LENS_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
  return B;
}

}  // namespace

namespace {

// ------------------------------------------------------------ call graphs
// lens_deflect / lens_map over a ray grid without a caller's plan: once the
// stars' bounding box is read back (the one wait), the rest of the call --
// tree build, upward pass, downward pass, evaluation -- is the same kernel
// sequence whenever the input addresses and sizes, the options, the smooth
// terms and the tree geometry repeat.  The second time such a call is seen
// that sequence is captured into a HIP graph (on a private stream, with the
// buffers it uses kept alive) and from then on replayed with one launch.
// The stage profiler needs eager launches, so calls made while it is on run
// eagerly.
std::atomic<uint64_t> g_call_ids{1};

struct CallExec {
  std::vector<uint64_t> key, skey;  // full key; its part independent of star positions
  uint64_t id = g_call_ids.fetch_add(1);  // never reused
  lens_plan *P = nullptr;
  GridExec ge;
  hipStream_t origin = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last = nullptr;

  ~CallExec() {
    if (last) (void)hipStreamSynchronize(last);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (P) {
      P->put_all(nullptr);
      delete P;
    }
    ge.put_all(nullptr);
    if (origin) (void)hipStreamDestroy(origin);
  }
};

constexpr size_t kCallCache = 4;
std::mutex g_call_mu;
std::vector<std::unique_ptr<CallExec>> g_calls;        // most recently used last
std::vector<std::vector<uint64_t>> g_call_seen;         // keys seen once

// A non-blocking stream beside a caller's stream (default priority) and an
// event to start it behind the caller's work: the speculative replay's
// bounding-box reduction runs there.  One per (device, stream) of the
// calling host thread, kept for the thread's life (a few at most).
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr;
};

const SideStream &side_stream_for(hipStream_t st) {
  thread_local std::vector<std::pair<std::pair<int, hipStream_t>, SideStream>> sides;
  int dev = 0;
  LENS_HIP(hipGetDevice(&dev));
  for (auto &e : sides)
    if (e.first.first == dev && e.first.second == st) return e.second;
  if (sides.size() >= 8) {
    // stale entries (streams the caller may have destroyed): drop the oldest
    SideStream &old = sides.front().second;
    (void)hipStreamSynchronize(old.stream);
    (void)hipEventDestroy(old.start);
    (void)hipStreamDestroy(old.stream);
    sides.erase(sides.begin());
  }
  SideStream s;
  LENS_HIP(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
  LENS_HIP(hipEventCreateWithFlags(&s.start, hipEventDisableTiming));
  sides.emplace_back(std::make_pair(dev, st), s);
  return sides.back().second;
}

// The parts of a call's key that do not depend on the stars' positions.
std::vector<uint64_t> call_key_static(const lens_field &f, const lens_grid &g, const lens_opts &o,
                                      const double *y_out, const lens_map_desc *map, int device,
                                      hipStream_t st) {
  std::vector<uint64_t> k;
  key_push(k, (int64_t)device);
  key_push(k, (const void *)st);  // replays on one stream are ordered; others get their own
  key_push(k, (const void *)f.xy);
  key_push(k, (const void *)f.m);
  key_push(k, f.n_stars);
  key_push(k, f.kappa_s);
  key_push(k, f.gamma);
  key_push(k, g.x0);
  key_push(k, g.y0);
  key_push(k, g.dx);
  key_push(k, g.dy);
  key_push(k, g.nx);
  key_push(k, g.ny);
  key_push(k, (int64_t)o.precision);
  key_push(k, (int64_t)o.order_p);
  key_push(k, (int64_t)o.fp32_levels);
  key_push(k, (int64_t)o.leaf_level);
  key_push(k, (const void *)y_out);
  if (map) {
    key_push(k, map->y1min);
    key_push(k, map->y2min);
    key_push(k, map->side);
    key_push(k, (int64_t)map->npix);
    key_push(k, (const void *)map->counts);
  }
  return k;
}

std::vector<uint64_t> call_key(const lens_field &f, const lens_grid &g, const lens_opts &o,
                               const double *y_out, const lens_map_desc *map, const lens_plan &P,
                               hipStream_t st) {
  std::vector<uint64_t> k = call_key_static(f, g, o, y_out, map, P.device, st);
  key_push(k, P.g.x0);
  key_push(k, P.g.y0);
  key_push(k, P.g.side);
  key_push(k, (int64_t)P.g.L);
  return k;
}

// The whole grid in one pass through the call-graph cache (see above).
void fmm_grid_call(const lens_field &f, const lens_grid &grid, const lens_opts &o, double c1,
                   double c2, double *y_out, const lens_map_desc *map, double S,
                   hipStream_t st,
                   double *dfdz = nullptr) {
  double bb[4];
  grid_bbox(grid, 0, grid.ny, bb);
  double sb[4];
  int64_t cnt = 0;
  // Speculation (outputs that the call overwrites, not maps that it adds
  // to): replay the latest graph of this call's arrays and parameters at
  // once, and check its tree against the stars' bounding box, reduced on a
  // side stream (it only reads the stars) while the graph runs; if the stars
  // have moved out of the tree, the call below runs again and overwrites the
  // outputs.  Without a graph to replay the reduction runs on the stream.
  int dev = 0;
  LENS_HIP(hipGetDevice(&dev));
  std::vector<uint64_t> skey;
  uint64_t spec = 0;  // id of the graph replayed speculatively
  BBoxRead rd;
  std::unique_lock<std::mutex> lk(g_call_mu);
  if (!map && !profiling_enabled()) {
    skey = call_key_static(f, grid, o, y_out, map, dev, st);
    key_push(skey, (const void *)dfdz);
    for (size_t i = g_calls.size(); i-- > 0;)
      if (g_calls[i]->skey == skey) {
        spec = g_calls[i]->id;
        const SideStream &side = side_stream_for(st);
        LENS_HIP(hipEventRecord(side.start, st));
        LENS_HIP(hipStreamWaitEvent(side.stream, side.start, 0));
        rd = bbox_enqueue(f.xy, f.n_stars, side.stream, bb);
        LENS_HIP(hipGraphLaunch(g_calls[i]->exec, st));
        g_calls[i]->last = st;
        break;
      }
  }
  lk.unlock();
  if (!spec) rd = bbox_enqueue(f.xy, f.n_stars, st, bb);
  bbox_finish(rd, sb, &cnt);
  const double rho_local = local_density(cnt, bb);
  const double area = std::max((bb[2] - bb[0]) * (bb[3] - bb[1]), 1e-300);
  const double density = (double)(grid.nx * grid.ny) / area;
  auto eager = [&] {
    lens_plan *P = build_plan(f, bb, &grid, density, o, st, nullptr, sb, rho_local);
    try {
      fmm_grid_rows(*P, grid, 0, grid.ny, c1, c2, y_out, map, S, st, dfdz);
    } catch (...) {
      lens_plan_destroy(P);
      throw;
    }
    release_owned(P, st);
  };
  if (profiling_enabled()) return eager();
  // host-side geometry only, to form the key
  lens_plan probe;
  LENS_HIP(hipGetDevice(&probe.device));
  plan_geometry(&probe, f.n_stars, sb, bb, &grid, density, o, rho_local);
  auto key = call_key(f, grid, o, y_out, map, probe, st);
  key_push(key, (const void *)dfdz);
  lk.lock();
  for (size_t i = 0; i < g_calls.size(); ++i)
    if (g_calls[i]->key == key) {
      std::unique_ptr<CallExec> c = std::move(g_calls[i]);
      g_calls.erase(g_calls.begin() + (long)i);
      if (c->id != spec) LENS_HIP(hipGraphLaunch(c->exec, st));  // else it already ran
      c->last = st;
      g_calls.push_back(std::move(c));
      return;
    }
  if (std::find(g_call_seen.begin(), g_call_seen.end(), key) == g_call_seen.end()) {
    g_call_seen.push_back(key);
    if (g_call_seen.size() > 16) g_call_seen.erase(g_call_seen.begin());
    return eager();
  }
  auto c = std::make_unique<CallExec>();
  c->key = key;
  c->skey = skey;
  auto *P = new lens_plan();
  c->P = P;
  P->device = probe.device;
  P->kappa_s = f.kappa_s;
  P->gamma = f.gamma;
  plan_geometry(P, f.n_stars, sb, bb, &grid, density, o, rho_local);
  std::copy(sb, sb + 4, P->star_bb);
  (void)op_tables(o.order_p, st);
  plan_alloc(P, st);
  gridexec_alloc(*P, grid, 0, grid.ny, c->ge, st);
  LENS_HIP(hipStreamCreateWithFlags(&c->origin, hipStreamNonBlocking));
  LENS_HIP(hipStreamSynchronize(st));  // the buffers above were handed out on st
  set_capturing(true);
  hipError_t began = hipStreamBeginCapture(c->origin, hipStreamCaptureModeThreadLocal);
  if (began != hipSuccess) {
    set_capturing(false);
    LENS_HIP(began);
  }
  try {
    plan_enqueue(P, f.xy, f.m, c->origin);
    gridexec_enqueue(*P, c->ge, c1, c2, y_out, map, c->origin, dfdz);
  } catch (...) {
    hipGraph_t tmp = nullptr;
    (void)hipStreamEndCapture(c->origin, &tmp);
    if (tmp) (void)hipGraphDestroy(tmp);
    set_capturing(false);
    (void)hipGetLastError();
    throw;
  }
  const hipError_t ended = hipStreamEndCapture(c->origin, &c->graph);
  set_capturing(false);
  LENS_HIP(ended);
  LENS_HIP(hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0));
  LENS_HIP(hipGraphLaunch(c->exec, st));
  c->last = st;
  if (g_calls.size() >= kCallCache) g_calls.erase(g_calls.begin());
  g_calls.push_back(std::move(c));
}

}  // namespace

namespace lensfmm {

// Grid deflection with a plan into a caller-provided device region: no
// device memory is allocated.  The grid is split into bands of whole rows
// whose per-call buffers (locals of every level, ray ranges) fit in
// `bytes`, evaluated one after another on the stream in the same region.
// Every band is planned on the host before anything is enqueued.
void deflect_grid_no_alloc(lens_plan *plan, const lens_field *field, const lens_grid *grid,
                           double *y_out, const lens_opts *opts, char *region, size_t bytes,
                           hipStream_t st, double *dfdz) {
  if (!plan) fail(LENS_EINVAL, "plan is NULL (the allocation-free deflection needs a plan)");
  const lens_opts o = resolve_opts(opts);
  FieldView fv = field_for(plan, field);
  check_plan_device(plan);
  if (!grid) fail(LENS_EINVAL, "grid is NULL");
  check_grid(grid);
  const int64_t n = grid->nx * grid->ny;
  if (n > (int64_t)std::numeric_limits<uint32_t>::max() - 1) fail(LENS_EINVAL, "grid exceeds 2^32-2 rays");
  if (n == 0) return;
  if (!y_out) fail(LENS_EINVAL, "y_out is NULL");
  const double c1 = (1.0 - fv.f.kappa_s) - fv.f.gamma;
  const double c2 = (1.0 - fv.f.kappa_s) + fv.f.gamma;
  NoTiming quiet;  // no stage events either
  if (o.method == LENS_DIRECT || fv.f.n_stars == 0) {
    DirectArgs d{};
    d.n_stars = fv.f.n_stars;
    d.sxy = fv.f.xy;
    d.sm = fv.f.m;
    d.grid_mode = 1;
    d.grid = *grid;
    d.n_rays = n;
    d.c1 = c1;
    d.c2 = c2;
    d.y_out = y_out;
    d.dfdz_out = dfdz;
    launch_direct(d, st);
    return;
  }
  if (!op_tables_if_built(plan->p))
    fail(LENS_EUNSUPPORTED, "operator tables of the plan's order are not on this device");
  double bb[4];
  grid_bbox(*grid, 0, grid->ny, bb);
  check_inside(*plan, bb);
  std::vector<std::pair<int64_t, int64_t>> bands;
  for (int64_t j0 = 0; j0 < grid->ny;) {
    const size_t one = gridexec_bytes(*plan, *grid, j0, j0 + 1);
    if (one > bytes)
      fail(LENS_ENOMEM, "one grid row needs " + std::to_string(one) +
                            " bytes of scratch, more than the " + std::to_string(bytes) +
                            " bytes of the allocation-free workspace");
    int64_t lo = j0 + 1, hi = grid->ny;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (gridexec_bytes(*plan, *grid, j0, mid) <= bytes) lo = mid; else hi = mid - 1;
    }
    bands.emplace_back(j0, lo);
    j0 = lo;
  }
  for (const auto &b : bands) {
    GridExec ge;
    gridexec_alloc(*plan, *grid, b.first, b.second, ge, st, region);
    gridexec_enqueue(*plan, ge, c1, c2, y_out, nullptr, st, dfdz);
  }
  plan->last_stream = st;
}

}  // namespace lensfmm

extern "C" {

void lens_opts_default(lens_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->method = LENS_FMM;
  o->precision = LENS_MIXED;
  o->order_p = 12;
  o->leaf_level = 0;
  o->max_rays_per_chunk = 0;
}

const char *lens_last_error(void) { return lensfmm::last_error().c_str(); }

const char *lens_version(void) { return "liblensfmm 0.1 (gfx950)"; }

lens_status lens_plan_create(const lens_field *field, const double *ray_box, const lens_grid *grid,
                             const lens_opts *opts, void *stream, lens_plan **out) {
  return guarded([&] {
    if (!out) fail(LENS_EINVAL, "out is NULL");
    check_field(field);
    lens_opts o = resolve_opts(opts);
    if (wants_auto(opts) && field->n_stars > 0) {
      if (!grid || grid->nx * grid->ny == 0)
        fail(LENS_EINVAL, "order_p = 0 with tol > 0 needs a grid to tune on");
      check_grid(grid);
      o = auto_opts(*field, *grid, nullptr, *opts, (hipStream_t)stream);
    }
    double gbox[4];
    if (grid) {
      check_grid(grid);
      if (grid->nx > 0 && grid->ny > 0) {
        grid_bbox(*grid, 0, grid->ny, gbox);
        if (ray_box) {
          gbox[0] = std::min(gbox[0], ray_box[0]);
          gbox[1] = std::min(gbox[1], ray_box[1]);
          gbox[2] = std::max(gbox[2], ray_box[2]);
          gbox[3] = std::max(gbox[3], ray_box[3]);
        }
        ray_box = gbox;
      }
    }
    if (ray_box) {
      for (int c = 0; c < 4; ++c)
        if (!is_finite(ray_box[c])) fail(LENS_EINVAL, "ray_box must be finite");
      if (ray_box[2] < ray_box[0] || ray_box[3] < ray_box[1]) fail(LENS_EINVAL, "ray_box is empty");
    }
    // with a grid, the leaf level is chosen for its ray density, as for the
    // plans lens_deflect and lens_map build themselves
    double density = 0.0;
    if (grid && grid->nx > 0 && grid->ny > 0) {
      const double area = std::max((gbox[2] - gbox[0]) * (gbox[3] - gbox[1]), 1e-300);
      density = (double)(grid->nx * grid->ny) / area;
    }
    *out = build_plan(*field, ray_box, grid, density, o, (hipStream_t)stream);
  });
}

void lens_plan_destroy(lens_plan *plan) {
  if (!plan) return;
  // stream-ordered: the buffers go back to the pool behind the plan's last
  // work, and a later reuse on another stream waits for it
  plan->put_all(plan->last_stream);
  delete plan;
}

lens_status lens_plan_info(const lens_plan *plan, int32_t *order_p, int32_t *leaf_level,
                           double *root_x0, double *root_y0, double *root_side) {
  return guarded([&] {
    if (!plan) fail(LENS_EINVAL, "plan is NULL");
    if (order_p) *order_p = plan->p;
    if (leaf_level) *leaf_level = plan->g.L;
    if (root_x0) *root_x0 = plan->g.x0;
    if (root_y0) *root_y0 = plan->g.y0;
    if (root_side) *root_side = plan->g.side;
  });
}

lens_status lens_deflect(lens_plan *plan, const lens_field *field, const lens_grid *grid,
                         const double *rays_xy, int64_t n_rays, double *y_out, double *dfdz_out,
                         const lens_opts *opts, void *stream) {
  return guarded([&] {
    hipStream_t st = (hipStream_t)stream;
    lens_opts o = resolve_opts(opts);
    FieldView fv = field_for(plan, field);
    if (plan) check_plan_device(plan);
    if ((grid == nullptr) == (rays_xy == nullptr) && !(grid == nullptr && n_rays == 0))
      fail(LENS_EINVAL, "give exactly one of grid and rays_xy");
    if (n_rays < 0) fail(LENS_EINVAL, "n_rays < 0");
    if (grid) {
      check_grid(grid);
      if (n_rays != grid->nx * grid->ny) fail(LENS_EINVAL, "n_rays must equal grid.nx * grid.ny");
    }
    if (n_rays > (int64_t)std::numeric_limits<uint32_t>::max() - 1)
      fail(LENS_EINVAL, "n_rays exceeds 2^32-2");
    if (n_rays > 0 && !y_out) fail(LENS_EINVAL, "y_out is NULL");
    if (n_rays == 0) return;
    const double c1 = (1.0 - fv.f.kappa_s) - fv.f.gamma;
    const double c2 = (1.0 - fv.f.kappa_s) + fv.f.gamma;

    if (plan && grid && o.workspace && o.method == LENS_FMM && fv.f.n_stars > 0) {
      // the caller's workspace instead of the pool, in bands of rows that fit
      deflect_grid_no_alloc(plan, field, grid, y_out, &o, static_cast<char *>(o.workspace),
                            o.workspace_bytes, st, dfdz_out);
      return;
    }
    if (o.method == LENS_DIRECT || fv.f.n_stars == 0) {
      DirectArgs d{};
      d.n_stars = fv.f.n_stars;
      d.sxy = fv.f.xy;
      d.sm = fv.f.m;
      d.grid_mode = grid != nullptr;
      if (grid) d.grid = *grid;
      d.rxy = rays_xy;
      d.n_rays = n_rays;
      d.c1 = c1;
      d.c2 = c2;
      d.y_out = y_out;
      d.dfdz_out = dfdz_out;
      StageTimer tm("direct", st);
      launch_direct(d, st);
      return;
    }

    if (!plan && grid) {
      if (wants_auto(opts)) o = auto_opts(fv.f, *grid, nullptr, *opts, st);
      fmm_grid_call(fv.f, *grid, o, c1, c2, y_out, nullptr, 0.0, st, dfdz_out);
      return;
    }
    double bb[4];
    if (grid) {
      grid_bbox(*grid, 0, grid->ny, bb);
    } else {
      device_bbox(rays_xy, n_rays, st, bb);
    }
    if (!plan && wants_auto(opts)) o = auto_opts(fv.f, tuning_grid(bb), nullptr, *opts, st);
    lens_plan *P = plan;
    lens_plan *owned = nullptr;
    if (!P) {
      const double area = std::max((bb[2] - bb[0]) * (bb[3] - bb[1]), 1e-300);
      owned = P = build_plan(fv.f, bb, grid, (double)n_rays / area, o, st);
    }
    try {
      if (grid)
        fmm_grid_rows(*P, *grid, 0, grid->ny, c1, c2, y_out, nullptr, 0.0, st, dfdz_out);
      else
        fmm_explicit(*P, rays_xy, n_rays, bb, c1, c2, y_out, st, dfdz_out);
    } catch (...) {
      if (owned) lens_plan_destroy(owned);
      throw;
    }
    if (owned) release_owned(owned, st);
  });
}

lens_status lens_map(lens_plan *plan, const lens_field *field, const lens_grid *grid,
                     const lens_map_desc *map, const lens_opts *opts, void *stream) {
  return guarded([&] {
    hipStream_t st = (hipStream_t)stream;
    lens_opts o = resolve_opts(opts);
    FieldView fv = field_for(plan, field);
    if (plan) check_plan_device(plan);
    if (!grid) fail(LENS_EINVAL, "grid is NULL");
    check_grid(grid);
    if (!map) fail(LENS_EINVAL, "map is NULL");
    if (map->npix <= 0) fail(LENS_EINVAL, "map.npix must be > 0");
    if ((int64_t)map->npix * map->npix > (int64_t)std::numeric_limits<int32_t>::max())
      fail(LENS_EINVAL, "map.npix^2 exceeds 2^31-1");
    if (!is_finite(map->y1min) || !is_finite(map->y2min) || !is_finite(map->side) || !(map->side > 0))
      fail(LENS_EINVAL, "map placement must be finite with side > 0");
    if (!map->counts) fail(LENS_EINVAL, "map.counts is NULL");
    const int64_t n = grid->nx * grid->ny;
    if (n > (int64_t)std::numeric_limits<int32_t>::max())
      fail(LENS_EINVAL, "a map call may shoot at most 2^31-1 rays (int32 counts)");
    if (n == 0) return;
    const double c1 = (1.0 - fv.f.kappa_s) - fv.f.gamma;
    const double c2 = (1.0 - fv.f.kappa_s) + fv.f.gamma;
    const double S = (double)map->npix / map->side;
    if (!plan && fv.f.n_stars > 0 && wants_auto(opts)) o = auto_opts(fv.f, *grid, map, *opts, st);
    const int64_t rows = std::max<int64_t>(1, o.max_rays_per_chunk / std::max<int64_t>(grid->nx, 1));

    if (o.method == LENS_DIRECT || fv.f.n_stars == 0) {
      for (int64_t j0 = 0; j0 < grid->ny; j0 += rows) {
        const int64_t j1 = std::min(grid->ny, j0 + rows);
        DirectArgs d{};
        d.n_stars = fv.f.n_stars;
        d.sxy = fv.f.xy;
        d.sm = fv.f.m;
        d.grid_mode = 1;
        d.grid = *grid;
        d.n_rays = (j1 - j0) * grid->nx;
        d.ray_offset = j0 * grid->nx;
        d.c1 = c1;
        d.c2 = c2;
        d.counts = map->counts;
        d.y1min = map->y1min;
        d.y2min = map->y2min;
        d.S = S;
        d.npix = map->npix;
        StageTimer tm("direct_map", st);
        launch_direct(d, st);
      }
      return;
    }
    if (!plan && rows >= grid->ny) {
      fmm_grid_call(fv.f, *grid, o, c1, c2, nullptr, map, S, st);
      return;
    }
    double bb[4];
    grid_bbox(*grid, 0, grid->ny, bb);
    lens_plan *P = plan;
    lens_plan *owned = nullptr;
    if (!P) {
      const double area = std::max((bb[2] - bb[0]) * (bb[3] - bb[1]), 1e-300);
      owned = P = build_plan(fv.f, bb, grid, (double)n / area, o, st);
    }
    try {
      for (int64_t j0 = 0; j0 < grid->ny; j0 += rows) {
        const int64_t j1 = std::min(grid->ny, j0 + rows);
        fmm_grid_rows(*P, *grid, j0, j1, c1, c2, nullptr, map, S, st);
      }
    } catch (...) {
      if (owned) lens_plan_destroy(owned);
      throw;
    }
    if (owned) release_owned(owned, st);
  });
}

lens_status lens_map_ipm(lens_plan *plan, const lens_field *field, const lens_grid *grid,
                         const lens_ipm_desc *map, const lens_opts *opts, void *stream) {
  return guarded([&] {
    hipStream_t st = (hipStream_t)stream;
    lens_opts o = resolve_opts(opts);
    FieldView fv = field_for(plan, field);
    if (plan) check_plan_device(plan);
    if (!grid) fail(LENS_EINVAL, "grid is NULL");
    check_grid(grid);
    if (!map) fail(LENS_EINVAL, "map is NULL");
    if (map->npix <= 0) fail(LENS_EINVAL, "map.npix must be > 0");
    if ((int64_t)map->npix * map->npix > (int64_t)std::numeric_limits<int32_t>::max())
      fail(LENS_EINVAL, "map.npix^2 exceeds 2^31-1");
    if (!is_finite(map->y1min) || !is_finite(map->y2min) || !is_finite(map->side) || !(map->side > 0))
      fail(LENS_EINVAL, "map placement must be finite with side > 0");
    if (!map->mu) fail(LENS_EINVAL, "map.mu is NULL");
    const int64_t nx = grid->nx, ny = grid->ny;
    if (nx < 2 || ny < 2) return;  // no cells
    const double c1 = (1.0 - fv.f.kappa_s) - fv.f.gamma;
    const double c2 = (1.0 - fv.f.kappa_s) + fv.f.gamma;
    const double S = (double)map->npix / map->side;
    const double cell_px = grid->dx * grid->dy * S * S;
    if (!plan && fv.f.n_stars > 0 && wants_auto(opts)) {
      // tuned for bin reassignment in a map of the same placement
      const lens_map_desc md{map->y1min, map->y2min, map->side, map->npix, nullptr};
      o = auto_opts(fv.f, *grid, &md, *opts, st);
    }
    // cell rows per pass (each pass deflects its rows plus the next one):
    // by default passes of about kIpmPassRays rays, and never more cells than
    // a pass's 32-bit cell indices can name
    const int64_t chunk = opts && opts->max_rays_per_chunk > 0 ? o.max_rays_per_chunk : kIpmPassRays;
    const int64_t rows = std::max<int64_t>(
        1, std::min<int64_t>({ny - 1, chunk / nx - 1, kIpmPassCellsMax / (nx - 1)}));
    Scratch sc(st);
    const int64_t npx = (int64_t)map->npix * map->npix;
    const int64_t ndiff = (int64_t)map->npix * (map->npix + 1);
    auto *acc = sc.get<unsigned long long>((size_t)npx);
    auto *diff = sc.get<unsigned long long>((size_t)ndiff);
    launch_ipm_zero(acc, npx, st);
    launch_ipm_zero(diff, ndiff, st);
    auto *queue = sc.get<uint32_t>((size_t)rows * (nx - 1));
    auto *qcount = sc.get<uint32_t>(1);
    double *ybuf = sc.get<double>((size_t)(rows + 1) * nx * 2);
    lens_plan *P = plan;
    lens_plan *owned = nullptr;
    const bool direct = o.method == LENS_DIRECT || fv.f.n_stars == 0;
    if (!P && !direct) {
      double bb[4];
      grid_bbox(*grid, 0, ny, bb);
      const double area = std::max((bb[2] - bb[0]) * (bb[3] - bb[1]), 1e-300);
      owned = P = build_plan(fv.f, bb, grid, (double)(nx * ny) / area, o, st);
    }
    try {
      for (int64_t j0 = 0; j0 < ny - 1; j0 += rows) {
        const int64_t j1 = std::min(ny - 1, j0 + rows);  // cell rows [j0, j1) need ray rows [j0, j1]
        // the kernels write ray (i, j) at y_out[2 (j nx + i)]: shift the base
        // so that row j0 lands at the start of ybuf
        double *y_out = reinterpret_cast<double *>(reinterpret_cast<uintptr_t>(ybuf) -
                                                   (uintptr_t)(j0 * nx) * 2 * sizeof(double));
        if (direct) {
          DirectArgs d{};
          d.n_stars = fv.f.n_stars;
          d.sxy = fv.f.xy;
          d.sm = fv.f.m;
          d.grid_mode = 1;
          d.grid = *grid;
          d.n_rays = (j1 + 1 - j0) * nx;
          d.ray_offset = j0 * nx;
          d.c1 = c1;
          d.c2 = c2;
          d.y_out = y_out;
          StageTimer tm("direct", st);
          launch_direct(d, st);
        } else {
          fmm_grid_rows(*P, *grid, j0, j1 + 1, c1, c2, y_out, nullptr, 0.0, st);
        }
        StageTimer tm("ipm", st);
        const IpmPass pass{ybuf, nx, j0, j0, j1, cell_px, map->y1min, map->y2min, S, map->npix,
                           acc, diff, queue, qcount};
        launch_ipm_cells(pass, st);
      }
      StageTimer tm("ipm", st);
      launch_ipm_finish(acc, diff, map->npix, map->mu, st);
    } catch (...) {
      if (owned) lens_plan_destroy(owned);
      throw;
    }
    if (owned) release_owned(owned, st);
  });
}

}  // extern "C"

namespace {

// Adjoint FMM with a forward plan: the rays (charges g_k) are sources in a
// tree of the plan's geometry, the plan's sorted stars are the targets (its
// leaf starts locate each box's stars, its permutation the caller's order).
void backward_with_plan(lens_plan &F, const double *rays, int64_t n_rays, const double rb[4],
                        const double *grad_y, double *grad_xy, double *grad_m, hipStream_t st) {
  const double x1 = F.g.x0 + F.g.side, y1 = F.g.y0 + F.g.side;
  if (rb[0] < F.g.x0 || rb[1] < F.g.y0 || rb[2] > x1 || rb[3] > y1)
    fail(LENS_EINVAL, "rays lie outside the plan's root square (pass ray_box to lens_plan_create)");
  Scratch sc(st);
  auto *A = new lens_plan();
  try {
    A->device = F.device;
    A->qdim = 2;
    A->p = F.p;
    A->precision = F.precision;
    A->fine_levels = F.fine_levels;
    A->n_stars = n_rays;
    A->g = F.g;
    std::copy(F.star_bb, F.star_bb + 4, A->target);
    A->domain[0] = F.g.x0, A->domain[1] = F.g.y0, A->domain[2] = x1, A->domain[3] = y1;
    std::copy(rb, rb + 4, A->star_bb);
    source_windows(A);
    plan_alloc(A, st);
    plan_enqueue(A, rays, grad_y, st);
    double *loc = nullptr;
    const Window wl = downward(*A, F.star_bb, sc, st, &loc);
    EvalArgs ea{};
    fill_star_side(*A, wl, loc, ea);
    const int64_t per = (F.n_stars + wl.count() - 1) / std::max<int64_t>(wl.count(), 1);
    ea.chunks_per_box =
        std::max<int64_t>(1, (per + adj_targets_per_unit() - 1) / adj_targets_per_unit());
    while (wl.count() * ea.chunks_per_box > (int64_t)0x7fffffff && ea.chunks_per_box > 1)
      ea.chunks_per_box = (ea.chunks_per_box + 1) / 2;
    AdjArgs d{static_cast<const double *>(A->sm.ptr), static_cast<const double *>(F.sxy.ptr),
              static_cast<const double *>(F.sm.ptr), F.perm,
              static_cast<const int32_t *>(F.leaf_start.ptr), grad_xy, grad_m, true};
    StageTimer tme("eval_adjoint", st);
    launch_eval_adj(ea, d, A->precision, st);
  } catch (...) {
    lens_plan_destroy(A);
    throw;
  }
  release_owned(A, st);
  F.last_stream = st;
}

// grad[0, n) = 0 by a kernel (no memset node if the caller captures a graph)
void zero_f64(double *p, int64_t n, hipStream_t st) {
  launch_fill_u32(reinterpret_cast<uint32_t *>(p), 2 * n, 0u, st);
}

// ---------------------------------------------- images, critical curves

// A ray grid deflected in passes of whole rows (by the plan or directly),
// each pass holding its cell rows plus the next ray row: the common frame of
// lens_find_images and lens_critical_curves.
struct GridPasses {
  const FieldView &fv;
  const lens_grid &grid;
  lens_plan *P;   // nullptr: direct sum
  double c1, c2;
  int64_t rows;   // cell rows per pass
  double *ybuf, *dbuf;

  // Deflect the ray rows [j0, j1] (y, and f' if dbuf) so that row j0 starts
  // the buffers.
  void deflect(int64_t j0, int64_t j1, hipStream_t st) {
    const int64_t nx = grid.nx;
    auto shifted = [&](double *b) {
      return b ? reinterpret_cast<double *>(reinterpret_cast<uintptr_t>(b) -
                                            (uintptr_t)(j0 * nx) * 2 * sizeof(double))
               : nullptr;
    };
    double *y_out = shifted(ybuf), *d_out = shifted(dbuf);
    if (!P) {
      DirectArgs d{};
      d.n_stars = fv.f.n_stars;
      d.sxy = fv.f.xy;
      d.sm = fv.f.m;
      d.grid_mode = 1;
      d.grid = grid;
      d.n_rays = (j1 + 1 - j0) * nx;
      d.ray_offset = j0 * nx;
      d.c1 = c1;
      d.c2 = c2;
      d.y_out = y_out;
      d.dfdz_out = d_out;
      StageTimer tm("direct", st);
      launch_direct(d, st);
    } else {
      fmm_grid_rows(*P, grid, j0, j1 + 1, c1, c2, y_out, nullptr, 0.0, st, d_out);
    }
  }
};

int64_t pass_rows(const lens_opts *opts, int64_t nx, int64_t ny) {
  const int64_t chunk = opts && opts->max_rays_per_chunk > 0 ? opts->max_rays_per_chunk : kIpmPassRays;
  return std::max<int64_t>(1, std::min<int64_t>({ny - 1, chunk / nx - 1, kIpmPassCellsMax / (nx - 1)}));
}

template <typename T>
T read_scalar(const T *d, hipStream_t st) {
  T v{};
  LENS_HIP(hipMemcpyAsync(&v, d, sizeof(T), hipMemcpyDeviceToHost, st));
  LENS_HIP(hipStreamSynchronize(st));
  return v;
}

// Re-raise a failed inner library call with its own status and message.
void check_inner(lens_status r) {
  if (r != LENS_OK) fail(r, last_error());
}

}  // namespace

extern "C" {

lens_status lens_deflect_backward(lens_plan *plan, const lens_field *field, const lens_grid *grid,
                                  const double *rays_xy, int64_t n_rays, const double *grad_y,
                                  double *grad_xy, double *grad_m, const lens_opts *opts,
                                  void *stream) {
  return guarded([&] {
    hipStream_t st = (hipStream_t)stream;
    const lens_opts o = resolve_opts(opts);
    if (plan) {
      check_plan_device(plan);
      if (plan->qdim != 1) fail(LENS_EINVAL, "plan is not a star plan");
      if (field && field->n_stars != plan->n_stars)
        fail(LENS_EINVAL, "field.n_stars differs from the plan's");
      if (field && !is_finite(field->kappa_s + field->gamma))
        fail(LENS_EINVAL, "kappa_s and gamma must be finite");
    } else {
      check_field(field);
    }
    if ((grid == nullptr) == (rays_xy == nullptr) && !(grid == nullptr && n_rays == 0))
      fail(LENS_EINVAL, "give exactly one of grid and rays_xy");
    if (n_rays < 0) fail(LENS_EINVAL, "n_rays < 0");
    if (grid) {
      check_grid(grid);
      if (n_rays != grid->nx * grid->ny) fail(LENS_EINVAL, "n_rays must equal grid.nx * grid.ny");
    }
    if (n_rays > (int64_t)std::numeric_limits<int32_t>::max())
      fail(LENS_EINVAL, "n_rays exceeds 2^31-1");
    const int64_t N = plan ? plan->n_stars : field->n_stars;
    if (N == 0) return;
    if (!grad_xy || !grad_m) fail(LENS_EINVAL, "grad_xy / grad_m is NULL");
    if (n_rays > 0 && !grad_y) fail(LENS_EINVAL, "grad_y is NULL");
    const bool direct = o.method == LENS_DIRECT;
    if (direct && (!field || !field->xy || !field->m))
      fail(LENS_EINVAL, "LENS_DIRECT needs the field's star arrays");
    if (n_rays == 0) {
      zero_f64(grad_xy, 2 * N, st);
      zero_f64(grad_m, N, st);
      return;
    }
    Scratch sc(st);
    const double *rays = rays_xy;
    if (grid) {
      double *r = sc.get<double>((size_t)n_rays * 2);
      launch_grid_rays(*grid, r, st);
      rays = r;
    }
    if (direct) {
      StageTimer tm("direct_adjoint", st);
      launch_direct_adj(N, field->xy, field->m, n_rays, rays, grad_y, grad_xy, grad_m, st);
      return;
    }
    if (plan) {
      double rb[4];
      if (grid)
        grid_bbox(*grid, 0, grid->ny, rb);
      else
        device_bbox(rays_xy, n_rays, st, rb);
      backward_with_plan(*plan, rays, n_rays, rb, grad_y, grad_xy, grad_m, st);
      return;
    }
    // sources: the rays with complex charges g_k; targets: the stars
    double tb[4];
    device_bbox(field->xy, N, st, tb);
    const double area = std::max((tb[2] - tb[0]) * (tb[3] - tb[1]), 1e-300);
    lens_field src{n_rays, rays, nullptr, 0.0, 0.0};
    lens_plan *P = build_plan(src, tb, nullptr, (double)N / area, o, st, grad_y);
    try {
      double *loc = nullptr;
      const Window wl = downward(*P, tb, sc, st, &loc);
      uint32_t *k = sc.get<uint32_t>(N), *v = sc.get<uint32_t>(N);
      uint32_t *kt = sc.get<uint32_t>(N), *vt = sc.get<uint32_t>(N);
      const size_t ncnt = radix_counts_len(N);
      uint32_t *cnt = sc.get<uint32_t>(ncnt);
      uint32_t *stmp = sc.get<uint32_t>(scan_tmp_len(ncnt));
      double *txy = sc.get<double>((size_t)N * 2), *tm = sc.get<double>((size_t)N);
      int32_t *tstart = sc.get<int32_t>(wl.count() + 1);
      {
        StageTimer tmr("adjoint_targets", st);
        launch_ray_keys(field->xy, N, P->g, wl, k, v, st);
        int bits = 1;
        while ((int64_t(1) << bits) < wl.count()) ++bits;
        const bool in_tmp = radix_sort_pairs(k, v, kt, vt, N, bits, cnt, stmp, st);
        const uint32_t *ks = in_tmp ? kt : k;
        v = in_tmp ? vt : v;
        launch_gather_stars(v, field->xy, field->m, 1, N, txy, tm, nullptr, st);
        launch_box_starts(ks, N, wl.count(), tstart,
                          sc.get<int32_t>(box_starts_coarse_len(wl.count())), st);
      }
      EvalArgs ea{};
      fill_star_side(*P, wl, loc, ea);
      const int64_t per = (N + wl.count() - 1) / std::max<int64_t>(wl.count(), 1);
      ea.chunks_per_box =
          std::max<int64_t>(1, (per + adj_targets_per_unit() - 1) / adj_targets_per_unit());
      while (wl.count() * ea.chunks_per_box > (int64_t)0x7fffffff && ea.chunks_per_box > 1)
        ea.chunks_per_box = (ea.chunks_per_box + 1) / 2;
      AdjArgs d{static_cast<const double *>(P->sm.ptr), txy, tm, v, tstart, grad_xy, grad_m};
      StageTimer tme("eval_adjoint", st);
      launch_eval_adj(ea, d, P->precision, st);
    } catch (...) {
      lens_plan_destroy(P);
      throw;
    }
    release_owned(P, st);
  });
}

lens_status lens_map_batched(int32_t n_fields, const lens_field *fields, const lens_grid *grids,
                             const lens_map_desc *maps, const lens_opts *opts, void *stream) {
  return guarded([&] {
    hipStream_t st = (hipStream_t)stream;
    const lens_opts o = resolve_opts(opts);
    if (opts && opts->order_p == 0 && !(opts->tol >= 0 && is_finite(opts->tol)))
      fail(LENS_EINVAL, "opts.tol must be finite and >= 0");
    if (n_fields < 0) fail(LENS_EINVAL, "n_fields < 0");
    if (n_fields == 0) return;
    if (!fields || !grids || !maps) fail(LENS_EINVAL, "fields / grids / maps is NULL");
    for (int i = 0; i < n_fields; ++i) {
      const std::string at = " (field " + std::to_string(i) + ")";
      try {
        check_field(&fields[i]);
        check_grid(&grids[i]);
      } catch (const LensError &e) {
        fail(e.status, e.msg + at);
      }
      const lens_map_desc &m = maps[i];
      if (m.npix <= 0 || (int64_t)m.npix * m.npix > (int64_t)std::numeric_limits<int32_t>::max())
        fail(LENS_EINVAL, "map.npix out of range" + at);
      if (!is_finite(m.y1min) || !is_finite(m.y2min) || !is_finite(m.side) || !(m.side > 0))
        fail(LENS_EINVAL, "map placement must be finite with side > 0" + at);
      if (!m.counts) fail(LENS_EINVAL, "map.counts is NULL" + at);
      if (grids[i].nx * grids[i].ny > (int64_t)std::numeric_limits<int32_t>::max())
        fail(LENS_EINVAL, "a field may shoot at most 2^31-1 rays" + at);
    }
    int dev = 0;
    LENS_HIP(hipGetDevice(&dev));
    // bounding boxes of every field's stars: one pass, one read-back
    std::vector<double> bbox((size_t)4 * n_fields, 0.0);
    {
      Scratch sc(st);
      std::vector<BBoxSet> sets(n_fields);
      int64_t nmax = 1;
      for (int i = 0; i < n_fields; ++i) {
        sets[i] = BBoxSet{fields[i].xy, fields[i].n_stars};
        nmax = std::max(nmax, fields[i].n_stars);
      }
      const int parts = bbox_parts(nmax);
      auto *sets_d = sc.get<BBoxSet>(n_fields);
      double *partial = sc.get<double>((size_t)n_fields * parts * 4);
      double *out = sc.get<double>((size_t)n_fields * 4);
      LENS_HIP(hipMemcpyAsync(sets_d, sets.data(), sizeof(BBoxSet) * n_fields,
                              hipMemcpyHostToDevice, st));
      launch_bbox_multi(sets_d, n_fields, parts, partial, out, st);
      LENS_HIP(hipMemcpyAsync(bbox.data(), out, sizeof(double) * 4 * n_fields,
                              hipMemcpyDeviceToHost, st));
      LENS_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < n_fields; ++i)
        if (fields[i].n_stars > 0)
          for (int c = 0; c < 4; ++c)
            if (!is_finite(bbox[4 * i + c]))
              fail(LENS_EINVAL, "non-finite star coordinates (field " + std::to_string(i) + ")");
    }
    const bool tune = opts && opts->order_p == 0 && opts->tol > 0 && o.method == LENS_FMM;
    auto key = batch_key(dev, n_fields, fields, grids, maps, o);
    key_push(key, (int64_t)tune);
    key_push(key, (const void *)st);  // replays on one stream are ordered; others get their own
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchExec *B = nullptr;
    for (auto it = g_batches.begin(); it != g_batches.end(); ++it) {
      if ((*it)->key != key) continue;
      bool ok = true;
      for (int i = 0; i < n_fields && ok; ++i)
        if ((*it)->plans[i]) ok = inside((*it)->plans[i]->domain, &bbox[4 * i]);
      if (ok) {
        B = it->get();
      } else {
        g_batches.erase(it);  // stars moved outside the captured trees
      }
      break;
    }
    if (!B) {
      auto nb = batch_build(n_fields, fields, grids, maps, o, bbox, tune, tune ? *opts : o, st);
      nb->key = key;
      if (g_batches.size() >= kBatchCache) g_batches.erase(g_batches.begin());
      g_batches.push_back(std::move(nb));
      B = g_batches.back().get();
    }
    StageTimer tm("batched_graph", st);
    LENS_HIP(hipGraphLaunch(B->exec, st));
    B->last = st;
  });
}

lens_status lens_autotune(const lens_field *field, const lens_grid *grid, const lens_map_desc *map,
                          double tol, const lens_opts *base, void *stream, lens_opts *out,
                          double *err_out, double *ms_out) {
  return guarded([&] {
    hipStream_t st = (hipStream_t)stream;
    const lens_opts b = resolve_opts(base);
    check_field(field);
    if (!grid) fail(LENS_EINVAL, "grid is NULL");
    check_grid(grid);
    if (!out) fail(LENS_EINVAL, "out is NULL");
    if (!is_finite(tol) || !(tol > 0)) fail(LENS_EINVAL, "tol must be finite and > 0");
    if (map && (map->npix <= 0 || (int64_t)map->npix * map->npix > (int64_t)std::numeric_limits<int32_t>::max() ||
                !is_finite(map->y1min) || !is_finite(map->y2min) || !is_finite(map->side) ||
                !(map->side > 0)))
      fail(LENS_EINVAL, "map placement must be finite with side > 0 and 0 < npix^2 <= 2^31-1");
    lens_opts ub = base ? *base : b;  // keep the caller's encodings
    if (!base) lens_opts_default(&ub);
    ub.method = b.method;
    ub.precision = b.precision;
    ub.order_p = 0;
    ub.tol = tol;
    const TuneOut t = tuned_cached(*field, *grid, map, ub, st);
    *out = t.o;
    if (err_out) *err_out = t.err;
    if (ms_out) *ms_out = t.ms;
    if (!t.met)
      fail(LENS_EUNSUPPORTED, "no expansion order up to " + std::to_string(LENS_MAX_ORDER) +
                                  " reaches tol (best sampled error " + std::to_string(t.err) + ")");
  });
}

lens_status lens_find_images(lens_plan *plan, const lens_field *field, const lens_grid *grid,
                             const double *sources, int32_t n_sources, double tol, int32_t max_iter,
                             double *images, int32_t *image_src, int64_t cap, int64_t *n_images,
                             const lens_opts *opts, void *stream) {
  return guarded([&] {
    hipStream_t st = (hipStream_t)stream;
    lens_opts o = resolve_opts(opts);
    FieldView fv = field_for(plan, field);
    if (plan) check_plan_device(plan);
    if (!grid) fail(LENS_EINVAL, "grid is NULL");
    check_grid(grid);
    if (!n_images) fail(LENS_EINVAL, "n_images is NULL");
    if (n_sources < 0) fail(LENS_EINVAL, "n_sources < 0");
    if (n_sources > 0 && !sources) fail(LENS_EINVAL, "sources is NULL");
    if (cap < 0) fail(LENS_EINVAL, "cap < 0");
    if (cap > 0 && (!images || !image_src)) fail(LENS_EINVAL, "images / image_src is NULL");
    if (!(tol > 0) || !is_finite(tol)) fail(LENS_EINVAL, "tol must be finite and > 0");
    if (max_iter < 0 || max_iter > 1000) fail(LENS_EINVAL, "max_iter must be in [0, 1000]");
    *n_images = 0;
    const int64_t nx = grid->nx, ny = grid->ny;
    if (nx < 2 || ny < 2 || n_sources == 0) return;
    const double c1 = (1.0 - fv.f.kappa_s) - fv.f.gamma;
    const double c2 = (1.0 - fv.f.kappa_s) + fv.f.gamma;
    const bool direct = o.method == LENS_DIRECT || fv.f.n_stars == 0;
    if (!plan && !direct && wants_auto(opts)) o = auto_opts(fv.f, *grid, nullptr, *opts, st);
    const int64_t rows = pass_rows(opts, nx, ny);
    double gbb[4];
    grid_bbox(*grid, 0, ny, gbb);
    lens_plan *P = direct ? nullptr : plan;
    lens_plan *owned = nullptr;
    if (!direct && !P) {
      const double area = std::max((gbb[2] - gbb[0]) * (gbb[3] - gbb[1]), 1e-300);
      owned = P = build_plan(fv.f, gbb, grid, (double)(nx * ny) / area, o, st);
    }
    try {
      Scratch sc(st);
      GridPasses gp{fv, *grid, P, c1, c2, rows, sc.get<double>((size_t)(rows + 1) * nx * 2), nullptr};
      auto *count = sc.get<unsigned long long>(1);
      // seeds: every mapped triangle that holds a source (a second sweep
      // with room for all of them if the first overflowed)
      int64_t capc = std::max<int64_t>(4096, 64 * (int64_t)n_sources);
      std::vector<DevBuf> cbufs;
      double *cand_x = nullptr;
      int32_t *cand_s = nullptr;
      int64_t n = 0;
      for (int attempt = 0; attempt < 2; ++attempt) {
        Scratch cs(st);
        cand_x = cs.get<double>((size_t)capc * 2);
        cand_s = cs.get<int32_t>((size_t)capc);
        launch_ipm_zero(count, 1, st);
        for (int64_t j0 = 0; j0 < ny - 1; j0 += rows) {
          const int64_t j1 = std::min(ny - 1, j0 + rows);
          gp.deflect(j0, j1, st);
          ImageCellArgs a{gp.ybuf, nx, j0, j0, j1, *grid, sources, n_sources, count, cand_x, cand_s, capc};
          StageTimer tm("images", st);
          launch_image_cells(a, st);
        }
        n = (int64_t)read_scalar(count, st);
        if (n <= capc) {
          cbufs.swap(cs.bufs);  // keep the candidates
          break;
        }
        capc = n;
      }
      struct Keep {
        std::vector<DevBuf> b;
        hipStream_t s;
        ~Keep() {
          std::vector<DevBuf *> ps;
          for (auto &x : b) ps.push_back(&x);
          pool_put_batch(ps.data(), ps.size(), s);
        }
      } keep{std::move(cbufs), st};
      if (n == 0) return;
      // Newton refinement
      double *yc = sc.get<double>((size_t)n * 2), *dc = sc.get<double>((size_t)n * 2);
      double *res = sc.get<double>((size_t)n), *det = sc.get<double>((size_t)n);
      uint32_t *unconv = sc.get<uint32_t>(1);
      ExplicitLocals el;
      if (P) el = explicit_locals(*P, gbb, sc, st);
      NewtonArgs na{n, cand_x, cand_s, sources, yc, dc, c1, c2, tol,
                    4.0 * std::hypot(grid->dx, grid->dy), {gbb[0], gbb[1], gbb[2], gbb[3]},
                    res, det, unconv, 1};
      for (int it = 0; it <= max_iter; ++it) {
        if (P) {
          fmm_explicit_eval(*P, el, cand_x, n, c1, c2, yc, st, dc);
        } else {
          DirectArgs d{};
          d.n_stars = fv.f.n_stars;
          d.sxy = fv.f.xy;
          d.sm = fv.f.m;
          d.rxy = cand_x;
          d.n_rays = n;
          d.c1 = c1;
          d.c2 = c2;
          d.y_out = yc;
          d.dfdz_out = dc;
          launch_direct(d, st);
        }
        launch_fill_u32(unconv, 1, 0u, st);
        na.step = it < max_iter;
        StageTimer tm("images", st);
        launch_newton(na, st);
        if (read_scalar(unconv, st) == 0) break;
      }
      // merge the converged candidates of each source (host: images are few)
      std::vector<double> hx((size_t)n * 2), hr((size_t)n), hd((size_t)n);
      std::vector<int32_t> hs((size_t)n);
      LENS_HIP(hipMemcpyAsync(hx.data(), cand_x, hx.size() * 8, hipMemcpyDeviceToHost, st));
      LENS_HIP(hipMemcpyAsync(hr.data(), res, hr.size() * 8, hipMemcpyDeviceToHost, st));
      LENS_HIP(hipMemcpyAsync(hd.data(), det, hd.size() * 8, hipMemcpyDeviceToHost, st));
      LENS_HIP(hipMemcpyAsync(hs.data(), cand_s, hs.size() * 4, hipMemcpyDeviceToHost, st));
      LENS_HIP(hipStreamSynchronize(st));
      std::vector<int64_t> ord;
      for (int64_t k = 0; k < n; ++k)
        if (hr[k] <= tol && std::isfinite(hd[k]) && hd[k] != 0.0) ord.push_back(k);
      std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
        if (hs[a] != hs[b]) return hs[a] < hs[b];
        if (hx[2 * a] != hx[2 * b]) return hx[2 * a] < hx[2 * b];
        if (hx[2 * a + 1] != hx[2 * b + 1]) return hx[2 * a + 1] < hx[2 * b + 1];
        return a < b;
      });
      const double eps = std::max(1e-3 * std::min(grid->dx, grid->dy), 1e3 * tol);
      std::vector<int64_t> kept;
      size_t first_of_src = 0;
      for (int64_t k : ord) {
        if (!kept.empty() && hs[kept.back()] != hs[k]) first_of_src = kept.size();
        bool dup = false;
        for (size_t q = kept.size(); q-- > first_of_src;) {
          const int64_t c = kept[q];
          if (hx[2 * k] - hx[2 * c] > eps) break;
          if (std::hypot(hx[2 * k] - hx[2 * c], hx[2 * k + 1] - hx[2 * c + 1]) <= eps) {
            if (hr[k] < hr[c]) kept[q] = k;  // the better-converged copy
            dup = true;
            break;
          }
        }
        if (!dup) kept.push_back(k);
      }
      // merging may have swapped in a copy at a slightly different x1: the
      // output stays ordered by source, then x1 to within eps
      *n_images = (int64_t)kept.size();
      const int64_t m = std::min<int64_t>(cap, (int64_t)kept.size());
      if (m > 0) {
        std::vector<double> out((size_t)m * 4);
        std::vector<int32_t> osrc((size_t)m);
        for (int64_t q = 0; q < m; ++q) {
          const int64_t k = kept[q];
          out[4 * q] = hx[2 * k];
          out[4 * q + 1] = hx[2 * k + 1];
          out[4 * q + 2] = 1.0 / hd[k];
          out[4 * q + 3] = hr[k];
          osrc[q] = hs[k];
        }
        LENS_HIP(hipMemcpyAsync(images, out.data(), out.size() * 8, hipMemcpyHostToDevice, st));
        LENS_HIP(hipMemcpyAsync(image_src, osrc.data(), osrc.size() * 4, hipMemcpyHostToDevice, st));
        LENS_HIP(hipStreamSynchronize(st));
      }
    } catch (...) {
      if (owned) lens_plan_destroy(owned);
      throw;
    }
    if (owned) release_owned(owned, st);
  });
}

lens_status lens_critical_curves(lens_plan *plan, const lens_field *field, const lens_grid *grid,
                                 double *seg_out, double *caustic_out, int64_t cap, int64_t *n_seg,
                                 const lens_opts *opts, void *stream) {
  return guarded([&] {
    hipStream_t st = (hipStream_t)stream;
    lens_opts o = resolve_opts(opts);
    FieldView fv = field_for(plan, field);
    if (plan) check_plan_device(plan);
    if (!grid) fail(LENS_EINVAL, "grid is NULL");
    check_grid(grid);
    if (!n_seg) fail(LENS_EINVAL, "n_seg is NULL");
    if (cap < 0) fail(LENS_EINVAL, "cap < 0");
    if (cap > 0 && !seg_out) fail(LENS_EINVAL, "seg_out is NULL");
    *n_seg = 0;
    const int64_t nx = grid->nx, ny = grid->ny;
    if (nx < 2 || ny < 2) return;
    const double c1 = (1.0 - fv.f.kappa_s) - fv.f.gamma;
    const double c2 = (1.0 - fv.f.kappa_s) + fv.f.gamma;
    const bool direct = o.method == LENS_DIRECT || fv.f.n_stars == 0;
    if (!plan && !direct && wants_auto(opts)) o = auto_opts(fv.f, *grid, nullptr, *opts, st);
    const int64_t rows = pass_rows(opts, nx, ny);
    double gbb[4];
    grid_bbox(*grid, 0, ny, gbb);
    lens_plan *P = direct ? nullptr : plan;
    lens_plan *owned = nullptr;
    if (!direct && !P) {
      const double area = std::max((gbb[2] - gbb[0]) * (gbb[3] - gbb[1]), 1e-300);
      owned = P = build_plan(fv.f, gbb, grid, (double)(nx * ny) / area, o, st);
    }
    try {
      Scratch sc(st);
      const size_t nb = (size_t)(rows + 1) * nx * 2;
      GridPasses gp{fv, *grid, P, c1, c2, rows, sc.get<double>(nb), sc.get<double>(nb)};
      auto *count = sc.get<unsigned long long>(1);
      launch_ipm_zero(count, 1, st);
      for (int64_t j0 = 0; j0 < ny - 1; j0 += rows) {
        const int64_t j1 = std::min(ny - 1, j0 + rows);
        gp.deflect(j0, j1, st);
        CritArgs a{gp.dbuf, nx, j0, j0, j1, *grid, c1, c2, seg_out, count, cap};
        StageTimer tm("critical", st);
        launch_crit_cells(a, st);
      }
      const int64_t n = (int64_t)read_scalar(count, st);
      *n_seg = n;
      const int64_t m = std::min(n, cap);
      if (caustic_out && m > 0) {
        // the segments' end points are 2m rays inside the grid's box
        if (P) {
          fmm_explicit(*P, seg_out, 2 * m, gbb, c1, c2, caustic_out, st);
        } else {
          DirectArgs d{};
          d.n_stars = fv.f.n_stars;
          d.sxy = fv.f.xy;
          d.sm = fv.f.m;
          d.rxy = seg_out;
          d.n_rays = 2 * m;
          d.c1 = c1;
          d.c2 = c2;
          d.y_out = caustic_out;
          launch_direct(d, st);
        }
        LENS_HIP(hipStreamSynchronize(st));
      }
    } catch (...) {
      if (owned) lens_plan_destroy(owned);
      throw;
    }
    if (owned) release_owned(owned, st);
  });
}

lens_status lens_deflect_multiplane(int32_t n_planes, const lens_field *fields, const double *beta,
                                    const lens_grid *grid, const double *rays_xy, int64_t n_rays,
                                    double *y_out, const lens_opts *opts, void *stream) {
  return guarded([&] {
    hipStream_t st = (hipStream_t)stream;
    resolve_opts(opts);
    if (n_planes < 1 || n_planes > kMaxPlanes)
      fail(LENS_EINVAL, "n_planes must be in [1, " + std::to_string(kMaxPlanes) + "]");
    if (!fields) fail(LENS_EINVAL, "fields is NULL");
    for (int32_t j = 0; j < n_planes; ++j) check_field(&fields[j]);
    if (n_planes > 1 && !beta) fail(LENS_EINVAL, "beta is NULL");
    for (int32_t j = 1; j < n_planes; ++j)
      for (int32_t i = 0; i < j; ++i)
        if (!is_finite(beta[(size_t)j * n_planes + i])) fail(LENS_EINVAL, "beta must be finite");
    if ((grid == nullptr) == (rays_xy == nullptr) && !(grid == nullptr && n_rays == 0))
      fail(LENS_EINVAL, "give exactly one of grid and rays_xy");
    if (n_rays < 0) fail(LENS_EINVAL, "n_rays < 0");
    if (grid) {
      check_grid(grid);
      if (n_rays != grid->nx * grid->ny) fail(LENS_EINVAL, "n_rays must equal grid.nx * grid.ny");
    }
    if (n_rays > (int64_t)std::numeric_limits<uint32_t>::max() - 1)
      fail(LENS_EINVAL, "n_rays exceeds 2^32-2");
    if (n_rays > 0 && !y_out) fail(LENS_EINVAL, "y_out is NULL");
    if (n_rays == 0) return;
    Scratch sc(st);
    const int64_t n = n_rays;
    double *alpha = sc.get<double>((size_t)n_planes * n * 2);
    double *x = sc.get<double>((size_t)n * 2);
    double *y = sc.get<double>((size_t)n * 2);
    MultiPlaneArgs a{};
    a.n = n;
    a.grid_mode = grid != nullptr;
    if (grid) a.grid = *grid;
    a.rays = rays_xy;
    a.alpha = alpha;
    for (int32_t j = 0; j < n_planes; ++j) {
      a.j = j;
      for (int32_t i = 0; i < j; ++i) a.beta[i] = beta[(size_t)j * n_planes + i];
      a.x_out = x;
      launch_mp_positions(a, st);  // x_j (x_0 itself for j = 0)
      if (j == 0 && grid)
        check_inner(lens_deflect(nullptr, &fields[0], grid, nullptr, n, y, nullptr, opts, stream));
      else
        check_inner(lens_deflect(nullptr, &fields[j], nullptr, x, n, y, nullptr, opts, stream));
      launch_mp_alpha(x, y, alpha + (size_t)j * n * 2, n, st);
    }
    // the source plane: every plane's deflection at full weight
    a.j = n_planes;
    for (int32_t i = 0; i < n_planes; ++i) a.beta[i] = 1.0;
    a.x_out = y_out;
    launch_mp_positions(a, st);
  });
}

void lens_release_cached(void) {
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    g_batches.clear();
  }
  std::lock_guard<std::mutex> lk(g_call_mu);
  g_calls.clear();
  g_call_seen.clear();
}

}  // extern "C"
