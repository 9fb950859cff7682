// Internal declarations shared by the host orchestration (api.cpp) and the
// HIP kernel translation units.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "lens.h"

namespace lensfmm {

// ------------------------------------------------------------------ errors
const std::string &last_error();

struct LensError {
  lens_status status;
  std::string msg;
};

void set_error(const std::string &msg);
[[noreturn]] void fail(lens_status st, const std::string &msg);
void check_hip(hipError_t e, const char *what);
#define LENS_HIP(call) ::lensfmm::check_hip((call), #call)

// ------------------------------------------------------------ device memory

// A cached device allocation.  Blocks return to a per-device free list and
// are reused by later requests; a block released on one stream and reused on
// another makes the new stream wait for the release point first.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  int device = -1;
};

DevBuf pool_get(size_t bytes, hipStream_t stream);
void pool_put(DevBuf &b, hipStream_t stream);
// release several buffers behind one event
void pool_put_batch(DevBuf *const *bufs, size_t n, hipStream_t stream);

// RAII list of scratch buffers released at scope exit (stream-ordered).
struct Scratch {
  hipStream_t stream;
  std::vector<DevBuf> bufs;
  explicit Scratch(hipStream_t s) : stream(s) {}
  ~Scratch() {
    std::vector<DevBuf *> ps;
    for (auto &b : bufs) ps.push_back(&b);
    pool_put_batch(ps.data(), ps.size(), stream);
  }
  template <typename T>
  T *get(size_t count) {
    DevBuf b = pool_get(count * sizeof(T) + 256, stream);
    bufs.push_back(b);
    return static_cast<T *>(b.ptr);
  }
  Scratch(const Scratch &) = delete;
  Scratch &operator=(const Scratch &) = delete;
};

// ------------------------------------------------------------------ geometry

// Root square of the quadtree and its depth.  Box (ix, iy) at level l has
// side s_l = side / 2^l and lower-left corner (x0 + ix s_l, y0 + iy s_l);
// boxes of a level are numbered row-major, iy * 2^l + ix.
struct Geometry {
  double x0, y0, side;
  int L;  // leaf level
};

// A rectangle of boxes at one level: columns [bx0, bx0+nbx), rows [by0, by0+nby).
struct Window {
  int64_t bx0, by0, nbx, nby;
  __host__ __device__ int64_t count() const { return nbx * nby; }
};

// ------------------------------------------------------------ kernel launchers
// (each returns after enqueueing on `stream`; sizes already validated)

// Tree build (tree.hip)
// out[0..4) = bounding box {x1min, x2min, x1max, x2max} of xy[0, n); with
// count_box (a host array {x1min, x2min, x1max, x2max}), out[4] holds the
// bits of the number of points inside that closed rectangle.  partial:
// device scratch of 5 * nparts doubles; out may be host-mapped memory.
void launch_bbox(const double *xy, int64_t n, double *partial, int nparts, const double *count_box,
                 double *out, hipStream_t stream);
int bbox_parts(int64_t n);
struct BBoxSet {
  const double *xy;
  int64_t n;
};
// out[s][4] = bounding box of set s (sets_dev: device array of nsets sets)
void launch_bbox_multi(const BBoxSet *sets_dev, int nsets, int nparts, double *partial,
                       double *out, hipStream_t stream);
void launch_leaf_keys(const double *xy, int64_t n, Geometry g, uint32_t *keys, uint32_t *vals,
                      uint32_t *box_count, hipStream_t stream);
// p[0..n) = v (a kernel, so it may be captured in a graph)
void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream);
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of key.
// Uses (k_tmp, v_tmp) as ping-pong storage; returns true if the sorted result
// ended up in the tmp buffers.
bool radix_sort_pairs(uint32_t *k, uint32_t *v, uint32_t *k_tmp, uint32_t *v_tmp, int64_t n,
                      int bits, uint32_t *counts, uint32_t *scan_tmp, hipStream_t stream);
size_t radix_counts_len(int64_t n);
size_t scan_tmp_len(size_t n);
void exclusive_scan_u32(const uint32_t *in, uint32_t *out, size_t n, uint32_t *tmp,
                        hipStream_t stream);
// sources (stars, or rays with complex charges) sorted by leaf box:
// positions [n][2] and charges [n][qdim] (qdim 1: real masses; 2: complex);
// with sq32 (qdim 1), also the masses rounded to FP32
void launch_gather_stars(const uint32_t *perm, const double *xy, const double *q, int qdim,
                         int64_t n, double *sxy, double *sq, float *sq32, hipStream_t stream);
void launch_gather_rays(const uint32_t *perm, const double *xy, int64_t n, double *sxy,
                        hipStream_t stream);
// start[b] = first sorted index with key >= b, for b in [0, nbox]
void launch_box_starts(const uint32_t *sorted_keys, int64_t n, int64_t nbox, int32_t *start,
                       int32_t *coarse, hipStream_t stream);
// int32 entries of the scratch `coarse` that launch_box_starts needs
int64_t box_starts_coarse_len(int64_t nbox);

// Expansion operator tables (host-built, uploaded once per order).
struct OpTables {
  int p = 0;
  double *m2m = nullptr;   // [4][p][p] complex, M[q][l][k]
  double *l2l = nullptr;   // [4][p][p] complex, L[q][j][l]
  double *m2l = nullptr;   // [49][p][p] complex, stored T[tau][k][l]
  float *m2l32 = nullptr;  // same in FP32
  // M2L as MFMA B fragments: [49][ks][nt][64 lanes]
  int ks = 0, nt = 0;
  double *bfrag64 = nullptr;
  float *bfrag32 = nullptr;
  double *l2l_frag = nullptr;  // L2L as FP64 MFMA B fragments: [4][ks][nt][64]
};
const OpTables &op_tables(int p, hipStream_t stream);
// The tables of order p on the current device if already built, else
// nullptr (never allocates).
const OpTables *op_tables_if_built(int p);

// Host-side table builders (also exported for tests through lens_debug_*).
void build_m2m_table(int p, std::vector<double> &out);
void build_l2l_table(int p, std::vector<double> &out);
void build_m2l_table(int p, std::vector<double> &out);
void build_m2l_bfrag(int p, std::vector<double> &out, int &ks_count, int &nt_count);
void build_l2l_bfrag(int p, int ks_count, int nt_count, std::vector<double> &out);

// Upward pass (upward.hip)
// (mp32 outputs are optional FP32 copies of the same coefficients)
// n_sources (all levels) picks a wave per box when boxes hold many sources.
// Trees of several fields sorted together (batched maps): field j's sources
// xy/q ([n][2], [n]) occupy elements [off, off + n) of the combined arrays;
// its sorted sources go to sxy/sq.
struct TreeJob {
  const double *xy, *q;
  double *sxy, *sq;
  float *sq32;  // FP32 copies of the sorted charges (or nullptr)
  Geometry g;
  int64_t off, n;
};
// keys (j << shift) | leaf key, values the field-local index
void launch_leaf_keys_multi(const TreeJob *jobs, int njobs, int64_t total, int shift, uint32_t *keys,
                            uint32_t *vals, hipStream_t stream);
// after the sort: gather each field's sources, keys &= mask (leaf keys)
void launch_gather_multi(const TreeJob *jobs, int njobs, int64_t total, uint32_t mask, uint32_t *keys,
                         const uint32_t *perm, hipStream_t stream);

// child_win / child_mp: the level below, already formed ([child_win][p] FP64;
// child_mp nullptr at the leaf level): boxes of more than 32 sources whose
// children it holds are formed from them by M2M.  win_sources: the sources
// expected in `win` (chooses a thread or a wave per box); clustered: some
// boxes may hold far more than that average.
void launch_p2m(Geometry g, int level, Window win, const double *sxy, const double *sq, int qdim,
                const int32_t *leaf_start, int p, double *mp, float *mp32, double win_sources,
                bool clustered, Window child_win, const double *child_mp, hipStream_t stream);
// M2M of levels level, level-1, ..., level-nlev+1 in one launch; the child
// level (level+1) is dense, [n][n][p] complex; out[i] / out32[i] (optional)
// receive level - i, dense.
constexpr int kMaxM2MChain = 4;
struct M2MChain {
  int level, nlev, p;
  const double *child;
  double *out[kMaxM2MChain];
  float *out32[kMaxM2MChain];
};
int m2m_chain_levels(int level);  // most levels one launch can take from `level` down
void launch_m2m_chain(const M2MChain &c, hipStream_t stream);

// Downward pass (downward.hip): local expansions of `win` at `level` from the
// parent's locals (level >= 3) and the multipoles of the interaction list.
struct DownArgs {
  int level, p;
  double s;              // box side at this level
  Window win, pwin;      // target window and parent window
  const double *mp;      // multipoles at this level, [swin][p] complex FP64
  const float *mp32;     // same in FP32 (mixed fine levels) or nullptr
  Window swin;           // boxes held in mp / mp32
  const double *ploc;    // parent locals [pwin][p] or nullptr (level 2)
  double *loc;           // output locals [win][p]
};
// loc += L2L(parent locals), FP64 (levels >= 3).
void launch_l2l(const DownArgs &a, const OpTables &t, hipStream_t stream);
// L2L down a chain of levels in one launch: the locals of `level` are final;
// levels level+1 .. level+nlev (nlev <= 3) get loc += L2L(parent) in turn.
// win[j] / loc[j]: window and locals [win][p] of level + j.
constexpr int kMaxL2LChain = 3;
struct L2LChain {
  int level, nlev, p;
  Window win[kMaxL2LChain + 1];
  double *loc[kMaxL2LChain + 1];
};
void launch_l2l_chain(const L2LChain &c, const OpTables &t, hipStream_t stream);

// M2L of several levels in one launch: loc = (1/s) sum over the interaction
// list (FP64 or FP32 arithmetic); runs on MFMA when the order's tile fits the
// LDS budget, else on VALU (one launch per level).
constexpr int kMaxBatchLevels = LENS_MAX_LEVEL + 1;
struct M2LLevel {
  int level;
  double s;
  Window win;
  const void *mp;       // multipoles of the level, FP64 or FP32
  double *loc;
  const double *ploc;   // fused L2L: parent locals (window pwin), or nullptr
  Window pwin;
  Window swin;          // boxes held in mp ([swin][p], row-major in the window)
};
struct M2LBatch {
  int count = 0, p = 0;
  M2LLevel lv[kMaxBatchLevels];
  int64_t tile_begin[kMaxBatchLevels + 1];
};
void launch_m2l_batch(M2LBatch &b, const OpTables &t, bool fp32, hipStream_t stream);
// One level with L2L fused: loc = (1/s) M2L + L2L(ploc), the L2L part on FP64
// MFMA; returns false (nothing launched) if the order has no MFMA tile.
bool launch_m2l_l2l(M2LBatch &b, const OpTables &t, bool fp32, hipStream_t stream);
void launch_to_f32(const double *src, float *dst, size_t n, hipStream_t stream);

// Evaluation (eval.hip): per leaf box of the window, local expansion at its
// rays + direct sum over the 3x3 neighbourhood + smooth term.
struct EvalArgs {
  Geometry g;
  int p;
  Window win;            // leaf-level target window
  const double *loc;     // [win][p] complex locals
  const double *sxy;     // sorted stars
  const double *sm;
  const float *sm32;     // their masses in FP32 (LENS_MIXED near field)
  const int32_t *leaf_start;  // [4^L + 1]
  // rays: grid or sorted explicit
  int grid_mode;
  lens_grid grid;
  const int32_t *col_start;   // grid: [win.nbx + 1] first ray column per box column
  const int32_t *row_start;   // grid: [win.nby + 1]
  const double *rxy;          // explicit, sorted by leaf box
  const uint32_t *rperm;      // explicit: sorted position -> caller index
  const int32_t *ray_start;   // explicit: [win.count() + 1]
  int64_t chunks_per_box;     // units (waves) per leaf box
  int rays_per_lane;          // R: rays held per lane (1..4), 64*R rays per unit
  int tile_shift;             // grid: a wave's 64 rays are a 2^tile_shift-wide tile
  double c1, c2;              // (1 - kappa_s - gamma), (1 - kappa_s + gamma)
  double *y_out;              // [n][2] or nullptr
  double *dfdz_out;           // [n][2] f'(z) (deflection only) or nullptr
  // map
  int32_t *counts;
  double y1min, y2min, S;
  int32_t npix;
};
void launch_eval(const EvalArgs &a, int precision, hipStream_t stream);
// col_start[c] = first grid column whose rays fall in box column win.bx0 + c
// (c = 0..nbx); row_start likewise over the rows [j_begin, j_end).
void launch_grid_ranges(const lens_grid &grid, Geometry g, Window win, int64_t j_begin,
                        int64_t j_end, int32_t *col_start, int32_t *row_start, hipStream_t stream);
void eval_shape(int64_t max_rays, int *R, int64_t *CH);
void grid_tile_shape(int64_t W, int64_t H, int *shift, int64_t *tiles);
void launch_ray_keys(const double *rxy, int64_t n, Geometry g, Window win, uint32_t *keys,
                     uint32_t *vals, hipStream_t stream);

// Adjoint (adjoint.hip): gradients at stars from rays with complex charges
struct AdjArgs {
  const double *sq;       // sorted source charges [n][2] (complex g_k)
  const double *txy;      // targets (stars) sorted by window box
  const double *tm;       // their masses
  const uint32_t *tperm;  // sorted position -> caller's star index
  const int32_t *tstart;  // [win.count() + 1], or [4^L + 1] if tglobal
  double *grad_xy;        // [N][2]
  double *grad_m;         // [N]
  bool tglobal = false;   // tstart indexed by global leaf box (a forward plan's)
};
void launch_eval_adj(const EvalArgs &a, const AdjArgs &d, int precision, hipStream_t stream);
void launch_direct_adj(int64_t n_stars, const double *star_xy, const double *star_m, int64_t n_rays,
                       const double *rays_xy, const double *grad_y, double *grad_xy,
                       double *grad_m, hipStream_t stream);
void launch_grid_rays(const lens_grid &g, double *out, hipStream_t stream);
int64_t adj_targets_per_unit();

// Direct FP64 sum (direct.hip)
struct DirectArgs {
  int64_t n_stars;
  const double *sxy, *sm;
  int grid_mode;
  lens_grid grid;
  const double *rxy;
  int64_t n_rays;
  int64_t ray_offset;    // first ray index (grid rows chunking)
  double c1, c2;
  double *y_out;
  double *dfdz_out;      // [n][2] f'(z) or nullptr (not with counts)
  int32_t *counts;
  double y1min, y2min, S;
  int32_t npix;
};
void launch_direct(const DirectArgs &a, hipStream_t stream);

// Inverse polygon mapping (ipm.hip).  acc is an npix^2 fixed-point
// accumulator (units of 2^-40 of a pixel's magnification) and diff an
// npix x (npix + 1) one of row differences (pixels a wide cell covers
// completely); launch_ipm_finish adds acc plus the row prefix sums of diff to
// the FP64 map mu.  y holds grid rows [ybase, ...) with nx rays per row;
// cells of rows [j0, j1) are mapped.  queue needs (nx - 1) (j1 - j0) entries.
struct IpmPass {
  const double *y;
  int64_t nx, ybase, j0, j1;
  double cell_px, y1min, y2min, S;
  int32_t npix;
  unsigned long long *acc, *diff;
  uint32_t *queue, *qcount;
};
// Image finding, critical curves, multi-plane chaining (images.hip).  Cells
// of grid rows [j0, j1) of a deflected grid held from row ybase on.
struct ImageCellArgs {
  const double *y;
  int64_t nx, ybase, j0, j1;
  lens_grid grid;
  const double *src;      // [n_src][2] source positions (device)
  int32_t n_src;
  unsigned long long *count;  // candidates found so far
  double *cand_x;         // [cap][2] seeds
  int32_t *cand_s;        // [cap] source index
  int64_t cap;
};
void launch_image_cells(const ImageCellArgs &a, hipStream_t stream);

struct NewtonArgs {
  int64_t n;
  double *cand_x;
  const int32_t *cand_s;
  const double *src, *y, *dfdz;
  double c1, c2, tol, max_step;
  double box[4];
  double *res, *det;
  uint32_t *unconverged;
  int step;               // 0: residual and det only
};
void launch_newton(const NewtonArgs &a, hipStream_t stream);

struct CritArgs {
  const double *dfdz;
  int64_t nx, ybase, j0, j1;
  lens_grid grid;
  double c1, c2;
  double *seg;            // [cap][4]
  unsigned long long *count;
  int64_t cap;
};
void launch_crit_cells(const CritArgs &a, hipStream_t stream);

constexpr int kMaxPlanes = 64;
struct MultiPlaneArgs {
  int64_t n;
  int grid_mode;
  lens_grid grid;
  const double *rays;     // explicit x_0 (grid_mode 0)
  const double *alpha;    // [j][n][2] deflections of planes 0..j-1
  double beta[kMaxPlanes];  // beta_ij, i < j
  int32_t j;
  double *x_out;          // [n][2]
};
void launch_mp_positions(const MultiPlaneArgs &a, hipStream_t stream);
void launch_mp_alpha(const double *x, const double *y, double *alpha, int64_t n, hipStream_t stream);
void launch_ipm_zero(unsigned long long *acc, int64_t n, hipStream_t stream);
void launch_ipm_cells(const IpmPass &p, hipStream_t stream);
void launch_ipm_finish(const unsigned long long *acc, const unsigned long long *diff, int32_t npix,
                       double *mu, hipStream_t stream);

}  // namespace lensfmm

namespace lensfmm {

// Per-stage timing with HIP events on the launching stream, enabled by
// lens_profile_enable().  A StageTimer brackets one stage of one call.
bool profiling_enabled();
// While a thread captures a HIP graph, StageTimer records nothing.
void set_capturing(bool on);
// Scope in which this thread's StageTimers record nothing (calls that must
// not create runtime objects).
struct NoTiming {
  NoTiming();
  ~NoTiming();
  NoTiming(const NoTiming &) = delete;
  NoTiming &operator=(const NoTiming &) = delete;
};

// Grid deflection with a plan into a caller-provided device region of
// `bytes` bytes (allocates no device memory); see lens_deflect_noalloc and
// lens_opts.workspace.  dfdz: f'(z) as in lens_deflect, or nullptr.
void deflect_grid_no_alloc(lens_plan *plan, const lens_field *field, const lens_grid *grid,
                           double *y_out, const lens_opts *opts, char *region, size_t bytes,
                           hipStream_t st, double *dfdz = nullptr);
struct StageTimer {
  const char *name;
  hipStream_t stream;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  StageTimer(const char *n, hipStream_t s);
  ~StageTimer();
  StageTimer(const StageTimer &) = delete;
  StageTimer &operator=(const StageTimer &) = delete;
};

}  // namespace lensfmm
