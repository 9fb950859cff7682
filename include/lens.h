/*
 * lens.h -- C ABI of liblensfmm, a fast-multipole evaluator of gravitational
 * lens deflection by many point masses on AMD Instinct MI355X (gfx950).
 *
 * The operation (Jimenez-Vicente & Mediavilla 2022, Section 1, eq. 1, with
 * the smooth-field term of its footnote and of step 3 of the map driver in
 * Section 2.4) maps each image-plane ray x to the source plane:
 *
 *     alpha(x) = sum_i m_i (x - x_i) / |x - x_i|^2
 *     y1 = (1 - kappa_s - gamma) x1 - alpha1
 *     y2 = (1 - kappa_s + gamma) x2 - alpha2
 *
 * in units of the Einstein radius of unit mass, with the shear along the x1
 * axis.  In complex form, z = x1 + i x2, alpha = conj(f) with
 * f(z) = sum_i m_i / (z - z_i) (Appendix A: the expansions take a simple
 * analytic form in complex variables).  A ray that coincides exactly with a
 * star skips that singular pair.
 *
 * LENS_FMM evaluates the sum with the fast multipole method of Appendix A
 * (quadtree, P2M, M2M, M2L, L2L, L2P and near-field P2P); LENS_DIRECT sums
 * it directly in FP64.  LENS_FP64 runs every FMM stage in FP64; LENS_MIXED
 * runs the near field and the fine-level translations in FP32 and keeps FP64
 * for coordinates relative to box centres, coarse-level translations and the
 * final y.
 *
 * Conventions shared by every entry point:
 *  - Every array pointer is a DEVICE pointer (hipMalloc / torch CUDA tensor
 *    memory) unless its comment says otherwise.  The caller owns every
 *    buffer; the library never frees or retains a caller pointer past the
 *    call (a plan copies what it needs).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All device work is enqueued on it; outputs are valid once the stream
 *    has completed.  The only calls that wait on the stream are noted below.
 *  - On any status other than LENS_OK nothing has been enqueued and the
 *    outputs are untouched, except LENS_EDEVICE, which reports a HIP runtime
 *    failure after work may have been enqueued.  lens_last_error() gives a
 *    thread-local description (host string, valid until the thread's next
 *    call into the library).
 *  - Positions are FP64 pairs laid out [n][2] = (x1, x2); masses FP64 [n].
 *    Masses may be any finite value; N_* = 0 is valid (alpha = 0); a call
 *    with zero rays is a no-op.
 *  - Distinct plans may be used from distinct threads on distinct streams.
 */
#ifndef LENS_H
#define LENS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define LENS_API __attribute__((visibility("default")))
#else
#define LENS_API
#endif

typedef enum {
  LENS_OK = 0,
  LENS_EINVAL = 1,       /* bad argument; nothing enqueued */
  LENS_ENOMEM = 2,       /* device allocation failed; nothing enqueued */
  LENS_EDEVICE = 3,      /* HIP runtime error */
  LENS_EUNSUPPORTED = 4  /* valid request this library does not implement */
} lens_status;

enum { LENS_FMM = 0, LENS_DIRECT = 1 };   /* lens_opts.method    */
enum { LENS_FP64 = 0, LENS_MIXED = 1 };   /* lens_opts.precision */

#define LENS_MAX_ORDER 40     /* largest expansion order p (terms k = 0..p-1) */
#define LENS_MAX_LEVEL 15     /* deepest quadtree level */

/* The lens: N_* point masses plus the smooth convergence and shear. */
typedef struct {
  int64_t n_stars;      /* N_* >= 0 */
  const double *xy;     /* [N_*][2] star positions (device) */
  const double *m;      /* [N_*] star masses (device) */
  double kappa_s;       /* smooth convergence (finite) */
  double gamma;         /* shear along x1 (finite) */
} lens_field;

/* A cell-centred ray grid: ray k = j*nx + i sits at
 * (x0 + (i + 0.5) dx, y0 + (j + 0.5) dy), each product and sum rounded once. */
typedef struct {
  double x0, y0;        /* lower-left corner of the grid */
  double dx, dy;        /* cell sizes, > 0 */
  int64_t nx, ny;       /* cells per side, >= 0 */
} lens_grid;

/* A source-plane inverse-ray-shooting map (Section 2.3): counts[v*npix + u]
 * counts the rays with u = floor((y1 - y1min) * S), v = floor((y2 - y2min) * S),
 * S = npix / side, 0 <= u, v < npix (half-open pixels; rays outside are
 * dropped).  Counts are ACCUMULATED (+=) so a map may be built over calls. */
typedef struct {
  double y1min, y2min;  /* lower-left corner of the map */
  double side;          /* side length, > 0 */
  int32_t npix;         /* pixels per side, npix*npix <= INT32_MAX */
  int32_t *counts;      /* [npix][npix] int32 (device) */
} lens_map_desc;

typedef struct {
  int32_t method;       /* LENS_FMM or LENS_DIRECT */
  int32_t precision;    /* LENS_FP64 or LENS_MIXED (LENS_DIRECT is always FP64) */
  int32_t order_p;      /* expansion terms p in [1, LENS_MAX_ORDER]; 0 = chosen
                           by the autotuner for `tol` (tol > 0, LENS_FMM;
                           see lens_autotune), else 12 */
  int32_t leaf_level;   /* quadtree leaf level in [2, LENS_MAX_LEVEL]; 0 = chosen
                           by the library's cost model */
  int64_t max_rays_per_chunk;  /* rays per pass of lens_map (0 = the whole
                                  grid in one pass: a map needs no per-ray
                                  memory) and lens_map_ipm (0 = 2^28) */
  int32_t fp32_levels;  /* LENS_MIXED: M2L of the finest fp32_levels quadtree
                           levels runs on FP32 MFMA, coarser levels on FP64;
                           0 = 2 levels, -1 = none (all M2L in FP64), at most
                           LENS_MAX_LEVEL.  Ignored for LENS_FP64. */
  double tol;           /* with order_p = 0: the target of the autotuner --
                           the largest per-ray relative deflection error
                           (lens_deflect, lens_plan_create with a grid) or the
                           expected bin-reassignment fraction (lens_map,
                           lens_map_ipm, lens_map_batched).  The first call
                           for a problem measures (it waits on the stream); the
                           choice is kept in-process and in an on-disk cache
                           ($LENS_TUNE_CACHE, "off" to disable; default
                           ~/.cache/lensfmm/autotune.txt) keyed by a coarse
                           description of the problem.  Unused otherwise */
  void *workspace;      /* NULL (default): per-call device memory comes from
                           the library's pool.  Otherwise a caller-owned
                           device buffer, 256-byte aligned, of
                           workspace_bytes bytes that lens_deflect with a plan
                           and a ray grid carves its per-call memory from
                           (local expansions of every level over the grid,
                           ray ranges): the grid then runs in bands of whole
                           rows that fit it, no device allocation is made,
                           and one row that does not fit gives LENS_ENOMEM.
                           Calls on one stream may share it; calls that
                           overlap in time must not.  Other calls, and the
                           direct method or a field without stars (which
                           need no per-call memory), ignore it. */
  size_t workspace_bytes;
} lens_opts;

/* Fill *o with the defaults (FMM, mixed, p = 12, automatic leaf level). */
LENS_API void lens_opts_default(lens_opts *o);

/* Star-side state reusable across calls: the quadtree over the stars and the
 * multipole expansions of every box (Appendix A, initialisation and upward
 * passes).  Opaque. */
typedef struct lens_plan lens_plan;

/*
 * Build a plan for `field` whose quadtree also covers the rectangle
 * ray_box = {x1min, x2min, x1max, x2max} (HOST array; every ray later
 * evaluated with this plan must lie inside it; NULL = the stars' extent only)
 * and, if `grid` is not NULL, every ray of that grid.  With a grid, leaf boxes
 * are aligned with its cells where the spacings allow (a leaf box then holds
 * a whole number of 64-ray waves).  Copies the stars (sorted by leaf box) into
 * plan-owned device memory, so the caller's star arrays may be freed
 * afterwards.  Waits on `stream` once, to read back the stars' bounding box.
 * *out receives the plan.
 */
LENS_API lens_status lens_plan_create(const lens_field *field, const double *ray_box,
                                      const lens_grid *grid, const lens_opts *opts, void *stream,
                                      lens_plan **out);

/* Release a plan.  Does not wait: its device buffers return to the library's
 * pool ordered after the work last enqueued with the plan (a later reuse on
 * another stream waits for that work). */
LENS_API void lens_plan_destroy(lens_plan *plan);

/* Query a plan: expansion order, leaf level, root square (x0, y0, side). */
LENS_API lens_status lens_plan_info(const lens_plan *plan, int32_t *order_p, int32_t *leaf_level,
                           double *root_x0, double *root_y0, double *root_side);

/*
 * Deflect rays: y_out[k][2] = y(x_k) (FP64, device), and, if dfdz_out is not
 * NULL, dfdz_out[k][2] = f'(z_k) = -sum_i m_i / (z_k - z_i)^2 (real, imaginary
 * parts; FP64, device), the derivative that Appendix A's expansions give in
 * closed form.  With alpha = conj(f) the deflection Jacobian is
 * d(alpha1, alpha2)/d(x1, x2) = [[Re f', -Im f'], [-Im f', -Re f']], so the
 * lens map's Jacobian determinant is (1 - kappa_s)^2 - |gamma + conj(f')|^2
 * (for the shear along x1).  A ray exactly on a star skips that pair in f'
 * too; LENS_MIXED forms the near-field pairs of f' in FP32 (partial sums
 * carried into FP64 every 128 stars; valid for pairs farther apart than
 * ~1e-9 Einstein radii).  Rays come from `grid` (then rays_xy must
 * be NULL and n_rays = grid->nx * grid->ny) or from the explicit device array
 * rays_xy[n_rays][2] (then grid must be NULL).
 * `plan` may be NULL: the library then builds the star tree for this call,
 * waiting on the stream once to read back the stars' (and, for explicit
 * rays, the rays') bounding box.  Grid calls without a plan are cached: from
 * the second call with the same stream, input addresses and sizes, options,
 * smooth terms and resulting tree geometry on, the call's kernels run as one
 * captured HIP graph (its buffers stay allocated until lens_release_cached;
 * calls made while the stage profiler is on run uncached).  Such a call
 * launches its latest graph before the bounding box has come back and then
 * waits for the bounding-box reduction only; if the tree geometry has
 * changed (the stars moved), it recomputes, so y_out and dfdz_out always
 * hold this call's result.
 * With a plan, the plan's (sorted) stars, expansion order, leaf level and
 * precision are used and opts->method still selects FMM or direct; `field`
 * may then be NULL (the plan's kappa_s and gamma apply) or supply only
 * kappa_s and gamma (its star pointers are ignored).  Grid calls with a plan
 * do not wait on the stream.
 */
LENS_API lens_status lens_deflect(lens_plan *plan, const lens_field *field, const lens_grid *grid,
                                  const double *rays_xy, int64_t n_rays, double *y_out,
                                  double *dfdz_out, const lens_opts *opts, void *stream);

/* Device scratch held by the allocation-free entry point (per GPU, for the
 * life of the process). */
#define LENS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * lens_deflect for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same result as lens_deflect(plan, field, grid, NULL, nx*ny, y_out, opts,
 * stream) -- bit for bit -- for a grid of rays and an existing plan (which
 * holds the star side, built once by lens_plan_create).  The per-call
 * buffers (local expansions of every level, ray ranges) live in a static
 * device array of LENS_NOALLOC_SCRATCH_BYTES per GPU instead of the
 * library's pool; the grid is evaluated in bands of whole rows whose buffers
 * fit, one after another on `stream`.  No hipMalloc, hipFree or pool call is
 * made and the stage profiler records nothing.  Every call on one GPU shares
 * that GPU's array: calls that overlap in time on one GPU (on different
 * streams, or from different threads) race and must not be made.
 * LENS_ENOMEM (nothing enqueued) if even a single grid row needs more than
 * LENS_NOALLOC_SCRATCH_BYTES; LENS_EINVAL for a NULL plan or grid, or rays
 * outside the plan's region.  opts->method = LENS_DIRECT sums directly (no
 * scratch).  All pointers as in lens_deflect.
 */
LENS_API lens_status lens_deflect_noalloc(lens_plan *plan, const lens_field *field,
                                          const lens_grid *grid, double *y_out,
                                          const lens_opts *opts, void *stream);

/*
 * Inverse ray shooting: deflect every ray of `grid` and add it to the map
 * (see lens_map_desc).  Rays are processed in chunks of whole grid rows of at
 * most opts->max_rays_per_chunk rays (the bounded passes of Section 2.4; by
 * default one pass, as the map needs no per-ray memory); the result does not
 * depend on the chunking.  `plan` may be NULL as in lens_deflect.
 */
LENS_API lens_status lens_map(lens_plan *plan, const lens_field *field, const lens_grid *grid,
                     const lens_map_desc *map, const lens_opts *opts, void *stream);

/* A source-plane magnification map for inverse polygon mapping:
 * mu[v*npix + u] (FP64, device) is accumulated (+=), pixel (u, v) as in
 * lens_map_desc. */
typedef struct {
  double y1min, y2min;  /* lower-left corner of the map */
  double side;          /* side length, > 0 */
  int32_t npix;         /* pixels per side, npix*npix <= INT32_MAX */
  double *mu;           /* [npix][npix] FP64 (device) */
} lens_ipm_desc;

/*
 * Inverse polygon mapping (Section 2.3, first order as in Section 2.4): the
 * rays of `grid` are deflected (as lens_deflect, by FMM or direct sum) and
 * taken as the corners of the (nx-1) x (ny-1) image-plane cells of area
 * dx*dy between adjacent rays.  Each cell maps to a quadrilateral in the
 * source plane whose area is shared exactly among the pixels it overlaps,
 * in proportion to the overlap areas (Green's theorem), however many pixels
 * that is, so map->mu receives the magnification (sum of image areas over
 * pixel area).  A cell that straddles a critical curve maps to a
 * quadrilateral whose edges cross; it is treated as if it were not critical
 * (Section 2.3): the region its edges enclose, the two triangles either side
 * of the crossing, takes the cell's area by overlap.  Only a cell whose image
 * has zero area gives a quarter of its area to the pixel of each corner.
 * Contributions are summed in fixed point (2^-40 of a pixel's
 * magnification), so the map does not depend on summation order.  Rays are
 * processed in passes of whole rows of at most opts->max_rays_per_chunk rays
 * (default 2^28; a pass also holds fewer than 2^32 cells), each pass
 * deflecting its rows plus the first row of the next, so that a grid of any
 * size (e.g. 1.5e11 rays) streams through one plan; a pass needs 16 bytes
 * of scratch per ray for the deflected corners plus 4 bytes per cell, and
 * the map 16 bytes per pixel.  The map does not depend on the pass size.
 * `plan` may be NULL as in lens_deflect.
 */
LENS_API lens_status lens_map_ipm(lens_plan *plan, const lens_field *field, const lens_grid *grid,
                                  const lens_ipm_desc *map, const lens_opts *opts, void *stream);

/*
 * Images of point sources: every x of the grid's region with y(x) =
 * sources[s] (the inverse lens equation; Section 2.5 finds the images of a
 * source behind a particle halo this way).  The grid rays are the corners
 * of (nx-1)(ny-1) cells, each split along its (i,j)-(i+1,j+1) diagonal into
 * two triangles; a triangle whose mapped corners contain a source seeds a
 * candidate at the source's preimage under the triangle's linear map.  Each
 * candidate is refined by up to max_iter Newton steps
 *     x <- x + A(x)^-1 (beta - y(x)),
 *     A = [[c1 - Re f', Im f'], [Im f', c2 + Re f']],  f' = -sum m/(z - z_i)^2,
 * with c1 = 1 - kappa_s - gamma, c2 = 1 - kappa_s + gamma (the derivative of
 * the expansions, Appendix A); a step is at most 4 cell diagonals long and x
 * stays inside the grid's rays' box.  A candidate whose |y(x) - beta| <= tol
 * is an image; images of one source closer than max(1e-3 min(dx, dy),
 * 1e3 tol) are one.  Every image inside the grid's box whose triangle sees
 * its source is found; two images closer than about a cell (a source within
 * a cell's image of a caustic) may come out as one, and the tiny images
 * next to each lens that no grid resolves are found only where a triangle
 * holds them.  Deflections are computed as lens_deflect computes them
 * (plan, method, precision and order from opts; the grid is deflected in
 * passes of whole rows as in lens_map_ipm), so tol should exceed the
 * evaluation's own error (~1e-6 |alpha| for LENS_MIXED).
 *   sources    [n_sources][2] FP64 (device)
 *   images     [cap][4] FP64 (device): x1, x2, magnification 1/det A
 *              (signed: negative for saddle images), residual |y - beta|;
 *              ordered by source, then x1
 *   image_src  [cap] int32 (device): the source of each image
 *   n_images   (host) number of images found; only the first cap are
 *              written
 * Synchronises `stream` (reads back candidate counts).  LENS_EINVAL for bad
 * arguments (tol <= 0, max_iter outside [0, 1000], NULL pointers).
 */
LENS_API lens_status lens_find_images(lens_plan *plan, const lens_field *field,
                                      const lens_grid *grid, const double *sources,
                                      int32_t n_sources, double tol, int32_t max_iter,
                                      double *images, int32_t *image_src, int64_t cap,
                                      int64_t *n_images, const lens_opts *opts, void *stream);

/*
 * Critical curves (det A = 0) over the grid's region, and optionally their
 * caustics.  det A = (c1 - Re f')(c2 + Re f') - (Im f')^2 at every grid ray
 * (f' as lens_deflect's dfdz_out); on each cell a corner-to-corner edge whose
 * end values differ in sign is cut where the linear interpolant of det A
 * vanishes and the cuts are joined into segments (marching squares; a cell
 * cut on all four edges is split by the sign of the mean of its corners).
 *   seg_out      [cap][4] FP64 (device): x1a, x2a, x1b, x2b per segment,
 *                in no particular order
 *   caustic_out  [cap][4] FP64 (device) or NULL: the images y of the same
 *                end points (the caustics)
 *   n_seg        (host) segments found; only the first cap are written
 * The segments' end points are within O(dx^2) of the curve where det A is
 * smooth on the scale of a cell.  Synchronises `stream`.
 */
LENS_API lens_status lens_critical_curves(lens_plan *plan, const lens_field *field,
                                          const lens_grid *grid, double *seg_out,
                                          double *caustic_out, int64_t cap, int64_t *n_seg,
                                          const lens_opts *opts, void *stream);

/*
 * Multi-plane ray tracing: a thick lens as a chain of thin planes (the
 * extension noted in the introduction).  Plane 0 is nearest the observer;
 * a ray starts at x_0 (grid or explicit rays, as lens_deflect) and reaches
 * plane j at
 *     x_j = x_0 - sum_{i<j} beta[j*n_planes + i] alpha_i(x_i),
 * and the source plane at y = x_0 - sum_i alpha_i(x_i), where alpha_i(x) =
 * x - y_i(x) is plane i's full deflection (its stars and its kappa_s and
 * gamma, y_i as lens_deflect computes it) and beta_ij = D_ij D_s / (D_j D_is)
 * are the distance ratios, plane deflections being scaled to the source
 * plane.  fields[n_planes]; beta: host, [n_planes][n_planes], only i < j
 * read (may be NULL for one plane); n_planes <= 64.  Each plane is
 * evaluated by lens_deflect with `opts` and no plan (planes after the first
 * see explicit rays, so each such call reads back a bounding box).  Scratch:
 * 16 (n_planes + 2) bytes per ray.
 */
LENS_API lens_status lens_deflect_multiplane(int32_t n_planes, const lens_field *fields,
                                             const double *beta, const lens_grid *grid,
                                             const double *rays_xy, int64_t n_rays,
                                             double *y_out, const lens_opts *opts, void *stream);

/*
 * Empirical autotuner for one field and ray grid: the expansion order p, the
 * leaf level and, for LENS_MIXED, fp32_levels (Appendix A leaves p and the
 * tree depth to the user; here they are measured).  A strided sample of at
 * most 256 x 256 rays of `grid` is deflected by the FP64 direct sum and by
 * the FMM at p = 6, 7, ... (a plan over the whole grid, as lens_deflect and
 * lens_map build it).  The error is the largest per-ray relative deflection
 * error |dalpha_k| / max(|alpha_k|, 1e-3 rms alpha) over the sample when
 * map is NULL, else the expected fraction of
 * rays binned into another pixel of `map`, mean(|dy1| + |dy2|) npix / side
 * (map->counts is not touched).  A setting reaches `tol` when its sampled
 * error is at most 0.5 tol (a margin for the rays outside the sample).  Of
 * the settings that reach `tol` the one
 * with the fastest whole lens_deflect (or lens_map) call is kept, and the
 * leaf level one either side of the library's choice is timed too (unless
 * base->leaf_level is set).  base: method and precision.  Runs full calls on
 * scratch memory and synchronises `stream`.  The choice is cached, as for
 * order_p = 0 (in-process by the call's arrays and parameters, on disk by a
 * coarse description of the problem): a cached answer returns without
 * measuring (from the disk cache with err_out and ms_out NaN).  *out receives the chosen
 * options; err_out and ms_out (may be NULL) the sampled error and the time
 * of one call in ms.  LENS_EUNSUPPORTED if no p up to LENS_MAX_ORDER reaches
 * tol; *out then holds the most accurate setting tried.
 */
LENS_API lens_status lens_autotune(const lens_field *field, const lens_grid *grid,
                                   const lens_map_desc *map, double tol, const lens_opts *base,
                                   void *stream, lens_opts *out, double *err_out, double *ms_out);

/*
 * Stage profiler.  lens_profile_enable(1) clears the totals and starts
 * bracketing every stage of every later call (tree, upward, downward, eval,
 * direct) with HIP events on the stream that runs it; (0) stops.
 * lens_profile_read waits for the recorded events, then fills up to `cap`
 * entries: stage names (host strings valid until the next enable), total
 * milliseconds and number of timed launches.  Returns the number of stages.
 * Process-wide; meant for benchmarks, not for concurrent calls.
 */
LENS_API void lens_profile_enable(int32_t on);
LENS_API int32_t lens_profile_read(int32_t cap, const char **names, double *total_ms,
                                   int64_t *launches);

/*
 * Adjoint of lens_deflect with respect to the lenses: given
 * grad_y[k][2] = dL/dy_k for the rays of `grid` (rays_xy NULL) or of
 * rays_xy[n_rays][2] (grid NULL), writes
 *     grad_xy[i][2] = dL/d(x_i),  grad_m[i] = dL/dm_i      (FP64, device)
 * for every star, in the caller's star order (kappa_s and gamma do not
 * enter).  With g_k = dL/dy1_k + i dL/dy2_k and h(z) = sum_k g_k / (z - z_k):
 * dL/dm_i = Re h(z_i) and dL/dx_i + i dL/dy_i = m_i conj(h'(z_i)), from
 * differentiating eq. 1.  LENS_FMM evaluates h and h' by the fast multipole
 * method with the rays as sources (complex charges) and the stars as
 * targets; LENS_DIRECT sums them directly in FP64 over the field's star
 * arrays (field required).  A ray exactly on a star is skipped, as in the
 * forward map.
 * With a `plan` (the forward call's; `field` may then be NULL) the stars,
 * their tree, expansion order, precision and quadtree geometry come from the
 * plan: the rays' tree takes the plan's geometry and the stars need no sort,
 * so a grid call does not wait on the stream (explicit rays: one read-back of
 * their bounding box, which must lie in the plan's root square).  Without a
 * plan the call waits on the stream to read back the bounding boxes of the
 * stars and the rays (FMM).
 */
LENS_API lens_status lens_deflect_backward(lens_plan *plan, const lens_field *field,
                                           const lens_grid *grid, const double *rays_xy,
                                           int64_t n_rays, const double *grad_y, double *grad_xy,
                                           double *grad_m, const lens_opts *opts, void *stream);

/*
 * Inverse ray shooting for n_fields independent fields in one call: the rays
 * of grids[i] lensed by fields[i] are added into maps[i] (see lens_map).
 * fields, grids and maps are HOST arrays of n_fields structs (their data
 * pointers are device pointers); one opts applies to every field (NULL =
 * defaults; the leaf level is chosen per field).  All fields' work --
 * tree builds, expansions, downward passes and binned evaluations -- is
 * allocated up front and captured once as a HIP graph whose branches run
 * the fields concurrently; the graph is cached (a few batches) by the
 * arrays, sizes and parameters, and replayed by later calls while every
 * field's stars stay inside its captured quadtree.  Waits on `stream` once
 * per call, to read back the fields' bounding boxes.  Fields may differ in
 * N_*, kappa_s, gamma, grid and map.
 */
LENS_API lens_status lens_map_batched(int32_t n_fields, const lens_field *fields,
                                      const lens_grid *grids, const lens_map_desc *maps,
                                      const lens_opts *opts, void *stream);

/* Release the cached graphs (lens_map_batched, and plan-less grid calls of
 * lens_deflect / lens_map) and their device buffers (waits for them). */
LENS_API void lens_release_cached(void);

/* Thread-local text for the last status other than LENS_OK (host string). */
LENS_API const char *lens_last_error(void);

/* Library version string (host string). */
LENS_API const char *lens_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LENS_H */
