// Quadtree construction (Appendix A, initialisation step): bounding boxes,
// leaf-box keys, a stable LSD radix sort of (key, index) pairs, gathers and
// per-box start offsets.  Keys are row-major leaf-box indices iy * 2^L + ix,
// so the 3 boxes of one row of a 3x3 neighbourhood are contiguous in the
// sorted order.  The sort is stable and every reduction runs in a fixed
// order, so the tree (and everything computed from it) is bitwise
// reproducible run to run.
#include <cfloat>

#include "device_common.h"

namespace lensfmm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// ------------------------------------------------------------ bounding box

// v = {x1min, x2min, x1max, x2max} of the grid-strided points of xy[0, n).
__device__ inline void bbox_accumulate(const double *__restrict__ xy, int64_t n, double v[4]) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double a = xy[2 * i], b = xy[2 * i + 1];
    v[0] = fmin(v[0], a);
    v[1] = fmin(v[1], b);
    v[2] = fmax(v[2], a);
    v[3] = fmax(v[3], b);
  }
}

// v = min/max over the parts [0, nparts) of partial boxes laid out [part][4].
__device__ inline void bbox_merge_parts(const double *__restrict__ pp, int nparts, double v[4]) {
  for (int i = threadIdx.x; i < nparts; i += kThreads) {
    v[0] = fmin(v[0], pp[4 * i + 0]);
    v[1] = fmin(v[1], pp[4 * i + 1]);
    v[2] = fmax(v[2], pp[4 * i + 2]);
    v[3] = fmax(v[3], pp[4 * i + 3]);
  }
}

// Reduces every thread's box v over the workgroup (a fixed tree order) and
// writes the result to out[0..3].
__device__ inline void bbox_block_store(const double v[4], double *__restrict__ out) {
  __shared__ double red[4][kThreads];
  for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + o]);
      red[1][threadIdx.x] = fmin(red[1][threadIdx.x], red[1][threadIdx.x + o]);
      red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + o]);
      red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = red[threadIdx.x][0];
}

// Per-workgroup bounding box of xy[0, n) (partial[part][4]) and, with
// has_box, the number of points inside the closed rectangle {b0, b1, b2, b3}
// (pcount[part]): one read of the points for both.
// Sum of one value per thread over the workgroup (the result in every thread).
__device__ inline unsigned long long block_sum_u64(unsigned long long c) {
  __shared__ unsigned long long red[kThreads];
  red[threadIdx.x] = c;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  return red[0];
}

__global__ __launch_bounds__(kThreads) void k_bbox_partial(const double *__restrict__ xy, int64_t n,
                                                           int has_box, double b0, double b1,
                                                           double b2, double b3,
                                                           double *__restrict__ partial,
                                                           unsigned long long *__restrict__ pcount) {
  double v[4] = {DBL_MAX, DBL_MAX, -DBL_MAX, -DBL_MAX};
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const double a = xy[2 * i], b = xy[2 * i + 1];
    v[0] = fmin(v[0], a);
    v[1] = fmin(v[1], b);
    v[2] = fmax(v[2], a);
    v[3] = fmax(v[3], b);
    c += (a >= b0 && a <= b2 && b >= b1 && b <= b3) ? 1ull : 0ull;
  }
  bbox_block_store(v, partial + 4 * blockIdx.x);
  if (has_box) {
    c = block_sum_u64(c);
    if (threadIdx.x == 0) pcount[blockIdx.x] = c;
  }
}

// out = {x1min, x2min, x1max, x2max} and, with has_box, the count as the
// bits of out[4]; out may be host-mapped memory (the read-back landing).
__global__ __launch_bounds__(kThreads) void k_bbox_final(const double *__restrict__ partial,
                                                         const unsigned long long *__restrict__ pcount,
                                                         int nparts, int has_box,
                                                         double *__restrict__ out) {
  double v[4] = {DBL_MAX, DBL_MAX, -DBL_MAX, -DBL_MAX};
  bbox_merge_parts(partial, nparts, v);
  bbox_block_store(v, out);
  if (has_box) {
    unsigned long long c = 0;
    for (int i = threadIdx.x; i < nparts; i += kThreads) c += pcount[i];
    c = block_sum_u64(c);
    if (threadIdx.x == 0) reinterpret_cast<unsigned long long *>(out)[4] = c;
  }
}

// Bounding boxes of several point sets at once: blockIdx.y = set; partial
// results [set][part][4], then one workgroup per set reduces its parts.
__global__ __launch_bounds__(kThreads) void k_bbox_multi_partial(const BBoxSet *__restrict__ sets,
                                                                 int nparts,
                                                                 double *__restrict__ partial) {
  const BBoxSet S = sets[blockIdx.y];
  double v[4] = {DBL_MAX, DBL_MAX, -DBL_MAX, -DBL_MAX};
  bbox_accumulate(S.xy, S.n, v);
  bbox_block_store(v, partial + ((size_t)blockIdx.y * nparts + blockIdx.x) * 4);
}

__global__ __launch_bounds__(kThreads) void k_bbox_multi_final(const double *__restrict__ partial,
                                                               int nparts, double *__restrict__ out) {
  double v[4] = {DBL_MAX, DBL_MAX, -DBL_MAX, -DBL_MAX};
  bbox_merge_parts(partial + (size_t)blockIdx.x * nparts * 4, nparts, v);
  bbox_block_store(v, out + (size_t)blockIdx.x * 4);
}

// --------------------------------------------------------------- leaf keys

// Leaf key (row-major box index) and identity index of every source; with
// box_count, also the number of sources per leaf box (integer atomics, so
// the counts are exact whatever the order).
__global__ __launch_bounds__(kThreads) void k_leaf_keys(const double *__restrict__ xy, int64_t n,
                                                        Geometry g, uint32_t *__restrict__ keys,
                                                        uint32_t *__restrict__ vals,
                                                        uint32_t *__restrict__ box_count) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t nb = int64_t(1) << g.L;
  const double s = ldexp(g.side, -g.L);
  const int64_t ix = box_coord(xy[2 * i], g.x0, s, nb);
  const int64_t iy = box_coord(xy[2 * i + 1], g.y0, s, nb);
  const uint32_t k = (uint32_t)(iy * nb + ix);
  keys[i] = k;
  vals[i] = (uint32_t)i;
  if (box_count) atomicAdd(&box_count[k], 1u);
}

__global__ __launch_bounds__(kThreads) void k_fill_u32(uint32_t *__restrict__ p, int64_t n,
                                                       uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    p[i] = v;
}

// ------------------------------------------------------------------ scans
// Exclusive scan of uint32 in three phases: tile sums, a single-workgroup
// scan of the tile sums (carried across chunks), tile scans with offsets.

constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive scan across the workgroup of one value per thread; returns the
// thread's exclusive prefix and writes the total to *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *sh /*[kWaves]*/,
                                                    uint32_t *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(x, lane);
  if (lane == 63) sh[w] = incl;
  __syncthreads();
  uint32_t woff = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) {
    if (q < w) woff += sh[q];
    tot += sh[q];
  }
  __syncthreads();
  *total = tot;
  return woff + incl - x;
}

__global__ __launch_bounds__(kThreads) void k_scan_tile_sums(const uint32_t *__restrict__ in,
                                                             size_t n, uint32_t *__restrict__ sums) {
  const size_t base = (size_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
  for (int it = 0; it < kScanItems; ++it) {
    const size_t i = base + (size_t)it * kThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  __shared__ uint32_t sh[kWaves];
  uint32_t tot;
  (void)block_excl_scan(s, sh, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Scan of one tile.  The tile's offset is the sum of the earlier tiles'
// sums, read directly when tiles are few (this replaces a separate scan of
// the sums); with PRE the offsets come already scanned (many tiles).
template <bool PRE>
__global__ __launch_bounds__(kThreads) void k_scan_tiles(const uint32_t *__restrict__ in, size_t n,
                                                         const uint32_t *__restrict__ sums,
                                                         uint32_t *__restrict__ out) {
  // thread t owns the kScanItems consecutive elements [t*items, (t+1)*items)
  __shared__ uint32_t tile[kScanTile];
  __shared__ uint32_t sh[kWaves];
  const size_t base = (size_t)blockIdx.x * kScanTile;
  for (int it = 0; it < kScanItems; ++it) {
    const size_t i = base + (size_t)it * kThreads + threadIdx.x;
    tile[it * kThreads + threadIdx.x] = (i < n) ? in[i] : 0u;
  }
  __syncthreads();
  uint32_t loc[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    loc[j] = s;
    s += tile[threadIdx.x * kScanItems + j];
  }
  uint32_t tile_off;
  if (PRE) {
    tile_off = sums[blockIdx.x];
  } else {
    uint32_t before = 0;
    for (unsigned i = threadIdx.x; i < blockIdx.x; i += kThreads) before += sums[i];
    (void)block_excl_scan(before, sh, &tile_off);
  }
  uint32_t tot;
  const uint32_t ex = block_excl_scan(s, sh, &tot);
  const uint32_t off = tile_off + ex;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) tile[threadIdx.x * kScanItems + j] = off + loc[j];
  __syncthreads();
  for (int it = 0; it < kScanItems; ++it) {
    const size_t i = base + (size_t)it * kThreads + threadIdx.x;
    if (i < n) out[i] = tile[it * kThreads + threadIdx.x];
  }
}

// ------------------------------------------------------------- radix sort

// Tiles of kThreads * ITEMS keys: 2048 (twice as many workgroups as 4096-key
// tiles, which measured faster for 1e6 keys: more waves in flight per CU)
// up to kLongSort keys, 4096 beyond (a digit's run in a tile is then twice
// as long, so the scatter writes fuller cache lines).
constexpr int kSortItems = 8, kLongSortItems = 16;
constexpr int kSortTile = kThreads * kSortItems;
constexpr int64_t kLongSort = int64_t(1) << 23;

template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_radix_count(const uint32_t *__restrict__ keys,
                                                          int64_t n, int shift,
                                                          uint32_t *__restrict__ counts,
                                                          int nblocks) {
  constexpr int TILE = kThreads * ITEMS;
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * TILE;
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t i = base + (int64_t)it * kThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  counts[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter.  Items of a tile are taken in global order (round `it`,
// then thread).  A key's destination is the digit's global offset for this
// tile + the keys of that digit in earlier (round, wave) pairs of the tile +
// those in lower lanes of its own wave (found with ballots on the digit
// bits).  Every item of the tile is ranked first, the per-(round, wave,
// digit) counts are turned into offsets by one thread per digit, and only
// then are the items written: three barriers per tile.
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ offsets,
    int nblocks) {
  constexpr int TILE = kThreads * ITEMS;
  __shared__ uint32_t run[256];
  // counts, then offsets within the tile (<= TILE, fits 16 bits)
  __shared__ uint16_t cnt[ITEMS][kWaves][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  run[t] = offsets[(size_t)t * nblocks + blockIdx.x];
  {
    uint32_t *c32 = reinterpret_cast<uint32_t *>(&cnt[0][0][0]);
    for (int e = t; e < ITEMS * kWaves * 256 / 2; e += kThreads) c32[e] = 0u;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * TILE;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t i = base + (int64_t)it * kThreads + t;
    const bool valid = i < n;
    key[it] = valid ? kin[i] : 0u;
    val[it] = valid ? vin[i] : 0u;
    const uint32_t d = (key[it] >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    rank[it] = (uint32_t)__popcll(peers & below);
    // the highest lane of each digit group records the group's size
    if (valid && (peers >> lane) == 1ull) cnt[it][w][d] = (uint16_t)__popcll(peers);
  }
  __syncthreads();
  {
    // thread t: exclusive prefix of digit t's counts over (round, wave)
    uint32_t pre = 0;
    for (int it = 0; it < ITEMS; ++it)
#pragma unroll
      for (int q = 0; q < kWaves; ++q) {
        const uint32_t c = cnt[it][q][t];
        cnt[it][q][t] = (uint16_t)pre;
        pre += c;
      }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int64_t i = base + (int64_t)it * kThreads + t;
    if (i < n) {
      const uint32_t d = (key[it] >> shift) & 255u;
      const uint32_t pos = run[d] + cnt[it][w][d] + rank[it];
      kout[pos] = key[it];
      vout[pos] = val[it];
    }
  }
}

// ----------------------------------------------------------------- gathers

// sources sorted by leaf box: positions and qdim charge components each
__global__ __launch_bounds__(kThreads) void k_gather_stars(const uint32_t *__restrict__ perm,
                                                           const double *__restrict__ xy,
                                                           const double *__restrict__ q, int qdim,
                                                           int64_t n, double *__restrict__ sxy,
                                                           double *__restrict__ sq,
                                                           float *__restrict__ sq32) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= n) return;
  const int64_t i = perm[j];
  sxy[2 * j] = xy[2 * i];
  sxy[2 * j + 1] = xy[2 * i + 1];
  for (int c = 0; c < qdim; ++c) sq[qdim * j + c] = q[qdim * i + c];
  if (sq32) sq32[j] = (float)q[i];
}

// Several fields' trees in one pass (batched maps): field j's sources are
// elements [off_j, off_j + n_j) of the combined key/value arrays, keyed
// (j << shift) | leaf key, so one stable sort orders every field by leaf box
// (within a field exactly as its own sort would).
__device__ __forceinline__ int tree_job_of(const TreeJob *__restrict__ jobs, int njobs, int64_t g) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].off <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kThreads) void k_leaf_keys_multi(const TreeJob *__restrict__ jobs,
                                                              int njobs, int64_t total, int shift,
                                                              uint32_t *__restrict__ keys,
                                                              uint32_t *__restrict__ vals) {
  const int64_t gi = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (gi >= total) return;
  const int j = tree_job_of(jobs, njobs, gi);
  const TreeJob &t = jobs[j];
  const int64_t i = gi - t.off;
  const int64_t nb = int64_t(1) << t.g.L;
  const double s = ldexp(t.g.side, -t.g.L);
  const int64_t ix = box_coord(t.xy[2 * i], t.g.x0, s, nb);
  const int64_t iy = box_coord(t.xy[2 * i + 1], t.g.y0, s, nb);
  keys[gi] = ((uint32_t)j << shift) | (uint32_t)(iy * nb + ix);
  vals[gi] = (uint32_t)i;
}

// Sorted position gi of the combined arrays: field j's source perm[gi]
// (a field-local index) into that field's sorted arrays; the key loses its
// field bits.
__global__ __launch_bounds__(kThreads) void k_gather_multi(const TreeJob *__restrict__ jobs, int njobs,
                                                           int64_t total, uint32_t mask,
                                                           uint32_t *__restrict__ keys,
                                                           const uint32_t *__restrict__ perm) {
  const int64_t gi = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (gi >= total) return;
  const int j = tree_job_of(jobs, njobs, gi);
  const TreeJob &t = jobs[j];
  const int64_t k = gi - t.off;
  const int64_t i = perm[gi];
  t.sxy[2 * k] = t.xy[2 * i];
  t.sxy[2 * k + 1] = t.xy[2 * i + 1];
  t.sq[k] = t.q[i];
  if (t.sq32) t.sq32[k] = (float)t.q[i];
  keys[gi] &= mask;
}

__global__ __launch_bounds__(kThreads) void k_gather_rays(const uint32_t *__restrict__ perm,
                                                          const double *__restrict__ xy, int64_t n,
                                                          double *__restrict__ sxy) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= n) return;
  const uint32_t i = perm[j];
  sxy[2 * j] = xy[2 * (int64_t)i];
  sxy[2 * j + 1] = xy[2 * (int64_t)i + 1];
}

// start[b] = lower_bound of box b in the sorted keys, b = 0..nbox, in two
// steps: every stride-th box searches the whole array; then a workgroup per
// stride of boxes counts the keys between its two coarse bounds per box
// (LDS histogram) and writes their exclusive prefix, so each key is read once
// and each entry written once, with no per-box search.  The stride is 256
// boxes (one per thread: more workgroups in flight) for trees of up to 2^22
// leaves and 4096 (16 per thread, so the per-workgroup cost stays small
// against its 16 KB of output) beyond; a stride without keys only fills its
// entries (the deep, mostly empty trees of clustered fields: 2.7e8 boxes).
constexpr int64_t kWideStartsFrom = int64_t(1) << 22;

__global__ __launch_bounds__(kThreads) void k_box_starts_coarse(const uint32_t *__restrict__ keys,
                                                                int64_t n, int64_t nbox,
                                                                int64_t stride,
                                                                int32_t *__restrict__ coarse) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t nc = nbox / stride + 1;
  if (c > nc) return;
  const int64_t b = c * stride < nbox ? c * stride : nbox;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  coarse[c] = (int32_t)lo;
}

template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_box_starts(const uint32_t *__restrict__ keys,
                                                         int64_t nbox,
                                                         const int32_t *__restrict__ coarse,
                                                         int32_t *__restrict__ start) {
  constexpr int64_t STRIDE = (int64_t)kThreads * ITEMS;
  __shared__ uint32_t cnt[STRIDE];
  __shared__ uint32_t sh[kWaves];
  const int t = threadIdx.x;
  const int64_t c = blockIdx.x, b0 = c * STRIDE;
  // the keys in [lo, hi) are those of boxes [b0, b0 + stride)
  const int32_t lo = coarse[c], hi = coarse[c + 1];
  const int64_t nb = nbox + 1 - b0 < STRIDE ? nbox + 1 - b0 : STRIDE;
  if (lo == hi) {  // no keys: every start is lo (workgroup-uniform)
    for (int64_t j = t; j < nb; j += kThreads) start[b0 + j] = lo;
    return;
  }
  for (int j = t; j < STRIDE; j += kThreads) cnt[j] = 0;
  __syncthreads();
  for (int64_t j = (int64_t)lo + t; j < hi; j += kThreads) atomicAdd(&cnt[keys[j] - b0], 1u);
  __syncthreads();
  // thread t: boxes [t * ITEMS, (t + 1) * ITEMS), prefixed within the
  // thread, then across the workgroup; the prefixes go back to LDS for
  // coalesced stores
  uint32_t v[ITEMS], sum = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    v[i] = sum;
    sum += cnt[t * ITEMS + i];
  }
  uint32_t tot;
  const uint32_t ex = block_excl_scan(sum, sh, &tot);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) cnt[t * ITEMS + i] = ex + v[i];
  __syncthreads();
  for (int64_t j = t; j < nb; j += kThreads) start[b0 + j] = lo + (int32_t)cnt[j];
}

inline unsigned blocks_for(int64_t n, int per = kThreads) {
  return (unsigned)((n + per - 1) / per);
}

}  // namespace

// ------------------------------------------------------------- launchers

int bbox_parts(int64_t n) {
  int64_t b = (n + kThreads * 8 - 1) / (kThreads * 8);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

void launch_bbox(const double *xy, int64_t n, double *partial, int nparts, const double *count_box,
                 double *out, hipStream_t stream) {
  const bool has = count_box != nullptr;
  const double b0 = has ? count_box[0] : 0.0, b1 = has ? count_box[1] : 0.0;
  const double b2 = has ? count_box[2] : -1.0, b3 = has ? count_box[3] : -1.0;
  auto *pcount = reinterpret_cast<unsigned long long *>(partial + 4 * (size_t)nparts);
  hipLaunchKernelGGL(k_bbox_partial, dim3(nparts), dim3(kThreads), 0, stream, xy, n, (int)has, b0,
                     b1, b2, b3, partial, pcount);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kThreads), 0, stream, partial, pcount, nparts,
                     (int)has, out);
  LENS_HIP(hipGetLastError());
}

void launch_bbox_multi(const BBoxSet *sets_dev, int nsets, int nparts, double *partial,
                       double *out, hipStream_t stream) {
  if (nsets == 0) return;
  hipLaunchKernelGGL(k_bbox_multi_partial, dim3(nparts, nsets), dim3(kThreads), 0, stream, sets_dev,
                     nparts, partial);
  hipLaunchKernelGGL(k_bbox_multi_final, dim3(nsets), dim3(kThreads), 0, stream, partial, nparts,
                     out);
  LENS_HIP(hipGetLastError());
}

void launch_leaf_keys(const double *xy, int64_t n, Geometry g, uint32_t *keys, uint32_t *vals,
                      uint32_t *box_count, hipStream_t stream) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_leaf_keys, dim3(blocks_for(n)), dim3(kThreads), 0, stream, xy, n, g, keys,
                     vals, box_count);
  LENS_HIP(hipGetLastError());
}

void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream) {
  if (n == 0) return;
  int64_t nb = blocks_for(n);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)nb), dim3(kThreads), 0, stream, p, n, v);
  LENS_HIP(hipGetLastError());
}

// Tiles up to which each tile sums its predecessors' totals itself; beyond,
// the totals are scanned first (recursively), so the work stays linear.
constexpr size_t kDirectTiles = 1024;

size_t scan_tmp_len(size_t n) {
  const size_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb <= kDirectTiles) return nb + 1;
  return 2 * nb + scan_tmp_len(nb) + 1;
}

void exclusive_scan_u32(const uint32_t *in, uint32_t *out, size_t n, uint32_t *tmp,
                        hipStream_t stream) {
  if (n == 0) return;
  const size_t nb = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)nb), dim3(kThreads), 0, stream, in, n, tmp);
  if (nb <= kDirectTiles) {
    hipLaunchKernelGGL(k_scan_tiles<false>, dim3((unsigned)nb), dim3(kThreads), 0, stream, in, n,
                       tmp, out);
  } else {
    uint32_t *offs = tmp + nb;
    exclusive_scan_u32(tmp, offs, nb, offs + nb, stream);
    hipLaunchKernelGGL(k_scan_tiles<true>, dim3((unsigned)nb), dim3(kThreads), 0, stream, in, n,
                       offs, out);
  }
  LENS_HIP(hipGetLastError());
}

size_t radix_counts_len(int64_t n) {
  const int64_t nb = (n + kSortTile - 1) / kSortTile;
  return (size_t)(nb < 1 ? 1 : nb) * 256;
}

template <int ITEMS>
static bool radix_passes(uint32_t *k, uint32_t *v, uint32_t *k_tmp, uint32_t *v_tmp, int64_t n,
                         int bits, uint32_t *counts, uint32_t *scan_tmp, hipStream_t stream) {
  constexpr int64_t TILE = kThreads * ITEMS;
  const int nb = (int)((n + TILE - 1) / TILE);
  bool in_tmp = false;
  for (int shift = 0; shift < bits; shift += 8) {
    uint32_t *ki = in_tmp ? k_tmp : k, *vi = in_tmp ? v_tmp : v;
    uint32_t *ko = in_tmp ? k : k_tmp, *vo = in_tmp ? v : v_tmp;
    hipLaunchKernelGGL((k_radix_count<ITEMS>), dim3(nb), dim3(kThreads), 0, stream, ki, n, shift,
                       counts, nb);
    exclusive_scan_u32(counts, counts, (size_t)nb * 256, scan_tmp, stream);
    hipLaunchKernelGGL((k_radix_scatter<ITEMS>), dim3(nb), dim3(kThreads), 0, stream, ki, vi, ko, vo,
                       n, shift, counts, nb);
    LENS_HIP(hipGetLastError());
    in_tmp = !in_tmp;
  }
  return in_tmp;
}

bool radix_sort_pairs(uint32_t *k, uint32_t *v, uint32_t *k_tmp, uint32_t *v_tmp, int64_t n,
                      int bits, uint32_t *counts, uint32_t *scan_tmp, hipStream_t stream) {
  if (n <= 1 || bits <= 0) return false;
  if (n > kLongSort)
    return radix_passes<kLongSortItems>(k, v, k_tmp, v_tmp, n, bits, counts, scan_tmp, stream);
  return radix_passes<kSortItems>(k, v, k_tmp, v_tmp, n, bits, counts, scan_tmp, stream);
}

void launch_gather_stars(const uint32_t *perm, const double *xy, const double *q, int qdim,
                         int64_t n, double *sxy, double *sq, float *sq32, hipStream_t stream) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather_stars, dim3(blocks_for(n)), dim3(kThreads), 0, stream, perm, xy, q,
                     qdim, n, sxy, sq, qdim == 1 ? sq32 : nullptr);
  LENS_HIP(hipGetLastError());
}

void launch_leaf_keys_multi(const TreeJob *jobs, int njobs, int64_t total, int shift, uint32_t *keys,
                            uint32_t *vals, hipStream_t stream) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_leaf_keys_multi, dim3(blocks_for(total)), dim3(kThreads), 0, stream, jobs,
                     njobs, total, shift, keys, vals);
  LENS_HIP(hipGetLastError());
}

void launch_gather_multi(const TreeJob *jobs, int njobs, int64_t total, uint32_t mask, uint32_t *keys,
                         const uint32_t *perm, hipStream_t stream) {
  if (total == 0) return;
  hipLaunchKernelGGL(k_gather_multi, dim3(blocks_for(total)), dim3(kThreads), 0, stream, jobs, njobs,
                     total, mask, keys, perm);
  LENS_HIP(hipGetLastError());
}

void launch_gather_rays(const uint32_t *perm, const double *xy, int64_t n, double *sxy,
                        hipStream_t stream) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather_rays, dim3(blocks_for(n)), dim3(kThreads), 0, stream, perm, xy, n,
                     sxy);
  LENS_HIP(hipGetLastError());
}

void launch_box_starts(const uint32_t *sorted_keys, int64_t n, int64_t nbox, int32_t *start,
                       int32_t *coarse, hipStream_t stream) {
  const bool wide = nbox >= kWideStartsFrom;
  const int64_t stride = wide ? (int64_t)kThreads * 16 : kThreads;
  const int64_t nc = nbox / stride + 2;
  hipLaunchKernelGGL(k_box_starts_coarse, dim3(blocks_for(nc)), dim3(kThreads), 0, stream,
                     sorted_keys, n, nbox, stride, coarse);
  const dim3 grid((unsigned)(nbox / stride + 1));
  if (wide)
    hipLaunchKernelGGL(k_box_starts<16>, grid, dim3(kThreads), 0, stream, sorted_keys, nbox, coarse, start);
  else
    hipLaunchKernelGGL(k_box_starts<1>, grid, dim3(kThreads), 0, stream, sorted_keys, nbox, coarse, start);
  LENS_HIP(hipGetLastError());
}

int64_t box_starts_coarse_len(int64_t nbox) { return nbox / kThreads + 2; }

}  // namespace lensfmm
