// One round of parallel nearest-neighbour-chain HAC (ParChain, Alg. 1), as
// HIP kernels for gfx950.
//
//   act pass        terminals (Alg. 1 last line), n_min (Sec. 4.1), grid bbox
//   grid            counting sort of active clusters by centroid cell; the
//                   flat stand-in for the per-round centroid k-d tree
//   nn search       per terminal: ring search outward from its own cell with
//                   the linkage's centroid bound (Table 1 radius, Sec. 4.1-4.3)
//                   as the stop rule; argmin on (distance, cluster ID)
//   full scan       terminals whose ring search gets too wide (and every
//                   terminal when pruning is off or d is large): one block
//                   scans all active clusters
//   pair tiles      exact complete/average distances of large cluster pairs,
//                   64x64 point tiles (deferred from the search)
//   chain           succ / WriteMin(pred) (Alg. 1, read as in DESIGN notes)
//   R-NN + merge    reciprocal pairs filtered and merged in parallel
//   compaction      active list, and for complete/average the point layout
//                   so that every cluster stays a contiguous range
//
// Distances are FP64 on float32 inputs. Values compared inside a search are
// "keys": Ward the squared distance, complete the largest squared point
// distance, average the mean distance; all are monotone in the linkage
// distance. Every value of a cluster pair is computed the same way whoever
// computes it, so decisions do not depend on the launch shape.
#include <float.h>
#include <math.h>

#include "pc_common.hpp"

namespace pc {

namespace {

constexpr int kCellBudget = 160;        // default: cells a thread may visit before handing off
constexpr double kSlack = 1.0 + 1e-9;   // bounds are applied with this margin
constexpr unsigned long long kNoKey = ~0ull;

__device__ __forceinline__ unsigned f32_bits_up(double h) {
  // float bits of h rounded toward +inf (an upper bound of h)
  float f = (float)h;
  if ((double)f < h) f = nextafterf(f, INFINITY);
  return __float_as_uint(f);
}

template <class T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, kWave);
    v = u < v ? u : v;
  }
  return v;
}
template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, kWave);
    v = u > v ? u : v;
  }
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// block-wide: add a per-thread count into a global counter with one atomic per wave
__device__ __forceinline__ void count_add(long long *dst, long long v) {
  v = wave_sum_ll(v);
  if ((threadIdx.x & (kWave - 1)) == 0 && v) atomicAdd((unsigned long long *)dst, (unsigned long long)v);
}

// One atomic per block: reduce within each wave, then across the block's waves.
template <class T, bool MIN>
__device__ __forceinline__ T block_reduce(T v) {
  __shared__ T red[kBlock / kWave];
  v = MIN ? wave_min(v) : wave_max(v);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  T r = red[0];
  for (int j = 1; j < kBlock / kWave; ++j) r = MIN ? (red[j] < r ? red[j] : r) : (red[j] > r ? red[j] : r);
  return r;
}

// (value, key) lexicographic improvement test
__device__ __forceinline__ bool better(double v, unsigned long long key, double bv, unsigned long long bkey) {
  return v < bv || (v == bv && key < bkey);
}

__device__ __forceinline__ unsigned long long make_key(int cid, int slot) {
  return ((unsigned long long)(unsigned)cid << 32) | (unsigned)slot;
}

// ------------------------------------------------------------------ init --
__global__ void k_reset_round(Counters *c) {
  c->n_ovf = 0;
  c->n_cand = 0;
  c->cand_overflow = 0;
  c->n_pend = 0;
  c->n_pairs = 0;
  c->pair_overflow = 0;
  c->n_min = 0x7fffffff;
  for (int a = 0; a < kMortonAxes; ++a) {
    c->bb_lo[a] = ~0ull;
    c->bb_hi[a] = 0ull;
  }
  c->n_tiles = 0;
}

// per Gram batch: the append counters start empty
__global__ void k_reset_batch(Counters *c) {
  c->n_small = 0;
  c->n_scr = 0;
  c->n_scr32 = 0;
  c->n_cand = 0;
  c->n_pairs = 0;
  c->n_pend = 0;
  c->cand_overflow = 0;
  c->pair_overflow = 0;
  c->n_tiles = 0;
  c->n_chunks = 0;
}

__global__ void k_check_finite(const float *x, long long count, Counters *c) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) c->nonfinite = 1;
}

__global__ void k_point_bbox(const float *x, int n, int d, int axes, Counters *c) {
  unsigned long long lo[kMortonAxes], hi[kMortonAxes];
#pragma unroll
  for (int a = 0; a < kMortonAxes; ++a) {
    lo[a] = ~0ull;
    hi[a] = 0ull;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
#pragma unroll
    for (int a = 0; a < kMortonAxes; ++a)
      if (a < axes) {
        unsigned long long b = ordered_bits((double)x[(size_t)i * d + a]);
        lo[a] = b < lo[a] ? b : lo[a];
        hi[a] = b > hi[a] ? b : hi[a];
      }
#pragma unroll
  for (int a = 0; a < kMortonAxes; ++a) {
    if (a >= axes) break;  // uniform: axes is a kernel argument
    unsigned long long l = block_reduce<unsigned long long, true>(lo[a]);
    unsigned long long h = block_reduce<unsigned long long, false>(hi[a]);
    if (threadIdx.x == 0) {
      atomicMin(&c->bb_lo[a], l);
      atomicMax(&c->bb_hi[a], h);
    }
  }
}

__device__ __forceinline__ unsigned spread16(unsigned v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

// Morton (Z-order) code of the first `axes` coordinates: spatially close
// clusters get close slots, so one wavefront's terminals search nearby cells
// (grid) or lie in one small box (box tree). One or two axes: 16 bits each;
// three to eight axes: 64 / axes bits each, interleaved into 64 bits.
__device__ __forceinline__ int morton_bits(int axes) { return axes <= 2 ? 16 : 64 / axes; }

__global__ void k_morton(const float *x, int n, int d, int axes, const Counters *c,
                         unsigned long long *key, unsigned *val) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int bits = morton_bits(axes);
  const double top = (double)((1u << bits) - 1u);
  unsigned q[kMortonAxes];
#pragma unroll
  for (int a = 0; a < kMortonAxes; ++a) {
    q[a] = 0;
    if (a < axes) {
      double lo = from_ordered_bits(c->bb_lo[a]), hi = from_ordered_bits(c->bb_hi[a]);
      double t = hi > lo ? ((double)x[(size_t)i * d + a] - lo) / (hi - lo) : 0.0;
      t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
      q[a] = (unsigned)(t * top);
    }
  }
  if (axes <= 2) {
    key[i] = axes == 2 ? (unsigned long long)(spread16(q[0]) | (spread16(q[1]) << 1)) : q[0];
  } else {
    unsigned long long k = 0;
    for (int b = bits - 1; b >= 0; --b)
#pragma unroll
      for (int a = 0; a < kMortonAxes; ++a)
        if (a < axes) k = (k << 1) | (unsigned long long)((q[a] >> b) & 1u);
    key[i] = k;
  }
  val[i] = (unsigned)i;
}

__global__ void k_init_slots(State S, const float *x, const unsigned *perm) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S.n) return;
  const int p = (int)perm[s];
  const int d = S.d;
  S.cid[s] = p;
  S.csize[s] = 1;
  S.node[s] = p;
  S.node2slot[p] = s;
  if (S.cache_mask) {
    S.nparent[s] = -1;
    S.nparent[S.n + s] = -1;
  }
  S.succ[s] = -1;
  S.succ_node[s] = -1;
  S.predd[s] = kInfBits;
  S.term_round[s] = -1;
  S.alive[s] = 1;
  S.mdst[s] = s;
  S.moff[s] = 0;
  S.eff[s] = 0.0;
  S.nn_h[s] = 0.0;
  S.act[s] = s;
  for (int k = 0; k < d; ++k) {
    const float v = x[(size_t)p * d + k];
    S.wsum[(size_t)s * d + k] = (double)v;
    S.wcen[(size_t)s * d + k] = (double)v;
  }
  if (!centroid_link(S.linkage)) S.crad[s] = 0.0;
  if (S.linkage != kWard) S.cvar[s] = 0.0;
  if (S.linkage == kAvgSq) S.cmv[s] = 0.0;
  if (S.linkage == kComplete) {
    if (d == 2)
      for (int k = 0; k < kSupDirs; ++k) S.sup[(size_t)s * kSupDirs + k] = p;
    if (d <= kExtMaxDim)
      for (int k = 0; k < 2 * d; ++k) S.ext[(size_t)s * 2 * d + k] = p;
  }
  if (!centroid_link(S.linkage)) {
    S.cbeg[s] = s;
    S.powner[s] = s;
    for (int k = 0; k < d; ++k) {
      const float v = x[(size_t)p * d + k];
      S.lo[(size_t)s * d + k] = v;
      S.hi[(size_t)s * d + k] = v;
      S.px[(size_t)s * d + k] = v;
    }
  }
}

__global__ void k_set_nact(Counters *c, int n) { c->n_act = n; }

// -------------------------------------------------------------- act pass --
__global__ void k_act_pass(State S, int round) {
  const int nact = S.cnt->n_act;
  const int axes = S.d >= 2 ? 2 : 1;
  int mn = 0x7fffffff;
  unsigned long long lo[2] = {~0ull, ~0ull}, hi[2] = {0ull, 0ull};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nact; i += gridDim.x * blockDim.x) {
    const int s = S.act[i];
    const int sc = S.succ[s];
    const bool term = sc < 0 || S.node[sc] != S.succ_node[s];  // dead slots carry node -1
    S.flags[i] = term ? 1 : 0;
    if (term) S.term_round[s] = round;
    S.mdst[s] = s;
    S.moff[s] = 0;
    const int sz = S.csize[s];
    mn = sz < mn ? sz : mn;
    for (int a = 0; a < axes; ++a) {
      unsigned long long b = ordered_bits(S.wcen[(size_t)s * S.d + a]);
      lo[a] = b < lo[a] ? b : lo[a];
      hi[a] = b > hi[a] ? b : hi[a];
    }
  }
  mn = block_reduce<int, true>(mn);
  for (int a = 0; a < 2; ++a) {
    lo[a] = block_reduce<unsigned long long, true>(lo[a]);
    hi[a] = block_reduce<unsigned long long, false>(hi[a]);
  }
  if (threadIdx.x == 0) {
    atomicMin(&S.cnt->n_min, mn);
    for (int a = 0; a < axes; ++a) {
      atomicMin(&S.cnt->bb_lo[a], lo[a]);
      atomicMax(&S.cnt->bb_hi[a], hi[a]);
    }
  }
}

__global__ void k_scatter_flagged(const int *src, const int *flags, const int *pos, const int *dlen, int *dst) {
  const int len = *dlen;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x)
    if (flags[i]) dst[pos[i]] = src[i];
}

// ------------------------------------------------------------------ grid --
// at most this many cells: the cell scan's length is then known on the host
// from the previous round's active count (an upper bound of this round's)
__host__ __device__ __forceinline__ int grid_cells_max(int cell_cap, int nact) {
  const long long m = 4LL * nact + 16;
  return m < cell_cap ? (int)m : cell_cap;
}

__global__ void k_grid_params(State S, int cell_cap) {
  GridParams g;
  const int axes = S.d >= 2 ? 2 : 1;
  const int nact = S.cnt->n_act;
  double lo[2] = {0, 0}, ext[2] = {0, 0};
  for (int a = 0; a < axes; ++a) {
    lo[a] = from_ordered_bits(S.cnt->bb_lo[a]);
    ext[a] = from_ordered_bits(S.cnt->bb_hi[a]) - lo[a];
    if (!(ext[a] > 0.0)) ext[a] = 0.0;
  }
  double target = (double)nact;  // about one cluster per cell
  if (target < 1.0) target = 1.0;
  if (target > (double)cell_cap) target = (double)cell_cap;
  double h;
  if (axes == 2 && ext[0] > 0.0 && ext[1] > 0.0) h = sqrt(ext[0] * ext[1] / target);
  else h = fmax(ext[0], ext[1]) / target;
  if (!(h > 0.0)) h = 1.0;
  int G0, G1;
  for (;;) {
    double g0 = floor(ext[0] / h) + 1.0, g1 = axes == 2 ? floor(ext[1] / h) + 1.0 : 1.0;
    if (g0 * g1 <= (double)grid_cells_max(cell_cap, nact)) {
      G0 = (int)g0;
      G1 = (int)g1;
      break;
    }
    h *= 1.25;
  }
  g.org[0] = lo[0];
  g.org[1] = lo[1];
  g.h = h;
  g.inv_h = 1.0 / h;
  g.eps = 1e-13 * (fabs(lo[0]) + fabs(lo[1]) + ext[0] + ext[1] + h);
  g.G[0] = G0;
  g.G[1] = G1;
  g.ncell = G0 * G1;
  g.ncell1 = G0 * G1 + 1;
  g.axes = axes;
  *S.grid = g;
  S.cnt->n_tiles = 0;
}

__device__ __forceinline__ int cell_coord(double c, double org, double inv_h, int G) {
  double t = floor((c - org) * inv_h);
  int i = t < 0.0 ? 0 : (t >= (double)G ? G - 1 : (int)t);
  return i;
}

__global__ void k_zero_cells(State S) {
  const int nc = S.grid->ncell + 1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
    S.cell_cnt[i] = 0;
    S.cell_nmin[i] = 0x7fffffff;
  }
}

__global__ void k_cell_count(State S) {
  const GridParams g = *S.grid;
  const int nact = S.cnt->n_act;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nact; i += gridDim.x * blockDim.x) {
    const int s = S.act[i];
    const double *c = S.wcen + (size_t)s * S.d;
    int cx = cell_coord(c[0], g.org[0], g.inv_h, g.G[0]);
    int cy = g.axes == 2 ? cell_coord(c[1], g.org[1], g.inv_h, g.G[1]) : 0;
    const int cell = cy * g.G[0] + cx;
    S.cell_of[i] = cell;
    S.cell_rank[i] = atomicAdd(&S.cell_cnt[cell], 1);
    atomicMin(&S.cell_nmin[cell], S.csize[s]);
  }
}

// Mean squared deviation of a cluster's points from its centroid (Var/|C|,
// the merge rule of Sec. 2.1), lowered by a relative 1e-6 for FP64 rounding:
// complete linkage's key is at least ||cA - cB||^2 + this for both clusters
// (the mean squared point distance never exceeds the largest).
__device__ __forceinline__ double spread_lo(const State &S, int s) {
  return S.cvar[s] / (double)S.csize[s] * (1.0 - 1e-6);
}

__device__ __forceinline__ int spread_bits(double v) {
  float f = (float)v;
  if ((double)f > v) f = nextafterf(f, 0.0f);
  return __float_as_int(f);
}

__global__ void k_cell_scatter(State S) {
  const int nact = S.cnt->n_act;
  const int d = S.d;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nact; i += gridDim.x * blockDim.x) {
    const int s = S.act[i];
    const int pos = S.cell_start[S.cell_of[i]] + S.cell_rank[i];
    if (pos < 0 || pos >= nact) {
      S.cnt->nonfinite = 3;
      continue;
    }
    S.item_slot[pos] = s;
    S.item_meta[pos] = make_int4(s, S.csize[s], S.cid[s], S.linkage == kComplete ? spread_bits(spread_lo(S, s)) : 0);
    for (int k = 0; k < d; ++k) S.item_cen[(size_t)pos * d + k] = S.wcen[(size_t)s * d + k];
    if (S.linkage == kAvgSq) S.item_v[pos] = S.cmv[s];
    if (!centroid_link(S.linkage))
      for (int k = 0; k < d; ++k) {
        S.item_lo[(size_t)pos * d + k] = S.lo[(size_t)s * d + k];
        S.item_hi[(size_t)pos * d + k] = S.hi[(size_t)s * d + k];
      }
  }
}

// ------------------------------------------------------- linkage values --
// Ward key: 2|A||B|/(|A|+|B|) * ||cA - cB||^2 (Table 1, squared). Sizes are
// integers below 2^53, so the weight is exact before the division.
template <int MAXD>
__device__ __forceinline__ double ward_key(const double *ct, double nt, const double *cc, double nc, int d) {
  double q = 0.0;
  if (MAXD > 0) {
#pragma unroll
    for (int k = 0; k < MAXD; ++k)
      if (k < d) {
        double t = ct[k] - cc[k];
        q += t * t;
      }
  } else {
    for (int k = 0; k < d; ++k) {
      double t = ct[k] - cc[k];
      q += t * t;
    }
  }
  const double w = (2.0 * nt * nc) / (nt + nc);
  return w * q;
}

// avg-2 key: ||cA - cB||^2 + (Var(A)/|A| + Var(B)/|B|) (Table 1, the mean
// squared point distance), v = Var/|.| per cluster. The two spread terms are
// added first, so the value does not depend on which side asks.
template <int MAXD>
__device__ __forceinline__ double avgsq_key(const double *ct, double vt, const double *cc, double vc, int d) {
  double q = 0.0;
  if (MAXD > 0) {
#pragma unroll
    for (int k = 0; k < MAXD; ++k)
      if (k < d) {
        double t = ct[k] - cc[k];
        q += t * t;
      }
  } else {
    for (int k = 0; k < d; ++k) {
      double t = ct[k] - cc[k];
      q += t * t;
    }
  }
  return q + (vt + vc);
}

// Key of a centroid linkage (Ward: sizes; avg-2: spread terms).
template <int LINK, int MAXD>
__device__ __forceinline__ double cen_key(const double *ct, double nt, double vt, const double *cc, double nc,
                                          double vc, int d) {
  if (LINK == kWard) return ward_key<MAXD>(ct, nt, cc, nc, d);
  return avgsq_key<MAXD>(ct, vt, cc, vc, d);
}

// Exact complete (largest squared distance) or average (mean distance) value
// of a small pair, rows = the cluster with the lower ID.
template <int LINK>
__device__ __forceinline__ double pair_exact_inline(const float *px, int d, int begR, int nR, int begS, int nS) {
  double acc = 0.0;
  for (int r = 0; r < nR; ++r) {
    const float *pr = px + (size_t)(begR + r) * d;
    for (int c = 0; c < nS; ++c) {
      const float *pc = px + (size_t)(begS + c) * d;
      double q = 0.0;
      for (int k = 0; k < d; ++k) {
        double t = (double)pr[k] - (double)pc[k];
        q += t * t;
      }
      if (LINK == kComplete) acc = q > acc ? q : acc;
      else acc += sqrt(q);
    }
  }
  if (LINK == kAverage) acc = acc / ((double)nR * (double)nS);
  return acc;
}

// Lower and upper bounds of a pair's key from centroids and tight boxes.
//   complete (squared units): LB = max(centroid distance, per-axis extent
//     max(hiC-loT, hiT-loC) -- every per-axis extent is attained by a real
//     point pair --, centroid distance + both spreads vs); UB = squared max
//     distance between the boxes.
//   average: LB = max(centroid distance (Sec. 4.2), min box distance);
//     UB = max box distance.
template <int LINK, int MAXD>
__device__ __forceinline__ void pair_bounds(const double *ct, const float *lt, const float *ht, const double *cc,
                                            const float *lc, const float *hc, int d, double &lb, double &ub,
                                            double vs = 0.0) {
  double cdist = 0.0, ext = 0.0, mind = 0.0, maxd = 0.0;
  const int D = MAXD > 0 ? MAXD : d;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (MAXD > 0 && k >= d) break;
    double t = ct[k] - cc[k];
    cdist += t * t;
    double a = (double)hc[k] - (double)lt[k], b = (double)ht[k] - (double)lc[k];
    double e = a > b ? a : b;  // farthest separation along axis k (>= 0)
    ext = e > ext ? e : ext;
    maxd += e * e;
    double g = (double)lc[k] - (double)ht[k], g2 = (double)lt[k] - (double)hc[k];
    double gap = g > g2 ? g : g2;
    if (gap > 0.0) mind += gap * gap;
  }
  if (LINK == kComplete) {
    double e2 = ext * ext;
    lb = cdist > e2 ? cdist : e2;
    const double sp = cdist * (1.0 - 1e-6) + vs;  // vs: both spreads, lowered
    lb = sp > lb ? sp : lb;
    ub = maxd;
  } else {
    double c1 = sqrt(cdist), m1 = sqrt(mind);
    lb = c1 > m1 ? c1 : m1;
    ub = sqrt(maxd);
  }
}

// ------------------------------------------------ cluster-pair cache ----
// Alg. 4 / Sec. 5: distances of cluster pairs are kept for reuse. Keys are
// (lower node id, higher node id); node ids are never reused, so an entry of
// a merged cluster can never match again (invalidation on merge) and is
// dropped at the next rebuild. A slot's value is PENDING from the moment a
// terminal claims the pair for evaluation until the value is stored, so a
// pair is evaluated once per round however many terminals want it (the
// paper's claim-before-compute entry).
constexpr unsigned long long kCacheEmpty = ~0ull;
constexpr unsigned long long kCachePending = 0xfff8000000000001ull;  // never a stored value
constexpr int kCacheProbe = 32;

__device__ __forceinline__ unsigned long long pair_key(int na, int nb) {
  const unsigned lo = (unsigned)min(na, nb), hi = (unsigned)max(na, nb);
  return ((unsigned long long)lo << 32) | hi;
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// 0: miss, 1: hit (value in v), 2: claimed this round, value not stored yet
__device__ __forceinline__ int cache_find(const State &S, unsigned long long key, double &v) {
  if (!S.cache_mask) return 0;
  const unsigned long long h = mix64(key);
  for (int i = 0; i < kCacheProbe; ++i) {
    const unsigned long long idx = (h + i) & S.cache_mask;
    const unsigned long long k = __atomic_load_n(&S.ck[idx], __ATOMIC_RELAXED);
    if (k == key) {
      const unsigned long long b = __atomic_load_n(&S.cv[idx], __ATOMIC_RELAXED);
      if (b == kCachePending) return 2;
      v = pos_from_bits(b);
      return 1;
    }
    if (k == kCacheEmpty) return 0;
  }
  return 0;
}

// 1: claimed (caller evaluates), 2: already present, 0: no free slot
__device__ __forceinline__ int cache_claim(const State &S, unsigned long long key) {
  const unsigned long long h = mix64(key);
  for (int i = 0; i < kCacheProbe; ++i) {
    const unsigned long long idx = (h + i) & S.cache_mask;
    const unsigned long long prev = atomicCAS(&S.ck[idx], kCacheEmpty, key);
    if (prev == kCacheEmpty) {
      atomicAdd((unsigned long long *)&S.cnt->cache_inserts, 1ull);
      return 1;
    }
    if (prev == key) return 2;
  }
  return 0;
}

// store a value (claimed slot or a new one); false if the probe window is full
__device__ __forceinline__ bool cache_fill(const State &S, unsigned long long key, double v) {
  const unsigned long long h = mix64(key);
  for (int i = 0; i < kCacheProbe; ++i) {
    const unsigned long long idx = (h + i) & S.cache_mask;
    const unsigned long long prev = atomicCAS(&S.ck[idx], kCacheEmpty, key);
    if (prev == kCacheEmpty || prev == key) {
      if (prev == kCacheEmpty) atomicAdd((unsigned long long *)&S.cnt->cache_inserts, 1ull);
      atomicExch(&S.cv[idx], pos_bits(v));
      return true;
    }
  }
  atomicAdd((unsigned long long *)&S.cnt->cache_fail, 1ull);
  return false;
}

__device__ __forceinline__ int node_size(const State &S, int v) { return v < S.n ? 1 : S.row_size[v - S.n]; }

// Value of the node pair (x, y) from the cache: stored directly, or combined
// from the stored values of the parts of the newer node (its two children,
// recursively up to DEPTH levels) by the Lance-Williams rules of Table 2 and
// Sec. 5: complete takes the larger value (keys are monotone in the
// distance), average the size-weighted mean (Eq. case 2; two levels give
// Eq. case 1). A pair being evaluated this round (pending) is not combined.
template <int DEPTH>
__device__ __forceinline__ bool cache_parts(const State &S, int x, int y, double &v) {
  const int r = cache_find(S, pair_key(x, y), v);
  if (r == 1) return true;
  if constexpr (DEPTH == 0) {
    return false;
  } else {
    if (r == 2) return false;
    const int z = x > y ? x : y, o = x > y ? y : x;  // node ids grow with merge order
    if (z < S.n) return false;
    const int a = S.row_na[z - S.n], b = S.row_nb[z - S.n];
    double va, vb;
    if (!cache_parts<DEPTH - 1>(S, a, o, va) || !cache_parts<DEPTH - 1>(S, b, o, vb)) return false;
    if (S.linkage == kComplete) {
      v = va > vb ? va : vb;
    } else {
      const double sa = (double)node_size(S, a), sb = (double)node_size(S, b);
      v = (sa * va + sb * vb) / (sa + sb);
    }
    return true;
  }
}

// cache_parts with the children of the newer node as the first split; a
// combined value is stored under (x, y) when `store` (then false if it could
// not be stored). The grid search stores nothing while it runs: its emission
// pass treats a stored value as one its bound pass already counted.
__device__ __forceinline__ bool cache_resolve(const State &S, int x, int y, double &v, bool store = true) {
  if (!S.cache_mask) return false;
  const int r = cache_find(S, pair_key(x, y), v);
  if (r == 1) return true;
  if (r == 2) return false;
  const int z = x > y ? x : y, o = x > y ? y : x;
  if (z < S.n) return false;
  const int a = S.row_na[z - S.n], b = S.row_nb[z - S.n];
  double va, vb;
  if (!cache_parts<1>(S, a, o, va) || !cache_parts<1>(S, b, o, vb)) return false;
  if (S.linkage == kComplete) {
    v = va > vb ? va : vb;
  } else {
    const double sa = (double)node_size(S, a), sb = (double)node_size(S, b);
    v = (sa * va + sb * vb) / (sa + sb);
  }
  if (store && !cache_fill(S, pair_key(x, y), v)) return false;
  atomicAdd((unsigned long long *)&S.cnt->cache_derived, 1ull);
  return true;
}

// A pair whose value combines from cached parts is not evaluated: it joins
// the list of pairs whose values are read back from the cache.
// Its value travels with the entry and is stored after the search.
__device__ __forceinline__ bool pend_if_resolved(const State &S, int ti, int c) {
  double v;
  if (!cache_resolve(S, S.node[S.term[ti]], S.node[c], v, false)) return false;
  const long long q = append_slot(&S.cnt->n_pend);
  if (q < S.pair_cap) {
    S.pd_t[q] = ti;
    S.pd_c[q] = c;
    S.pd_v[q] = v;
  } else {
    S.cnt->pair_overflow = 1;
  }
  return true;
}

__global__ void k_cache_clear(unsigned long long *keys, unsigned long long *vals, unsigned long long mask) {
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i <= mask;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    keys[i] = kCacheEmpty;
    vals[i] = kCachePending;
  }
}

__device__ __forceinline__ bool node_alive(const State &S, int v) {
  const int sl = S.node2slot[v];
  return sl >= 0 && S.node[sl] == v;
}

// alive, or a child or grandchild of a live node: its entries can still be
// combined into a live pair's value
__device__ __forceinline__ bool node_recent(const State &S, int v) {
  if (node_alive(S, v)) return true;
  const int p = S.nparent[v];
  if (p < 0) return false;
  if (node_alive(S, p)) return true;
  const int g = S.nparent[p];
  return g >= 0 && node_alive(S, g);
}

// Move the valued entries of live pairs (and of their recent parts) of an old
// table into the (cleared) current one.
__global__ void k_cache_rebuild(State S, const unsigned long long *okeys, const unsigned long long *ovals,
                                unsigned long long omask) {
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i <= omask;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const unsigned long long k = okeys[i], b = ovals[i];
    if (k == kCacheEmpty || b == kCachePending) continue;
    const int a = (int)(k >> 32), c = (int)(k & 0xffffffffu);
    if (!node_recent(S, a) || !node_recent(S, c)) continue;
    cache_fill(S, k, pos_from_bits(b));
  }
}

// Drop claims whose value never arrived (a round being redone).
__global__ void k_cache_unclaim(State S) {
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i <= S.cache_mask;
       i += (unsigned long long)gridDim.x * blockDim.x)
    if (S.ck[i] != kCacheEmpty && S.cv[i] == kCachePending) S.ck[i] = kCacheEmpty;
}

// ---- d == 2 support polygons (complete linkage) --------------------------
// For unit directions u_k = (cos, sin)(2 pi k / K) a cluster keeps a point
// s_k maximising u_k . x. The farthest pair of two clusters is attained at
// points extreme in opposite directions, so pairs s_k(A), s_{k+K/2+j}(B) for
// small j give a real point pair within ~(1 - cos(pi/K)) of it (lower bound).
// The half-planes u_k . x <= u_k . s_k enclose the cluster; the farthest
// distance from a point to the cluster is at most its farthest distance to
// that K-gon's vertices (upper bound).
__constant__ double c_dir[2][kSupDirs];  // cos, sin of 2 pi k / kSupDirs (set by the host)

__device__ __forceinline__ void sup_dir(int k, double &c, double &s) {
  c = c_dir[0][k];
  s = c_dir[1][k];
}

// farthest pair among exactly opposite support points: for the farthest pair
// (a*, b*) and the direction u_k nearest to a* - b*, |s_k(A) - s_{k+K/2}(B)|
// >= u_k . (a* - b*) >= cos(pi/K) |a* - b*|
__device__ double sup_pair_lb(const float *x, const int *sa, const int *sb) {
  double m = 0.0;
  for (int k = 0; k < kSupDirs; ++k) {
    const float *pa = x + (size_t)sa[k] * 2;
    const float *pb = x + (size_t)sb[(k + kSupDirs / 2) % kSupDirs] * 2;
    const double u = (double)pa[0] - (double)pb[0], v = (double)pa[1] - (double)pb[1];
    const double q = u * u + v * v;
    m = q > m ? q : m;
  }
  return m;
}

// vertex k of the enclosing K-gon: intersection of support lines k and k+1,
// pushed outward by a small margin so rounding cannot shrink the polygon
__device__ __forceinline__ void sup_vertex(const float *x, const int *sp, int k, double &vx, double &vy) {
  const int k1 = (k + 1) % kSupDirs;
  double c0, s0, c1, s1;
  sup_dir(k, c0, s0);
  sup_dir(k1, c1, s1);
  const float *p0 = x + (size_t)sp[k] * 2, *p1 = x + (size_t)sp[k1] * 2;
  double h0 = c0 * (double)p0[0] + s0 * (double)p0[1];
  double h1 = c1 * (double)p1[0] + s1 * (double)p1[1];
  h0 += 1e-12 * (fabs(h0) + 1.0);
  h1 += 1e-12 * (fabs(h1) + 1.0);
  const double den = c0 * s1 - s0 * c1;  // sin(2 pi / K)
  vx = (h0 * s1 - h1 * s0) / den;
  vy = (h1 * c0 - h0 * c1) / den;
}

// Complete linkage, pairs too large to evaluate inline: tighter bounds.
//   comp_ub_refine: (|cA - cB| + rA + rB)^2 with rA, rB radius bounds (cheap;
//     used while the search bound is still being lowered)
//   comp_lb_refine: a real point pair's squared distance never exceeds the
//     key: the farthest pair among the two clusters' extreme points
//     (d <= kExtMaxDim) and among their opposite support points (d == 2)
__device__ __forceinline__ void comp_ub_refine(const State &S, int t, int c, const double *ct, const double *cc,
                                               int d, double &ub) {
  double c2 = 0.0;
  for (int k = 0; k < d; ++k) {
    double u = ct[k] - cc[k];
    c2 += u * u;
  }
  double us = sqrt(c2) + S.crad[t] + S.crad[c];
  us = us * us * (1.0 + 1e-12);
  ub = us < ub ? us : ub;
}

__device__ __forceinline__ void comp_lb_refine(const State &S, int t, int c, int d, double &lb,
                                               double stop = INFINITY) {
  if (d <= kExtMaxDim) {
    const int *et = S.ext + (size_t)t * 2 * d, *ec = S.ext + (size_t)c * 2 * d;
    double m = 0.0;
    for (int i = 0; i < 2 * d; ++i) {
      const float *pa = S.xin + (size_t)et[i] * d;
      for (int j = 0; j < 2 * d; ++j) {
        const float *pb = S.xin + (size_t)ec[j] * d;
        double q = 0.0;
        for (int k = 0; k < d; ++k) {
          double u = (double)pa[k] - (double)pb[k];
          q += u * u;
        }
        m = q > m ? q : m;
      }
    }
    lb = m > lb ? m : lb;
  }
  if (d == 2 && lb <= stop) {
    const double m = sup_pair_lb(S.xin, S.sup + (size_t)t * kSupDirs, S.sup + (size_t)c * kSupDirs);
    lb = m > lb ? m : lb;
  }
}

__device__ __forceinline__ void comp_refine(const State &S, int t, int c, const double *ct, const double *cc,
                                            int d, double &lb, double &ub) {
  comp_lb_refine(S, t, c, d, lb);
  comp_ub_refine(S, t, c, ct, cc, d, ub);
}

// Stop rule of the ring search: a lower bound on the key of any cluster whose
// centroid lies at least `D` away from the terminal's centroid.
template <int LINK>
__device__ __forceinline__ double ring_key_lb(double D, double nt, double nmin) {
  if (LINK == kWard) return D * D * ((2.0 * nt * nmin) / (nt + nmin));  // Sec. 4.1 radius
  if (LINK == kComplete) return D * D;  // Sec. 4.3: centroid distance <= complete distance
  if (LINK == kAvgSq) return D * D;     // Sec. 4.2: squared centroid distance <= avg-2 (+ spreads)
  return D;                             // Sec. 4.2: centroid distance <= average distance
}

// Initial search bound from the predecessor distance (Alg. 2), in key units.
template <int LINK>
__device__ __forceinline__ double beta_key(unsigned predbits) {
  if (predbits >= kInfBits) return INFINITY;
  double b = (double)__uint_as_float(predbits);
  if (LINK == kAverage || LINK == kAvgSq) return b * kSlack;
  return b * b * kSlack;
}

// Heights: complete and Ward keys are squared distances; average and avg-2
// keys are the heights themselves.
__device__ __forceinline__ double key_to_height(int link, double v) {
  return (link == kAverage || link == kAvgSq) ? v : sqrt(v);
}

// ------------------------------------------------------ ring search kernel --
// One thread per terminal. PASS 0: Ward (final result) or, for complete and
// average, the search bound plus the best inline-evaluated candidate. PASS 1
// (complete/average): re-walk the rings under the final bound and emit the
// large pairs whose lower bound does not exceed it.
// CACHE: the call keeps a pair cache (compiled out otherwise: its probes
// cost registers, hence occupancy, in every search)
template <int LINK, int MAXD, int PASS, bool CACHE>
__global__ __launch_bounds__(kBlock) void k_nn_grid(State S, int *t_ovf) {
  const int nterm = S.cnt->n_term;
  const int ti = blockIdx.x * blockDim.x + threadIdx.x;
  long long evals = 0, ppairs = 0, visits = 0, hits = 0;
  if (ti < nterm) {
    const GridParams g = *S.grid;
    const int d = S.d;
    const int t = S.term[ti];
    const int cid_t = S.cid[t];
    const int n_t = S.csize[t];
    const double nt = (double)n_t, nmin = (double)S.cnt->n_min;
    double ct[MAXD];
    float lt[MAXD], ht[MAXD];
#pragma unroll
    for (int k = 0; k < MAXD; ++k) {
      ct[k] = k < d ? S.wcen[(size_t)t * d + k] : 0.0;
      if (!centroid_link(LINK)) {
        lt[k] = k < d ? S.lo[(size_t)t * d + k] : 0.f;
        ht[k] = k < d ? S.hi[(size_t)t * d + k] : 0.f;
      }
    }
    const int beg_t = !centroid_link(LINK) ? S.cbeg[t] : 0;
    const double vt = LINK == kAvgSq ? S.cmv[t] : 0.0;
    // complete: own spread (lowered); avg-2: own spread term (exact, every
    // key is at least the squared centroid distance plus it)
    const double sp_t = LINK == kComplete ? spread_lo(S, t) : vt;
    bool skip = false;
    double bound;
    double bestv = INFINITY;
    unsigned long long bestk = kNoKey;
    if (PASS == 0) {
      bound = beta_key<LINK>(S.predd[t]);
    } else {
      skip = t_ovf[ti] != 0;
      bound = S.t_beta[ti] * kSlack;
    }
    if (!skip) {
      const int cx = cell_coord(ct[0], g.org[0], g.inv_h, g.G[0]);
      const int cy = g.axes == 2 ? cell_coord(ct[1], g.org[1], g.inv_h, g.G[1]) : 0;
      double m = 0.5;
      {
        double f = (ct[0] - g.org[0]) * g.inv_h - (double)cx;
        f = f < 0 ? 0 : (f > 1 ? 1 : f);
        m = fmin(m, fmin(f, 1.0 - f));
        if (g.axes == 2) {
          double f1 = (ct[1] - g.org[1]) * g.inv_h - (double)cy;
          f1 = f1 < 0 ? 0 : (f1 > 1 ? 1 : f1);
          m = fmin(m, fmin(f1, 1.0 - f1));
        }
      }
      const int kmax = max(max(cx, g.G[0] - 1 - cx), max(cy, g.G[1] - 1 - cy));
      int visited = 0;
      bool overflow = false;
      for (int k = 0; k <= kmax && !overflow; ++k) {
        if (k >= 1) {
          const double D = fmax(0.0, ((double)(k - 1) + m) * g.h * (1.0 - 1e-9) - g.eps);
          const double lbk = ring_key_lb<LINK>(D, nt, nmin) + sp_t;  // complete: + own spread
          const double cur = PASS == 0 ? fmin(bound, bestv) : bound;
          if (lbk > cur) break;
        }
        visited += k == 0 ? 1 : 8 * k;
        if (PASS == 0 && visited > S.cell_budget) {
          overflow = true;
          break;
        }
        // the ring: two full rows (contiguous item ranges) and two column strips
        for (int part = 0; part < 4; ++part) {
          int y, x0, x1, ystep = 0, ny = 1;
          if (k == 0) {
            if (part) break;
            y = cy;
            x0 = x1 = cx;
          } else if (part < 2) {
            y = part == 0 ? cy - k : cy + k;
            if (y < 0 || y >= g.G[1]) continue;
            x0 = max(cx - k, 0);
            x1 = min(cx + k, g.G[0] - 1);
          } else {
            const int x = part == 2 ? cx - k : cx + k;
            if (x < 0 || x >= g.G[0]) continue;
            const int ylo = max(cy - k + 1, 0), yhi = min(cy + k - 1, g.G[1] - 1);
            if (ylo > yhi) continue;
            y = ylo;
            x0 = x1 = x;
            ny = yhi - ylo + 1;
            ystep = 1;
          }
          for (int yy = 0; yy < ny; ++yy) {
            const int row = y + yy * ystep;
            const int a = S.cell_start[row * g.G[0] + x0], b = S.cell_start[row * g.G[0] + x1 + 1];
            visits += b - a;
            for (int it = a; it < b; ++it) {
              const int4 mt = S.item_meta[it];
              const int s = mt.x;
              if (s == t) continue;
              const double *cc = S.item_cen + (size_t)it * d;
              const unsigned long long key = make_key(mt.z, s);
              if (centroid_link(LINK)) {
                double cv[MAXD];
#pragma unroll
                for (int q = 0; q < MAXD; ++q) cv[q] = q < d ? cc[q] : 0.0;
                const double v =
                    cen_key<LINK, MAXD>(ct, nt, vt, cv, (double)mt.y, LINK == kAvgSq ? S.item_v[it] : 0.0, d);
                ++evals;
                if (v <= bound && better(v, key, bestv, bestk)) {
                  bestv = v;
                  bestk = key;
                }
              } else {
                double cv[MAXD];
                float lc[MAXD], hc[MAXD];
#pragma unroll
                for (int q = 0; q < MAXD; ++q) {
                  cv[q] = q < d ? cc[q] : 0.0;
                  lc[q] = q < d ? S.item_lo[(size_t)it * d + q] : 0.f;
                  hc[q] = q < d ? S.item_hi[(size_t)it * d + q] : 0.f;
                }
                double lb, ub;
                pair_bounds<LINK, MAXD>(ct, lt, ht, cv, lc, hc, d, lb, ub, sp_t + (double)__int_as_float(mt.w));
                const double cur = PASS == 0 ? fmin(bound, bestv) : bound;
                if (lb > cur * kSlack) continue;
                const long long cost = (long long)n_t * (long long)mt.y;
                if (CACHE && PASS == 0 && cost > kInlinePairs) {
                  double v;
                  if (cache_find(S, pair_key(S.node[t], S.node[s]), v) == 1) {
                    ++hits;
                    if (better(v, key, bestv, bestk)) {
                      bestv = v;
                      bestk = key;
                    }
                    continue;
                  }
                }
                if (PASS == 0 && cost > kInlinePairs) {
                  // remember it: the final bound decides later whether it is evaluated
                  const long long ci = append_slot(&S.cnt->n_cand);
                  if (ci < S.cand_cap) {
                    S.cd_t[ci] = ti;
                    S.cd_c[ci] = s;
                    S.cd_lb[ci] = lb;
                  } else {
                    S.cnt->cand_overflow = 1;
                  }
                }
                if (LINK == kComplete && cost > kInlinePairs) {
                  if (PASS == 0) {
                    comp_ub_refine(S, t, s, ct, cv, d, ub);
                  } else {
                    comp_lb_refine(S, t, s, d, lb, cur * kSlack);
                    if (lb > cur * kSlack) continue;
                  }
                }
                if (cost <= kInlinePairs) {
                  if (PASS == 0) {
                    double v;
                    if (cost == 1) {
                      // two singletons: the FP64 centroids are the widened points, so
                      // this is the same sum as the point-pair evaluation
                      double q = 0.0;
#pragma unroll
                      for (int k = 0; k < MAXD; ++k)
                        if (k < d) {
                          const double u = ct[k] - cv[k];
                          q += u * u;
                        }
                      v = LINK == kComplete ? q : sqrt(q);
                    } else {
                      const int beg_c = S.cbeg[s];
                      v = (mt.z < cid_t) ? pair_exact_inline<LINK>(S.px, d, beg_c, mt.y, beg_t, n_t)
                                         : pair_exact_inline<LINK>(S.px, d, beg_t, n_t, beg_c, mt.y);
                    }
                    ++evals;
                    ppairs += cost;
                    if (better(v, key, bestv, bestk)) {
                      bestv = v;
                      bestk = key;
                    }
                  }
                } else if (PASS == 0) {
                  if (ub < bound) bound = ub;
                } else {
                  if (CACHE) {
                    double v;
                    if (cache_find(S, pair_key(S.node[t], S.node[s]), v) == 1) continue;  // counted in pass 0
                    if (pend_if_resolved(S, ti, s)) continue;
                  }
                  const long long p = append_slot(&S.cnt->n_pairs);
                  if (p < S.pair_cap) {
                    S.pr_t[p] = ti;
                    S.pr_c[p] = s;
                    S.pr_v[p] = -1.0;
                  } else {
                    S.cnt->pair_overflow = 1;
                  }
                }
              }
            }
          }
        }
      }
      if (PASS == 0) {
        if (overflow) {
          t_ovf[ti] = 1;
          const int o = atomicAdd(&S.cnt->n_ovf, 1);
          S.ovf[o] = ti;
        } else {
          t_ovf[ti] = 0;
          if (centroid_link(LINK) && bestk == kNoKey) {
            // the predecessor bound was not met (cannot happen for an exact
            // bound); hand the terminal to the full scan without a bound
            t_ovf[ti] = 1;
            const int o = atomicAdd(&S.cnt->n_ovf, 1);
            S.ovf[o] = ti;
          } else {
            S.t_best[ti] = bestv;
            S.t_key[ti] = bestk;
            if (!centroid_link(LINK)) {
              S.t_beta[ti] = fmin(bound, bestv);
              S.t_min[ti] = pos_bits(bestv);
            }
          }
        }
      }
    }
  }
  count_add(&S.cnt->cluster_evals, evals);
  count_add(&S.cnt->point_pairs, ppairs);
  count_add(&S.cnt->visits[PASS == 0 ? 0 : 3], visits);
  count_add(&S.cnt->cache_hits, hits);
}

// ------------------------------------------ ring search, wave per terminal --
// Rounds with few terminals leave most of the chip idle under one thread per
// terminal, and each thread's walk is a long chain of dependent loads. Here
// the 64 lanes of a wavefront share one terminal: a ring is cut into its row
// and column segments (contiguous item ranges), the items of all segments are
// dealt out to the lanes, and the lanes' bounds and best candidates are
// combined at the end of every ring, where the stop rule is applied. Inside a
// ring a lane prunes with its own bound, never below the combined one, so it
// keeps every item the thread search would keep; the exact best candidate,
// hence the row, is the same. Pass 0 only, no pair cache: it writes what
// pass 1 and the candidate emission read (best candidate, final bound,
// hand-off flag, recorded large candidates).
template <int LINK, int MAXD>
__device__ __forceinline__ void grid_item_p0(const State &S, int it, int t, int cid_t, int n_t, int beg_t,
                                             const double *ct, const float *lt, const float *ht, double nt,
                                             double vt, double sp_t, int ti, double &bound, double &bestv,
                                             unsigned long long &bestk, long long &evals, long long &ppairs) {
  const int d = S.d;
  const int4 mt = S.item_meta[it];
  const int s = mt.x;
  if (s == t) return;
  const double *cc = S.item_cen + (size_t)it * d;
  const unsigned long long key = make_key(mt.z, s);
  double cv[MAXD];
  if (centroid_link(LINK)) {
#pragma unroll
    for (int q = 0; q < MAXD; ++q) cv[q] = q < d ? cc[q] : 0.0;
    const double v = cen_key<LINK, MAXD>(ct, nt, vt, cv, (double)mt.y, LINK == kAvgSq ? S.item_v[it] : 0.0, d);
    ++evals;
    if (v <= bound && better(v, key, bestv, bestk)) {
      bestv = v;
      bestk = key;
    }
    return;
  }
  float lc[MAXD], hc[MAXD];
#pragma unroll
  for (int q = 0; q < MAXD; ++q) {
    cv[q] = q < d ? cc[q] : 0.0;
    lc[q] = q < d ? S.item_lo[(size_t)it * d + q] : 0.f;
    hc[q] = q < d ? S.item_hi[(size_t)it * d + q] : 0.f;
  }
  double lb, ub;
  pair_bounds<LINK, MAXD>(ct, lt, ht, cv, lc, hc, d, lb, ub, sp_t + (double)__int_as_float(mt.w));
  if (lb > fmin(bound, bestv) * kSlack) return;
  const long long cost = (long long)n_t * (long long)mt.y;
  if (cost > kInlinePairs) {
    // remember it: the final bound decides later whether it is evaluated
    const long long ci = append_slot(&S.cnt->n_cand);
    if (ci < S.cand_cap) {
      S.cd_t[ci] = ti;
      S.cd_c[ci] = s;
      S.cd_lb[ci] = lb;
    } else {
      S.cnt->cand_overflow = 1;
    }
    if (LINK == kComplete) comp_ub_refine(S, t, s, ct, cv, d, ub);
    if (ub < bound) bound = ub;
    return;
  }
  double v;
  if (cost == 1) {
    double q = 0.0;
#pragma unroll
    for (int k = 0; k < MAXD; ++k)
      if (k < d) {
        const double u = ct[k] - cv[k];
        q += u * u;
      }
    v = LINK == kComplete ? q : sqrt(q);
  } else {
    const int beg_c = S.cbeg[s];
    v = (mt.z < cid_t) ? pair_exact_inline<LINK>(S.px, d, beg_c, mt.y, beg_t, n_t)
                       : pair_exact_inline<LINK>(S.px, d, beg_t, n_t, beg_c, mt.y);
  }
  ++evals;
  ppairs += cost;
  if (better(v, key, bestv, bestk)) {
    bestv = v;
    bestk = key;
  }
}

template <int LINK, int MAXD>
__global__ __launch_bounds__(kBlock) void k_nn_grid_wave(State S, int *t_ovf) {
  constexpr int kW = kBlock / kWave;
  const int nterm = S.cnt->n_term;
  const int lane = threadIdx.x & (kWave - 1);
  long long evals = 0, ppairs = 0, visits = 0;
  const GridParams g = *S.grid;
  const int d = S.d;
  const double nmin = (double)S.cnt->n_min;
  // the loop bound depends on the wavefront only: every lane of a wave runs
  // the same terminals, so the shuffles below see all 64 lanes
  for (int ti = blockIdx.x * kW + (int)(threadIdx.x / kWave); ti < nterm; ti += gridDim.x * kW) {
    const int t = S.term[ti];
    const int cid_t = S.cid[t];
    const int n_t = S.csize[t];
    const double nt = (double)n_t;
    double ct[MAXD];
    float lt[MAXD], ht[MAXD];
#pragma unroll
    for (int k = 0; k < MAXD; ++k) {
      ct[k] = k < d ? S.wcen[(size_t)t * d + k] : 0.0;
      lt[k] = (!centroid_link(LINK) && k < d) ? S.lo[(size_t)t * d + k] : 0.f;
      ht[k] = (!centroid_link(LINK) && k < d) ? S.hi[(size_t)t * d + k] : 0.f;
    }
    const int beg_t = !centroid_link(LINK) ? S.cbeg[t] : 0;
    const double vt = LINK == kAvgSq ? S.cmv[t] : 0.0;
    const double sp_t = LINK == kComplete ? spread_lo(S, t) : vt;
    double bound = beta_key<LINK>(S.predd[t]);
    double bestv = INFINITY;
    unsigned long long bestk = kNoKey;
    const int cx = cell_coord(ct[0], g.org[0], g.inv_h, g.G[0]);
    const int cy = g.axes == 2 ? cell_coord(ct[1], g.org[1], g.inv_h, g.G[1]) : 0;
    double m = 0.5;
    {
      double f = (ct[0] - g.org[0]) * g.inv_h - (double)cx;
      f = f < 0 ? 0 : (f > 1 ? 1 : f);
      m = fmin(m, fmin(f, 1.0 - f));
      if (g.axes == 2) {
        double f1 = (ct[1] - g.org[1]) * g.inv_h - (double)cy;
        f1 = f1 < 0 ? 0 : (f1 > 1 ? 1 : f1);
        m = fmin(m, fmin(f1, 1.0 - f1));
      }
    }
    const int kmax = max(max(cx, g.G[0] - 1 - cx), max(cy, g.G[1] - 1 - cy));
    int visited = 0;
    bool overflow = false;
    for (int k = 0; k <= kmax; ++k) {
      if (k >= 1) {
        const double D = fmax(0.0, ((double)(k - 1) + m) * g.h * (1.0 - 1e-9) - g.eps);
        const double lbk = ring_key_lb<LINK>(D, nt, nmin) + sp_t;
        if (lbk > fmin(bound, bestv)) break;
      }
      visited += k == 0 ? 1 : 8 * k;
      if (visited > S.wave_budget) {
        overflow = true;
        break;
      }
      // segments of ring k: 0 and 1 the rows above and below (full width),
      // then the left and right column cells between them
      const int ylo = k == 0 ? 0 : max(cy - k + 1, 0), yhi = k == 0 ? -1 : min(cy + k - 1, g.G[1] - 1);
      const int ncol = max(0, yhi - ylo + 1);
      const int nseg = k == 0 ? 1 : 2 + 2 * ncol;
      for (int s0 = 0; s0 < nseg; s0 += kWave) {
        const int j = s0 + lane;
        int a = 0, b = 0;
        if (j < nseg) {
          int y, x0, x1;
          if (k == 0) {
            y = cy;
            x0 = x1 = cx;
          } else if (j < 2) {
            y = j == 0 ? cy - k : cy + k;
            x0 = max(cx - k, 0);
            x1 = min(cx + k, g.G[0] - 1);
          } else {
            const int jj = j - 2;
            y = ylo + (jj < ncol ? jj : jj - ncol);
            x0 = x1 = jj < ncol ? cx - k : cx + k;
          }
          if (y >= 0 && y < g.G[1] && x0 >= 0 && x1 < g.G[0] && x0 <= x1) {
            a = S.cell_start[y * g.G[0] + x0];
            b = S.cell_start[y * g.G[0] + x1 + 1];
          }
        }
        // exclusive prefix of the segment lengths over the lanes
        int incl = b - a;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const int u = __shfl_up(incl, o, kWave);
          if (lane >= o) incl += u;
        }
        const int excl = incl - (b - a);
        const int total = __shfl(incl, kWave - 1, kWave);
        const int nsc = min(nseg - s0, kWave);
        if (lane == 0) visits += total;
        for (int base = 0; base < total; base += kWave) {
          const int i = base + lane;
          // the last segment whose start is at or before i (empty segments
          // share their start with the next one, so the last is non-empty)
          int sg = 0;
#pragma unroll
          for (int step = kWave / 2; step > 0; step >>= 1) {
            const int c = sg + step;
            const int pc = __shfl(excl, c < nsc ? c : 0, kWave);
            if (c < nsc && pc <= i) sg = c;
          }
          const int sa = __shfl(a, sg, kWave), sp = __shfl(excl, sg, kWave);
          if (i < total)
            grid_item_p0<LINK, MAXD>(S, sa + (i - sp), t, cid_t, n_t, beg_t, ct, lt, ht, nt, vt, sp_t, ti, bound,
                                     bestv, bestk, evals, ppairs);
        }
      }
      // combine the lanes: smallest bound, best (value, key)
      bound = wave_min(bound);
#pragma unroll
      for (int o = kWave / 2; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bestv, o, kWave);
        const unsigned long long ok = __shfl_xor(bestk, o, kWave);
        if (better(ov, ok, bestv, bestk)) {
          bestv = ov;
          bestk = ok;
        }
      }
    }
    if (lane == 0) {
      bool hand_off = overflow;
      // the predecessor bound was not met (cannot happen for an exact
      // bound): the full scan takes the terminal without a bound
      if (!overflow && centroid_link(LINK) && bestk == kNoKey) hand_off = true;
      t_ovf[ti] = hand_off ? 1 : 0;
      if (hand_off) {
        const int o = atomicAdd(&S.cnt->n_ovf, 1);
        S.ovf[o] = ti;
      } else {
        S.t_best[ti] = bestv;
        S.t_key[ti] = bestk;
        if (!centroid_link(LINK)) {
          S.t_beta[ti] = fmin(bound, bestv);
          S.t_min[ti] = pos_bits(bestv);
        }
      }
    }
  }
  count_add(&S.cnt->cluster_evals, evals);
  count_add(&S.cnt->point_pairs, ppairs);
  count_add(&S.cnt->visits[0], visits);
}

// Recorded large candidates: keep those whose lower bound does not exceed
// their terminal's final bound (refined bounds for complete), emit them as
// pairs. Does nothing if the record overflowed (the host then re-walks the
// rings instead).
template <int LINK>
__global__ void k_cand_emit(State S, const int *t_ovf) {
  if (S.cnt->cand_overflow) return;
  const int nc = (int)min(S.cnt->n_cand, S.cand_cap);
  const int d = S.d;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
    const int ti = S.cd_t[i];
    if (t_ovf[ti]) continue;
    const double beta = S.t_beta[ti] * kSlack;
    double lb = S.cd_lb[i];
    if (lb > beta * kSlack) continue;
    const int c = S.cd_c[i];
    if (S.cache_mask && pend_if_resolved(S, ti, c)) continue;
    if (LINK == kComplete) {
      comp_lb_refine(S, S.term[ti], c, d, lb, beta * kSlack);
      if (lb > beta * kSlack) continue;
    }
    if (S.cache_mask) {
      // claim the pair; if another terminal already did, wait for its value
      const int r = cache_claim(S, pair_key(S.node[S.term[ti]], S.node[c]));
      if (r == 2) {
        const long long q = append_slot(&S.cnt->n_pend);
        if (q < S.pair_cap) {
          S.pd_t[q] = ti;
          S.pd_c[q] = c;
          S.pd_v[q] = -1.0;
        } else {
          S.cnt->pair_overflow = 1;
        }
        continue;
      }
    }
    const long long p = append_slot(&S.cnt->n_pairs);
    if (p < S.pair_cap) {
      S.pr_t[p] = ti;
      S.pr_c[p] = c;
      S.pr_v[p] = LINK == kComplete ? lb : -1.0;  // complete: the refined lower bound, reused
    } else {
      S.cnt->pair_overflow = 1;
    }
  }
}

// ------------------------------------------------ block ring search ------
// One block per terminal handed off by the thread search. The block walks the
// same rings; thread j takes ring cell j (row cells first, then the column
// cells) and skips it when the cell's own lower bound -- its rectangle's
// distance to the centroid and, for Ward, its smallest cluster size --
// exceeds the current bound. After each ring the block agrees on the best
// candidate and the bound, so the stop rule is uniform.
template <int LINK>
__device__ __forceinline__ double cell_key_lb(double D, double nt, int cnmin) {
  if (LINK == kWard) {
    const double nm = (double)cnmin;
    return D * D * ((2.0 * nt * nm) / (nt + nm));
  }
  if (LINK == kComplete || LINK == kAvgSq) return D * D;
  return D;
}

template <int LINK, int MAXD, bool CACHE>
__global__ __launch_bounds__(kBlock) void k_nn_ringblk(State S) {
  __shared__ double red_v[kBlock / kWave], red_b[kBlock / kWave];
  __shared__ unsigned long long red_k[kBlock / kWave];
  __shared__ double sh_bound, sh_best;
  __shared__ unsigned long long sh_key;
  const int count = S.cnt->n_ovf;
  const GridParams g = *S.grid;
  const int d = S.d;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  long long evals = 0, ppairs = 0, visits = 0, hits = 0;
  for (int qi = blockIdx.x; qi < count; qi += gridDim.x) {
    const int ti = S.ovf[qi];
    const int t = S.term[ti];
    const int cid_t = S.cid[t];
    const int n_t = S.csize[t];
    const double nt = (double)n_t;
    double ct[MAXD];
    float lt[MAXD], ht[MAXD];
#pragma unroll
    for (int k = 0; k < MAXD; ++k) {
      ct[k] = k < d ? S.wcen[(size_t)t * d + k] : 0.0;
      lt[k] = (!centroid_link(LINK) && k < d) ? S.lo[(size_t)t * d + k] : 0.f;
      ht[k] = (!centroid_link(LINK) && k < d) ? S.hi[(size_t)t * d + k] : 0.f;
    }
    const int beg_t = !centroid_link(LINK) ? S.cbeg[t] : 0;
    const double vt = LINK == kAvgSq ? S.cmv[t] : 0.0;
    const double sp_t = LINK == kComplete ? spread_lo(S, t) : vt;
    const int cx = cell_coord(ct[0], g.org[0], g.inv_h, g.G[0]);
    const int cy = g.axes == 2 ? cell_coord(ct[1], g.org[1], g.inv_h, g.G[1]) : 0;
    const int kmax = max(max(cx, g.G[0] - 1 - cx), max(cy, g.G[1] - 1 - cy));
    double beta_final = 0.0;
    bool use_pred = true;
    for (int pass = 0; pass < (centroid_link(LINK) ? 1 : 2); ++pass) {
      double bound = pass == 0 ? (use_pred ? beta_key<LINK>(S.predd[t]) : INFINITY) : beta_final * kSlack;
      double bestv = INFINITY;
      unsigned long long bestk = kNoKey;
      double cur = bound;  // block-uniform bound
      for (int k = 0; k <= kmax; ++k) {
        const int ncell = k == 0 ? 1 : 8 * k;
        for (int j0 = 0; j0 < ncell; j0 += kBlock) {
          const int j = j0 + threadIdx.x;
          int x = -1, y = -1;
          if (j < ncell) {
            if (k == 0) {
              x = cx;
              y = cy;
            } else if (j < 2 * k + 1) {
              x = cx - k + j;
              y = cy - k;
            } else if (j < 4 * k + 2) {
              x = cx - k + (j - 2 * k - 1);
              y = cy + k;
            } else if (j < 6 * k + 1) {
              x = cx - k;
              y = cy - k + 1 + (j - 4 * k - 2);
            } else {
              x = cx + k;
              y = cy - k + 1 + (j - 6 * k - 1);
            }
          }
          if (x < 0 || y < 0 || x >= g.G[0] || y >= g.G[1]) continue;
          const int cell = y * g.G[0] + x;
          const int a = S.cell_start[cell], b = S.cell_start[cell + 1];
          if (a == b) continue;
          // distance from the centroid to this cell's rectangle
          double dx = 0.0, dy = 0.0;
          {
            const double x0 = g.org[0] + x * g.h, x1 = x0 + g.h;
            dx = ct[0] < x0 ? x0 - ct[0] : (ct[0] > x1 ? ct[0] - x1 : 0.0);
            if (g.axes == 2) {
              const double y0 = g.org[1] + y * g.h, y1 = y0 + g.h;
              dy = ct[1] < y0 ? y0 - ct[1] : (ct[1] > y1 ? ct[1] - y1 : 0.0);
            }
          }
          const double Dc = fmax(0.0, sqrt(dx * dx + dy * dy) * (1.0 - 1e-9) - g.eps);
          const double mycur = pass == 0 ? fmin(cur, fmin(bound, bestv)) : cur;
          if (cell_key_lb<LINK>(Dc, nt, S.cell_nmin[cell]) + sp_t > mycur) continue;
          visits += b - a;
          for (int it = a; it < b; ++it) {
            const int4 mt = S.item_meta[it];
            const int sl = mt.x;
            if (sl == t) continue;
            const double *cc = S.item_cen + (size_t)it * d;
            const unsigned long long key = make_key(mt.z, sl);
            double cv[MAXD];
#pragma unroll
            for (int q = 0; q < MAXD; ++q) cv[q] = q < d ? cc[q] : 0.0;
            if (centroid_link(LINK)) {
              const double v =
                  cen_key<LINK, MAXD>(ct, nt, vt, cv, (double)mt.y, LINK == kAvgSq ? S.item_v[it] : 0.0, d);
              ++evals;
              if (v <= bound && better(v, key, bestv, bestk)) {
                bestv = v;
                bestk = key;
              }
            } else {
              float lc[MAXD], hc[MAXD];
#pragma unroll
              for (int q = 0; q < MAXD; ++q) {
                lc[q] = q < d ? S.item_lo[(size_t)it * d + q] : 0.f;
                hc[q] = q < d ? S.item_hi[(size_t)it * d + q] : 0.f;
              }
              double lb, ub;
              pair_bounds<LINK, MAXD>(ct, lt, ht, cv, lc, hc, d, lb, ub, sp_t + (double)__int_as_float(mt.w));
              const double c2 = pass == 0 ? fmin(cur, fmin(bound, bestv)) : cur;
              if (lb > c2 * kSlack) continue;
              const long long cost = (long long)n_t * (long long)mt.y;
              if (CACHE && pass == 0 && cost > kInlinePairs) {
                double v;
                if (cache_find(S, pair_key(S.node[t], S.node[sl]), v) == 1) {
                  ++hits;
                  if (better(v, key, bestv, bestk)) {
                    bestv = v;
                    bestk = key;
                  }
                  continue;
                }
              }
              if (LINK == kComplete && cost > kInlinePairs) {
                if (pass == 0) {
                  comp_ub_refine(S, t, sl, ct, cv, d, ub);
                } else {
                  comp_lb_refine(S, t, sl, d, lb, c2 * kSlack);
                  if (lb > c2 * kSlack) continue;
                }
              }
              if (cost <= kInlinePairs) {
                if (pass == 0) {
                  const int beg_c = S.cbeg[sl];
                  const double v = (mt.z < cid_t) ? pair_exact_inline<LINK>(S.px, d, beg_c, mt.y, beg_t, n_t)
                                                  : pair_exact_inline<LINK>(S.px, d, beg_t, n_t, beg_c, mt.y);
                  ++evals;
                  ppairs += cost;
                  if (better(v, key, bestv, bestk)) {
                    bestv = v;
                    bestk = key;
                  }
                }
              } else if (pass == 0) {
                if (ub < bound) bound = ub;
              } else {
                if (CACHE) {
                  double v;
                  if (cache_find(S, pair_key(S.node[t], S.node[sl]), v) == 1) continue;  // counted in pass 0
                  if (pend_if_resolved(S, ti, sl)) continue;
                }
                const long long pp = append_slot(&S.cnt->n_pairs);
                if (pp < S.pair_cap) {
                  S.pr_t[pp] = ti;
                  S.pr_c[pp] = sl;
                  S.pr_v[pp] = -1.0;
                } else {
                  S.cnt->pair_overflow = 1;
                }
              }
            }
          }
        }
        if (pass == 0) {
          // agree on the best candidate and the bound
          double bv = bestv, bb = bound;
          unsigned long long bk = bestk;
          for (int o = kWave / 2; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o, kWave), ob = __shfl_xor(bb, o, kWave);
            const unsigned long long ok = __shfl_xor(bk, o, kWave);
            if (better(ov, ok, bv, bk)) {
              bv = ov;
              bk = ok;
            }
            bb = fmin(bb, ob);
          }
          if (lane == 0) {
            red_v[wv] = bv;
            red_k[wv] = bk;
            red_b[wv] = bb;
          }
          __syncthreads();
          if (threadIdx.x == 0) {
            double v0 = red_v[0], b0 = red_b[0];
            unsigned long long k0 = red_k[0];
            for (int q = 1; q < kBlock / kWave; ++q) {
              if (better(red_v[q], red_k[q], v0, k0)) {
                v0 = red_v[q];
                k0 = red_k[q];
              }
              b0 = fmin(b0, red_b[q]);
            }
            sh_best = v0;
            sh_key = k0;
            sh_bound = b0;
          }
          __syncthreads();
          bestv = sh_best;
          bestk = sh_key;
          bound = sh_bound;
          cur = fmin(bound, bestv);
          __syncthreads();
        }
        // stop when the next ring cannot hold anything better
        if (k + 1 <= kmax) {
          double m = 0.5;
          {
            double f = (ct[0] - g.org[0]) * g.inv_h - (double)cx;
            f = f < 0 ? 0 : (f > 1 ? 1 : f);
            m = fmin(m, fmin(f, 1.0 - f));
            if (g.axes == 2) {
              double f1 = (ct[1] - g.org[1]) * g.inv_h - (double)cy;
              f1 = f1 < 0 ? 0 : (f1 > 1 ? 1 : f1);
              m = fmin(m, fmin(f1, 1.0 - f1));
            }
          }
          const double D = fmax(0.0, ((double)k + m) * g.h * (1.0 - 1e-9) - g.eps);
          if (ring_key_lb<LINK>(D, nt, (double)S.cnt->n_min) + sp_t > cur) break;
        }
      }
      if (centroid_link(LINK) && pass == 0 && bestk == kNoKey && use_pred) {
        // the predecessor bound held nothing (cannot happen for an exact
        // bound): search again without it
        use_pred = false;
        pass = -1;
        __syncthreads();
        continue;
      }
      if (pass == 0) {
        beta_final = fmin(bound, bestv);
        if (threadIdx.x == 0) {
          S.t_best[ti] = bestv;
          S.t_key[ti] = bestk;
          if (!centroid_link(LINK)) {
            S.t_beta[ti] = beta_final;
            S.t_min[ti] = pos_bits(bestv);
          }
        }
      }
      __syncthreads();
    }
  }
  count_add(&S.cnt->cluster_evals, evals);
  count_add(&S.cnt->point_pairs, ppairs);
  count_add(&S.cnt->visits[1], visits);
  count_add(&S.cnt->cache_hits, hits);
}

// ---------------------------------------------------- full scan kernel ----
// One block per handed-off terminal; every active cluster is a candidate.
// Same keys, bounds and tie-break as the ring search.
template <int LINK>
__global__ __launch_bounds__(kBlock) void k_nn_full(State S, const int *list, const int *dcount) {
  extern __shared__ unsigned char smem[];
  const int count = dcount ? *dcount : S.cnt->n_term;
  const int nact = S.cnt->n_act;
  const int d = S.d;
  double *ct = (double *)smem;
  float *lt = (float *)(ct + d);
  float *ht = lt + d;
  __shared__ double red_v[kBlock / kWave];
  __shared__ unsigned long long red_k[kBlock / kWave];
  __shared__ double red_b[kBlock / kWave];
  long long evals = 0, ppairs = 0, visits = 0, hits = 0;
  for (int q = blockIdx.x; q < count; q += gridDim.x) {
    const int ti = list ? list[q] : q;
    const int t = S.term[ti];
    const int cid_t = S.cid[t];
    const int n_t = S.csize[t];
    const double nt = (double)n_t;
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
      ct[k] = S.wcen[(size_t)t * d + k];
      if (!centroid_link(LINK)) {
        lt[k] = S.lo[(size_t)t * d + k];
        ht[k] = S.hi[(size_t)t * d + k];
      }
    }
    __syncthreads();
    const int beg_t = !centroid_link(LINK) ? S.cbeg[t] : 0;
    const double vt = LINK == kAvgSq ? S.cmv[t] : 0.0;
    double bound = S.prune ? beta_key<LINK>(S.predd[t]) : INFINITY;
    double bestv = INFINITY;
    unsigned long long bestk = kNoKey;
    for (int i = threadIdx.x; i < nact; i += blockDim.x) {
      const int s = S.act[i];
      ++visits;
      if (s == t) continue;
      const unsigned long long key = make_key(S.cid[s], s);
      const int n_c = S.csize[s];
      const double *cc = S.wcen + (size_t)s * d;
      if (centroid_link(LINK)) {
        // a full scan needs no bound for Ward / avg-2: every candidate is evaluated
        const double v = cen_key<LINK, 0>(ct, nt, vt, cc, (double)n_c, LINK == kAvgSq ? S.cmv[s] : 0.0, d);
        ++evals;
        if (better(v, key, bestv, bestk)) {
          bestv = v;
          bestk = key;
        }
      } else {
        double lb, ub;
        pair_bounds<LINK, 0>(ct, lt, ht, cc, S.lo + (size_t)s * d, S.hi + (size_t)s * d, d, lb, ub,
                             LINK == kComplete ? spread_lo(S, t) + spread_lo(S, s) : 0.0);
        if (S.prune && lb > fmin(bound, bestv) * kSlack) continue;
        const long long cost = (long long)n_t * n_c;
        if (cost > kInlinePairs && S.cache_mask) {
          double v;
          if (cache_find(S, pair_key(S.node[t], S.node[s]), v) == 1) {
            ++hits;
            if (better(v, key, bestv, bestk)) {
              bestv = v;
              bestk = key;
            }
            continue;
          }
        }
        if (LINK == kComplete && cost > kInlinePairs) comp_ub_refine(S, t, s, ct, cc, d, ub);
        if (cost <= kInlinePairs) {
          const int beg_c = S.cbeg[s];
          const double v = (S.cid[s] < cid_t) ? pair_exact_inline<LINK>(S.px, d, beg_c, n_c, beg_t, n_t)
                                              : pair_exact_inline<LINK>(S.px, d, beg_t, n_t, beg_c, n_c);
          ++evals;
          ppairs += cost;
          if (better(v, key, bestv, bestk)) {
            bestv = v;
            bestk = key;
          }
        } else if (ub < bound) {
          bound = ub;
        }
      }
    }
    // block argmin of (value, key) and min of the bound
    {
      const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
      for (int o = kWave / 2; o > 0; o >>= 1) {
        double ov = __shfl_xor(bestv, o, kWave);
        unsigned long long ok = __shfl_xor(bestk, o, kWave);
        double ob = __shfl_xor(bound, o, kWave);
        if (better(ov, ok, bestv, bestk)) {
          bestv = ov;
          bestk = ok;
        }
        bound = fmin(bound, ob);
      }
      if (lane == 0) {
        red_v[w] = bestv;
        red_k[w] = bestk;
        red_b[w] = bound;
      }
      __syncthreads();
      bestv = red_v[0];
      bestk = red_k[0];
      bound = red_b[0];
      for (int j = 1; j < kBlock / kWave; ++j) {
        if (better(red_v[j], red_k[j], bestv, bestk)) {
          bestv = red_v[j];
          bestk = red_k[j];
        }
        bound = fmin(bound, red_b[j]);
      }
    }
    const double beta = fmin(bound, bestv);
    if (threadIdx.x == 0) {
      S.t_best[ti] = bestv;
      S.t_key[ti] = bestk;
      if (!centroid_link(LINK)) {
        S.t_beta[ti] = beta;
        S.t_min[ti] = pos_bits(bestv);
      }
    }
    if (!centroid_link(LINK)) {
      // emit the large pairs that the final bound does not exclude
      for (int i = threadIdx.x; i < nact; i += blockDim.x) {
        const int s = S.act[i];
        if (s == t) continue;
        const int n_c = S.csize[s];
        if ((long long)n_t * n_c <= kInlinePairs) continue;
        if (S.cache_mask) {
          double v;
          if (cache_find(S, pair_key(S.node[t], S.node[s]), v) == 1) continue;  // already counted
        }
        if (S.prune) {
          double lb, ub;
          pair_bounds<LINK, 0>(ct, lt, ht, S.wcen + (size_t)s * d, S.lo + (size_t)s * d, S.hi + (size_t)s * d,
                               d, lb, ub, LINK == kComplete ? spread_lo(S, t) + spread_lo(S, s) : 0.0);
          if (lb > beta * kSlack) continue;
          if (LINK == kComplete) {
            comp_lb_refine(S, t, s, d, lb, beta * kSlack);
            if (lb > beta * kSlack) continue;
          }
        }
        if (S.cache_mask && pend_if_resolved(S, ti, s)) continue;
        const long long p = append_slot(&S.cnt->n_pairs);
        if (p < S.pair_cap) {
          S.pr_t[p] = ti;
          S.pr_c[p] = s;
          S.pr_v[p] = -1.0;
        } else {
          S.cnt->pair_overflow = 1;
        }
      }
    }
    __syncthreads();
  }
  count_add(&S.cnt->cluster_evals, evals);
  count_add(&S.cnt->point_pairs, ppairs);
  count_add(&S.cnt->visits[1], visits);
  count_add(&S.cnt->cache_hits, hits);
}

// ------------------------------------------------------ box-tree search ----
// Ward and avg-2 at 3 <= d <= kTreeMaxDim. The active list is in slot order,
// a Morton order over up to eight axes (clusters inherit the slot of their
// lower-ID child, so the order stays spatially coherent as they merge). An
// implicit 16-ary tree is built over it every round: leaves of kTreeFan
// consecutive clusters, each level above grouping kTreeFan nodes, every node
// with the FP64 box of its centroids, its smallest size and smallest spread
// term (the range query of Alg. 3 over a bounding-box tree instead of a k-d
// tree). One thread per terminal evaluates its own leaf first (a near
// neighbour and a tight bound), then walks outward, bottom up, depth first
// and without a stack (a node's parent is its index / 16), entering a node
// only if its lower bound does not exceed the thread's bound (Sec. 4.1, 4.2:
// the Ward and avg-2 keys grow with the centroid distance). Every loop step
// does one box test or one candidate, so lanes of a wavefront stay in step.
// A bound takes the key's FP64 operations in the same order on values no
// larger than the key's operands, so it never exceeds a key (rounding is
// monotone); pruning is strict, so equal keys reach the tie-break.
constexpr int kTreeFan = 16;

__global__ void k_tree_items(State S) {
  const int nact = S.cnt->n_act, d = S.d;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nact; i += gridDim.x * blockDim.x) {
    const int s = S.act[i];
    S.item_meta[i] = make_int4(s, S.csize[s], S.cid[s], 0);
    for (int k = 0; k < d; ++k) S.item_cen[(size_t)i * d + k] = S.wcen[(size_t)s * d + k];
    if (S.linkage == kAvgSq) S.item_v[i] = S.cmv[s];
  }
}

// one thread per node of level `lev`: the box of its (up to kTreeFan)
// children, which are items for the leaves (lev 0)
__global__ void k_tree_level(State S, int lev) {
  const int d = S.d;
  const int cnt = S.tree_cnt[lev];
  const int nsrc = lev == 0 ? S.cnt->n_act : S.tree_cnt[lev - 1];
  const int src0 = lev == 0 ? 0 : S.tree_off[lev - 1];
  const int dst0 = S.tree_off[lev];
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += gridDim.x * blockDim.x) {
    const int c0 = j * kTreeFan, c1 = min(c0 + kTreeFan, nsrc);
    int nm = 0x7fffffff;
    double vm = INFINITY;
    for (int c = c0; c < c1; ++c) {
      const int sz = lev == 0 ? S.item_meta[c].y : S.tree_nmin[src0 + c];
      nm = sz < nm ? sz : nm;
      if (S.linkage == kAvgSq) {
        const double v = lev == 0 ? S.item_v[c] : S.tree_vmin[src0 + c];
        vm = v < vm ? v : vm;
      }
    }
    for (int k = 0; k < d; ++k) {
      double lo = INFINITY, hi = -INFINITY;
      for (int c = c0; c < c1; ++c) {
        const double a = lev == 0 ? S.item_cen[(size_t)c * d + k] : S.tree_lo[(size_t)(src0 + c) * d + k];
        const double b = lev == 0 ? a : S.tree_hi[(size_t)(src0 + c) * d + k];
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
      }
      S.tree_lo[(size_t)(dst0 + j) * d + k] = lo;
      S.tree_hi[(size_t)(dst0 + j) * d + k] = hi;
    }
    S.tree_nmin[dst0 + j] = nm;
    S.tree_vmin[dst0 + j] = vm;
  }
}

// lower bound of the key of the terminal (centroid ct, size nt, spread term
// vt) and any cluster inside node `node`
template <int LINK, int MAXD>
__device__ __forceinline__ double tree_lb(const State &S, int node, const double *ct, double nt, double vt, int d) {
  double q = 0.0;
#pragma unroll
  for (int k = 0; k < MAXD; ++k)
    if (k < d) {
      const double lo = S.tree_lo[(size_t)node * d + k], hi = S.tree_hi[(size_t)node * d + k];
      const double g = lo > ct[k] ? lo - ct[k] : (ct[k] > hi ? ct[k] - hi : 0.0);
      q += g * g;
    }
  if (LINK == kWard) {
    const double nm = (double)S.tree_nmin[node];
    return ((2.0 * nt * nm) / (nt + nm)) * q;
  }
  return q + (vt + S.tree_vmin[node]);
}

template <int LINK, int MAXD>
__global__ __launch_bounds__(kBlock) void k_nn_tree(State S) {
  const int nterm = S.cnt->n_term, nact = S.cnt->n_act, d = S.d;
  const int ti = blockIdx.x * blockDim.x + threadIdx.x;
  long long evals = 0, boxes = 0;
  if (ti < nterm) {
    const int t = S.term[ti];
    double ct[MAXD];
#pragma unroll
    for (int k = 0; k < MAXD; ++k) ct[k] = k < d ? S.wcen[(size_t)t * d + k] : 0.0;
    const double nt = (double)S.csize[t];
    const double vt = LINK == kAvgSq ? S.cmv[t] : 0.0;
    const double bound = beta_key<LINK>(S.predd[t]);
    double bestv = INFINITY;
    unsigned long long bestk = kNoKey;
    const int own = S.term_pos[ti] / kTreeFan;  // the terminal's own leaf
    const int top = S.tree_top;
    // Bottom up: the own leaf, then the subtrees of its siblings, then those
    // of its parent's siblings, ... (nearest in Morton order first, so the
    // bound tightens early). (al, anc): the ancestor whose subtree is done;
    // sib: the sibling subtree being walked (-1: none yet at this level);
    // (level, idx): the node to test next, item >= 0: walking leaf idx.
    int al = 0, anc = own, sib = -1;
    int level = 0, idx = own, item = 0;
    bool done = false;
    while (!done) {
      if (item >= 0) {
        const int i = idx * kTreeFan + item;
        const int4 mt = S.item_meta[i];
        double cv[MAXD];
#pragma unroll
        for (int k = 0; k < MAXD; ++k) cv[k] = k < d ? S.item_cen[(size_t)i * d + k] : 0.0;
        const double v = cen_key<LINK, MAXD>(ct, nt, vt, cv, (double)mt.y, LINK == kAvgSq ? S.item_v[i] : 0.0, d);
        ++evals;
        const unsigned long long key = make_key(mt.z, mt.x);
        if (mt.x != t && v <= bound && better(v, key, bestv, bestk)) {
          bestv = v;
          bestk = key;
        }
        if (++item < kTreeFan && i + 1 < nact) continue;
        item = -1;
      } else {
        ++boxes;
        const double lb = tree_lb<LINK, MAXD>(S, S.tree_off[level] + idx, ct, nt, vt, d);
        if (!(lb > fmin(bound, bestv))) {
          if (level > 0) {
            --level;
            idx *= kTreeFan;  // first child
          } else {
            item = 0;
          }
          continue;
        }
      }
      // the node (level, idx) is finished: next node of the walk
      for (;;) {
        if (level == al) {
          // a subtree at level al is finished: the next sibling of anc
          const int p0 = (anc / kTreeFan) * kTreeFan, p1 = min(p0 + kTreeFan, S.tree_cnt[al]);
          int nx = sib < 0 ? p0 : sib + 1;
          if (nx == anc) ++nx;
          if (nx < p1) {
            sib = nx;
            idx = nx;
            break;
          }
          // every sibling done: the parent's subtree is done
          if (al == top) {
            done = true;
            break;
          }
          anc /= kTreeFan;
          ++al;
          sib = -1;
          level = al;
          if (al == top) {  // the root has no siblings
            done = true;
            break;
          }
          continue;
        }
        if ((idx & (kTreeFan - 1)) != kTreeFan - 1 && idx + 1 < S.tree_cnt[level]) {
          ++idx;
          break;
        }
        idx /= kTreeFan;
        ++level;
      }
    }
    if (bestk == kNoKey) {
      // the predecessor bound held nothing (cannot happen for an exact bound):
      // the full scan takes the terminal without a bound
      const int o = atomicAdd(&S.cnt->n_ovf, 1);
      S.ovf[o] = ti;
    } else {
      S.t_best[ti] = bestv;
      S.t_key[ti] = bestk;
    }
  }
  count_add(&S.cnt->cluster_evals, evals);
  count_add(&S.cnt->visits[0], evals + boxes);
}

// ---------------------------------------------------------- pair tiles ----
__device__ __forceinline__ void pair_orient(const State &S, int p, int &begR, int &nR, int &begS, int &nS) {
  const int t = S.term[S.pr_t[p]];
  const int c = S.pr_c[p];
  const bool tlow = S.cid[t] < S.cid[c];
  const int r = tlow ? t : c, q = tlow ? c : t;
  begR = S.cbeg[r];
  nR = S.csize[r];
  begS = S.cbeg[q];
  nS = S.csize[q];
}

// Tile walks: block b takes the contiguous tiles [a, e) of `total` and finds
// the owner of its first tile by binary search over the exclusive prefix
// `start` (entries with no tiles share the next entry's start); later tiles
// advance the owner.
__device__ __forceinline__ void tile_share(long long total, long long &a, long long &e) {
  const long long per = (total + gridDim.x - 1) / gridDim.x;
  a = (long long)blockIdx.x * per;
  e = a + per < total ? a + per : total;
}

__device__ __forceinline__ int tile_owner(const long long *start, int cnt, long long tile) {
  int lo = 0, hi = cnt - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int tile_advance(const long long *start, int cnt, int i, long long tile) {
  while (i + 1 < cnt && start[i + 1] <= tile) ++i;
  return i;
}

__global__ void k_pair_tiles(State S, long long *ntl) {
  const int np = (int)min(S.cnt->n_pairs, S.pair_cap);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    int br, nr, bs, ns;
    pair_orient(S, p, br, nr, bs, ns);
    ntl[p] = (long long)((nr + kTile - 1) / kTile) * (long long)((ns + kTile - 1) / kTile);
    S.pr_v[p] = 0.0;
  }
}

// Average linkage: one wavefront per 64x64 tile of a pair's point ranges,
// rows = the cluster with the lower ID. Rows are staged in LDS as FP64; lane
// j owns column point j; the tile's FP64 sum of point distances goes to
// tile_v[tile] and is added up per pair in a fixed order later.
template <int MAXD>
__global__ __launch_bounds__(kBlock) void k_tiles_avg(State S, long long ntiles) {
  constexpr int kW = kBlock / kWave;
  constexpr int MD = MAXD > 0 ? MAXD : 1;
  __shared__ double rows[kW][kTile][MD];
  const int np = (int)min(S.cnt->n_pairs, S.pair_cap);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int d = S.d;
  long long ppairs = 0;
  const long long ngroups = (ntiles + kW - 1) / kW;
  long long ga, ge;
  tile_share(ngroups, ga, ge);
  int p = ga < ge && ga * kW + w < ntiles ? tile_owner(S.pr_tile0, np, ga * kW + w) : 0;
  for (long long gg = ga; gg < ge; ++gg) {
    const long long gt = gg * kW + w;
    const bool active = gt < ntiles;
    int br = 0, r0 = 0, nrow = 0, col = 0, ns = 0, bs = 0;
    if (active) {
      p = tile_advance(S.pr_tile0, np, p, gt);
      int nr;
      pair_orient(S, p, br, nr, bs, ns);
      const long long local = gt - S.pr_tile0[p];
      const int ntc = (ns + kTile - 1) / kTile;
      const int rt = (int)(local / ntc), ctl = (int)(local % ntc);
      r0 = rt * kTile;
      nrow = min(nr, r0 + kTile) - r0;
      col = ctl * kTile + lane;
    }
    __syncthreads();
    if (MAXD > 0 && active && lane < nrow) {
      const float *pr = S.px + (size_t)(br + r0 + lane) * d;
#pragma unroll
      for (int k = 0; k < MD; ++k) rows[w][lane][k] = k < d ? (double)pr[k] : 0.0;
    }
    __syncthreads();
    double acc = 0.0;
    if (active && col < ns) {
      const float *pc = S.px + (size_t)(bs + col) * d;
      if (MAXD > 0) {
        double cv[MD];
#pragma unroll
        for (int k = 0; k < MD; ++k) cv[k] = k < d ? (double)pc[k] : 0.0;
        for (int rr = 0; rr < nrow; ++rr) {
          double qd = 0.0;
#pragma unroll
          for (int k = 0; k < MD; ++k)
            if (k < d) {
              double u = rows[w][rr][k] - cv[k];
              qd = __builtin_fma(u, u, qd);  // average: held to 1e-12, not bitwise
            }
          acc += sqrt(qd);
        }
      } else {
        for (int rr = 0; rr < nrow; ++rr) {
          const float *pr = S.px + (size_t)(br + r0 + rr) * d;
          double qd = 0.0;
          for (int k = 0; k < d; ++k) {
            double u = (double)pr[k] - (double)pc[k];
            qd += u * u;
          }
          acc += sqrt(qd);
        }
      }
      ppairs += nrow;
    }
    acc = wave_sum(acc);
    if (active && lane == 0) S.tile_v[gt] = acc;
  }
  count_add(&S.cnt->point_pairs, ppairs);
}

// ---- complete linkage: exact pruning inside a pair -----------------------
// With L a lower bound of the pair's key, only a point whose farthest possible
// distance to the other cluster exceeds L can end the farthest pair; the key is
// max(L, max over the kept points' pairs). The farthest pair itself is always
// kept, and if nothing is kept the key is L.
__device__ __forceinline__ void pair_slots(const State &S, int p, int &r, int &q) {
  const int t = S.term[S.pr_t[p]];
  const int c = S.pr_c[p];
  const bool tlow = S.cid[t] < S.cid[c];
  r = tlow ? t : c;
  q = tlow ? c : t;
}

__global__ void k_pair_prep_comp(State S, long long *nch) {
  const int np = (int)min(S.cnt->n_pairs, S.pair_cap);
  const int d = S.d;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    int r, q;
    pair_slots(S, p, r, q);
    if (!(S.pr_v[p] >= 0.0)) {
      // no bound yet (a screened pair brings its L): box / spread bounds and
      // the extreme-point pairs
      const double *cr = S.wcen + (size_t)r * d, *cq = S.wcen + (size_t)q * d;
      double lb, ub;
      pair_bounds<kComplete, 0>(cr, S.lo + (size_t)r * d, S.hi + (size_t)r * d, cq, S.lo + (size_t)q * d,
                                S.hi + (size_t)q * d, d, lb, ub, spread_lo(S, r) + spread_lo(S, q));
      // the (2d)^2 extreme-point pairs pay off for large pairs (above 4-D
      // their count grows faster than the filter saves on small ones)
      if (d <= 4 || (long long)S.csize[r] * S.csize[q] >= 4096) comp_lb_refine(S, r, q, d, lb);
      S.pr_v[p] = lb;
    }
    S.pr_kR[p] = 0;
    S.pr_kS[p] = 0;
    nch[p] = (S.csize[r] + S.csize[q] + kChunk - 1) / kChunk;
  }
}

// squared farthest-distance bound from a point to a cluster: min of the box
// corner bound and (|x - c| + radius)^2
__device__ __forceinline__ double point_far_ub(const float *x, const State &S, int c, int d) {
  const float *lo = S.lo + (size_t)c * d, *hi = S.hi + (size_t)c * d;
  const double *cc = S.wcen + (size_t)c * d;
  double box = 0.0, c2 = 0.0;
  for (int k = 0; k < d; ++k) {
    const double v = (double)x[k];
    const double a = v - (double)lo[k], b = (double)hi[k] - v;
    const double e = a > b ? a : b;
    box += e * e;
    const double u = v - cc[k];
    c2 += u * u;
  }
  double sp = sqrt(c2) + S.crad[c];
  sp = sp * sp;
  return (box < sp ? box : sp) * (1.0 + 1e-12);
}

// one block per 256-point chunk of a pair's points (both sides)
__global__ __launch_bounds__(kBlock) void k_filter_comp(State S, long long nchunks) {
  __shared__ int sp;
  __shared__ double vtx[2][kSupDirs][2];  // enclosing polygons of R (0) and S (1), d == 2
  const int np = (int)min(S.cnt->n_pairs, S.pair_cap);
  const int d = S.d;
  long long ca, ce;
  tile_share(nchunks, ca, ce);
  int owner = 0;
  if (threadIdx.x == 0 && ca < ce) owner = tile_owner(S.pr_cbase, np, ca);
  for (long long ch = ca; ch < ce; ++ch) {
    if (threadIdx.x == 0) {
      owner = tile_advance(S.pr_cbase, np, owner, ch);
      sp = owner;
    }
    __syncthreads();
    const int p = sp;
    int r, q;
    pair_slots(S, p, r, q);
    if (d == 2 && threadIdx.x < 2 * kSupDirs) {
      const int side = threadIdx.x / kSupDirs, k = threadIdx.x % kSupDirs;
      double vx, vy;
      sup_vertex(S.xin, S.sup + (size_t)(side ? q : r) * kSupDirs, k, vx, vy);
      vtx[side][k][0] = vx;
      vtx[side][k][1] = vy;
    }
    __syncthreads();
    const int nR = S.csize[r], nS = S.csize[q];
    const long long region = S.pr_cbase[p] * kChunk;
    const int local = (int)((ch - S.pr_cbase[p]) * kChunk) + threadIdx.x;
    if (local < nR + nS) {
      const bool rside = local < nR;
      const int pos = rside ? S.cbeg[r] + local : S.cbeg[q] + (local - nR);
      const float *xp = S.px + (size_t)pos * d;
      double ub = point_far_ub(xp, S, rside ? q : r, d);
      if (d == 2 && ub >= S.pr_v[p]) {
        // farthest distance to the other cluster's enclosing polygon
        const int side = rside ? 1 : 0;
        const double px0 = (double)xp[0], px1 = (double)xp[1];
        double m = 0.0;
        for (int k = 0; k < kSupDirs; ++k) {
          const double u = px0 - vtx[side][k][0], v = px1 - vtx[side][k][1];
          const double qd = u * u + v * v;
          m = qd > m ? qd : m;
        }
        m *= 1.0 + 1e-10;
        ub = m < ub ? m : ub;
      }
      if (ub >= S.pr_v[p]) {
        const int k = atomicAdd(rside ? &S.pr_kR[p] : &S.pr_kS[p], 1);
        S.fidx[region + (rside ? 0 : nR) + k] = pos;
      }
    }
    __syncthreads();
  }
}

__global__ void k_pair_tiles_f(State S, long long *ntl) {
  const int np = (int)min(S.cnt->n_pairs, S.pair_cap);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    const int kr = S.pr_kR[p], ks = S.pr_kS[p];
    ntl[p] = (long long)((kr + kTile - 1) / kTile) * (long long)((ks + kTile - 1) / kTile);
  }
}

// Tiles of kept points. A block takes four consecutive tiles per step (one per
// wavefront; the loop bound is uniform over the block so barriers are safe).
// Each wavefront stages its tile's 64 row points in LDS as FP64; lane j owns
// kept column point j and sweeps the rows with broadcast LDS reads.
template <int MAXD>
__global__ __launch_bounds__(kBlock) void k_tiles_comp(State S) {
  constexpr int kW = kBlock / kWave;
  constexpr int MD = MAXD > 0 ? MAXD : 1;
  __shared__ double rows[kW][kTile][MD];
  const int np = (int)min(S.cnt->n_pairs, S.pair_cap);
  const long long ntiles = S.cnt->n_tiles;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int d = S.d;
  long long ppairs = 0;
  const long long ngroups = (ntiles + kW - 1) / kW;
  long long ga, ge;
  tile_share(ngroups, ga, ge);
  int p = ga < ge && ga * kW + w < ntiles ? tile_owner(S.pr_tile0, np, ga * kW + w) : 0;
  for (long long gg = ga; gg < ge; ++gg) {
    const long long gt = gg * kW + w;
    const bool active = gt < ntiles;
    int r0 = 0, nrow = 0, col = 0, ks = 0, nR = 0;
    long long region = 0;
    if (active) {
      p = tile_advance(S.pr_tile0, np, p, gt);
      int r, q;
      pair_slots(S, p, r, q);
      nR = S.csize[r];
      const int kr = S.pr_kR[p];
      ks = S.pr_kS[p];
      region = S.pr_cbase[p] * kChunk;
      const long long local = gt - S.pr_tile0[p];
      const int ntc = (ks + kTile - 1) / kTile;
      const int rt = (int)(local / ntc), ctl = (int)(local % ntc);
      r0 = rt * kTile;
      nrow = min(kr, r0 + kTile) - r0;
      col = ctl * kTile + lane;
    }
    __syncthreads();
    if (MAXD > 0 && active && lane < nrow) {
      const float *pr = S.px + (size_t)S.fidx[region + r0 + lane] * d;
#pragma unroll
      for (int k = 0; k < MD; ++k) rows[w][lane][k] = k < d ? (double)pr[k] : 0.0;
    }
    __syncthreads();
    double acc = 0.0;
    if (active && col < ks) {
      const float *pc = S.px + (size_t)S.fidx[region + nR + col] * d;
      if (MAXD > 0) {
        double cv[MD];
#pragma unroll
        for (int k = 0; k < MD; ++k) cv[k] = k < d ? (double)pc[k] : 0.0;
        for (int rr = 0; rr < nrow; ++rr) {
          double qd = 0.0;
#pragma unroll
          for (int k = 0; k < MD; ++k)
            if (k < d) {
              double u = rows[w][rr][k] - cv[k];
              qd += u * u;
            }
          acc = qd > acc ? qd : acc;
        }
      } else {
        for (int rr = 0; rr < nrow; ++rr) {
          const float *pr = S.px + (size_t)S.fidx[region + r0 + rr] * d;
          double qd = 0.0;
          for (int k = 0; k < d; ++k) {
            double u = (double)pr[k] - (double)pc[k];
            qd += u * u;
          }
          acc = qd > acc ? qd : acc;
        }
      }
      ppairs += nrow;
    }
    acc = wave_max(acc);
    if (active && lane == 0) atomicMax((unsigned long long *)&S.pr_v[p], pos_bits(acc));
  }
  count_add(&S.cnt->point_pairs, ppairs);
}

// Exact tiles for 16 < d <= kGramMaxDim: one block per 64x64 tile, both point
// sets staged in LDS (coordinate-major, FP32 as given), each thread a 4x4
// block of pairs. Squared distances are summed over the coordinates in order
// with separate multiply and add, as the oracle does. Average adds the roots
// into the tile's sum; complete takes the largest square.
template <int LINK>
__global__ __launch_bounds__(kBlock) void k_tiles_hd(State S) {
  __shared__ __attribute__((aligned(16))) float As[kGramMaxDim][kTile];
  __shared__ __attribute__((aligned(16))) float Bs[kGramMaxDim][kTile];
  __shared__ double red[kBlock / kWave];
  const int np = (int)min(S.cnt->n_pairs, S.pair_cap);
  const long long ntiles = S.cnt->n_tiles;
  const int d = S.d;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  long long ppairs = 0;
  long long ta, te;
  tile_share(ntiles, ta, te);
  int p = ta < te ? tile_owner(S.pr_tile0, np, ta) : 0;
  for (long long gt = ta; gt < te; ++gt) {
    p = tile_advance(S.pr_tile0, np, p, gt);
    const long long local = gt - S.pr_tile0[p];
    int nA, nB, begA = 0, begB = 0;
    long long region = 0;
    if (LINK == kAverage) {
      pair_orient(S, p, begA, nA, begB, nB);
    } else {
      int r, q;
      pair_slots(S, p, r, q);
      nA = S.pr_kR[p];
      nB = S.pr_kS[p];
      region = S.pr_cbase[p] * kChunk;
      begB = S.csize[r];  // column indices follow the row cluster's slots
    }
    const int ntc = (nB + kTile - 1) / kTile;
    const int r0 = (int)(local / ntc) * kTile, c0 = (int)(local % ntc) * kTile;
    const int nr = min(kTile, nA - r0), nc = min(kTile, nB - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < kTile * d; j += kBlock) {
      const int i = j / d, k = j % d;
      float a = 0.0f, b = 0.0f;
      if (i < nr) {
        const int pa = LINK == kAverage ? begA + r0 + i : S.fidx[region + r0 + i];
        a = S.px[(size_t)pa * d + k];
      }
      if (i < nc) {
        const int pb = LINK == kAverage ? begB + c0 + i : S.fidx[region + begB + c0 + i];
        b = S.px[(size_t)pb * d + k];
      }
      // column position swizzled by k (XOR of a multiple of 4): the lanes of a
      // wavefront store to eight banks instead of one, and every aligned
      // group of four stays contiguous for the float4 reads below
      const int sw = i ^ ((k & 7) << 2);
      As[k][sw] = a;
      Bs[k][sw] = b;
    }
    __syncthreads();
    double q[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) q[a][b] = 0.0;
    for (int k = 0; k < d; ++k) {
      const int sk = (k & 7) << 2;
      const float4 av = *(const float4 *)&As[k][(ty * 4) ^ sk];
      const float4 bv = *(const float4 *)&Bs[k][(tx * 4) ^ sk];
      const double ar[4] = {(double)av.x, (double)av.y, (double)av.z, (double)av.w};
      const double br[4] = {(double)bv.x, (double)bv.y, (double)bv.z, (double)bv.w};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const double u = ar[a] - br[b];
          // complete: separate multiply and add (bit-identical maxima);
          // average: fused (held to 1e-12)
          if (LINK == kAverage) q[a][b] = __builtin_fma(u, u, q[a][b]);
          else q[a][b] += u * u;
        }
    }
    double part = LINK == kAverage ? 0.0 : -1.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (ty * 4 + a >= nr || tx * 4 + b >= nc) continue;
        if (LINK == kAverage) part += sqrt(q[a][b]);
        else part = q[a][b] > part ? q[a][b] : part;
      }
    part = LINK == kAverage ? wave_sum(part) : wave_max(part);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      double v = red[0];
      for (int j = 1; j < kBlock / kWave; ++j) v = LINK == kAverage ? v + red[j] : (red[j] > v ? red[j] : v);
      if (LINK == kAverage) S.tile_v[gt] = v;
      else atomicMax((unsigned long long *)&S.pr_v[p], pos_bits(v));
      ppairs += (long long)nr * nc;
    }
  }
  count_add(&S.cnt->point_pairs, ppairs);  // nonzero in thread 0 only
}

// Per pair: finish the value, then WriteMin into its terminal's best value.
__global__ __launch_bounds__(kBlock) void k_pair_finish(State S, int link) {
  const int np = (int)min(S.cnt->n_pairs, S.pair_cap);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave0 = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nwaves = (gridDim.x * blockDim.x) / kWave;
  long long evals = 0;
  if (link == kComplete) {
    // the value is already in place (tile maxima): a thread per pair
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
      const double v = S.pr_v[p];
      atomicMin(&S.t_min[S.pr_t[p]], pos_bits(v));
      ++evals;
      if (S.cache_mask) cache_fill(S, pair_key(S.node[S.term[S.pr_t[p]]], S.node[S.pr_c[p]]), v);
    }
    count_add(&S.cnt->cluster_evals, evals);
    return;
  }
  for (int p = wave0; p < np; p += nwaves) {
    double v;
    {
      const long long a = S.pr_tile0[p], b = (p + 1 < np) ? S.pr_tile0[p + 1] : S.cnt->n_tiles;
      double s = 0.0;
      for (long long g = a + lane; g < b; g += kWave) s += S.tile_v[g];
      s = wave_sum(s);
      int br, nr, bs, ns;
      pair_orient(S, p, br, nr, bs, ns);
      v = s / ((double)nr * (double)ns);
    }
    if (lane == 0) {
      S.pr_v[p] = v;
      atomicMin(&S.t_min[S.pr_t[p]], pos_bits(v));
      ++evals;
      if (S.cache_mask) cache_fill(S, pair_key(S.node[S.term[S.pr_t[p]]], S.node[S.pr_c[p]]), v);
    }
  }
  count_add(&S.cnt->cluster_evals, evals);
}

__global__ void k_term_key_reset(State S) {
  const int nterm = min(S.tb1, S.cnt->n_term);
  for (int ti = S.tb0 + blockIdx.x * blockDim.x + threadIdx.x; ti < nterm; ti += gridDim.x * blockDim.x)
    if (pos_bits(S.t_best[ti]) != S.t_min[ti]) S.t_key[ti] = kNoKey;
}

__global__ void k_pair_key(State S) {
  const int np = (int)min(S.cnt->n_pairs, S.pair_cap);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    const int ti = S.pr_t[p];
    if (pos_bits(S.pr_v[p]) == S.t_min[ti]) {
      const int c = S.pr_c[p];
      atomicMin(&S.t_key[ti], make_key(S.cid[c], c));
    }
  }
}

// Pairs another terminal evaluated this round: take the stored value.
__global__ void k_pending_min(State S) {
  const int np = (int)min(S.cnt->n_pend, S.pair_cap);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
    const int ti = S.pd_t[i], c = S.pd_c[i];
    double v = S.pd_v[i];
    if (v >= 0.0) {
      // combined from cached parts during the search: store it now
      cache_fill(S, pair_key(S.node[S.term[ti]], S.node[c]), v);
    } else if (cache_find(S, pair_key(S.node[S.term[ti]], S.node[c]), v) != 1) {
      S.cnt->nonfinite = 4;  // a claimed pair was not evaluated
      continue;
    }
    atomicMin(&S.t_min[ti], pos_bits(v));
  }
}

__global__ void k_pending_key(State S) {
  const int np = (int)min(S.cnt->n_pend, S.pair_cap);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
    const int ti = S.pd_t[i], c = S.pd_c[i];
    double v = S.pd_v[i];
    const bool have = v >= 0.0 || cache_find(S, pair_key(S.node[S.term[ti]], S.node[c]), v) == 1;
    if (have && pos_bits(v) == S.t_min[ti]) atomicMin(&S.t_key[ti], make_key(S.cid[c], c));
  }
}

// ------------------------------------------------------------ Gram search --
// For d >= kGramMinDim the centroid grid prunes poorly, so every terminal is
// compared with every active cluster through MFMA Gram tiles, and every
// candidate that the rounding bounds cannot rule out is evaluated exactly in
// FP64 afterwards:
//   * centroids are recentred on the middle of their range, scaled into
//     [-1, 1] (distances scale by sc) and rounded to FP16 (x~);
//   * per cluster the prep pass keeps |x~|^2, the FP64 norm eta of the
//     rounding error x - x~ (rounded up) and an allowance e for the FP32
//     accumulation of the dot products; with T = |x~ - y~| and D the scaled
//     centroid distance, |D - T| <= eta_x + eta_y, and
//     d2 = |x~|^2 + |y~|^2 - 2 x~.y~ is within e_x + e_y of T^2;
//   * pass 0 (bound pass) picks, per terminal, the cluster with the smallest
//     cheap key estimate (|x~-y~|^2 scaled by the Ward size factor, or plus
//     the two spreads; the norm terms ride in two augmented coordinates, so
//     the MFMA produces the estimate itself) and evaluates an FP64 upper bound
//     of that cluster's key: exact for Ward (Table 1), exact for complete and
//     average when the pair is cached or small, else the centroid-distance
//     radius and spread bounds. Any upper bound of the nearest key will do;
//   * pass 1 records every cluster whose rigorous lower bound (FP32 with
//     outward margins) does not exceed that bound: Ward w D^2, complete
//     D^2 + spreads (mean squared point distance <= largest), average D
//     (centroid distance <= mean distance, Sec. 4.2).
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float float16v __attribute__((ext_vector_type(16)));

// Element type of the screening tiles (pc_options.precision): FP16 or BF16
// operands on the 32x32x16 MFMA, or FP32 operands on the 32x32x2 MFMA; FP32
// accumulation in every case. The rounding error of each rounded vector is
// measured from its actual rounded values (eta below), so every bound holds
// for any of them; FP32 products are not exact, which the accumulation
// allowance covers (kElAllow).
template <int E> struct El;
template <> struct El<kElF16> {
  typedef _Float16 T;
  static constexpr int KS = 16;  // K of one MFMA
  __device__ static T from(float f) { return (T)f; }
  __device__ static float to(T v) { return (float)v; }
  __device__ static float16v mma(const T *a, const T *b, float16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(*(const half8 *)a, *(const half8 *)b, c, 0, 0, 0);
  }
};
template <> struct El<kElBF16> {
  typedef __bf16 T;
  static constexpr int KS = 16;
  __device__ static T from(float f) { return (T)f; }
  __device__ static float to(T v) { return (float)v; }
  __device__ static float16v mma(const T *a, const T *b, float16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8 *)a, *(const bf16x8 *)b, c, 0, 0, 0);
  }
};
template <> struct El<kElF32> {
  typedef float T;
  static constexpr int KS = 2;
  __device__ static T from(float f) { return f; }
  __device__ static float to(T v) { return v; }
  __device__ static float16v mma(const T *a, const T *b, float16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(*a, *b, c, 0, 0, 0);
  }
};
// elements per 16-byte chunk; LDS rows are padded by one chunk
template <int E> constexpr int el_chunk() { return 16 / (int)sizeof(typename El<E>::T); }
// the FP32 accumulation allowance per vector, in units of 2^-24 |x~|^2 per
// term: products of 16-bit operands are exact in FP32, FP32 products round
__host__ __device__ constexpr double kElAllow(int e) { return e == kElF32 ? 3.0 : 2.0; }
constexpr int kGT = 64;                      // block tile: 64 terminals x 64 candidates
constexpr float kGMargin = 1.0f + 1.0f / 16384.0f;  // outward margin of the FP32 tests

__device__ __forceinline__ float f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}

__device__ __forceinline__ float f32_dn(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return f;
}

// per-dimension range of the active centroids: a wave per item, lanes over dims
__global__ void k_gram_range(State S) {
  const int nact = S.cnt->n_act, d = S.d;
  const int lane = threadIdx.x & (kWave - 1);
  const int w0 = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, nw = (gridDim.x * blockDim.x) / kWave;
  unsigned long long lo[2] = {~0ull, ~0ull}, hi[2] = {0ull, 0ull};
  for (int i = w0; i < nact; i += nw) {
    const double *c = S.wcen + (size_t)S.act[i] * d;
    for (int j = 0; j < 2; ++j) {
      const int k = lane + j * kWave;
      if (k < d) {
        const unsigned long long b = ordered_bits(c[k]);
        lo[j] = b < lo[j] ? b : lo[j];
        hi[j] = b > hi[j] ? b : hi[j];
      }
    }
  }
  for (int j = 0; j < 2; ++j) {
    const int k = lane + j * kWave;
    if (k < d && lo[j] != ~0ull) {
      atomicMin(&S.gmin[k], lo[j]);
      atomicMax(&S.gmax[k], hi[j]);
    }
  }
}

__global__ void k_gram_setup(State S) {
  const int k = threadIdx.x;
  __shared__ double rr[kGramMaxDim];
  double r = 0.0;
  if (k < S.d) {
    const double lo = from_ordered_bits(S.gmin[k]), hi = from_ordered_bits(S.gmax[k]);
    S.gorg[k] = 0.5 * (lo + hi);
    r = 0.5 * (hi - lo);
  }
  rr[k] = r;
  __syncthreads();
  if (k == 0) {
    double m = 0.0;
    for (int j = 0; j < S.d; ++j) m = rr[j] > m ? rr[j] : m;
    *S.gscale = m > 0.0 ? 1.0 / m : 1.0;
  }
}

__global__ void k_gram_reset(State S) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < S.d) {
    S.gmin[k] = ~0ull;
    S.gmax[k] = 0ull;
  }
}

// FP16 copy of every active centroid (active-list order, zero beyond d) and
// its FP32 terms: x = |x~|^2 (+ mean squared spread for complete/average:
// the bound pass estimate), y = |x~|^2 - e rounded down, z = eta rounded up,
// w = 1/size (Ward) or the mean squared spread rounded down (complete, avg-2).
// A wave per item, lanes over dims.
template <int E>
__global__ void k_gram_prep(State S) {
  typedef typename El<E>::T T;
  T *g = reinterpret_cast<T *>(S.g16);
  const int nact = S.cnt->n_act, d = S.d, kp = S.gkp;
  const double sc = *S.gscale;
  const int lane = threadIdx.x & (kWave - 1);
  const int w0 = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, nw = (gridDim.x * blockDim.x) / kWave;
  for (int i = w0; i < nact; i += nw) {
    const int sl = S.act[i];
    const double *c = S.wcen + (size_t)sl * d;
    double nrm = 0.0, err = 0.0;
    for (int k = lane; k < kp; k += kWave) {
      T h = El<E>::from(0.0f);
      if (k < d) {
        const double xs = (c[k] - S.gorg[k]) * sc;
        h = El<E>::from((float)xs);
        const double hv = (double)El<E>::to(h);
        nrm += hv * hv;
        err += (xs - hv) * (xs - hv);
      }
      g[(size_t)i * kp + k] = h;
    }
    nrm = wave_sum(nrm);
    err = wave_sum(err);
    if (lane == 0) {
      // FP32 accumulation of kp exact products (FP32 operands: rounded
      // products too), plus the FP32 roundings of the norms and of
      // |x~|^2 + |y~|^2 - 2 x~.y~, with a factor 2 to spare
      const double e = kElAllow(E) * (double)(kp + 8) * 5.9604644775390625e-8 * nrm + 1e-30;
      // eta: the rounding error, plus the FP64 error of the scaled centroid
      const double eta = sqrt(err) * (1.0 + 1e-12) + 1e-15 * sqrt(nrm) + 1e-18;
      double v = 0.0;
      if (S.linkage != kWard) v = S.cvar[sl] / (double)S.csize[sl] * sc * sc;
      float4 q;
      q.x = (float)(nrm + v);
      q.y = f32_dn(nrm - e);
      q.z = f32_up(eta * (double)kGMargin);
      if (S.linkage == kWard) {
        q.w = (float)(1.0 / (double)S.csize[sl]);
      } else {
        const double vdn = v * (1.0 - 1e-6) - 0.5e-12;
        q.w = f32_dn(vdn > 0.0 ? vdn : 0.0);
      }
      S.gq[i] = q;
    }
  }
}

__global__ void k_term_pos(State S) {
  const int nact = S.cnt->n_act;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nact; i += gridDim.x * blockDim.x)
    if (S.flags[i]) S.term_pos[S.scan[i]] = i;
}

template <int LINK>
__global__ void k_gram_init(State S, int *t_ovf) {
  const int nterm = min(S.tb1, S.cnt->n_term);
  for (int ti = S.tb0 + blockIdx.x * blockDim.x + threadIdx.x; ti < nterm; ti += gridDim.x * blockDim.x) {
    S.t_best[ti] = INFINITY;
    S.t_key[ti] = kNoKey;
    S.t_min[ti] = pos_bits(INFINITY);
    S.t_beta[ti] = beta_key<LINK>(S.predd[S.term[ti]]);
    t_ovf[ti] = 0;
  }
}

// FP64 upper bound of the key of terminal t and cluster c (the pass-0 pick).
template <int LINK>
__device__ double gram_pick_upper(const State &S, int t, int c) {
  const int d = S.d;
  const double *ct = S.wcen + (size_t)t * d, *cc = S.wcen + (size_t)c * d;
  if (LINK == kWard) return ward_key<0>(ct, (double)S.csize[t], cc, (double)S.csize[c], d);
  if (LINK == kAvgSq) return avgsq_key<0>(ct, S.cmv[t], cc, S.cmv[c], d);
  double v;
  if (cache_resolve(S, S.node[t], S.node[c], v)) return v;
  const int nt = S.csize[t], nc = S.csize[c];
  if ((long long)nt * nc <= kInlinePairs)
    return (S.cid[c] < S.cid[t]) ? pair_exact_inline<LINK>(S.px, d, S.cbeg[c], nc, S.cbeg[t], nt)
                                 : pair_exact_inline<LINK>(S.px, d, S.cbeg[t], nt, S.cbeg[c], nc);
  double D2 = 0.0;
  for (int k = 0; k < d; ++k) {
    const double x = ct[k] - cc[k];
    D2 += x * x;
  }
  // complete: farthest pair <= D + rt + rc; average: also <= the root of the
  // mean squared point distance D^2 + spreads (Jensen)
  const double u1 = sqrt(D2) + S.crad[t] + S.crad[c];
  if (LINK == kComplete) return u1 * u1 * (1.0 + 1e-12);
  const double sc = *S.gscale;
  const double vs = (S.cvar[t] / (double)nt + S.cvar[c] / (double)nc) * (1.0 + 1e-6) + 1e-12 / (sc * sc);
  const double u2 = sqrt(D2 + vs);
  return (u1 < u2 ? u1 : u2) * (1.0 + 1e-12);
}

// Stage a 64-row tile of FP16 vectors in LDS. Pass 0 augments them so that
// the MFMA result is the bound pass estimate: rows get (x~, a, 1), columns
// (-2 y~, 1, b), with a, b the norm terms, so the product is a + b - 2 x~.y~.
template <int KP, int PASS, bool ROW, int E>
__device__ __forceinline__ void gram_stage(const State &S, typename El<E>::T (*dst)[KP + el_chunk<E>()],
                                           const int *src_idx, const float *aug, int nvalid, int d) {
  typedef typename El<E>::T T;
  constexpr int EPC = el_chunk<E>();  // elements per 16-byte chunk
  constexpr int CH = KP / EPC;        // chunks per row
  const T *g = reinterpret_cast<const T *>(S.g16);
  for (int j = threadIdx.x; j < kGT * CH; j += kBlock) {
    const int r = j / CH, c8 = j % CH;
    uint4 raw = make_uint4(0, 0, 0, 0);
    if (r < nvalid) {
      raw = *(const uint4 *)(g + (size_t)src_idx[r] * KP + c8 * EPC);
      if (PASS == 0) {
        T v[EPC];
        __builtin_memcpy(v, &raw, 16);
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
          const int k = c8 * EPC + e;
          if (!ROW && k < d) v[e] = El<E>::from(El<E>::to(v[e]) * -2.0f);  // exact
          if (k == d) v[e] = El<E>::from(ROW ? aug[r] : 1.0f);
          if (k == d + 1) v[e] = El<E>::from(ROW ? 1.0f : aug[r]);
        }
        __builtin_memcpy(&raw, v, 16);
      }
    }
    *(uint4 *)&dst[r][c8 * EPC] = raw;
  }
}

template <int LINK, int KP, int PASS, int E>
__global__ __launch_bounds__(kBlock) void k_gram(State S) {
  typedef typename El<E>::T T;
  constexpr int KS = El<E>::KS;
  __shared__ __attribute__((aligned(16))) T sq[kGT][KP + el_chunk<E>()];
  __shared__ __attribute__((aligned(16))) T sc[kGT][KP + el_chunk<E>()];
  __shared__ float4 qd[kGT], cd[kGT];
  __shared__ float qaug[kGT], caug[kGT], qthr[kGT];
  __shared__ int qs[kGT], qt[kGT], qp[kGT], cs[kGT], cidx[kGT];
  __shared__ float rbest[4][32];
  __shared__ int rarg[4][32];
  const int nterm = min(S.tb1, S.cnt->n_term), nact = S.cnt->n_act;  // this batch: [tb0, nterm)
  const int q0 = S.tb0 + blockIdx.x * kGT;
  if (q0 >= nterm) return;  // uniform per block
  const int nq = min(kGT, nterm - q0);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int d = S.d;
  const double scale = *S.gscale;
  if (threadIdx.x < kGT) {
    const int r = threadIdx.x, ti = q0 + r;
    if (r < nq) {
      const int pi = S.term_pos[ti];
      const float4 g = S.gq[pi];
      qs[r] = S.term[ti];
      qt[r] = ti;
      qp[r] = pi;
      cidx[r] = pi;  // staging source for the rows
      qd[r] = g;
      qaug[r] = g.x;
      if (PASS == 1) {
        // threshold in scaled key units, rounded up with margin
        const double u = S.t_beta[ti] * kSlack;
        const double us = LINK == kAverage ? u * scale : u * scale * scale;
        float uf = f32_up(us * (double)kGMargin);
        uf = uf > 1e-30f ? uf : 1e-30f;
        if (LINK == kWard) qthr[r] = 0.5f * uf;
        else if (LINK == kComplete || LINK == kAvgSq) qthr[r] = uf - g.w;
        else qthr[r] = uf + g.z;
      }
    } else {
      qs[r] = -1;
      qt[r] = -1;
      qp[r] = -1;
      cidx[r] = 0;
      qd[r] = make_float4(NAN, NAN, NAN, NAN);
      qaug[r] = 0.0f;
      if (PASS == 1) qthr[r] = NAN;
    }
  }
  __syncthreads();
  gram_stage<KP, PASS, true, E>(S, sq, cidx, qaug, nq, d);
  // this lane's 16 rows (MFMA 32x32 output layout)
  float rq[16], rz[16], rt[16], re[16];
  int pmin = 0x7fffffff, pmax = -1;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = wr + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
    const float4 g = qd[row];
    rq[i] = PASS == 0 ? g.x : g.y;
    rz[i] = g.w;
    re[i] = g.z;
    rt[i] = PASS == 1 ? qthr[row] : 0.0f;
  }
  for (int r = 0; r < nq; ++r) {
    pmin = min(pmin, qp[r]);
    pmax = max(pmax, qp[r]);
  }
  float best[16];
  int barg[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    best[i] = INFINITY;
    barg[i] = -1;
  }
  long long pairs = 0;
  for (int c0 = blockIdx.y * kGT; c0 < nact; c0 += gridDim.y * kGT) {
    const int nc = min(kGT, nact - c0);
    __syncthreads();
    if (threadIdx.x < kGT) {
      const int r = threadIdx.x;
      if (r < nc) {
        const float4 g = S.gq[c0 + r];
        cd[r] = g;
        caug[r] = g.x;
        cs[r] = S.act[c0 + r];
        cidx[r] = c0 + r;
      } else {
        // padding columns: an infinite norm term keeps them out of both passes
        cd[r] = make_float4(INFINITY, INFINITY, 0.0f, 1.0f);
        caug[r] = 0.0f;
        cs[r] = -2;
        cidx[r] = 0;
      }
    }
    __syncthreads();
    gram_stage<KP, PASS, false, E>(S, sc, cidx, caug, nc, d);
    __syncthreads();
    if (threadIdx.x == 0) pairs += (long long)nq * nc;
    float16v acc = {};
    // lanes 0-31 hold k values [kk, kk + KS/2) of their row, lanes 32-63 the rest
#pragma unroll
    for (int kk = 0; kk < KP; kk += KS)
      acc = El<E>::mma(&sq[wr + (lane & 31)][kk + (lane >> 5) * (KS / 2)],
                       &sc[wc + (lane & 31)][kk + (lane >> 5) * (KS / 2)], acc);
    const int col = wc + (lane & 31);
    const int ci = c0 + col;
    const float4 cg = cd[col];
    // the terminals' own columns lie in [pmin, pmax]; only those tiles check
    const bool selfs = c0 <= pmax && c0 + kGT > pmin;
    if (PASS == 0) {
      const float cz = cg.w;
      const bool padc = col >= nc;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        float g = acc[i];
        if (LINK == kWard) g = g * __builtin_amdgcn_rcpf(rz[i] + cz);
        if (padc) g = INFINITY;
        if (selfs) {
          const int row = wr + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
          if (qp[row] == ci) g = INFINITY;
        }
        if (g < best[i]) {
          best[i] = g;
          barg[i] = ci;
        }
      }
    } else {
      const float cm = cg.y, ce = cg.z, cw = cg.w;
      const int cslot = cs[col];
      unsigned rmask = 0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        // lower bound of T^2 against the square of (threshold distance + eta)
        const float lhs = __builtin_fmaf(-2.0f, acc[i], rq[i] + cm);
        float rr;
        if (LINK == kWard) rr = __builtin_amdgcn_sqrtf(rt[i] * (rz[i] + cw)) + (re[i] + ce);
        else if (LINK == kComplete || LINK == kAvgSq) rr = __builtin_amdgcn_sqrtf(rt[i] - cw) + (re[i] + ce);
        else rr = rt[i] + ce;
        rmask |= (lhs <= rr * rr ? 1u : 0u) << i;
      }
      if (cslot < 0) rmask = 0;
      if (selfs && rmask) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int row = wr + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
          if (qp[row] == ci) rmask &= ~(1u << i);
        }
      }
      // one atomic per wavefront and tile: exclusive prefix of the lanes' counts
      if (__ballot(rmask != 0)) {
        const int cnt = __popc(rmask);
        int incl = cnt;
        for (int o = 1; o < kWave; o <<= 1) {
          const int y = __shfl_up(incl, o, kWave);
          if (lane >= o) incl += y;
        }
        long long base = 0;
        if (lane == kWave - 1 && incl > 0) base = (long long)atomicAdd((unsigned long long *)&S.cnt->n_cand, (unsigned long long)incl);
        base = __shfl(base, kWave - 1, kWave);
        long long k = base + incl - cnt;
        while (rmask) {
          const int i = __ffs(rmask) - 1;
          rmask &= rmask - 1;
          const int row = wr + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
          if (k < S.cand_cap) {
            S.cd_t[k] = qt[row];
            S.cd_c[k] = cslot;
            S.cd_lb[k] = 0.0;
          } else {
            S.cnt->cand_overflow = 1;
          }
          ++k;
        }
      }
    }
  }
  if (PASS == 0) {
    // each row's pick: over the 32 lanes holding the row, then over the two
    // wavefronts that share the rows; then its FP64 upper bound
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      float v = best[i];
      int a = barg[i];
      for (int o = 16; o > 0; o >>= 1) {
        const float u = __shfl_xor(v, o, kWave);
        const int b = __shfl_xor(a, o, kWave);
        if (u < v || (u == v && b >= 0 && (a < 0 || b < a))) {
          v = u;
          a = b;
        }
      }
      best[i] = v;
      barg[i] = a;
    }
    __syncthreads();
    if ((lane & 31) == 0)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int rl = (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
        rbest[w][rl] = best[i];
        rarg[w][rl] = barg[i];
      }
    __syncthreads();
    if (threadIdx.x < kGT) {
      const int r = threadIdx.x, wq = (r >> 5) * 2;
      const float b0 = rbest[wq][r & 31], b1 = rbest[wq + 1][r & 31];
      const int a0 = rarg[wq][r & 31], a1 = rarg[wq + 1][r & 31];
      const int a = (b1 < b0 || (b1 == b0 && a1 >= 0 && (a0 < 0 || a1 < a0))) ? a1 : a0;
      if (qt[r] >= 0 && a >= 0) {
        const double u = gram_pick_upper<LINK>(S, qs[r], S.act[a]);
        atomicMin((unsigned long long *)&S.t_beta[qt[r]], pos_bits(u));
      }
    }
  }
  count_add(&S.cnt->visits[PASS == 0 ? 0 : 3], pairs);  // nonzero in thread 0 only
}

// ---- Gram search: interval screening of large candidate pairs -----------
// A complete/average candidate whose exact value would cost many point
// distances first gets a rigorous interval [L, H] from FP16 MFMA tiles over
// its point pairs: the points are recentred and scaled once per call (psc),
// rounded to FP16 with the same per-point terms as the centroids (|x~|^2, the
// accumulation allowance e and the rounding norm eta). Per point pair with
// s = sqrt(max(d2, 0)) and T = |x~ - y~|: |s - T| <= min(sqrt(E), E / s) for
// E = e_x + e_y, and ||x - y| - T| <= eta_x + eta_y. Average sums s over the
// tile; complete takes the largest d2. Each terminal's bound drops to its
// smallest H, and only candidates with L <= bound are evaluated exactly.
constexpr long long kIntervalWork = 16384;  // point pairs x d from which a pair is screened first
constexpr int kIntervalMinDim = 32;         // average: below it exact FP64 tiles are cheaper than screening
                                            // (complete screens at every Gram dimension: its tile
                                            // maximum brackets tightly and costs ~3 ops per pair)

// per-dimension range of all points (once per call)
__global__ void k_pt_range(const float *x, int n, int d, unsigned long long *gmin, unsigned long long *gmax) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w0 = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, nw = (gridDim.x * blockDim.x) / kWave;
  unsigned long long lo[2] = {~0ull, ~0ull}, hi[2] = {0ull, 0ull};
  for (int i = w0; i < n; i += nw)
    for (int j = 0; j < 2; ++j) {
      const int k = lane + j * kWave;
      if (k < d) {
        const unsigned long long b = ordered_bits((double)x[(size_t)i * d + k]);
        lo[j] = b < lo[j] ? b : lo[j];
        hi[j] = b > hi[j] ? b : hi[j];
      }
    }
  for (int j = 0; j < 2; ++j) {
    const int k = lane + j * kWave;
    if (k < d && lo[j] != ~0ull) {
      atomicMin(&gmin[k], lo[j]);
      atomicMax(&gmax[k], hi[j]);
    }
  }
}

__global__ void k_pt_setup(State S) {
  const int k = threadIdx.x;
  __shared__ double rr[kGramMaxDim];
  double r = 0.0;
  if (k < S.d) {
    const double lo = from_ordered_bits(S.gmin[k]), hi = from_ordered_bits(S.gmax[k]);
    S.porg[k] = 0.5 * (lo + hi);
    r = 0.5 * (hi - lo);
  }
  rr[k] = r;
  __syncthreads();
  if (k == 0) {
    double m = 0.0;
    for (int j = 0; j < S.d; ++j) m = rr[j] > m ? rr[j] : m;
    *S.pscale = m > 0.0 ? 1.0 / m : 1.0;
  }
}

// FP16 copy of every point in its current (permuted) place, and its FP32
// terms: x = |x~|^2, y = e, z = eta (rounded up). A wave per point.
template <int E>
__global__ void k_pt_prep(State S) {
  typedef typename El<E>::T T;
  T *g = reinterpret_cast<T *>(S.p16);
  const int n = S.n, d = S.d, kp = S.pkp;
  const double sc = *S.pscale;
  const int lane = threadIdx.x & (kWave - 1);
  const int w0 = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, nw = (gridDim.x * blockDim.x) / kWave;
  for (int i = w0; i < n; i += nw) {
    const float *p = S.px + (size_t)i * d;
    double nrm = 0.0, err = 0.0;
    for (int k = lane; k < kp; k += kWave) {
      T h = El<E>::from(0.0f);
      if (k < d) {
        const double xs = ((double)p[k] - S.porg[k]) * sc;
        h = El<E>::from((float)xs);
        const double hv = (double)El<E>::to(h);
        nrm += hv * hv;
        err += (xs - hv) * (xs - hv);
      }
      g[(size_t)i * kp + k] = h;
    }
    nrm = wave_sum(nrm);
    err = wave_sum(err);
    if (lane == 0) {
      const double e = kElAllow(E) * (double)(kp + 8) * 5.9604644775390625e-8 * nrm + 1e-30;
      const double eta = sqrt(err) * (1.0 + 1e-12) + 1e-15 * sqrt(nrm) + 1e-18;
      S.pq[i] = make_float4((float)nrm, f32_up(e), f32_up(eta * (double)kGMargin), 0.0f);
    }
  }
}

// Candidates: small pairs (at most kInlinePairs point pairs) are listed for
// an exact evaluation now, which also tightens the terminal's bound; large
// pairs get their tile count and point ranges for the interval pass (the
// cache is consulted only for the pairs that survive it). cd_lb < 0 marks a
// candidate whose exact value is in cd_v.
// complete, d <= kBlkMaxDim: the box of every 64-position block of the points
// in their current places (FP32, exact), once per round
__global__ void k_blk_boxes(State S) {
  const int n = S.n, d = S.d;
  const int nb = (n + 63) / 64;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
    const int p0 = b * 64, p1 = min(p0 + 64, n);
    for (int k = 0; k < d; ++k) {
      float lo = INFINITY, hi = -INFINITY;
      for (int p = p0; p < p1; ++p) {
        const float v = S.px[(size_t)p * d + k];
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
      }
      S.blk_lo[(size_t)b * d + k] = lo;
      S.blk_hi[(size_t)b * d + k] = hi;
    }
  }
}

// Upper bound of the squared distance of any point at positions [a, a + na)
// and any at [b, b + nb): per coordinate the farthest ends of the two unions
// of block boxes (at most two blocks per side), summed in FP64 and rounded up.
__device__ __forceinline__ double blk_far_ub(const State &S, int a, int na, int b, int nb) {
  const int d = S.d;
  const int a0 = a / 64, a1 = (a + na - 1) / 64, b0 = b / 64, b1 = (b + nb - 1) / 64;
  double q = 0.0;
  for (int k = 0; k < d; ++k) {
    const double la = fmin((double)S.blk_lo[(size_t)a0 * d + k], (double)S.blk_lo[(size_t)a1 * d + k]);
    const double ha = fmax((double)S.blk_hi[(size_t)a0 * d + k], (double)S.blk_hi[(size_t)a1 * d + k]);
    const double lb = fmin((double)S.blk_lo[(size_t)b0 * d + k], (double)S.blk_lo[(size_t)b1 * d + k]);
    const double hb = fmax((double)S.blk_hi[(size_t)b0 * d + k], (double)S.blk_hi[(size_t)b1 * d + k]);
    const double e = fmax(ha - lb, hb - la);
    q += e * e;
  }
  return q * (1.0 + 1e-12);
}

template <int LINK>
__global__ void k_cand_triage(State S, int ncand) {
  const int d = S.d;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncand; i += gridDim.x * blockDim.x) {
    const int ti = S.cd_t[i], c = S.cd_c[i];
    const int t = S.term[ti];
    const int nt = S.csize[t], nc = S.csize[c];
    const long long cost = (long long)nt * nc;
    if (cost <= kInlinePairs) {
      const long long k = append_slot(&S.cnt->n_small);
      S.cd_small[k] = i;  // k < ncand: every candidate appends at most once
    } else if (d >= (LINK == kComplete ? kGramMinDim : kIntervalMinDim) &&
               (cost * d >= kIntervalWork || (LINK == kComplete && tiles_settle_complete(S.pkp, d)))) {
      // (complete, settled in the tiles: every candidate above the inline
      // size, the tiles being far cheaper than FP64 tiles of padded pairs)
      // dense list of screened candidates: tile count, point ranges, index
      const long long k = append_slot(&S.cnt->n_scr);
      S.cd_tile0[k] = (long long)((nt + kGT - 1) / kGT) * ((nc + kGT - 1) / kGT);
      S.cd_desc[k] = make_int4(S.cbeg[t], nt, S.cbeg[c], nc);
      S.cd_scr[k] = i;
      double l0 = 0.0;
      if (LINK == kComplete) {
        // a lower bound of the key before any tile: the spread and box bounds
        // and, up to d = kExtMaxDim, the largest distance among the two
        // clusters' extreme points (a real pair); tiles whose block boxes
        // stay below it cannot hold the farthest pair
        double lb, ub;
        pair_bounds<kComplete, 0>(S.wcen + (size_t)t * d, S.lo + (size_t)t * d, S.hi + (size_t)t * d,
                                  S.wcen + (size_t)c * d, S.lo + (size_t)c * d, S.hi + (size_t)c * d, d, lb, ub,
                                  spread_lo(S, t) + spread_lo(S, c));
        comp_lb_refine(S, t, c, d, lb);
        l0 = lb > 0.0 ? lb * (1.0 - 1e-9) : 0.0;
      }
      S.cd_l0[k] = l0;
      S.cd_x[k] = LINK == kComplete && tiles_settle_complete(S.pkp, d) ? 0ull : kNoExact;
      S.cd_lb[i] = l0;
      S.cd_v[i] = 0.0;
    }
  }
}

__global__ void k_scr_count(Counters *c) { c->n_scr32 = (int)c->n_scr; }

// Complete, d <= kBlkMaxDim: a tighter fixed bound for each large screened
// candidate before its tiles, from real point pairs found by farthest-point
// steps (one block per candidate): the row point farthest from the column
// cluster's centroid, the column point farthest from it, and the row point
// farthest from that. Their squared distances are keys of real pairs, so the
// largest is a lower bound of the candidate's key (lowered by 1e-12 for the
// summation order).
constexpr long long kSeedTiles = 16;  // candidates with fewer tiles keep L0

// the point of [beg, beg + cnt) farthest from ref (FP32 distance picks it)
__device__ int far_point(const State &S, int beg, int cnt, const double *ref) {
  const int d = S.d;
  unsigned long long best = 0;
  for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
    const float *x = S.px + (size_t)(beg + j) * d;
    double q = 0.0;
    for (int k = 0; k < d; ++k) {
      const double u = (double)x[k] - ref[k];
      q += u * u;
    }
    const unsigned long long key = ((unsigned long long)__float_as_uint((float)q) << 32) | (unsigned)j;
    best = key > best ? key : best;
  }
  best = block_reduce<unsigned long long, false>(best);
  return beg + (int)(best & 0xffffffffu);
}

__device__ __forceinline__ double point_sq(const State &S, int a, int b) {
  const int d = S.d;
  double q = 0.0;
  for (int k = 0; k < d; ++k) {
    const double u = (double)S.px[(size_t)a * d + k] - (double)S.px[(size_t)b * d + k];
    q += u * u;
  }
  return q;
}

__global__ __launch_bounds__(kBlock) void k_cand_seed(State S) {
  __shared__ double ref[kBlkMaxDim];
  const int nscr = S.cnt->n_scr32, d = S.d;
  for (int k = blockIdx.x; k < nscr; k += gridDim.x) {
    const int4 ds = S.cd_desc[k];
    const long long tiles = (long long)((ds.y + kGT - 1) / kGT) * ((ds.w + kGT - 1) / kGT);
    if (tiles < kSeedTiles) continue;  // uniform per block
    const int i = S.cd_scr[k];
    const int c = S.cd_c[i];
    __syncthreads();
    if (threadIdx.x < d) ref[threadIdx.x] = S.wcen[(size_t)c * d + threadIdx.x];
    __syncthreads();
    const int r1 = far_point(S, ds.x, ds.y, ref);
    __syncthreads();
    if (threadIdx.x < d) ref[threadIdx.x] = (double)S.px[(size_t)r1 * d + threadIdx.x];
    __syncthreads();
    const int c1 = far_point(S, ds.z, ds.w, ref);
    __syncthreads();
    if (threadIdx.x < d) ref[threadIdx.x] = (double)S.px[(size_t)c1 * d + threadIdx.x];
    __syncthreads();
    const int r2 = far_point(S, ds.x, ds.y, ref);
    if (threadIdx.x == 0) {
      const double a = point_sq(S, r1, c1), b = point_sq(S, r2, c1);
      const double l = (a > b ? a : b) * (1.0 - 1e-12);
      if (l > S.cd_l0[k]) {
        S.cd_l0[k] = l;
        if (l > S.cd_lb[i]) S.cd_lb[i] = l;
      }
    }
  }
}

// Small candidates: a wavefront per candidate, a lane per point pair (rows:
// the cluster with the lower ID), coordinates summed in order; points are
// read in 16-byte pieces when d is a multiple of 4.
template <int LINK>
__global__ void k_cand_small(State S) {
  const int nsm = (int)S.cnt->n_small, d = S.d;
  const int lane = threadIdx.x & (kWave - 1);
  const int w0 = (blockIdx.x * blockDim.x + threadIdx.x) / kWave, nw = (gridDim.x * blockDim.x) / kWave;
  long long evals = 0, ppairs = 0;
  for (int j = w0; j < nsm; j += nw) {
    const int i = S.cd_small[j];
    const int ti = S.cd_t[i], c = S.cd_c[i];
    const int t = S.term[ti];
    const bool tl = S.cid[t] < S.cid[c];
    const int r = tl ? t : c, q = tl ? c : t;
    const int nS = S.csize[q], cost = S.csize[r] * nS;
    double val = 0.0;
    if (lane < cost) {
      const float *pr = S.px + (size_t)(S.cbeg[r] + lane / nS) * d;
      const float *pc = S.px + (size_t)(S.cbeg[q] + lane % nS) * d;
      double q2 = 0.0;
      if ((d & 3) == 0) {
        for (int k = 0; k < d; k += 4) {
          const float4 a = *(const float4 *)(pr + k), b = *(const float4 *)(pc + k);
          double u = (double)a.x - (double)b.x;
          q2 += u * u;
          u = (double)a.y - (double)b.y;
          q2 += u * u;
          u = (double)a.z - (double)b.z;
          q2 += u * u;
          u = (double)a.w - (double)b.w;
          q2 += u * u;
        }
      } else {
        for (int k = 0; k < d; ++k) {
          const double u = (double)pr[k] - (double)pc[k];
          q2 += u * u;
        }
      }
      val = LINK == kComplete ? q2 : sqrt(q2);
    }
    val = LINK == kComplete ? wave_max(val) : wave_sum(val) / (double)cost;
    if (lane == 0) {
      S.cd_v[i] = val;
      S.cd_lb[i] = -1.0;
      atomicMin((unsigned long long *)&S.t_beta[ti], pos_bits(val));
      ++evals;
      ppairs += cost;
    }
  }
  count_add(&S.cnt->cluster_evals, evals);
  count_add(&S.cnt->point_pairs, ppairs);
}

// Squared distance of points a and b in FP64, coordinates summed in order
// (the complete-linkage key of a point pair); 16-byte reads when d is a
// multiple of 4.
__device__ __forceinline__ double pair_sq_exact(const float *px, int a, int b, int d) {
  const float *x = px + (size_t)a * d, *y = px + (size_t)b * d;
  double q = 0.0;
  if ((d & 3) == 0) {
    for (int k = 0; k < d; k += 4) {
      const float4 u4 = *(const float4 *)(x + k), v4 = *(const float4 *)(y + k);
      double u = (double)u4.x - (double)v4.x;
      q += u * u;
      u = (double)u4.y - (double)v4.y;
      q += u * u;
      u = (double)u4.z - (double)v4.z;
      q += u * u;
      u = (double)u4.w - (double)v4.w;
      q += u * u;
    }
  } else {
    for (int k = 0; k < d; ++k) {
      const double u = (double)x[k] - (double)y[k];
      q += u * u;
    }
  }
  return q;
}

// Position of the r-th set bit (from 0) of m, which has more than r set bits.
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int r) {
  int base = 0;
#pragma unroll
  for (int w = 32; w > 0; w >>= 1) {
    const unsigned long long low = m & ((1ull << w) - 1);
    const int c = __popcll(low);
    if (r >= c) {
      r -= c;
      m >>= w;
      base += w;
    } else {
      m = low;
    }
  }
  return base;
}

// exact point-pair keys a wavefront takes per tile before it leaves the
// candidate to the exact pass instead
constexpr int kSettleCap = 4 * kWave;

// One block per 64x64 tile of a screened candidate's point pairs (rows: the
// terminal's points), four 32x32 MFMA sub-tiles; the tile's bound
// contributions are added (average) or maxed (complete) into the candidate.
// Each block walks a contiguous range of tiles; the next tile's points are
// loaded into registers while the current one is computed.
// SETTLE (complete): the same tiles again, for the candidates that survived
// their terminal's bound only (cd_l0 >= 0: sqrt(L) in tile units, L the
// candidate's final lower bound). A pair whose upper bound reaches L gets its
// exact FP64 key, the largest of which is the candidate's key: the farthest
// pair's upper bound reaches L. A wavefront that meets more than kSettleCap
// such pairs in one tile (near-equal distances) leaves the candidate to the
// exact pass instead (cd_x = kNoExact).
template <int LINK, int KP, int EL, bool SETTLE>
__global__ __launch_bounds__(kBlock, 4) void k_cand_tiles(State S, int ncand) {
  typedef typename El<EL>::T T;
  constexpr int KS = El<EL>::KS;
  constexpr int EPC = el_chunk<EL>();                   // elements per 16-byte chunk
  constexpr int CH = KP / EPC;                         // 16-byte chunks per point
  constexpr int NCH = (2 * kGT * CH + kBlock - 1) / kBlock;  // chunks per thread (both sides)
  __shared__ __attribute__((aligned(16))) T sab[2][kGT][KP + EPC];
  const T *pts = reinterpret_cast<const T *>(S.p16);
  __shared__ float an[2][kGT];
  __shared__ float side[2][3];  // per side: sum eta, max eta, max e
  __shared__ float red[3][kBlock / kWave];
  const long long ntiles = S.cnt->n_ctiles;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const double isc = 1.0 / *S.pscale;
  long long pairs = 0, settled = 0;
  const int nscr = S.cnt->n_scr32;
  long long ta, te;
  tile_share(ntiles, ta, te);
  if (ta >= te) {
    count_add(&S.cnt->visits[1], 0);
    return;
  }
  // the current screened entry and the next one (its metadata loaded one
  // entry ahead); every entry has at least one tile
  int own = tile_owner(S.cd_tile0, nscr, ta);
  int4 ds = S.cd_desc[own];
  int oi = S.cd_scr[own];
  long long ostart = S.cd_tile0[own];
  long long oend = own + 1 < nscr ? S.cd_tile0[own + 1] : ntiles;
  int4 nds = make_int4(0, 0, 0, 0);
  int ni = 0;
  long long nend = ntiles;
  auto ahead = [&]() {
    if (own + 1 < nscr) {
      nds = S.cd_desc[own + 1];
      ni = S.cd_scr[own + 1];
      nend = own + 2 < nscr ? S.cd_tile0[own + 2] : ntiles;
    }
  };
  ahead();
  uint4 reg[NCH];
  float4 rq = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  int cur_i = 0, cur_nr = 0, cur_nc = 0, cur_k = 0, cur_ba = 0, cur_bb = 0;
  // complete, d <= kBlkMaxDim: a tile whose block boxes cannot reach the
  // candidate's fixed lower bound holds no farthest pair and is skipped (the
  // tile holding the farthest pair always reaches it, so L and H stay valid);
  // the decision uses values no thread writes during the kernel, so it is
  // uniform over the block
  const bool prune = !SETTLE && LINK == kComplete && KP <= 32 && S.d <= kBlkMaxDim;  // compiled out above K = 32
  static_assert(!SETTLE || LINK == kComplete, "settling takes complete linkage's maximum");
  int ba = 0, bb = 0, nr = 0, nc = 0;
  auto locate = [&](long long tile) {
    if (tile >= oend) {
      ++own;
      ostart = oend;
      oend = nend;
      ds = nds;
      oi = ni;
      ahead();
    }
    const long long local = tile - ostart;
    const int ntc = (ds.w + kGT - 1) / kGT;
    const int r0 = (int)(local / ntc) * kGT, c0 = (int)(local % ntc) * kGT;
    // uniform over the block by construction: kept in scalar registers
    nr = __builtin_amdgcn_readfirstlane(min(kGT, ds.y - r0));
    nc = __builtin_amdgcn_readfirstlane(min(kGT, ds.w - c0));
    ba = __builtin_amdgcn_readfirstlane(ds.x + r0);
    bb = __builtin_amdgcn_readfirstlane(ds.z + c0);
  };
  // consecutive tiles of a candidate share their rows (tiles run row by
  // row): above K = 32 those are kept in LDS and only the columns are loaded
  // again (at small K the operands are cheap and the test costs more)
  constexpr bool kKeepRows = KP > 32;
  int last_ba = -1, last_nr = -1;
  bool cur_reuse = false;
  auto fetch = [&](long long tile) {
    locate(tile);
    const bool reuse = kKeepRows && ba == last_ba && nr == last_nr;
    last_ba = ba;
    last_nr = nr;
#pragma unroll
    for (int u = 0; u < NCH; ++u) {
      const int j = threadIdx.x + u * kBlock;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (j < 2 * kGT * CH) {
        const int sd = j / (kGT * CH), r = (j / CH) % kGT, c8 = j % CH;
        if (r < (sd ? nc : nr) && (sd || !reuse))
          v = *(const uint4 *)(pts + (size_t)((sd ? bb : ba) + r) * KP + c8 * EPC);
      }
      reg[u] = v;
    }
    rq = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (w < 2 && lane < (w ? nc : nr) && (w || !reuse)) rq = S.pq[(w ? bb : ba) + lane];
    cur_reuse = reuse;
    cur_i = oi;
    cur_nr = nr;
    cur_nc = nc;
    cur_k = own;
    cur_ba = ba;
    cur_bb = bb;
  };
  // the first tile at or after `tile` that is not skipped (its points
  // loaded), or te. The bound is the entry's fixed L0, raised for the entry
  // of the last snapshot to the running lower bound that thread 0 read into
  // LDS before the last barrier (the same value for every thread).
  // (tiles are visited one by one in order, so locate() crosses at most one
  // entry per tile, and locating a tile twice changes nothing)
  // With pruning, the block tests a window of up to kBlock tiles of one
  // entry at once (a thread per tile) and takes the first one kept.
  __shared__ double snap_lb;
  __shared__ int snap_own;
  __shared__ long long win_first[kBlock / kWave];
  if (threadIdx.x == 0) snap_own = -1;
  __syncthreads();
  auto next_tile = [&](long long tile) -> long long {
    if (SETTLE) {
      // the rest of an entry that did not survive is skipped
      while (tile < te) {
        locate(tile);
        if (S.cd_l0[own] >= 0.0) {
          fetch(tile);
          return tile;
        }
        tile = oend;
      }
      return te;
    }
    if (!prune) {
      if (tile < te) fetch(tile);
      return tile < te ? tile : te;
    }
    while (tile < te) {
      locate(tile);  // enters the tile's entry (at most one crossing)
      const long long wend = min(min(oend, te), tile + (long long)kBlock);
      double thr = S.cd_l0[own];
      if (own == snap_own) thr = fmax(thr, snap_lb);
      const long long my = tile + threadIdx.x;
      long long cand = LLONG_MAX;
      if (my < wend) {
        const long long local = my - ostart;
        const int ntc = (ds.w + kGT - 1) / kGT;
        const int r0 = (int)(local / ntc) * kGT, c0 = (int)(local % ntc) * kGT;
        const int mr = min(kGT, ds.y - r0), mc = min(kGT, ds.w - c0);
        if (!(blk_far_ub(S, ds.x + r0, mr, ds.z + c0, mc) < thr)) cand = my;
      }
      cand = wave_min(cand);
      __syncthreads();  // the previous window's reads of win_first are done
      if ((threadIdx.x & (kWave - 1)) == 0) win_first[threadIdx.x / kWave] = cand;
      __syncthreads();
      long long first = win_first[0];
      for (int q = 1; q < kBlock / kWave; ++q) first = win_first[q] < first ? win_first[q] : first;
      if (first < wend) {
        fetch(first);  // inside the entry located above: no crossing
        return first;
      }
      tile = wend;
    }
    return te;
  };
  long long tile = next_tile(ta);
  while (tile < te) {
    const int i = cur_i, nr = cur_nr, ncl = cur_nc, kc = cur_k, ta0 = cur_ba, tb0 = cur_bb;
    const bool keep_rows = cur_reuse;  // the rows in LDS are this tile's
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NCH; ++u) {
      const int j = threadIdx.x + u * kBlock;
      if (j < 2 * kGT * CH) {
        const int sd = j / (kGT * CH), r = (j / CH) % kGT, c8 = j % CH;
        if (sd || !keep_rows) *(uint4 *)&sab[sd][r][c8 * EPC] = reg[u];
      }
    }
    if (prune && threadIdx.x == 0) {
      // the running lower bound of the current entry (tiles raise it)
      snap_lb = __hip_atomic_load(&S.cd_lb[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      snap_own = own;
    }
    if (w < 2 && (w || !keep_rows)) {
      an[w][lane] = rq.x;
      float se = rq.z, me = rq.z, mx = rq.y;
      for (int o = kWave / 2; o > 0; o >>= 1) {
        se += __shfl_xor(se, o, kWave);
        me = fmaxf(me, __shfl_xor(me, o, kWave));
        mx = fmaxf(mx, __shfl_xor(mx, o, kWave));
      }
      if (lane == 0) {
        side[w][0] = se;
        side[w][1] = me;
        side[w][2] = mx;
      }
    }
    __syncthreads();
    const long long nxt = next_tile(tile + 1);  // its points in flight during the tile's arithmetic
    // above K = 32, a wavefront whose 32 x 32 quarter holds no point pair
    // (small clusters) skips its matrix and epilogue work; it still meets
    // every barrier
    const bool wlive = !kKeepRows || (wr < nr && wc < ncl);
    float16v acc = {};
    if (wlive) {
#pragma unroll
      for (int kk = 0; kk < KP; kk += KS)
        acc = El<EL>::mma(&sab[0][wr + (lane & 31)][kk + (lane >> 5) * (KS / 2)],
                         &sab[1][wc + (lane & 31)][kk + (lane >> 5) * (KS / 2)], acc);
    }
    const int col = wc + (lane & 31);
    const bool cval = col < ncl;
    const float cn = an[1][col];
    // accumulation allowance of the tile (rounded up), and its root
    const float Ef = (side[0][2] + side[1][2]) * kGMargin;
    const float rE = __builtin_amdgcn_sqrtf(Ef) * kGMargin;
    float sum = 0.0f, smin = INFINITY, mx = -INFINITY;
    int cnt = 16;
    if (!wlive) {
      cnt = 0;
    } else if (nr == kGT && ncl == kGT) {
      // full tile: no masks
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int row = wr + (k >> 2) * 8 + (lane >> 5) * 4 + (k & 3);
        const float d2 = __builtin_fmaf(-2.0f, acc[k], an[0][row] + cn);
        if (LINK == kAverage) {
          const float s = __builtin_amdgcn_sqrtf(fmaxf(d2, 0.0f));
          sum += s;
          smin = fminf(smin, s);
        } else {
          mx = fmaxf(mx, d2);
        }
      }
    } else {
      cnt = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int row = wr + (k >> 2) * 8 + (lane >> 5) * 4 + (k & 3);
        const bool v = cval && row < nr;
        const float d2 = __builtin_fmaf(-2.0f, acc[k], an[0][row] + cn);
        if (LINK == kAverage) {
          const float s = __builtin_amdgcn_sqrtf(fmaxf(d2, 0.0f));
          sum += v ? s : 0.0f;
          smin = fminf(smin, v ? s : INFINITY);
          cnt += v ? 1 : 0;
        } else {
          mx = fmaxf(mx, v ? d2 : -INFINITY);
        }
      }
    }
    // every pair of this lane: |s - T| <= min(sqrt(E), E / s) <= min(sqrt(E), E / smin)
    float eps = 0.0f;
    if (LINK == kAverage)
      eps = (float)cnt * fminf(rE, Ef * __builtin_amdgcn_rcpf(smin) * kGMargin) * kGMargin;
    for (int o = kWave / 2; o > 0; o >>= 1) {
      sum += __shfl_xor(sum, o, kWave);
      eps += __shfl_xor(eps, o, kWave);
      mx = fmaxf(mx, __shfl_xor(mx, o, kWave));
    }
    if (SETTLE && mx > -INFINITY) {
      // per pair: exact key <= ((sqrt(d2 + E) (1 + 1e-6) + em) isc)^2, the
      // tile's bracket applied to one pair. Pairs with d2 below T cannot
      // reach L (T lowered for its own roundings).
      const double E = (double)side[0][2] + (double)side[1][2];
      const double em = (double)side[0][1] + (double)side[1][1];
      const double a = S.cd_l0[kc] - em;
      float T = -INFINITY;
      if (a > 0.0) {
        double t2 = a * a - E;
        t2 -= fabs(t2) * 1e-6 + a * a * 1e-6;
        T = (float)t2;
      }
      if (mx >= T) {
        // the ballot of accumulator k: which lanes' pair k qualifies
        auto qual = [&](int k) -> unsigned long long {
          const int row = wr + (k >> 2) * 8 + (lane >> 5) * 4 + (k & 3);
          const float d2 = __builtin_fmaf(-2.0f, acc[k], an[0][row] + cn);
          return __ballot(cval && row < nr && d2 >= T);
        };
        int tot = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) tot += __popcll(qual(k));
        if (tot > kSettleCap) {
          if (lane == 0) atomicMax(&S.cd_x[kc], kNoExact);
        } else if (tot > 0) {
          // lane j takes the j-th qualifying pair (k-major, then lane order)
          double best = -1.0;
          for (int j0 = 0; j0 < tot; j0 += kWave) {
            const int j = j0 + lane;
            int rem = j, ks = -1;
            unsigned long long m = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
              const unsigned long long b = qual(k);
              const int c = __popcll(b);
              if (ks < 0) {
                if (rem < c) {
                  ks = k;
                  m = b;
                } else {
                  rem -= c;
                }
              }
            }
            if (j >= tot) continue;
            const int src = nth_set_bit(m, rem);
            const int row = wr + (ks >> 2) * 8 + (src >> 5) * 4 + (ks & 3);
            const int cl = wc + (src & 31);
            best = fmax(best, pair_sq_exact(S.px, ta0 + row, tb0 + cl, S.d));
          }
          best = wave_max(best);
          if (lane == 0) {
            atomicMax(&S.cd_x[kc], pos_bits(best));
            settled += tot;
          }
        }
      }
    }
    if (SETTLE) {
      tile = nxt;
      continue;
    }
    if (lane == 0) {
      red[0][w] = sum;
      red[1][w] = eps;
      red[2][w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0, ep = 0.0, m = -INFINITY;
      for (int j = 0; j < kBlock / kWave; ++j) {
        s += (double)red[0][j];
        ep += (double)red[1][j];
        m = fmax(m, (double)red[2][j]);
      }
      const double E = (double)side[0][2] + (double)side[1][2];
      pairs += (long long)nr * ncl;
      if (LINK == kAverage) {
        // FP32 sums of at most 16 + 6 terms per partial: relative 4e-6 covers them
        const double err = (double)ncl * side[0][0] + (double)nr * side[1][0] + ep * (1.0 + 4e-6) + s * 4e-6;
        const double l = s - err > 0.0 ? s - err : 0.0;
        atomicAdd(&S.cd_lb[i], l * isc);
        atomicAdd(&S.cd_v[i], (s + err) * isc);
      } else {
        const double em = (double)side[0][1] + (double)side[1][1];
        const double tl = sqrt(m - E > 0.0 ? m - E : 0.0) * (1.0 - 1e-6) - em;
        const double th = sqrt(m + E > 0.0 ? m + E : 0.0) * (1.0 + 1e-6) + em;
        const double kl = tl > 0.0 ? tl * tl * isc * isc : 0.0;
        atomicMax((unsigned long long *)&S.cd_lb[i], pos_bits(kl));
        atomicMax((unsigned long long *)&S.cd_v[i], pos_bits(th * th * isc * isc));
      }
    }
    tile = nxt;
  }
  if (SETTLE)
    count_add(&S.cnt->point_pairs, settled);
  else
    count_add(&S.cnt->visits[1], pairs);  // nonzero in thread 0 only
}

// Screened candidates: L kept as the candidate's lower bound, H lowers the
// terminal's bound.
template <int LINK>
__global__ void k_cand_bound(State S) {
  const int nscr = S.cnt->n_scr32;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nscr; k += gridDim.x * blockDim.x) {
    const int i = S.cd_scr[k];
    const int ti = S.cd_t[i], c = S.cd_c[i];
    double l = S.cd_lb[i], h = S.cd_v[i];
    if (LINK == kAverage) {
      const double np = (double)S.csize[S.term[ti]] * (double)S.csize[c];
      l = l / np * (1.0 - 1e-12);
      h = h / np * (1.0 + 1e-12);
    } else {
      l *= 1.0 - 1e-12;
      h *= 1.0 + 1e-12;
    }
    S.cd_lb[i] = l;
    atomicMin((unsigned long long *)&S.t_beta[ti], pos_bits(h));
  }
}

// Complete, settled in the tiles: the screened candidates that survive their
// terminal's final bound (the test of k_gram_exact) get sqrt(L) in tile units
// (the threshold of the SETTLE tile pass); the others -1.
__global__ void k_settle_select(State S) {
  const int nscr = S.cnt->n_scr32;
  const double sc = *S.pscale;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nscr; k += gridDim.x * blockDim.x) {
    const int i = S.cd_scr[k];
    const double l = S.cd_lb[i];
    S.cd_l0[k] = l <= S.t_beta[S.cd_t[i]] * kSlack ? sqrt(l) * sc / (1.0 + 1e-6) : -1.0;
  }
}

// Settled survivors: the largest exact pair key is the candidate's value (an
// exact value, like a small pair's); a survivor the tiles could not settle
// keeps its lower bound and goes to the exact pass.
__global__ void k_settle_finish(State S) {
  const int nscr = S.cnt->n_scr32;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nscr; k += gridDim.x * blockDim.x) {
    if (!(S.cd_l0[k] >= 0.0)) continue;
    const unsigned long long x = S.cd_x[k];
    const int i = S.cd_scr[k];
    if (x == kNoExact || (x == 0ull && S.cd_lb[i] > 0.0)) continue;
    S.cd_lb[i] = -1.0;
    S.cd_v[i] = pos_from_bits(x);
  }
}

// Recorded candidates: exact FP64 value (Ward, small complete/average pairs,
// cache hits) or a claim on the pair for the tile pass.
template <int LINK>
__global__ void k_gram_exact(State S) {
  if (S.cnt->cand_overflow) return;  // the round is redone with a larger record
  const int nc = (int)min(S.cnt->n_cand, S.cand_cap), d = S.d;
  long long evals = 0, ppairs = 0, hits = 0, refined = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
    const int ti = S.cd_t[i], c = S.cd_c[i];
    const double lb = S.cd_lb[i];
    if (!centroid_link(LINK) && lb < 0.0) {
      // exact value of a small pair, from the triage pass
      atomicMin(&S.t_min[ti], pos_bits(S.cd_v[i]));
      ++refined;
      continue;
    }
    S.cd_v[i] = NAN;
    if (lb > S.t_beta[ti] * kSlack) continue;
    ++refined;
    const int t = S.term[ti];
    double v;
    if (centroid_link(LINK)) {
      v = cen_key<LINK, 0>(S.wcen + (size_t)t * d, (double)S.csize[t], LINK == kAvgSq ? S.cmv[t] : 0.0,
                           S.wcen + (size_t)c * d, (double)S.csize[c], LINK == kAvgSq ? S.cmv[c] : 0.0, d);
      ++evals;
    } else {
      const int nt = S.csize[t], ncs = S.csize[c];
      const long long cost = (long long)nt * ncs;
      if (cost <= kInlinePairs) {
        v = (S.cid[c] < S.cid[t]) ? pair_exact_inline<LINK>(S.px, d, S.cbeg[c], ncs, S.cbeg[t], nt)
                                  : pair_exact_inline<LINK>(S.px, d, S.cbeg[t], nt, S.cbeg[c], ncs);
        ++evals;
        ppairs += cost;
      } else {
        const unsigned long long pk = pair_key(S.node[t], S.node[c]);
        if (cache_resolve(S, S.node[t], S.node[c], v)) {
          ++hits;
        } else {
          if (S.cache_mask && cache_claim(S, pk) == 2) {
            const long long q = append_slot(&S.cnt->n_pend);
            if (q < S.pair_cap) {
              S.pd_t[q] = ti;
              S.pd_c[q] = c;
              S.pd_v[q] = -1.0;
            } else {
              S.cnt->pair_overflow = 1;
            }
            continue;
          }
          const long long p = append_slot(&S.cnt->n_pairs);
          if (p < S.pair_cap) {
            S.pr_t[p] = ti;
            S.pr_c[p] = c;
            // complete: a screened candidate's lower bound L (within the
            // FP16 error of the value) starts the exact pass; others get
            // theirs from the pair prep
            S.pr_v[p] = LINK == kComplete && lb > 0.0 ? lb : -1.0;
          } else {
            S.cnt->pair_overflow = 1;
          }
          continue;
        }
      }
    }
    S.cd_v[i] = v;
    atomicMin(&S.t_min[ti], pos_bits(v));
  }
  count_add(&S.cnt->cluster_evals, evals);
  count_add(&S.cnt->point_pairs, ppairs);
  count_add(&S.cnt->cache_hits, hits);
  count_add(&S.cnt->refined, refined);
}

// After every value of the round is in t_min: the lowest cluster ID among the
// recorded candidates that reach it.
__global__ void k_gram_key(State S) {
  if (S.cnt->cand_overflow) return;
  const int nc = (int)min(S.cnt->n_cand, S.cand_cap);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
    const double v = S.cd_v[i];
    if (!(v >= 0.0)) continue;
    const int ti = S.cd_t[i], c = S.cd_c[i];
    if (pos_bits(v) == S.t_min[ti]) atomicMin(&S.t_key[ti], make_key(S.cid[c], c));
  }
}

// ---------------------------------------------------------------- chain --
// succ := nearest neighbour; WriteMin of the distance into the neighbour's
// predecessor slot (Alg. 1 chain update, the neighbour's pred is written).
__global__ void k_chain(State S) {
  const int nterm = S.cnt->n_term;
  for (int ti = blockIdx.x * blockDim.x + threadIdx.x; ti < nterm; ti += gridDim.x * blockDim.x) {
    const int t = S.term[ti];
    const unsigned long long key = S.t_key[ti];
    if (key == kNoKey) {
      S.cnt->nonfinite = 2;  // no neighbour found: reported as a device error
      S.succ[t] = -1;
      continue;
    }
    const int u = (int)(key & 0xffffffffu);
    const double v = ((centroid_link(S.linkage) || S.single) && !S.gram) ? S.t_best[ti] : pos_from_bits(S.t_min[ti]);
    const double h = key_to_height(S.linkage, v);
    S.succ[t] = u;
    S.succ_node[t] = S.node[u];
    S.nn_h[t] = h;
    atomicMin(&S.predd[u], f32_bits_up(h));
  }
}

// Reciprocal pairs: t with succ[succ[t]] == t, kept once (from the lower ID
// when both ends are terminals of this round).
__global__ void k_rnn_flags(State S, int round) {
  const int nterm = S.cnt->n_term;
  for (int ti = blockIdx.x * blockDim.x + threadIdx.x; ti < nterm; ti += gridDim.x * blockDim.x) {
    const int t = S.term[ti];
    const int u = S.succ[t];
    int f = 0;
    if (u >= 0 && S.succ[u] == t && S.succ_node[u] == S.node[t])
      f = (S.term_round[u] != round || S.cid[t] < S.cid[u]) ? 1 : 0;
    S.flags[ti] = f;
  }
}

__global__ void k_rnn_scatter(State S) {
  const int nterm = S.cnt->n_term;
  for (int ti = blockIdx.x * blockDim.x + threadIdx.x; ti < nterm; ti += gridDim.x * blockDim.x) {
    if (!S.flags[ti]) continue;
    const int m = S.scan[ti];
    if (m < 0 || m > S.n / 2) {
      S.cnt->nonfinite = 3;
      continue;
    }
    const int t = S.term[ti], u = S.succ[t];
    const bool tl = S.cid[t] < S.cid[u];
    S.m_a[m] = tl ? t : u;
    S.m_b[m] = tl ? u : t;
    S.m_h[m] = S.nn_h[t];
  }
}

// Merge every reciprocal pair (Alg. 1 merge): the new cluster lives in the
// slot of the child with the lower ID; Ward/centroid sums in FP64.
__global__ void k_merge(State S, int base) {
  const int nm = S.cnt->n_merge;
  const int d = S.d;
  const int n = S.n;
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < nm; m += gridDim.x * blockDim.x) {
    const int a = S.m_a[m], b = S.m_b[m];
    const double h = S.m_h[m];
    const int r = base + m;
    if (r < 0 || r >= n - 1) {
      S.cnt->nonfinite = 3;
      continue;
    }
    const int sa = S.csize[a], sb = S.csize[b];
    S.row_na[r] = S.node[a];
    S.row_nb[r] = S.node[b];
    S.row_h[r] = h;
    S.row_size[r] = sa + sb;
    S.row_lo[r] = S.cid[a];
    double e = h;
    e = S.eff[a] > e ? S.eff[a] : e;
    e = S.eff[b] > e ? S.eff[b] : e;
    S.row_eff[r] = e;
    S.eff[a] = e;
    const int ns = sa + sb;
    S.csize[a] = ns;
    if (!centroid_link(S.linkage)) {
      // radius bound of the union: max over children of |c_new - c_child| + r_child
      // (old centroids are still in place here)
      double da = 0.0, db = 0.0;
      for (int k = 0; k < d; ++k) {
        const double c = (S.wsum[(size_t)a * d + k] + S.wsum[(size_t)b * d + k]) / (double)ns;
        const double ta = c - S.wcen[(size_t)a * d + k], tb = c - S.wcen[(size_t)b * d + k];
        da += ta * ta;
        db += tb * tb;
      }
      const double ra = sqrt(da) + S.crad[a], rb = sqrt(db) + S.crad[b];
      S.crad[a] = (ra > rb ? ra : rb) * (1.0 + 1e-12);
    }
    if (S.linkage != kWard) {
      // Var(A u B) = Var(A) + Var(B) + |A||B|/(|A|+|B|) |cA - cB|^2 (sums of
      // squared deviations; the merge rule of Sec. 2.1 with its size factor)
      double cab = 0.0;
      for (int k = 0; k < d; ++k) {
        const double t = S.wcen[(size_t)a * d + k] - S.wcen[(size_t)b * d + k];
        cab += t * t;
      }
      S.cvar[a] = S.cvar[a] + S.cvar[b] + ((double)sa * (double)sb / (double)ns) * cab;
      if (S.linkage == kAvgSq) S.cmv[a] = S.cvar[a] / (double)ns;
    }
    if (S.linkage == kComplete) {
      if (d <= kExtMaxDim)
        for (int k = 0; k < d; ++k) {
          int *ea = S.ext + (size_t)a * 2 * d, *eb = S.ext + (size_t)b * 2 * d;
          const float la = S.xin[(size_t)ea[2 * k] * d + k], lb = S.xin[(size_t)eb[2 * k] * d + k];
          if (lb < la || (lb == la && eb[2 * k] < ea[2 * k])) ea[2 * k] = eb[2 * k];
          const float ha = S.xin[(size_t)ea[2 * k + 1] * d + k], hb = S.xin[(size_t)eb[2 * k + 1] * d + k];
          if (hb > ha || (hb == ha && eb[2 * k + 1] < ea[2 * k + 1])) ea[2 * k + 1] = eb[2 * k + 1];
        }
    }
    for (int k = 0; k < d; ++k) {
      const double sum = S.wsum[(size_t)a * d + k] + S.wsum[(size_t)b * d + k];
      S.wsum[(size_t)a * d + k] = sum;
      S.wcen[(size_t)a * d + k] = sum / (double)ns;
    }
    if (!centroid_link(S.linkage)) {
      for (int k = 0; k < d; ++k) {
        S.lo[(size_t)a * d + k] = fminf(S.lo[(size_t)a * d + k], S.lo[(size_t)b * d + k]);
        S.hi[(size_t)a * d + k] = fmaxf(S.hi[(size_t)a * d + k], S.hi[(size_t)b * d + k]);
      }
      S.mdst[b] = a;
      S.moff[b] = sa;
    }
    if (S.cache_mask) {
      S.nparent[S.node[a]] = n + r;
      S.nparent[S.node[b]] = n + r;
    }
    S.node[a] = n + r;
    S.node2slot[n + r] = a;
    S.succ[a] = -1;
    S.succ_node[a] = -1;
    S.predd[a] = kInfBits;
    S.alive[b] = 0;
    S.succ[b] = -1;
    S.node[b] = -1;
  }
}

// support points of merged clusters (d == 2): thread per (merge, direction)
__global__ void k_merge_sup(State S) {
  const long long total = (long long)S.cnt->n_merge * kSupDirs;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(i / kSupDirs), k = (int)(i % kSupDirs);
    const int a = S.m_a[m], b = S.m_b[m];
    int *sa = S.sup + (size_t)a * kSupDirs + k;
    const int sb = S.sup[(size_t)b * kSupDirs + k];
    double c, sn;
    sup_dir(k, c, sn);
    const float *pa = S.xin + (size_t)(*sa) * 2, *pb = S.xin + (size_t)sb * 2;
    const double va = c * (double)pa[0] + sn * (double)pa[1], vb = c * (double)pb[0] + sn * (double)pb[1];
    if (vb > va || (vb == va && sb < *sa)) *sa = sb;
  }
}

__global__ void k_alive_flags(State S) {
  const int nact = S.cnt->n_act;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nact; i += gridDim.x * blockDim.x)
    S.flags[i] = S.alive[S.act[i]];
}

__global__ void k_sizes_of_act(State S) {
  const int nact = S.cnt->n_act;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nact; i += gridDim.x * blockDim.x)
    S.flags[i] = S.csize[S.act[i]];
}

__global__ void k_set_nbeg(State S) {
  const int nact = S.cnt->n_act;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nact; i += gridDim.x * blockDim.x)
    S.nbeg[S.act[i]] = S.scan[i];
}

// Every point moves to its cluster's new contiguous range: merged clusters
// are the lower-ID child's points followed by the other child's.
__global__ void k_move_points(State S) {
  const int n = S.n, d = S.d;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    const int s = S.powner[p];
    const int a = S.mdst[s];
    const int dst = S.nbeg[a] + S.moff[s] + (p - S.cbeg[s]);
    if (dst < 0 || dst >= n) {  // layout inconsistency: report, never write out of range
      S.cnt->nonfinite = 3;
      continue;
    }
    for (int k = 0; k < d; ++k) S.px2[(size_t)dst * d + k] = S.px[(size_t)p * d + k];
    S.powner2[dst] = a;
  }
}

__global__ void k_copy_beg(State S) {
  const int nact = S.cnt->n_act;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nact; i += gridDim.x * blockDim.x) {
    const int s = S.act[i];
    S.cbeg[s] = S.nbeg[s];
  }
}

__global__ void k_swap_count(Counters *c, int *total_slot) { c->n_act = *total_slot; }

// --------------------------------------------------------------- finalize --
// (size, lowest point index): both below 2^lob, packed into 2 lob bits
__global__ void k_row_keys2(State S, int m, int lob) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  S.sk0[r] = ((unsigned long long)(unsigned)S.row_size[r] << lob) | (unsigned)S.row_lo[r];
  S.sv0[r] = (unsigned)r;
}
__global__ void k_row_keys1(State S, int m) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  S.sk0[i] = pos_bits(S.row_eff[S.sv0[i]]);
}
__global__ void k_newid(State S, int m) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  S.scan[S.sv0[i]] = S.n + i;
}
struct OutRow {
  long long a, b;
  double h;
  long long size;
};
__global__ void k_write_rows(State S, int m, OutRow *out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int r = S.sv0[i];
  const int n = S.n;
  int a = S.row_na[r], b = S.row_nb[r];
  a = a < n ? a : S.scan[a - n];
  b = b < n ? b : S.scan[b - n];
  OutRow o;
  o.a = a < b ? a : b;
  o.b = a < b ? b : a;
  o.h = S.row_h[r];
  o.size = S.row_size[r];
  out[i] = o;
}

inline int nblk(long long n, int cap = 4096) {
  long long b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (int)(b < cap ? b : cap);
}

inline void tmark(State &S, int k, bool end, hipStream_t s) {
  if (!S.timing) return;
  KTimer &t = *S.kt;
  int idx;
  if (t.take(idx) != hipSuccess) return;  // (no event: this launch goes untimed)
  (void)hipEventRecord(t.pool[idx], s);
  if (!end) {
    t.open[k] = idx;
  } else if (t.open[k] >= 0) {
    t.done.push_back(k);
    t.done.push_back(t.open[k]);
    t.done.push_back(idx);
    t.open[k] = -1;
  }
}

// the ring searches with or without the cache probes (centroid linkages
// never probe)
template <int LINK, int MAXD, int PASS>
void launch_grid(State &S, int tb, hipStream_t s, int *t_ovf) {
  if constexpr (!centroid_link(LINK)) {
    if (S.cache_mask) {
      k_nn_grid<LINK, MAXD, PASS, true><<<tb, kBlock, 0, s>>>(S, t_ovf);
      return;
    }
  }
  k_nn_grid<LINK, MAXD, PASS, false><<<tb, kBlock, 0, s>>>(S, t_ovf);
}
template <int LINK, int MAXD>
void launch_ringblk(State &S, int ob, hipStream_t s) {
  if constexpr (!centroid_link(LINK)) {
    if (S.cache_mask) {
      k_nn_ringblk<LINK, MAXD, true><<<ob, kBlock, 0, s>>>(S);
      return;
    }
  }
  k_nn_ringblk<LINK, MAXD, false><<<ob, kBlock, 0, s>>>(S);
}

// pass 0 of the ring search: a wavefront per terminal in rounds with few
// active clusters (no pair cache), else a thread per terminal
template <int LINK, int MAXD>
void launch_grid_p0(State &S, int nact, hipStream_t s, int *t_ovf) {
  if ((centroid_link(LINK) || !S.cache_mask) && nact <= S.wave_terms)
    k_nn_grid_wave<LINK, MAXD><<<nblk((long long)nact * kWave, 1 << 16), kBlock, 0, s>>>(S, t_ovf);
  else
    launch_grid<LINK, MAXD, 0>(S, nblk(nact, 1 << 20), s, t_ovf);
}

template <int LINK>
void launch_search(State &S, int nact, hipStream_t s, int *t_ovf) {
  const size_t sm = (size_t)S.d * (sizeof(double) + 2 * sizeof(float));
  if (S.d <= kGridMaxDim && S.prune) {
    tmark(S, 0, false, s);
    if (S.d <= 2) launch_grid_p0<LINK, 2>(S, nact, s, t_ovf);
    else if (S.d <= 4) launch_grid_p0<LINK, 4>(S, nact, s, t_ovf);
    else if (S.d <= 8) launch_grid_p0<LINK, 8>(S, nact, s, t_ovf);
    else launch_grid_p0<LINK, 16>(S, nact, s, t_ovf);
    tmark(S, 0, true, s);
    tmark(S, 1, false, s);
    const int ob = nblk((long long)nact * kBlock, 2048);
    if (S.d <= 2) launch_ringblk<LINK, 2>(S, ob, s);
    else if (S.d <= 4) launch_ringblk<LINK, 4>(S, ob, s);
    else if (S.d <= 8) launch_ringblk<LINK, 8>(S, ob, s);
    else launch_ringblk<LINK, 16>(S, ob, s);
    tmark(S, 1, true, s);
  } else {
    tmark(S, 1, false, s);
    k_nn_full<LINK><<<nblk((long long)nact * kBlock, 2048), kBlock, sm, s>>>(S, nullptr, nullptr);
    tmark(S, 1, true, s);
  }
}

// box tree: items in active-list order, the node boxes level by level, the
// search, then the full scan for any terminal it handed back
template <int LINK>
void launch_tree_search(State &S, int nact, hipStream_t s) {
  int cnt = (nact + kTreeFan - 1) / kTreeFan, off = 0, lev = 0;
  for (;;) {
    S.tree_cnt[lev] = cnt;
    S.tree_off[lev] = off;
    off += cnt;
    if (cnt == 1) break;
    cnt = (cnt + kTreeFan - 1) / kTreeFan;
    ++lev;
  }
  S.tree_top = lev;
  k_tree_items<<<nblk(nact, 1 << 20), kBlock, 0, s>>>(S);
  for (int l = 0; l <= S.tree_top; ++l) k_tree_level<<<nblk(S.tree_cnt[l], 1 << 20), kBlock, 0, s>>>(S, l);
  tmark(S, 0, false, s);
  if (S.d <= 4) k_nn_tree<LINK, 4><<<nblk(nact, 1 << 20), kBlock, 0, s>>>(S);
  else k_nn_tree<LINK, 8><<<nblk(nact, 1 << 20), kBlock, 0, s>>>(S);
  tmark(S, 0, true, s);
  tmark(S, 1, false, s);
  const size_t sm = (size_t)S.d * (sizeof(double) + 2 * sizeof(float));
  k_nn_full<LINK><<<256, kBlock, sm, s>>>(S, S.ovf, &S.cnt->n_ovf);
  tmark(S, 1, true, s);
}

template <int LINK>
void launch_emit(State &S, int nact, hipStream_t s, int *t_ovf) {
  // pass 1 of the ring search; the full-scan kernel already emitted its pairs
  if (S.d <= kGridMaxDim && S.prune) {
    const int tb = nblk(nact, 1 << 20);
    tmark(S, 3, false, s);
    if (S.d <= 2) launch_grid<LINK, 2, 1>(S, tb, s, t_ovf);
    else if (S.d <= 4) launch_grid<LINK, 4, 1>(S, tb, s, t_ovf);
    else if (S.d <= 8) launch_grid<LINK, 8, 1>(S, tb, s, t_ovf);
    else launch_grid<LINK, 16, 1>(S, tb, s, t_ovf);
    tmark(S, 3, true, s);
  }
}

template <int LINK, int KP, int E>
void launch_gram_kpe(State &S, int nact, hipStream_t s) {
  const int nb = S.tb1 - S.tb0;
  const int gx = (nb + kGT - 1) / kGT;
  int gy = 4096 / (gx > 0 ? gx : 1);
  const int maxy = (nact + kGT - 1) / kGT;
  gy = gy < 1 ? 1 : (gy > maxy ? maxy : gy);
  tmark(S, 0, false, s);
  k_gram<LINK, KP, 0, E><<<dim3(gx, gy), kBlock, 0, s>>>(S);
  tmark(S, 0, true, s);
  tmark(S, 3, false, s);
  k_gram<LINK, KP, 1, E><<<dim3(gx, gy), kBlock, 0, s>>>(S);
  tmark(S, 3, true, s);
}

template <int LINK, int KP>
void launch_gram_kp(State &S, int nact, hipStream_t s) {
  switch (S.elem) {
  case kElBF16: launch_gram_kpe<LINK, KP, kElBF16>(S, nact, s); break;
  case kElF32: launch_gram_kpe<LINK, KP, kElF32>(S, nact, s); break;
  default: launch_gram_kpe<LINK, KP, kElF16>(S, nact, s); break;
  }
}

template <int LINK, int KP, bool SETTLE>
void launch_cand_tiles(State &S, int ncand, hipStream_t s) {
  switch (S.elem) {
  case kElBF16: k_cand_tiles<LINK, KP, kElBF16, SETTLE><<<8192, kBlock, 0, s>>>(S, ncand); break;
  case kElF32: k_cand_tiles<LINK, KP, kElF32, SETTLE><<<8192, kBlock, 0, s>>>(S, ncand); break;
  default: k_cand_tiles<LINK, KP, kElF16, SETTLE><<<8192, kBlock, 0, s>>>(S, ncand); break;
  }
}

// Candidates of a batch: interval screening (complete/average), then exact
// values or claims.
template <int LINK>
void launch_gram_refine_t(State &S, int ncand, hipStream_t s) {
  if constexpr (!centroid_link(LINK)) {
    if (!S.p16 || ncand <= 0) goto exact;
    k_cand_triage<LINK><<<nblk(ncand, 4096), kBlock, 0, s>>>(S, ncand);
    k_cand_small<LINK><<<8192, kBlock, 0, s>>>(S);
    k_scr_count<<<1, 1, 0, s>>>(S.cnt);
    if (LINK == kComplete && S.d <= kBlkMaxDim) k_cand_seed<<<2048, kBlock, 0, s>>>(S);
    scan_exclusive_i64(S.cd_tile0, S.cd_tile0, ncand, &S.cnt->n_scr32, &S.cnt->n_ctiles, S.sws, s);
    tmark(S, 1, false, s);  // the interval tiles alone
    switch (S.pkp) {
    case 16: launch_cand_tiles<LINK, 16, false>(S, ncand, s); break;
    case 32: launch_cand_tiles<LINK, 32, false>(S, ncand, s); break;
    case 64: launch_cand_tiles<LINK, 64, false>(S, ncand, s); break;
    case 80: launch_cand_tiles<LINK, 80, false>(S, ncand, s); break;
    default: launch_cand_tiles<LINK, 128, false>(S, ncand, s); break;
    }
    tmark(S, 1, true, s);
    k_cand_bound<LINK><<<nblk(ncand, 4096), kBlock, 0, s>>>(S);
    if (LINK == kComplete && tiles_settle_complete(S.pkp, S.d)) {
      // the survivors' tiles again: exact keys of the pairs that may be the
      // farthest (counted with the exact pair tiles)
      k_settle_select<<<nblk(ncand, 4096), kBlock, 0, s>>>(S);
      tmark(S, 2, false, s);
      switch (S.pkp) {
      case 32: launch_cand_tiles<kComplete, 32, true>(S, ncand, s); break;
      case 64: launch_cand_tiles<kComplete, 64, true>(S, ncand, s); break;
      case 80: launch_cand_tiles<kComplete, 80, true>(S, ncand, s); break;
      default: launch_cand_tiles<kComplete, 128, true>(S, ncand, s); break;
      }
      tmark(S, 2, true, s);
      k_settle_finish<<<nblk(ncand, 4096), kBlock, 0, s>>>(S);
    }
  }
exact:
  tmark(S, 3, false, s);
  k_gram_exact<LINK><<<2048, kBlock, 0, s>>>(S);
  tmark(S, 3, true, s);
}

// once per round: FP16 centroids (the terminals are batched afterwards)
void launch_gram_setup(State &S, int nact, hipStream_t s) {
  k_gram_reset<<<1, kGramMaxDim, 0, s>>>(S);
  k_gram_range<<<nblk((long long)nact * kWave, 1024), kBlock, 0, s>>>(S);
  k_gram_setup<<<1, kGramMaxDim, 0, s>>>(S);
  const int gp = nblk((long long)nact * kWave, 4096), pp = nblk((long long)S.n * kWave, 4096);
  switch (S.elem) {
  case kElBF16:
    k_gram_prep<kElBF16><<<gp, kBlock, 0, s>>>(S);
    if (S.p16) k_pt_prep<kElBF16><<<pp, kBlock, 0, s>>>(S);
    break;
  case kElF32:
    k_gram_prep<kElF32><<<gp, kBlock, 0, s>>>(S);
    if (S.p16) k_pt_prep<kElF32><<<pp, kBlock, 0, s>>>(S);
    break;
  default:
    k_gram_prep<kElF16><<<gp, kBlock, 0, s>>>(S);
    if (S.p16) k_pt_prep<kElF16><<<pp, kBlock, 0, s>>>(S);
    break;
  }
  if (S.p16 && S.linkage == kComplete && S.d <= kBlkMaxDim)
    k_blk_boxes<<<nblk((S.n + 63) / 64, 4096), kBlock, 0, s>>>(S);
}

template <int LINK>
void launch_gram_batch_t(State &S, int nact, hipStream_t s) {
  k_reset_batch<<<1, 1, 0, s>>>(S.cnt);
  k_gram_init<LINK><<<nblk(S.tb1 - S.tb0, 2048), kBlock, 0, s>>>(S, S.cell_rank);
  switch (S.gkp) {
  case 16: launch_gram_kp<LINK, 16>(S, nact, s); break;
  case 32: launch_gram_kp<LINK, 32>(S, nact, s); break;
  case 64: launch_gram_kp<LINK, 64>(S, nact, s); break;
  case 80: launch_gram_kp<LINK, 80>(S, nact, s); break;
  case 128: launch_gram_kp<LINK, 128>(S, nact, s); break;
  default: launch_gram_kp<LINK, 144>(S, nact, s); break;
  }
}

}  // namespace

void launch_gram_keys(State &S, hipStream_t s) { k_gram_key<<<2048, kBlock, 0, s>>>(S); }

void launch_gram_refine(State &S, int ncand, hipStream_t s) {
  switch (S.linkage) {
  case kWard: launch_gram_refine_t<kWard>(S, ncand, s); break;
  case kAvgSq: launch_gram_refine_t<kAvgSq>(S, ncand, s); break;
  case kComplete: launch_gram_refine_t<kComplete>(S, ncand, s); break;
  default: launch_gram_refine_t<kAverage>(S, ncand, s); break;
  }
}

void launch_gram_batch(State &S, int nact, hipStream_t s) {
  switch (S.linkage) {
  case kWard: launch_gram_batch_t<kWard>(S, nact, s); break;
  case kAvgSq: launch_gram_batch_t<kAvgSq>(S, nact, s); break;
  case kComplete: launch_gram_batch_t<kComplete>(S, nact, s); break;
  default: launch_gram_batch_t<kAverage>(S, nact, s); break;
  }
}

void launch_cache_clear(State &S, unsigned long long *keys, unsigned long long *vals, unsigned long long mask,
                        hipStream_t s) {
  (void)S;
  k_cache_clear<<<nblk((long long)mask + 1, 8192), kBlock, 0, s>>>(keys, vals, mask);
}

void launch_cache_rebuild(State &S, const unsigned long long *okeys, const unsigned long long *ovals,
                          unsigned long long omask, hipStream_t s) {
  k_cache_rebuild<<<nblk((long long)omask + 1, 8192), kBlock, 0, s>>>(S, okeys, ovals, omask);
}

void launch_cache_unclaim(State &S, hipStream_t s) {
  if (S.cache_mask) k_cache_unclaim<<<nblk((long long)S.cache_mask + 1, 8192), kBlock, 0, s>>>(S);
}

hipError_t set_direction_table() {
  double t[2][kSupDirs];
  for (int k = 0; k < kSupDirs; ++k) {
    const double a = 2.0 * M_PI * (double)k / (double)kSupDirs;
    t[0][k] = cos(a);
    t[1][k] = sin(a);
  }
  return hipMemcpyToSymbol(HIP_SYMBOL(c_dir), t, sizeof(t));
}

void launch_check_finite(const float *x, long long count, Counters *cnt, hipStream_t s) {
  k_check_finite<<<nblk(count, 2048), kBlock, 0, s>>>(x, count, cnt);
}

void launch_init(State &S, const float *x, hipStream_t s) {
  const int n = S.n;
  // the box tree orders points over all (up to 8) axes, the grid over two
  const int axes = S.tree ? std::min(S.d, kMortonAxes) : (S.d >= 2 ? 2 : 1);
  const int key_bits = axes <= 2 ? 16 * axes : axes * (64 / axes);
  k_reset_round<<<1, 1, 0, s>>>(S.cnt);
  k_point_bbox<<<nblk(n, 1024), kBlock, 0, s>>>(x, n, S.d, axes, S.cnt);
  k_morton<<<nblk(n, 1 << 22), kBlock, 0, s>>>(x, n, S.d, axes, S.cnt, S.sk0, S.sv0);
  radix_sort_pairs(S.sk0, S.sk1, S.sv0, S.sv1, n, key_bits, S.hist, S.sws, s);
  k_init_slots<<<nblk(n, 1 << 22), kBlock, 0, s>>>(S, x, S.sv0);
  k_set_nact<<<1, 1, 0, s>>>(S.cnt, n);
  if (S.p16) {
    // point scaling of the interval tiles, fixed for the call
    k_gram_reset<<<1, kGramMaxDim, 0, s>>>(S);
    k_pt_range<<<nblk((long long)n * kWave, 1024), kBlock, 0, s>>>(x, n, S.d, S.gmin, S.gmax);
    k_pt_setup<<<1, kGramMaxDim, 0, s>>>(S);
  }
}

// First half of a round: terminals, grid, nearest-neighbour search (Ward
// complete; complete/average up to the emitted pair list and its tile prefix).
void launch_round(State &S, int round, int nact, hipStream_t s, bool &need_pairs) {
  const int gb = nblk(nact, 2048);
  S.single = 0;
  k_reset_round<<<1, 1, 0, s>>>(S.cnt);
  k_act_pass<<<gb, kBlock, 0, s>>>(S, round);
  scan_exclusive_i32(S.flags, S.scan, nact, &S.cnt->n_act, &S.cnt->n_term, S.sws, s);
  k_scatter_flagged<<<gb, kBlock, 0, s>>>(S.act, S.flags, S.scan, &S.cnt->n_act, S.term);
  // Few active clusters: a block per terminal scans all of them (every
  // candidate's bounds and values are those of the ring search, so the rows
  // are the same), which beats a thread walking grid rings in latency; the
  // grid is then not built.
  const bool full = S.full_scan_max > 0 && nact <= S.full_scan_max && round > 0 && S.d <= kGridMaxDim &&
                    S.prune && !S.gram && !S.tree;
  if (S.d <= kGridMaxDim && S.prune && !S.gram && !S.tree && !full) {
    k_grid_params<<<1, 1, 0, s>>>(S, S.cell_cap);
    k_zero_cells<<<nblk(nact + 1, 2048), kBlock, 0, s>>>(S);
    k_cell_count<<<gb, kBlock, 0, s>>>(S);
    // cells <= cell_cap; scan length ncell + 1 (the extra zero gives the total)
    scan_exclusive_i32(S.cell_cnt, S.cell_start, grid_cells_max(S.cell_cap, nact) + 1, &S.grid->ncell1, nullptr,
                       S.sws, s);
    k_cell_scatter<<<gb, kBlock, 0, s>>>(S);
  }
  int *t_ovf = S.cell_rank;  // per-terminal hand-off flags (cell ranks are no longer needed)
  need_pairs = false;
  if (S.gram) {
    // the host then runs the terminals in batches (launch_gram_batch)
    k_term_pos<<<gb, kBlock, 0, s>>>(S);
    launch_gram_setup(S, nact, s);
    need_pairs = !centroid_link(S.linkage);
    return;
  }
  if (S.tree) {
    k_term_pos<<<gb, kBlock, 0, s>>>(S);
    if (S.linkage == kWard) launch_tree_search<kWard>(S, nact, s);
    else launch_tree_search<kAvgSq>(S, nact, s);
    return;
  }
  if (full) {
    const size_t sm = (size_t)S.d * (sizeof(double) + 2 * sizeof(float));
    const int fb = nblk((long long)nact * kBlock, 2048);
    tmark(S, 1, false, s);
    switch (S.linkage) {
    case kWard: k_nn_full<kWard><<<fb, kBlock, sm, s>>>(S, nullptr, nullptr); break;
    case kAvgSq: k_nn_full<kAvgSq><<<fb, kBlock, sm, s>>>(S, nullptr, nullptr); break;
    case kComplete: k_nn_full<kComplete><<<fb, kBlock, sm, s>>>(S, nullptr, nullptr); break;
    default: k_nn_full<kAverage><<<fb, kBlock, sm, s>>>(S, nullptr, nullptr); break;
    }
    tmark(S, 1, true, s);
    need_pairs = !centroid_link(S.linkage);
    return;
  }
  // Round 0 of complete linkage: every cluster is one point, where the
  // complete key (largest squared point distance) is the squared distance and
  // so is the Ward key (weight 2*1*1/(1+1) = 1, exact), summed in the same
  // order with the same tie-break: Ward's lighter search gives the same
  // neighbours and values, and no pair needs evaluating.
  S.single = (round == 0 && S.linkage == kComplete && S.d <= kGridMaxDim && S.prune) ? 1 : 0;
  if (S.single) {
    launch_search<kWard>(S, nact, s, t_ovf);
    return;
  }
  switch (S.linkage) {
  case kWard: launch_search<kWard>(S, nact, s, t_ovf); break;
  case kAvgSq: launch_search<kAvgSq>(S, nact, s, t_ovf); break;
  case kComplete:
    launch_search<kComplete>(S, nact, s, t_ovf);
    if (S.d <= kGridMaxDim && S.prune) {
      tmark(S, 3, false, s);
      k_cand_emit<kComplete><<<2048, kBlock, 0, s>>>(S, t_ovf);
      tmark(S, 3, true, s);
    }
    need_pairs = true;
    break;
  default:
    launch_search<kAverage>(S, nact, s, t_ovf);
    if (S.d <= kGridMaxDim && S.prune) {
      tmark(S, 3, false, s);
      k_cand_emit<kAverage><<<2048, kBlock, 0, s>>>(S, t_ovf);
      tmark(S, 3, true, s);
    }
    need_pairs = true;
    break;
  }
}

// The record of large candidates overflowed: emit by re-walking the rings.
void launch_emit_fallback(State &S, int nact, hipStream_t s) {
  int *t_ovf = S.cell_rank;
  if (S.linkage == kComplete) launch_emit<kComplete>(S, nact, s, t_ovf);
  else if (S.linkage == kAverage) launch_emit<kAverage>(S, nact, s, t_ovf);
}

void launch_pairs_prefix(State &S, int npairs, hipStream_t s) {
  long long *tmp = S.pr_tile0;  // per-pair counts, then their exclusive prefix (in place)
  if (S.linkage == kComplete) {
    k_pair_prep_comp<<<nblk(npairs, 2048), kBlock, 0, s>>>(S, S.pr_cbase);
    scan_exclusive_i64(S.pr_cbase, S.pr_cbase, npairs, nullptr, &S.cnt->n_chunks, S.sws, s);
  } else {
    k_pair_tiles<<<nblk(npairs, 2048), kBlock, 0, s>>>(S, tmp);
    scan_exclusive_i64(tmp, S.pr_tile0, npairs, nullptr, &S.cnt->n_tiles, S.sws, s);
  }
}

// complete: `work` = filter chunks; average: `work` = tiles
void launch_pairs(State &S, int round, int npairs, long long work, hipStream_t s) {
  (void)round;
  if (npairs > 0) {
    if (S.linkage == kComplete) {
      k_filter_comp<<<(int)std::min<long long>(work, 1 << 20), kBlock, 0, s>>>(S, work);
      k_pair_tiles_f<<<nblk(npairs, 2048), kBlock, 0, s>>>(S, S.pr_tile0);
      scan_exclusive_i64(S.pr_tile0, S.pr_tile0, npairs, nullptr, &S.cnt->n_tiles, S.sws, s);
      tmark(S, 2, false, s);
      if (S.d <= 2) k_tiles_comp<2><<<2048, kBlock, 0, s>>>(S);
      else if (S.d <= 4) k_tiles_comp<4><<<2048, kBlock, 0, s>>>(S);
      else if (S.d <= 16) k_tiles_comp<16><<<2048, kBlock, 0, s>>>(S);
      else if (S.d <= kGramMaxDim) k_tiles_hd<kComplete><<<4096, kBlock, 0, s>>>(S);
      else k_tiles_comp<0><<<2048, kBlock, 0, s>>>(S);
      tmark(S, 2, true, s);
    } else {
      const long long ntiles = work;
      const int tb = (int)std::min<long long>((ntiles * kWave + kBlock - 1) / kBlock, 8192);
      tmark(S, 2, false, s);
      if (S.d <= 2) k_tiles_avg<2><<<tb, kBlock, 0, s>>>(S, ntiles);
      else if (S.d <= 4) k_tiles_avg<4><<<tb, kBlock, 0, s>>>(S, ntiles);
      else if (S.d <= kGramMaxDim) k_tiles_hd<kAverage><<<(int)std::min<long long>(ntiles, 8192), kBlock, 0, s>>>(S);
      else k_tiles_avg<0><<<tb, kBlock, 0, s>>>(S, ntiles);
      tmark(S, 2, true, s);
    }
    k_pair_finish<<<S.linkage == kComplete ? nblk(npairs, 2048) : nblk((long long)npairs * kWave, 4096), kBlock, 0,
                    s>>>(S, S.linkage);
  }
  if (S.cache_mask) k_pending_min<<<2048, kBlock, 0, s>>>(S);
  k_term_key_reset<<<nblk(S.n, 2048), kBlock, 0, s>>>(S);
  if (npairs > 0) k_pair_key<<<nblk(npairs, 2048), kBlock, 0, s>>>(S);
  if (S.cache_mask) k_pending_key<<<2048, kBlock, 0, s>>>(S);
  if (S.gram) k_gram_key<<<2048, kBlock, 0, s>>>(S);
}

// Second half of a round: chains, R-NN pairs, merges, compaction.
void launch_round_tail(State &S, int round, int nact, int merges_before, hipStream_t s) {
  const int gb = nblk(nact, 2048);
  k_chain<<<gb, kBlock, 0, s>>>(S);
  k_rnn_flags<<<gb, kBlock, 0, s>>>(S, round);
  scan_exclusive_i32(S.flags, S.scan, nact, &S.cnt->n_term, &S.cnt->n_merge, S.sws, s);
  k_rnn_scatter<<<gb, kBlock, 0, s>>>(S);
  k_merge<<<nblk(nact / 2 + 1, 2048), kBlock, 0, s>>>(S, merges_before);
  if (S.linkage == kComplete && S.d == 2)
    k_merge_sup<<<nblk((long long)(nact / 2 + 1) * kSupDirs, 8192), kBlock, 0, s>>>(S);
  if (S.phases) (void)hipEventRecord(S.rev[2], s);
  k_alive_flags<<<gb, kBlock, 0, s>>>(S);
  int *total = S.scan + S.n;  // one spare int past the scan array
  scan_exclusive_i32(S.flags, S.scan, nact, &S.cnt->n_act, total, S.sws, s);
  k_scatter_flagged<<<gb, kBlock, 0, s>>>(S.act, S.flags, S.scan, &S.cnt->n_act, S.act2);
  k_swap_count<<<1, 1, 0, s>>>(S.cnt, total);
  std::swap(S.act, S.act2);
  if (!centroid_link(S.linkage)) {
    k_sizes_of_act<<<gb, kBlock, 0, s>>>(S);
    scan_exclusive_i32(S.flags, S.scan, nact, &S.cnt->n_act, nullptr, S.sws, s);
    k_set_nbeg<<<gb, kBlock, 0, s>>>(S);
    k_move_points<<<nblk(S.n, 4096), kBlock, 0, s>>>(S);
    k_copy_beg<<<gb, kBlock, 0, s>>>(S);
    std::swap(S.px, S.px2);
    std::swap(S.powner, S.powner2);
  }
}

void launch_finalize(State &S, void *out_rows, hipStream_t s) {
  const int m = S.n - 1;
  if (m <= 0) return;
  const int b = nblk(m, 1 << 22);
  // sizes and point indices are at most n: the key needs 2 lob bits only
  int lob = 1;
  while ((1LL << lob) <= (long long)S.n) ++lob;
  k_row_keys2<<<b, kBlock, 0, s>>>(S, m, lob);
  radix_sort_pairs(S.sk0, S.sk1, S.sv0, S.sv1, m, 2 * lob, S.hist, S.sws, s);
  k_row_keys1<<<b, kBlock, 0, s>>>(S, m);
  radix_sort_pairs(S.sk0, S.sk1, S.sv0, S.sv1, m, 64, S.hist, S.sws, s);
  k_newid<<<b, kBlock, 0, s>>>(S, m);
  k_write_rows<<<b, kBlock, 0, s>>>(S, m, (OutRow *)out_rows);
}

}  // namespace pc
