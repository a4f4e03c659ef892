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

constexpr int kCellBudget = 160;        // cells a thread may visit before handing off
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
  c->n_pairs = 0;
  c->pair_overflow = 0;
  c->n_min = 0x7fffffff;
  c->bb_lo[0] = c->bb_lo[1] = ~0ull;
  c->bb_hi[0] = c->bb_hi[1] = 0ull;
  c->n_tiles = 0;
}

__global__ void k_check_finite(const float *x, long long count, Counters *c) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) c->nonfinite = 1;
}

__global__ void k_point_bbox(const float *x, int n, int d, int axes, Counters *c) {
  unsigned long long lo[2] = {~0ull, ~0ull}, hi[2] = {0ull, 0ull};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    for (int a = 0; a < axes; ++a) {
      unsigned long long b = ordered_bits((double)x[(size_t)i * d + a]);
      lo[a] = b < lo[a] ? b : lo[a];
      hi[a] = b > hi[a] ? b : hi[a];
    }
  for (int a = 0; a < 2; ++a) {
    unsigned long long l = block_reduce<unsigned long long, true>(lo[a]);
    unsigned long long h = block_reduce<unsigned long long, false>(hi[a]);
    if (threadIdx.x == 0 && a < axes) {
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

// Morton (Z-order) code of the first one or two coordinates: spatially close
// clusters get close slots, so one wavefront's terminals search nearby cells.
__global__ void k_morton(const float *x, int n, int d, int axes, const Counters *c,
                         unsigned long long *key, unsigned *val) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned q[2] = {0, 0};
  for (int a = 0; a < axes; ++a) {
    double lo = from_ordered_bits(c->bb_lo[a]), hi = from_ordered_bits(c->bb_hi[a]);
    double t = hi > lo ? ((double)x[(size_t)i * d + a] - lo) / (hi - lo) : 0.0;
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    q[a] = (unsigned)(t * 65535.0);
  }
  key[i] = axes == 2 ? (unsigned long long)(spread16(q[0]) | (spread16(q[1]) << 1)) : q[0];
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
  if (S.linkage != kWard) {
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
    if (g0 * g1 <= (double)cell_cap) {
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
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) S.cell_cnt[i] = 0;
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
  }
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
    S.item_meta[pos] = make_int4(s, S.csize[s], S.cid[s], 0);
    for (int k = 0; k < d; ++k) S.item_cen[(size_t)pos * d + k] = S.wcen[(size_t)s * d + k];
    if (S.linkage != kWard)
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

// Exact complete (largest squared distance) or average (mean distance) value
// of a small pair, rows = the cluster with the lower ID.
template <int LINK>
__device__ double pair_exact_inline(const float *px, int d, int begR, int nR, int begS, int nS) {
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
//     max(hiC-loT, hiT-loC)) -- every per-axis extent is attained by a real
//     point pair; UB = squared max distance between the boxes.
//   average: LB = max(centroid distance (Sec. 4.2), min box distance);
//     UB = max box distance.
template <int LINK, int MAXD>
__device__ __forceinline__ void pair_bounds(const double *ct, const float *lt, const float *ht, const double *cc,
                                            const float *lc, const float *hc, int d, double &lb, double &ub) {
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
    ub = maxd;
  } else {
    double c1 = sqrt(cdist), m1 = sqrt(mind);
    lb = c1 > m1 ? c1 : m1;
    ub = sqrt(maxd);
  }
}

// Stop rule of the ring search: a lower bound on the key of any cluster whose
// centroid lies at least `D` away from the terminal's centroid.
template <int LINK>
__device__ __forceinline__ double ring_key_lb(double D, double nt, double nmin) {
  if (LINK == kWard) return D * D * ((2.0 * nt * nmin) / (nt + nmin));  // Sec. 4.1 radius
  if (LINK == kComplete) return D * D;  // Sec. 4.3: centroid distance <= complete distance
  return D;                             // Sec. 4.2: centroid distance <= average distance
}

// Initial search bound from the predecessor distance (Alg. 2), in key units.
template <int LINK>
__device__ __forceinline__ double beta_key(unsigned predbits) {
  if (predbits >= kInfBits) return INFINITY;
  double b = (double)__uint_as_float(predbits);
  if (LINK == kAverage) return b * kSlack;
  return b * b * kSlack;
}

__device__ __forceinline__ double key_to_height(int link, double v) { return link == kAverage ? v : sqrt(v); }

// ------------------------------------------------------ ring search kernel --
// One thread per terminal. PASS 0: Ward (final result) or, for complete and
// average, the search bound plus the best inline-evaluated candidate. PASS 1
// (complete/average): re-walk the rings under the final bound and emit the
// large pairs whose lower bound does not exceed it.
template <int LINK, int MAXD, int PASS>
__global__ __launch_bounds__(kBlock) void k_nn_grid(State S, int *t_ovf) {
  const int nterm = S.cnt->n_term;
  const int ti = blockIdx.x * blockDim.x + threadIdx.x;
  long long evals = 0, ppairs = 0;
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
      if (LINK != kWard) {
        lt[k] = k < d ? S.lo[(size_t)t * d + k] : 0.f;
        ht[k] = k < d ? S.hi[(size_t)t * d + k] : 0.f;
      }
    }
    const int beg_t = LINK != kWard ? S.cbeg[t] : 0;
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
          const double D = ((double)(k - 1) + m) * g.h * (1.0 - 1e-9);
          const double lbk = ring_key_lb<LINK>(D, nt, nmin);
          const double cur = PASS == 0 ? fmin(bound, bestv) : bound;
          if (lbk > cur) break;
        }
        visited += k == 0 ? 1 : 8 * k;
        if (PASS == 0 && visited > kCellBudget) {
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
            for (int it = a; it < b; ++it) {
              const int4 mt = S.item_meta[it];
              const int s = mt.x;
              if (s == t) continue;
              const double *cc = S.item_cen + (size_t)it * d;
              const unsigned long long key = make_key(mt.z, s);
              if (LINK == kWard) {
                double cv[MAXD];
#pragma unroll
                for (int q = 0; q < MAXD; ++q) cv[q] = q < d ? cc[q] : 0.0;
                const double v = ward_key<MAXD>(ct, nt, cv, (double)mt.y, d);
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
                pair_bounds<LINK, MAXD>(ct, lt, ht, cv, lc, hc, d, lb, ub);
                const double cur = PASS == 0 ? fmin(bound, bestv) : bound;
                if (lb > cur * kSlack) continue;
                const long long cost = (long long)n_t * (long long)mt.y;
                if (cost <= kInlinePairs) {
                  if (PASS == 0) {
                    const int beg_c = S.cbeg[s];
                    const double v = (mt.z < cid_t)
                                         ? pair_exact_inline<LINK>(S.px, d, beg_c, mt.y, beg_t, n_t)
                                         : pair_exact_inline<LINK>(S.px, d, beg_t, n_t, beg_c, mt.y);
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
                  const int p = atomicAdd(&S.cnt->n_pairs, 1);
                  if (p < S.pair_cap) {
                    S.pr_t[p] = ti;
                    S.pr_c[p] = s;
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
          if (LINK == kWard && bestk == kNoKey) {
            // the predecessor bound was not met (cannot happen for an exact
            // bound); hand the terminal to the full scan without a bound
            t_ovf[ti] = 1;
            const int o = atomicAdd(&S.cnt->n_ovf, 1);
            S.ovf[o] = ti;
          } else {
            S.t_best[ti] = bestv;
            S.t_key[ti] = bestk;
            if (LINK != kWard) {
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
  long long evals = 0, ppairs = 0;
  for (int q = blockIdx.x; q < count; q += gridDim.x) {
    const int ti = list ? list[q] : q;
    const int t = S.term[ti];
    const int cid_t = S.cid[t];
    const int n_t = S.csize[t];
    const double nt = (double)n_t;
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
      ct[k] = S.wcen[(size_t)t * d + k];
      if (LINK != kWard) {
        lt[k] = S.lo[(size_t)t * d + k];
        ht[k] = S.hi[(size_t)t * d + k];
      }
    }
    __syncthreads();
    const int beg_t = LINK != kWard ? S.cbeg[t] : 0;
    double bound = S.prune ? beta_key<LINK>(S.predd[t]) : INFINITY;
    double bestv = INFINITY;
    unsigned long long bestk = kNoKey;
    for (int i = threadIdx.x; i < nact; i += blockDim.x) {
      const int s = S.act[i];
      if (s == t) continue;
      const unsigned long long key = make_key(S.cid[s], s);
      const int n_c = S.csize[s];
      const double *cc = S.wcen + (size_t)s * d;
      if (LINK == kWard) {
        // a full scan needs no bound for Ward: every candidate is evaluated
        const double v = ward_key<0>(ct, nt, cc, (double)n_c, d);
        ++evals;
        if (better(v, key, bestv, bestk)) {
          bestv = v;
          bestk = key;
        }
      } else {
        double lb, ub;
        pair_bounds<LINK, 0>(ct, lt, ht, cc, S.lo + (size_t)s * d, S.hi + (size_t)s * d, d, lb, ub);
        if (S.prune && lb > fmin(bound, bestv) * kSlack) continue;
        const long long cost = (long long)n_t * n_c;
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
      if (LINK != kWard) {
        S.t_beta[ti] = beta;
        S.t_min[ti] = pos_bits(bestv);
      }
    }
    if (LINK != kWard) {
      // emit the large pairs that the final bound does not exclude
      for (int i = threadIdx.x; i < nact; i += blockDim.x) {
        const int s = S.act[i];
        if (s == t) continue;
        const int n_c = S.csize[s];
        if ((long long)n_t * n_c <= kInlinePairs) continue;
        if (S.prune) {
          double lb, ub;
          pair_bounds<LINK, 0>(ct, lt, ht, S.wcen + (size_t)s * d, S.lo + (size_t)s * d, S.hi + (size_t)s * d,
                               d, lb, ub);
          if (lb > beta * kSlack) continue;
        }
        const int p = atomicAdd(&S.cnt->n_pairs, 1);
        if (p < S.pair_cap) {
          S.pr_t[p] = ti;
          S.pr_c[p] = s;
        } else {
          S.cnt->pair_overflow = 1;
        }
      }
    }
    __syncthreads();
  }
  count_add(&S.cnt->cluster_evals, evals);
  count_add(&S.cnt->point_pairs, ppairs);
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

__global__ void k_pair_tiles(State S, long long *ntl) {
  const int np = S.cnt->n_pairs;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    int br, nr, bs, ns;
    pair_orient(S, p, br, nr, bs, ns);
    ntl[p] = (long long)((nr + kTile - 1) / kTile) * (long long)((ns + kTile - 1) / kTile);
    S.pr_v[p] = 0.0;
  }
}

// One wavefront per 64x64 tile: lane j owns column point j of the pair's S
// side and walks the tile's R rows (row points are wave-uniform loads).
template <int LINK, int MAXD>
__global__ __launch_bounds__(kBlock) void k_tiles(State S, long long ntiles) {
  const int np = S.cnt->n_pairs;
  const int lane = threadIdx.x & (kWave - 1);
  const long long wave0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) / kWave;
  const int d = S.d;
  long long ppairs = 0;
  for (long long gt = wave0; gt < ntiles; gt += nwaves) {
    // pair of this tile: last p with pr_tile0[p] <= gt
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (S.pr_tile0[mid] <= gt) lo = mid;
      else hi = mid - 1;
    }
    const int p = lo;
    int br, nr, bs, ns;
    pair_orient(S, p, br, nr, bs, ns);
    const long long local = gt - S.pr_tile0[p];
    const int ntc = (ns + kTile - 1) / kTile;
    const int rt = (int)(local / ntc), ctl = (int)(local % ntc);
    const int r0 = rt * kTile, r1 = min(nr, r0 + kTile);
    const int col = ctl * kTile + lane;
    const bool valid = col < ns;
    double acc = 0.0;
    if (valid) {
      const float *pc = S.px + (size_t)(bs + col) * d;
      if (MAXD > 0) {
        double cv[MAXD > 0 ? MAXD : 1];
#pragma unroll
        for (int k = 0; k < MAXD; ++k) cv[k] = k < d ? (double)pc[k] : 0.0;
        for (int r = r0; r < r1; ++r) {
          const float *pr = S.px + (size_t)(br + r) * d;
          double q = 0.0;
#pragma unroll
          for (int k = 0; k < MAXD; ++k)
            if (k < d) {
              double t = (double)pr[k] - cv[k];
              q += t * t;
            }
          if (LINK == kComplete) acc = q > acc ? q : acc;
          else acc += sqrt(q);
        }
      } else {
        for (int r = r0; r < r1; ++r) {
          const float *pr = S.px + (size_t)(br + r) * d;
          double q = 0.0;
          for (int k = 0; k < d; ++k) {
            double t = (double)pr[k] - (double)pc[k];
            q += t * t;
          }
          if (LINK == kComplete) acc = q > acc ? q : acc;
          else acc += sqrt(q);
        }
      }
      ppairs += r1 - r0;
    }
    if (LINK == kComplete) {
      acc = wave_max(acc);
      if (lane == 0) atomicMax((unsigned long long *)&S.pr_v[p], pos_bits(acc));
    } else {
      acc = wave_sum(acc);
      if (lane == 0) S.tile_v[gt] = acc;
    }
  }
  count_add(&S.cnt->point_pairs, ppairs);
}

// Per pair: finish the value, then WriteMin into its terminal's best value.
__global__ __launch_bounds__(kBlock) void k_pair_finish(State S, int link) {
  const int np = S.cnt->n_pairs;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave0 = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nwaves = (gridDim.x * blockDim.x) / kWave;
  long long evals = 0;
  for (int p = wave0; p < np; p += nwaves) {
    double v;
    if (link == kComplete) {
      v = S.pr_v[p];
    } else {
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
    }
  }
  count_add(&S.cnt->cluster_evals, evals);
}

__global__ void k_term_key_reset(State S) {
  const int nterm = S.cnt->n_term;
  for (int ti = blockIdx.x * blockDim.x + threadIdx.x; ti < nterm; ti += gridDim.x * blockDim.x)
    if (pos_bits(S.t_best[ti]) != S.t_min[ti]) S.t_key[ti] = kNoKey;
}

__global__ void k_pair_key(State S) {
  const int np = S.cnt->n_pairs;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    const int ti = S.pr_t[p];
    if (pos_bits(S.pr_v[p]) == S.t_min[ti]) {
      const int c = S.pr_c[p];
      atomicMin(&S.t_key[ti], make_key(S.cid[c], c));
    }
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
    const double v = S.linkage == kWard ? S.t_best[ti] : pos_from_bits(S.t_min[ti]);
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
    for (int k = 0; k < d; ++k) {
      const double sum = S.wsum[(size_t)a * d + k] + S.wsum[(size_t)b * d + k];
      S.wsum[(size_t)a * d + k] = sum;
      S.wcen[(size_t)a * d + k] = sum / (double)ns;
    }
    if (S.linkage != kWard) {
      for (int k = 0; k < d; ++k) {
        S.lo[(size_t)a * d + k] = fminf(S.lo[(size_t)a * d + k], S.lo[(size_t)b * d + k]);
        S.hi[(size_t)a * d + k] = fmaxf(S.hi[(size_t)a * d + k], S.hi[(size_t)b * d + k]);
      }
      S.mdst[b] = a;
      S.moff[b] = sa;
    }
    S.node[a] = n + r;
    S.succ[a] = -1;
    S.succ_node[a] = -1;
    S.predd[a] = kInfBits;
    S.alive[b] = 0;
    S.succ[b] = -1;
    S.node[b] = -1;
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
__global__ void k_row_keys2(State S, int m) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  S.sk0[r] = ((unsigned long long)(unsigned)S.row_size[r] << 32) | (unsigned)S.row_lo[r];
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
  hipEventRecord(S.tev[2 * k + (end ? 1 : 0)], s);
  if (end) S.tlaunched[k] = 1;
}

template <int LINK>
void launch_search(State &S, int nact, hipStream_t s, int *t_ovf) {
  const int tb = nblk(nact, 1 << 20);
  const size_t sm = (size_t)S.d * (sizeof(double) + 2 * sizeof(float));
  if (S.d <= kGridMaxDim && S.prune) {
    tmark(S, 0, false, s);
    if (S.d <= 2) k_nn_grid<LINK, 2, 0><<<tb, kBlock, 0, s>>>(S, t_ovf);
    else if (S.d <= 4) k_nn_grid<LINK, 4, 0><<<tb, kBlock, 0, s>>>(S, t_ovf);
    else if (S.d <= 8) k_nn_grid<LINK, 8, 0><<<tb, kBlock, 0, s>>>(S, t_ovf);
    else k_nn_grid<LINK, 16, 0><<<tb, kBlock, 0, s>>>(S, t_ovf);
    tmark(S, 0, true, s);
    tmark(S, 1, false, s);
    k_nn_full<LINK><<<nblk((long long)nact * kBlock, 2048), kBlock, sm, s>>>(S, S.ovf, &S.cnt->n_ovf);
    tmark(S, 1, true, s);
  } else {
    tmark(S, 1, false, s);
    k_nn_full<LINK><<<nblk((long long)nact * kBlock, 2048), kBlock, sm, s>>>(S, nullptr, nullptr);
    tmark(S, 1, true, s);
  }
}

template <int LINK>
void launch_emit(State &S, int nact, hipStream_t s, int *t_ovf) {
  // pass 1 of the ring search; the full-scan kernel already emitted its pairs
  if (S.d <= kGridMaxDim && S.prune) {
    const int tb = nblk(nact, 1 << 20);
    if (S.d <= 2) k_nn_grid<LINK, 2, 1><<<tb, kBlock, 0, s>>>(S, t_ovf);
    else if (S.d <= 4) k_nn_grid<LINK, 4, 1><<<tb, kBlock, 0, s>>>(S, t_ovf);
    else if (S.d <= 8) k_nn_grid<LINK, 8, 1><<<tb, kBlock, 0, s>>>(S, t_ovf);
    else k_nn_grid<LINK, 16, 1><<<tb, kBlock, 0, s>>>(S, t_ovf);
  }
}

}  // namespace

void launch_check_finite(const float *x, long long count, Counters *cnt, hipStream_t s) {
  k_check_finite<<<nblk(count, 2048), kBlock, 0, s>>>(x, count, cnt);
}

void launch_init(State &S, const float *x, hipStream_t s) {
  const int n = S.n;
  const int axes = S.d >= 2 ? 2 : 1;
  k_reset_round<<<1, 1, 0, s>>>(S.cnt);
  k_point_bbox<<<nblk(n, 1024), kBlock, 0, s>>>(x, n, S.d, axes, S.cnt);
  k_morton<<<nblk(n, 1 << 22), kBlock, 0, s>>>(x, n, S.d, axes, S.cnt, S.sk0, S.sv0);
  radix_sort_pairs(S.sk0, S.sk1, S.sv0, S.sv1, n, axes == 2 ? 32 : 16, S.hist, S.part, s);
  k_init_slots<<<nblk(n, 1 << 22), kBlock, 0, s>>>(S, x, S.sv0);
  k_set_nact<<<1, 1, 0, s>>>(S.cnt, n);
}

// First half of a round: terminals, grid, nearest-neighbour search (Ward
// complete; complete/average up to the emitted pair list and its tile prefix).
void launch_round(State &S, int round, int nact, hipStream_t s, bool &need_pairs) {
  const int gb = nblk(nact, 2048);
  k_reset_round<<<1, 1, 0, s>>>(S.cnt);
  k_act_pass<<<gb, kBlock, 0, s>>>(S, round);
  scan_exclusive_i32(S.flags, S.scan, nact, &S.cnt->n_act, &S.cnt->n_term, S.part, s);
  k_scatter_flagged<<<gb, kBlock, 0, s>>>(S.act, S.flags, S.scan, &S.cnt->n_act, S.term);
  if (S.d <= kGridMaxDim && S.prune) {
    k_grid_params<<<1, 1, 0, s>>>(S, S.cell_cap);
    k_zero_cells<<<nblk(nact + 1, 2048), kBlock, 0, s>>>(S);
    k_cell_count<<<gb, kBlock, 0, s>>>(S);
    // cells <= cell_cap; scan length ncell + 1 (the extra zero gives the total)
    scan_exclusive_i32(S.cell_cnt, S.cell_start, S.cell_cap + 1, &S.grid->ncell1, nullptr, S.part, s);
    k_cell_scatter<<<gb, kBlock, 0, s>>>(S);
  }
  int *t_ovf = S.cell_rank;  // per-terminal hand-off flags (cell ranks are no longer needed)
  need_pairs = false;
  switch (S.linkage) {
  case kWard: launch_search<kWard>(S, nact, s, t_ovf); break;
  case kComplete: launch_search<kComplete>(S, nact, s, t_ovf); launch_emit<kComplete>(S, nact, s, t_ovf); need_pairs = true; break;
  default: launch_search<kAverage>(S, nact, s, t_ovf); launch_emit<kAverage>(S, nact, s, t_ovf); need_pairs = true; break;
  }
}

void launch_pairs_prefix(State &S, int npairs, hipStream_t s) {
  long long *ntl = (long long *)S.pr_tile0;
  // per-pair tile counts, then their exclusive prefix (in place)
  k_pair_tiles<<<nblk(npairs, 2048), kBlock, 0, s>>>(S, ntl);
  scan_exclusive_i64(ntl, S.pr_tile0, npairs, &S.cnt->n_pairs, &S.cnt->n_tiles, S.part, s);
}

void launch_pairs(State &S, int round, int npairs, long long ntiles, hipStream_t s) {
  (void)round;
  if (npairs > 0) {
    const int tb = (int)std::min<long long>((ntiles * kWave + kBlock - 1) / kBlock, 8192);
    tmark(S, 2, false, s);
    if (S.linkage == kComplete) {
      if (S.d <= 2) k_tiles<kComplete, 2><<<tb, kBlock, 0, s>>>(S, ntiles);
      else if (S.d <= 4) k_tiles<kComplete, 4><<<tb, kBlock, 0, s>>>(S, ntiles);
      else if (S.d <= 16) k_tiles<kComplete, 16><<<tb, kBlock, 0, s>>>(S, ntiles);
      else k_tiles<kComplete, 0><<<tb, kBlock, 0, s>>>(S, ntiles);
    } else {
      if (S.d <= 2) k_tiles<kAverage, 2><<<tb, kBlock, 0, s>>>(S, ntiles);
      else if (S.d <= 4) k_tiles<kAverage, 4><<<tb, kBlock, 0, s>>>(S, ntiles);
      else if (S.d <= 16) k_tiles<kAverage, 16><<<tb, kBlock, 0, s>>>(S, ntiles);
      else k_tiles<kAverage, 0><<<tb, kBlock, 0, s>>>(S, ntiles);
    }
    tmark(S, 2, true, s);
    k_pair_finish<<<nblk((long long)npairs * kWave, 4096), kBlock, 0, s>>>(S, S.linkage);
  }
  k_term_key_reset<<<nblk(S.n, 2048), kBlock, 0, s>>>(S);
  if (npairs > 0) k_pair_key<<<nblk(npairs, 2048), kBlock, 0, s>>>(S);
}

// Second half of a round: chains, R-NN pairs, merges, compaction.
void launch_round_tail(State &S, int round, int nact, int merges_before, hipStream_t s) {
  const int gb = nblk(nact, 2048);
  k_chain<<<gb, kBlock, 0, s>>>(S);
  k_rnn_flags<<<gb, kBlock, 0, s>>>(S, round);
  scan_exclusive_i32(S.flags, S.scan, nact, &S.cnt->n_term, &S.cnt->n_merge, S.part, s);
  k_rnn_scatter<<<gb, kBlock, 0, s>>>(S);
  k_merge<<<nblk(nact / 2 + 1, 2048), kBlock, 0, s>>>(S, merges_before);
  k_alive_flags<<<gb, kBlock, 0, s>>>(S);
  int *total = S.scan + S.n;  // one spare int past the scan array
  scan_exclusive_i32(S.flags, S.scan, nact, &S.cnt->n_act, total, S.part, s);
  k_scatter_flagged<<<gb, kBlock, 0, s>>>(S.act, S.flags, S.scan, &S.cnt->n_act, S.act2);
  k_swap_count<<<1, 1, 0, s>>>(S.cnt, total);
  std::swap(S.act, S.act2);
  if (S.linkage != kWard) {
    k_sizes_of_act<<<gb, kBlock, 0, s>>>(S);
    scan_exclusive_i32(S.flags, S.scan, nact, &S.cnt->n_act, nullptr, S.part, s);
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
  k_row_keys2<<<b, kBlock, 0, s>>>(S, m);
  radix_sort_pairs(S.sk0, S.sk1, S.sv0, S.sv1, m, 64, S.hist, S.part, s);
  k_row_keys1<<<b, kBlock, 0, s>>>(S, m);
  radix_sort_pairs(S.sk0, S.sk1, S.sv0, S.sv1, m, 64, S.hist, S.part, s);
  k_newid<<<b, kBlock, 0, s>>>(S, m);
  k_write_rows<<<b, kBlock, 0, s>>>(S, m, (OutRow *)out_rows);
}

}  // namespace pc
