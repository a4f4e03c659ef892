// Shared declarations of libparchain: device helpers, the per-call device
// state, and the launch wrappers each translation unit exports to the host
// driver. gfx950 only (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace pc {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kMaxDim = 2048;      // largest d accepted (full-scan kernel stages d coords in LDS)
constexpr int kGridMaxDim = 16;    // ring search over a centroid grid up to this d
constexpr int kInlinePairs = 64;   // |t|*|C| at or below this: evaluated inside the search
constexpr int kTile = 64;          // point-pair tile edge for deferred evaluations
constexpr int kChunk = 256;        // points per filter block (complete linkage)
constexpr int kExtMaxDim = 8;      // extreme-point bounds kept up to this d
constexpr int kBlkMaxDim = 16;     // complete: 64-point block boxes prune interval tiles up to this d
constexpr int kSupDirs = 64;       // d == 2, complete: support points in 64 fixed directions
constexpr int kGramMinDim = 4;     // Gram (MFMA) search from this d on
constexpr int kGramMaxDim = 128;   // largest d of the Gram search (K = 128 in LDS)
constexpr int kTreeMaxDim = 8;     // Ward / avg-2: box-tree search over Morton-ordered centroids up to this d
constexpr int kMortonAxes = 8;     // at most this many axes in the initial Morton order
// MFMA depth of the Gram tiles: the dimension plus two augmented
// coordinates (the norm terms of the bound pass), in steps of 16
inline int gram_kp(int d) {
  if (d + 2 <= 16) return 16;
  if (d + 2 <= 32) return 32;
  if (d + 2 <= 64) return 64;
  if (d + 2 <= 80) return 80;
  if (d + 2 <= 128) return 128;
  return 144;
}
// MFMA depth of the point tiles of the interval screening: the dimension
// alone (their norm terms are added outside the MFMA), in the same steps
inline int point_kp(int d) {
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  if (d <= 64) return 64;
  if (d <= 80) return 80;
  return 128;
}
constexpr uint32_t kInfBits = 0x7f800000u;
// complete linkage: the interval tiles settled no exact key for this candidate
constexpr unsigned long long kNoExact = ~0ull;
// complete linkage above these point depths: exact keys of the pairs that may
// be the farthest are taken inside the interval tiles (see k_cand_tiles)
__host__ __device__ inline bool tiles_settle_complete(int pkp, int d) { return !(pkp <= 32 && d <= kBlkMaxDim); }

// element type of the MFMA screening tiles (pc_options.precision)
enum ScreenElem { kElF16 = 0, kElBF16 = 1, kElF32 = 2 };
inline int screen_elem_bytes(int e) { return e == kElF32 ? 4 : 2; }

// avg-1 is the mean Euclidean distance, avg-2 the mean squared distance
enum Linkage { kComplete = 0, kAverage = 1, kWard = 2, kAvgSq = 3 };

// Ward and avg-2 values follow from centroids, sizes (and for avg-2 the
// spreads) alone, in O(1) (Table 1); these linkages keep no points.
__host__ __device__ constexpr bool centroid_link(int l) { return l == kWard || l == kAvgSq; }

// ---------------------------------------------------------------- helpers --
// Reserve one slot of a 64-bit append counter; returns the slot index.

__device__ __forceinline__ unsigned long long ordered_bits(double v) {
  // monotone map of doubles to unsigned 64-bit integers (for atomic min/max)
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ordered_bits(unsigned long long b) {
  b = (b >> 63) ? (b & 0x7fffffffffffffffull) : ~b;
  return __longlong_as_double((long long)b);
}
// For non-negative doubles the raw IEEE bits already order like the values.
__device__ __forceinline__ unsigned long long pos_bits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}
__device__ __forceinline__ double pos_from_bits(unsigned long long b) {
  return __longlong_as_double((long long)b);
}
__device__ __forceinline__ unsigned long long lanemask_lt() {
  const int lane = threadIdx.x & (kWave - 1);
  return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}
// Next free index of an append-only list: one atomic per wavefront for all
// lanes that call it together (every caller passes the same counter).
__device__ __forceinline__ long long append_slot(long long *counter) {
  const unsigned long long m = __ballot(1);
  const int leader = __ffsll((unsigned long long)m) - 1;
  const int lane = threadIdx.x & (kWave - 1);
  long long base = 0;
  if (lane == leader) base = (long long)atomicAdd((unsigned long long *)counter, (unsigned long long)__popcll(m));
  base = __shfl(base, leader, kWave);
  return base + __popcll(m & lanemask_lt());
}

// --------------------------------------------------------- device state ----
// Grid over cluster centroids (first one or two coordinates), square cells.
struct GridParams {
  double org[2];
  double h;
  double inv_h;
  double eps;  // absolute slack for cell-boundary rounding
  int G[2];
  int ncell;
  int ncell1;  // ncell + 1 (scan length of the cell counts)
  int axes;
};

// Counters the device updates and the host reads once per round.
struct Counters {
  int n_act;
  int n_term;
  int n_merge;
  int n_ovf;
  int pair_overflow;
  int n_min;
  int nonfinite;
  int cand_overflow;
  // append counters are 64-bit: a round can propose more than 2^31 candidates,
  // and an index is only ever used after a 64-bit check against its capacity
  long long n_pairs;
  long long n_cand;
  long long n_pend;
  unsigned long long bb_lo[kMortonAxes];  // ordered bits of the per-axis range
  unsigned long long bb_hi[kMortonAxes];  // (points at init, active centroids per round)
  long long cluster_evals;
  long long point_pairs;
  long long n_tiles;
  long long n_chunks;
  long long visits[4];  // per timed search kernel
  long long cache_hits;
  long long cache_inserts;
  long long cache_fail;
  long long cache_derived;
  long long n_ctiles;  // interval tiles of the current batch
  long long n_small;   // small candidates of the current batch
  long long n_scr;     // screened candidates of the current batch
  int n_scr32;
  int scan_err;        // a prefix scan's look-back gave up (see ScanWs)
  long long refined;   // screened candidates given an exact FP64 value
};

// Workspace of the single-pass prefix scans (decoupled look-back): two status
// arrays taken in turn, each scan clearing the other one for the next scan
// (launches on one stream run in order), their two block tickets, and the
// error flag a look-back raises if it gives up (it never hangs).
struct ScanWs {
  unsigned long long *st[2];
  int *ticket;  // two ints, one per status array
  int cap;      // status words per array (one per 1024 scanned elements)
  int turn;     // host: the array the next scan uses
  int fresh;    // host: the arrays hold stale words (new memory): clear first
  int *err;     // device: Counters::scan_err
};

// Kernel timing (host side): every timed launch records a start and an end
// event from a pool the context keeps across calls; the elapsed times are
// read once, after the call's last synchronisation, so no round waits on
// them. Marks recorded since the last commit belong to an attempt that may
// be redone and are dropped with it.
struct KTimer {
  std::vector<hipEvent_t> pool;
  int next = 0;                      // next unused event of this call
  int open[4] = {-1, -1, -1, -1};    // start event of each slot's running launch
  std::vector<int> done;             // (slot, start, end) triples
  size_t kept = 0;                   // entries of `done` committed
  hipError_t take(int &idx) {
    if (next == (int)pool.size()) {
      // timing only, read after a stream synchronisation: no system-scope
      // fence (its cache writeback would slow the work that follows)
      hipEvent_t e;
      hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
      if (r != hipSuccess) return r;
      pool.push_back(e);
    }
    idx = next++;
    return hipSuccess;
  }
  void begin_call() {
    next = 0;
    done.clear();
    kept = 0;
    for (int &o : open) o = -1;
  }
  void commit() { kept = done.size(); }
  void drop() { done.resize(kept); }
};

// All device arrays of one clustering call. Slots are storage indices of
// clusters (capacity n); a merged cluster keeps the slot of its child with
// the lower cluster ID. Lists hold slots.
struct State {
  int n, d, linkage, prune;
  // per slot
  int *cid;        // cluster ID = lowest original point index
  int *csize;
  int *node;       // dendrogram node id (leaf: point index; merge k: n+k)
  int *succ;       // slot of the nearest neighbour, -1 if none
  int *succ_node;  // node id of that neighbour when it was found
  unsigned *predd; // float bits (rounded up) of the smallest distance from a predecessor
  int *term_round; // round in which the slot was last a terminal
  int *alive;
  int *mdst, *moff;  // where a slot's points go in the next layout
  int *cbeg, *nbeg;  // start of the cluster's point range (current / next)
  double *eff;     // largest height in the cluster's subtree
  double *nn_h;    // linkage distance to succ
  double *wsum;    // d coordinate sums per slot (FP64)
  double *wcen;    // d centroid coordinates per slot (wsum / csize)
  float *lo, *hi;  // d-dimensional bounding box per slot (complete, average)
  int *ext;        // complete: 2d original point indices attaining the box faces (lo_k, hi_k)
  double *crad;    // complete, average: upper bound of the largest centroid-to-point distance
  double *cvar;    // complete, average, avg-2: sum of squared deviations from the centroid (FP64)
  double *cmv;     // avg-2: cvar / size, the spread term of the linkage value
  int *sup;        // complete, d == 2: kSupDirs original point indices, the cluster's
                   // support point in direction (cos, sin)(2 pi k / kSupDirs)
  const float *xin;  // the caller's points (original order)
  // lists
  int *act, *act2, *term, *flags, *scan, *ovf;
  // grid over active centroids
  int *cell_cnt, *cell_start, *cell_of, *cell_rank;
  int *cell_nmin;  // smallest cluster size in each cell
  int *item_slot;
  int4 *item_meta;    // (slot, size, cid, 0)
  double *item_cen;   // d per item
  double *item_v;     // avg-2: the cluster's spread term (cmv)
  float *item_lo, *item_hi;
  // per terminal
  double *t_best;                 // value of the best inline candidate
  unsigned long long *t_key;      // (cid << 32 | slot) of the best candidate
  double *t_beta;                 // search bound (complete, average)
  unsigned long long *t_min;      // bits of the smallest value (complete, average)
  // merges
  int *m_a, *m_b;
  double *m_h;
  // rows, creation order
  int *row_na, *row_nb, *row_size, *row_lo;
  double *row_h, *row_eff;
  // points, permuted so that every cluster is a contiguous range
  float *px, *px2;
  int *powner, *powner2;
  // sort scratch
  unsigned long long *sk0, *sk1;
  unsigned *sv0, *sv1;
  int *hist;
  long long *part;  // scan workspace (growable with the pair list)
  long long part_cap;
  ScanWs sws;
  GridParams *grid;
  Counters *cnt;
  // deferred pair evaluations (growable, owned by the context)
  int *pr_t, *pr_c;
  double *pr_v;
  long long *pr_tile0;  // exclusive prefix of tiles per pair
  long long *pr_cbase;  // complete: exclusive prefix of 256-point filter chunks per pair
  int *pr_kR, *pr_kS;   // complete: points of each side kept by the filter
  int *fidx;            // complete: kept point positions, 256-aligned region per pair
  long long fidx_cap;
  // cluster-pair cache (Sec. 5): open addressing, key = (lower node << 32 | higher
  // node), value = the pair's key value (bits); cache_mask + 1 slots, 0 = off
  unsigned long long *ck, *cv;
  unsigned long long cache_mask;
  int *node2slot;       // node id -> slot (valid while the node is alive)
  int *pd_t, *pd_c;     // pairs whose value another terminal is computing this round,
  double *pd_v;         // or whose value was combined from cached parts (else -1)
  // large candidates recorded by the bound pass (terminal index, slot, lower bound)
  int *cd_t, *cd_c;
  double *cd_lb;
  double *cd_v;         // Gram search: exact value of a recorded candidate (NaN if deferred)
  long long cand_cap;
  // Gram search (d >= kGramMinDim): FP16 copies of the active centroids,
  // recentred on gorg and scaled by gscale, with FP64 norms of the rounded values
  int gram;             // 1: this call searches with MFMA Gram tiles
  int gkp;              // padded K of the centroid tiles (multiple of 16)
  int pkp;              // padded K of the point tiles (d rounded up to 16, 32, 64, 80, 128)
  int elem;             // ScreenElem: FP16 / BF16 / FP32 operands of the screening tiles
  _Float16 *g16;        // n x gkp elements of that type, in active-list order
  float4 *gq;  // per active item: pass-0 norm term, rigorous norm, rounding error, size/spread term
  // interval screening (complete/average): FP16 points in their current
  // places and their terms (|x~|^2, e, eta), the fixed point scaling, and the
  // candidates' tile prefix
  _Float16 *p16;        // n x gkp elements of the screening type
  float4 *pq;
  double *porg, *pscale;
  long long *cd_tile0;
  int *cd_small;  // small candidates (exact now)
  int4 *cd_desc;  // screened candidates (dense): row begin, rows, column begin, columns
  int *cd_scr;    // screened candidates (dense): candidate index
  double *cd_l0;  // screened candidates (dense), complete: a lower bound of the key fixed before the tiles
  unsigned long long *cd_x;  // screened candidates (dense), complete: bits of the largest exact point-pair key
                            // found by the tiles (kNoExact: the tiles did not settle the key)
  float *blk_lo, *blk_hi;  // complete, d <= kBlkMaxDim: box of each 64-position block of points (d each)
  int *nparent;  // node -> parent node (-1: none yet); kept when the cache is on
  double *gorg;         // d
  unsigned long long *gmin, *gmax;  // per-dimension ordered bits of the centroid range
  double *gscale;       // 1 value
  int *term_pos;        // active-list index of each terminal
  // box tree (Ward / avg-2, 3 <= d <= kTreeMaxDim): an implicit 16-ary tree
  // over the active list (leaves of 16 consecutive clusters); per node the FP64
  // box of the centroids below it, the smallest size and smallest spread term.
  // Level l holds tree_cnt[l] nodes from node tree_off[l]; level tree_top is the root.
  int tree;
  int tree_top;
  int tree_cnt[8], tree_off[8];
  double *tree_lo, *tree_hi;  // d per node
  int *tree_nmin;
  double *tree_vmin;
  int tb0, tb1;      // terminals [tb0, tb1) of the current Gram batch
  int cell_budget;  // grid cells a thread-per-terminal search visits before handing off
  int wave_terms;   // rounds with at most this many active clusters search a wavefront per terminal
  int wave_budget;  // grid cells a wavefront-per-terminal search visits before handing off
  int full_scan_max;  // rounds with at most this many active clusters scan them all (grid paths)
  int single;       // this round's clusters are all single points and the search wrote t_best
  double *tile_v;
  long long pair_cap, tile_cap;
  int cell_cap;
  // optional kernel timing: event pairs around ring search, full scan, tiles
  int timing;
  int phases;           // (host) also time the rounds by phase
  struct KTimer *kt;    // kernel event log (host), owned by the context
  hipEvent_t *rev;      // 4 events per round (start, search done, merge done, end)

};

// ------------------------------------------------------ launch wrappers ----
// primitives (pc_prims.hip)
// the scan workspace over `words` long longs at `base`
void scan_ws_carve(ScanWs &ws, long long *base, long long words, int *err);
void scan_exclusive_i32(const int *in, int *out, int nmax, const int *dlen, int *dtotal, ScanWs &ws,
                        hipStream_t s);
void scan_exclusive_i64(const long long *in, long long *out, int nmax, const int *dlen,
                        long long *dtotal, ScanWs &ws, hipStream_t s);
// stable radix sort of (key, value) pairs by the low `bits` bits of key
void radix_sort_pairs(unsigned long long *&k0, unsigned long long *&k1, unsigned *&v0,
                      unsigned *&v1, int n, int bits, int *hist, ScanWs &ws, hipStream_t s);
int radix_hist_len(int n);

// round kernels (pc_round.hip)
hipError_t set_direction_table();  // once per device, before the first call
void launch_check_finite(const float *x, long long count, Counters *cnt, hipStream_t s);
void launch_init(State &S, const float *x, hipStream_t s);
void launch_round(State &S, int round, int nact_host, hipStream_t s, bool &need_pairs);
void launch_emit_fallback(State &S, int nact_host, hipStream_t s);
void launch_gram_keys(State &S, hipStream_t s);
void launch_gram_batch(State &S, int nact_host, hipStream_t s);
void launch_gram_refine(State &S, int ncand, hipStream_t s);
void launch_cache_clear(State &S, unsigned long long *keys, unsigned long long *vals,
                        unsigned long long mask, hipStream_t s);
void launch_cache_rebuild(State &S, const unsigned long long *okeys, const unsigned long long *ovals,
                          unsigned long long omask, hipStream_t s);
void launch_cache_unclaim(State &S, hipStream_t s);
void launch_pairs(State &S, int round, int npairs_host, long long ntiles_host, hipStream_t s);
void launch_pairs_prefix(State &S, int npairs_host, hipStream_t s);
void launch_round_tail(State &S, int round, int nact_host, int merges_before, hipStream_t s);
void launch_finalize(State &S, void *out_rows, hipStream_t s);

}  // namespace pc
