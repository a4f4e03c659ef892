// C ABI of libparchain.so (declared in include/parchain.h) and the host side
// of the round loop: validation, workspace layout, the per-round launches and
// the few counter reads that size the next launches.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/parchain.h"
#include "pc_common.hpp"

using namespace pc;

namespace {

thread_local std::string g_err;

pc_status fail(pc_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(call)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(e_ == hipErrorOutOfMemory ? PC_ERR_OUT_OF_MEMORY : PC_ERR_DEVICE,            \
                  std::string(#call) + ": " + hipGetErrorString(e_));                          \
  } while (0)

// Carves typed arrays out of one device allocation (or only counts bytes when
// base is null), 256-byte aligned.
struct Carver {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

size_t layout(State &S, char *base, int64_t n64, int d, int linkage, bool host_points, int elem,
              float **xin = nullptr, pc_merge **rows_out = nullptr) {
  Carver c{base};
  const size_t n = (size_t)n64;
  const bool pts = !centroid_link(linkage);
  const bool avgsq = linkage == kAvgSq;
  S.cid = c.take<int>(n);
  S.csize = c.take<int>(n);
  S.node = c.take<int>(n);
  S.node2slot = c.take<int>(2 * n);
  S.nparent = c.take<int>(pts ? 2 * n : 1);
  S.succ = c.take<int>(n);
  S.succ_node = c.take<int>(n);
  S.predd = c.take<unsigned>(n);
  S.term_round = c.take<int>(n);
  S.alive = c.take<int>(n);
  S.mdst = c.take<int>(n);
  S.moff = c.take<int>(n);
  S.cbeg = c.take<int>(pts ? n : 1);
  S.nbeg = c.take<int>(pts ? n : 1);
  S.eff = c.take<double>(n);
  S.nn_h = c.take<double>(n);
  S.wsum = c.take<double>(n * d);
  S.wcen = c.take<double>(n * d);
  S.lo = c.take<float>(pts ? n * d : 1);
  S.hi = c.take<float>(pts ? n * d : 1);
  const bool comp = linkage == kComplete;
  S.ext = c.take<int>(comp && d <= kExtMaxDim ? n * 2 * d : 1);
  S.crad = c.take<double>(pts ? n : 1);  // radius bounds: complete and average
  S.cvar = c.take<double>(linkage != kWard ? n : 1);
  S.cmv = c.take<double>(avgsq ? n : 1);
  S.sup = c.take<int>(comp && d == 2 ? n * kSupDirs : 1);
  S.act = c.take<int>(n);
  S.act2 = c.take<int>(n);
  S.term = c.take<int>(n);
  S.flags = c.take<int>(n);
  S.scan = c.take<int>(n + 1);
  S.ovf = c.take<int>(n);
  const bool grid = d <= kGridMaxDim;
  const size_t cells = grid ? 2 * n + 16 : 1;
  S.cell_cap = (int)cells;
  S.cell_cnt = c.take<int>(cells + 1);
  S.cell_start = c.take<int>(cells + 1);
  S.cell_nmin = c.take<int>(cells + 1);
  S.cell_of = c.take<int>(n);
  S.cell_rank = c.take<int>(n);
  S.item_slot = c.take<int>(grid ? n : 1);
  S.item_meta = c.take<int4>(grid ? n : 1);
  S.item_cen = c.take<double>(grid ? n * d : 1);
  S.item_v = c.take<double>(grid && avgsq ? n : 1);
  S.item_lo = c.take<float>(grid && pts ? n * d : 1);
  S.item_hi = c.take<float>(grid && pts ? n * d : 1);
  const bool gram = d >= kGramMinDim && d <= kGramMaxDim;
  const int kp = gram_kp(d);
  S.gkp = kp;
  S.pkp = point_kp(d);
  S.elem = elem;
  const size_t ew = (size_t)screen_elem_bytes(elem) / 2;  // in 16-bit units
  S.g16 = c.take<_Float16>(gram ? n * kp * ew : 1);
  S.gq = c.take<float4>(gram ? n : 1);
  S.p16 = gram && pts ? c.take<_Float16>(n * (size_t)S.pkp * ew) : nullptr;
  S.pq = c.take<float4>(gram && pts ? n : 1);
  const bool blk = gram && comp && d <= kBlkMaxDim;
  S.blk_lo = c.take<float>(blk ? (n / 64 + 2) * d : 1);
  S.blk_hi = c.take<float>(blk ? (n / 64 + 2) * d : 1);
  S.porg = c.take<double>(gram ? d : 1);
  S.pscale = c.take<double>(1);
  S.gorg = c.take<double>(gram ? d : 1);
  S.gmin = c.take<unsigned long long>(gram ? d : 1);
  S.gmax = c.take<unsigned long long>(gram ? d : 1);
  S.gscale = c.take<double>(1);
  // box tree: Ward / avg-2 at 3 <= d <= kTreeMaxDim (the call may still use another search)
  const bool tree = centroid_link(linkage) && d >= 3 && d <= kTreeMaxDim;
  S.term_pos = c.take<int>(gram || tree ? n : 1);
  const size_t tnodes = n / 15 + 16;  // a 16-ary tree over n / 16 leaves (8 levels at most)
  S.tree_lo = c.take<double>(tree ? tnodes * d : 1);
  S.tree_hi = c.take<double>(tree ? tnodes * d : 1);
  S.tree_nmin = c.take<int>(tree ? tnodes : 1);
  S.tree_vmin = c.take<double>(tree ? tnodes : 1);
  S.t_best = c.take<double>(n);
  S.t_key = c.take<unsigned long long>(n);
  S.t_beta = c.take<double>(n);
  S.t_min = c.take<unsigned long long>(n);
  S.m_a = c.take<int>(n / 2 + 1);
  S.m_b = c.take<int>(n / 2 + 1);
  S.m_h = c.take<double>(n / 2 + 1);
  S.row_na = c.take<int>(n);
  S.row_nb = c.take<int>(n);
  S.row_size = c.take<int>(n);
  S.row_lo = c.take<int>(n);
  S.row_h = c.take<double>(n);
  S.row_eff = c.take<double>(n);
  S.px = c.take<float>(pts ? n * d : 1);
  S.px2 = c.take<float>(pts ? n * d : 1);
  S.powner = c.take<int>(pts ? n : 1);
  S.powner2 = c.take<int>(pts ? n : 1);
  S.sk0 = c.take<unsigned long long>(n);
  S.sk1 = c.take<unsigned long long>(n);
  S.sv0 = c.take<unsigned>(n);
  S.sv1 = c.take<unsigned>(n);
  S.hist = c.take<int>((size_t)radix_hist_len((int)n) + 1);
  S.grid = c.take<GridParams>(1);
  S.cnt = c.take<Counters>(1);
  // staging: input points (if on the host) and output rows (if on the host)
  float *x = c.take<float>(host_points ? n * d : 1);
  pc_merge *r = c.take<pc_merge>(n);
  if (xin) *xin = x;
  if (rows_out) *rows_out = r;
  return c.off + 256;
}

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};

// The allocation-free entry point (pc_hac_noalloc) carves every buffer of its
// call out of this array; each device that loads the library holds its own
// copy until the process ends. Host code must not pass the array's name to a
// kernel: on the host it is only a stand-in. Its device address is taken once
// per device with hipGetSymbolAddress (scratch_address) and used instead.
static __device__ __align__(256) unsigned char scratch[PC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch array; call with `dev` current
hipError_t scratch_address(int dev, void **out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// The device buffers of a call: the context's own (grown on demand, kept
// between calls) or windows of the static scratch array (fixed: never grown).
struct Bufs {
  Buf ws, pairs, tiles, part, fidx, cand, cache[2];
  bool fixed = false;
};

}  // namespace

struct pc_context {
  int device = 0;
  size_t budget = 0;         // most device bytes the context may hold (0: no limit)
  bool over_budget = false;  // the last call stopped at the budget
  Bufs own;
  Bufs *cur = &own;          // the buffers of the running call
  void *scratch = nullptr;   // this device's static scratch array (device address)
  hipError_t scratch_error = hipSuccess;
  Counters *hcnt = nullptr;  // pinned host mirror of the device counters
  hipEvent_t ev[4] = {};
  KTimer ktimer;              // kernel event pool and log
  hipEvent_t rev[4] = {};    // per round: start, search done, merge done, end
  std::atomic<int> busy{0};
};

namespace {

size_t held_bytes(const pc_context *c) {
  const Bufs &o = c->own;
  size_t b = o.ws.bytes + o.pairs.bytes + o.tiles.bytes + o.part.bytes + o.fidx.bytes + o.cand.bytes;
  return b + o.cache[0].bytes + o.cache[1].bytes;
}

// can b hold `bytes`, growing within the context's budget if need be?
// (fixed buffers never grow)
bool fits(const pc_context *c, const Buf &b, size_t bytes) {
  if (b.bytes >= bytes) return true;
  if (c->cur->fixed) return false;
  if (!c->budget) return true;
  return held_bytes(c) - b.bytes + bytes <= c->budget;
}

hipError_t grow(pc_context *c, Buf &b, size_t bytes) {
  if (b.bytes >= bytes) return hipSuccess;
  if (!fits(c, b, bytes)) {
    c->over_budget = true;  // b is left as it was
    return hipErrorOutOfMemory;
  }
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e == hipSuccess) b.bytes = bytes;
  return e;
}

}  // namespace

extern "C" {

const char *pc_last_error(void) { return g_err.c_str(); }

const char *pc_version(void) { return "parchain-mi355x 0.1 (gfx950)"; }

pc_status pc_context_create(int device, size_t hbm_budget_bytes, pc_context **out) {
  if (!out) return fail(PC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int dev = device;
  if (dev < 0) HIPCHK(hipGetDevice(&dev));
  int count = 0;
  HIPCHK(hipGetDeviceCount(&count));
  if (dev >= count) return fail(PC_ERR_INVALID_ARG, "device index out of range");
  HIPCHK(hipSetDevice(dev));
  pc_context *c = new (std::nothrow) pc_context();
  if (!c) return fail(PC_ERR_OUT_OF_MEMORY, "host allocation failed");
  c->device = dev;
  c->budget = hbm_budget_bytes;
  hipError_t e = set_direction_table();
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->hcnt, sizeof(Counters), hipHostMallocDefault);
  for (int i = 0; e == hipSuccess && i < 4; ++i) e = hipEventCreate(&c->ev[i]);
  for (int i = 0; e == hipSuccess && i < 4; ++i) e = hipEventCreateWithFlags(&c->rev[i], hipEventDisableSystemFence);
  if (e == hipSuccess) {
    // the allocation-free entry point's array on this device; a failure here
    // is reported by that entry point (c->scratch stays null), not by pc_hac
    const hipError_t se = scratch_address(dev, &c->scratch);
    if (se != hipSuccess) {
      c->scratch = nullptr;
      c->scratch_error = se;
      (void)hipGetLastError();
    }
  }
  if (e != hipSuccess) {
    pc_context_destroy(c);
    return fail(PC_ERR_DEVICE, std::string("context setup: ") + hipGetErrorString(e));
  }
  *out = c;
  g_err.clear();
  return PC_OK;
}

}  // extern "C"

namespace pc {
void set_error(const char *msg) { g_err = msg; }

// Device bytes a context holds, and release of its growable buffers (the
// serving layer keeps each slot within its share of the budget).
size_t context_bytes(const pc_context *c) { return held_bytes(c); }

// the serving layer caps a slot's context at the request's reservation
void context_set_budget(pc_context *c, size_t bytes) { c->budget = bytes; }
bool context_over_budget(const pc_context *c) { return c->over_budget; }
int context_device(const pc_context *c) { return c->device; }

void context_trim(pc_context *c) {
  hipSetDevice(c->device);
  Bufs &o = c->own;
  for (Buf *b : {&o.ws, &o.pairs, &o.tiles, &o.part, &o.fidx, &o.cand, &o.cache[0], &o.cache[1]}) {
    if (b->p) hipFree(b->p);
    b->p = nullptr;
    b->bytes = 0;
  }
}
}  // namespace pc

extern "C" {

void pc_context_destroy(pc_context *c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  Bufs &o = c->own;
  for (Buf *b : {&o.ws, &o.pairs, &o.tiles, &o.part, &o.fidx, &o.cand, &o.cache[0], &o.cache[1]})
    if (b->p) hipFree(b->p);
  if (c->hcnt) hipHostFree(c->hcnt);
  for (int i = 0; i < 4; ++i)
    if (c->ev[i]) hipEventDestroy(c->ev[i]);
  for (hipEvent_t ev : c->ktimer.pool) hipEventDestroy(ev);
  for (int i = 0; i < 4; ++i)
    if (c->rev[i]) hipEventDestroy(c->rev[i]);
  delete c;
}

size_t pc_hac_workspace_bytes(int64_t n, int32_t d, int32_t linkage, const pc_options *opt) {
  if (n < 1 || d < 1 || d > kMaxDim || n > 2147483646LL || linkage < 0 || linkage > 3) return 0;
  if (opt && (opt->precision < 0 || opt->precision > 2)) return 0;
  State S;
  size_t bytes = layout(S, nullptr, n, d, linkage, true, opt ? opt->precision : 0);
  const bool gram = d >= kGramMinDim && d <= kGramMaxDim;
  // initial candidate record (grown on demand), pair list, tiles and filter
  const size_t cand = (size_t)std::max<int64_t>(1 << 22, 4 * n);
  const size_t per_cand = 3 * sizeof(double) + sizeof(long long) + sizeof(int4) + 4 * sizeof(int);
  if (!centroid_link(linkage) || gram) bytes += cand * per_cand + 1024;
  bytes += ((size_t)(2 * n + 64) / 1024 + 1024) * sizeof(long long);
  if (!centroid_link(linkage)) {
    const size_t pc = (size_t)std::max<int64_t>(1 << 20, 2 * n);
    bytes += pc * (4 * sizeof(long long) + 6 * sizeof(int)) + 1024;
    if (linkage == kAverage) bytes += ((size_t)1 << 22) * sizeof(double);
    if (linkage == kComplete) bytes += cand * sizeof(int);
    int cs = opt ? opt->cache_slots : -1;
    if (cs < 0) cs = linkage == kAverage ? 64 : 0;
    if (cs > 0) {
      size_t cap = (size_t)1 << 16;
      while (cap < (size_t)n * (size_t)cs && cap < ((size_t)1 << 31)) cap <<= 1;
      bytes += 2 * cap * 2 * sizeof(unsigned long long);
    }
  }
  return bytes;
}

// Largest candidate record / pair list a round may use (entries). Beyond it a
// call fails with PC_ERR_OUT_OF_MEMORY instead of growing without bound.
constexpr long long kMaxRecord = 1LL << 30;

// Scan workspace: two status words per 1024 elements of the longest scan of
// the call (two arrays taken in turn), plus the tickets.
static pc_status grow_part(pc_context *ctx, State &S, long long longest_scan) {
  const long long need = 2 * (longest_scan / 1024 + 1024) + 1;
  const void *old = ctx->cur->part.p;
  const size_t old_bytes = ctx->cur->part.bytes;
  HIPCHK(grow(ctx, ctx->cur->part, (size_t)need * sizeof(long long)));
  S.part = (long long *)ctx->cur->part.p;
  S.part_cap = (long long)(ctx->cur->part.bytes / sizeof(long long));
  // new memory (a reallocation can return the same address, so its size is
  // compared too) or a first use in this call: stale status words, and the
  // capacity to take from the new size
  if (ctx->cur->part.p != old || ctx->cur->part.bytes != old_bytes ||
      S.sws.st[0] != (unsigned long long *)S.part || S.sws.cap != (int)std::min<long long>((S.part_cap - 1) / 2, 0x7fffffffLL))
    scan_ws_carve(S.sws, S.part, S.part_cap, &S.cnt->scan_err);
  return PC_OK;
}

// per pair: tile prefix (i64), chunk prefix (i64), value (f64), pending
// value (f64), t, c, kR, kS, pending t, pending c (i32)
constexpr size_t kPairBytes = 4 * sizeof(long long) + 6 * sizeof(int);
// per candidate: lower bound, value, screening bound (f64), tile prefix
// (i64), point ranges (int4), terminal, cluster, small-list entry (i32)
constexpr size_t kCandBytes = 3 * sizeof(double) + sizeof(long long) + sizeof(int4) + 8 + 4 * sizeof(int);

static pc_status grow_pairs(pc_context *ctx, State &S, long long cap) {
  if (cap > kMaxRecord) return fail(PC_ERR_OUT_OF_MEMORY, "a round needs more than 2^30 cluster pairs");
  const size_t per = kPairBytes;
  HIPCHK(grow(ctx, ctx->cur->pairs, (size_t)cap * per + 1024));
  char *b = (char *)ctx->cur->pairs.p;
  const long long pc = (long long)((ctx->cur->pairs.bytes - 1024) / per);
  S.pair_cap = pc;
  S.pr_tile0 = (long long *)b;
  S.pr_cbase = S.pr_tile0 + pc;
  S.pr_v = (double *)(S.pr_cbase + pc);
  S.pd_v = S.pr_v + pc;
  S.pr_t = (int *)(S.pd_v + pc);
  S.pr_c = S.pr_t + pc;
  S.pr_kR = S.pr_c + pc;
  S.pr_kS = S.pr_kR + pc;
  S.pd_t = S.pr_kS + pc;
  S.pd_c = S.pd_t + pc;
  return grow_part(ctx, S, std::max<long long>(S.pair_cap, 2LL * S.n + 64));
}

static pc_status grow_fidx(pc_context *ctx, State &S, long long cap) {
  if (cap > 8 * kMaxRecord) return fail(PC_ERR_OUT_OF_MEMORY, "a round's pair filter needs too many points");
  HIPCHK(grow(ctx, ctx->cur->fidx, (size_t)cap * sizeof(int)));
  S.fidx = (int *)ctx->cur->fidx.p;
  S.fidx_cap = (long long)(ctx->cur->fidx.bytes / sizeof(int));
  return PC_OK;
}

static pc_status grow_tiles(pc_context *ctx, State &S, long long cap) {
  HIPCHK(grow(ctx, ctx->cur->tiles, (size_t)cap * sizeof(double)));
  S.tile_v = (double *)ctx->cur->tiles.p;
  S.tile_cap = (long long)(ctx->cur->tiles.bytes / sizeof(double));
  return PC_OK;
}

static pc_status grow_cand(pc_context *ctx, State &S, long long cap) {
  if (cap > kMaxRecord) return fail(PC_ERR_OUT_OF_MEMORY, "a round needs more than 2^30 recorded candidates");
  const size_t per = kCandBytes;
  HIPCHK(grow(ctx, ctx->cur->cand, (size_t)cap * per + 1024));
  const long long cc = (long long)((ctx->cur->cand.bytes - 1024) / per);
  S.cand_cap = cc;
  S.cd_lb = (double *)ctx->cur->cand.p;
  S.cd_v = S.cd_lb + cc;
  S.cd_l0 = S.cd_v + cc;
  S.cd_tile0 = (long long *)(S.cd_l0 + cc);  // 32 cc bytes in: the int4 records stay 16-byte aligned
  S.cd_desc = (int4 *)(S.cd_tile0 + cc);
  S.cd_x = (unsigned long long *)(S.cd_desc + cc);
  S.cd_t = (int *)(S.cd_x + cc);
  S.cd_c = S.cd_t + cc;
  S.cd_small = S.cd_c + cc;
  S.cd_scr = S.cd_small + cc;
  return grow_part(ctx, S, std::max<long long>(cc, 2LL * S.n + 64));
}

// Windows of the scratch array for one allocation-free call: the layout
// (`ws` bytes), the scan partials, then the candidate record, pair list, tile
// partials or filter indices and the two cache tables in fixed shares of what
// is left. cache_cap: entries per cache table (a power of two, 0: no cache).
static pc_status carve_scratch(char *base, size_t ws, int64_t n, int d, int linkage, int cache_slots, Bufs &B,
                               unsigned long long &cache_cap) {
  const size_t total = PC_NOALLOC_SCRATCH_BYTES;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t off = 0;
  auto take = [&](Buf &b, size_t bytes) {
    b.p = base + off;
    b.bytes = bytes;
    off = al(off + bytes);
  };
  cache_cap = 0;
  if (al(ws) + (1u << 20) > total)
    return fail(PC_ERR_OUT_OF_MEMORY, "input too large for the allocation-free scratch buffer");
  take(B.ws, ws);
  // scan partials for the longest scan a record of this scratch can need
  const size_t left = total - off;
  const long long longest = std::max<long long>(2 * n + 64, (long long)(left / kPairBytes) + 1);
  take(B.part, (size_t)(2 * (longest / 1024 + 1024) + 1) * sizeof(long long));
  if (off + (1u << 20) > total)
    return fail(PC_ERR_OUT_OF_MEMORY, "input too large for the allocation-free scratch buffer");
  const size_t rest = total - off - 8 * 256;  // alignment slack of the windows below
  const bool gram = d >= kGramMinDim && d <= kGramMaxDim;
  double fc = 0.0, fp = 0.0, ft = 0.0, ff = 0.0, fk = 0.0;  // shares of the rest
  if (centroid_link(linkage)) {
    fc = gram ? 1.0 : 0.0;
  } else if (linkage == kComplete) {
    fk = cache_slots > 0 ? 0.15 : 0.0;
    fc = 0.3;
    fp = 0.2;
    ff = 0.5 - fk;
  } else {
    fk = cache_slots > 0 ? 0.15 : 0.0;
    fc = 0.3;
    fp = 0.25;
    ft = 0.45 - fk;
  }
  auto share = [&](double f) { return std::max<size_t>((size_t)(f * (double)rest) & ~(size_t)255, 256); };
  take(B.cand, share(fc));
  take(B.pairs, share(fp));
  take(B.tiles, share(ft));
  take(B.fidx, share(ff));
  if (fk > 0.0) {
    unsigned long long cap = 1;
    while (2 * (cap * 2) * 2 * sizeof(unsigned long long) <= share(fk)) cap *= 2;
    if (cap >= 1024) {
      cache_cap = cap;
      take(B.cache[0], cap * 2 * sizeof(unsigned long long));
      take(B.cache[1], cap * 2 * sizeof(unsigned long long));
    }
  }
  if (off > total) return fail(PC_ERR_OUT_OF_MEMORY, "allocation-free scratch buffer overrun");
  if ((!centroid_link(linkage) || gram) && B.cand.bytes < 4096 * kCandBytes + 1024)
    return fail(PC_ERR_OUT_OF_MEMORY, "input too large for the allocation-free scratch buffer");
  B.fixed = true;
  return PC_OK;
}

// the initial size of a record: `want` entries, or what a fixed window holds
static long long initial_cap(const pc_context *ctx, const Buf &b, long long want, size_t per, size_t extra) {
  if (!ctx->cur->fixed) return want;
  const long long c = (long long)((b.bytes > extra ? b.bytes - extra : 0) / per);
  return std::max<long long>(1, std::min(want, c));
}

static pc_status hac_impl(pc_context *ctx, const float *points, int64_t n, int32_t d, int points_on_device,
                          int32_t linkage, const pc_options *opt, pc_merge *out, int out_on_device, void *stream,
                          pc_stats *stats, bool noalloc) {
  if (!ctx) return fail(PC_ERR_INVALID_ARG, "context is NULL");
  if (!points) return fail(PC_ERR_INVALID_ARG, "points is NULL");
  if (n < 1) return fail(PC_ERR_INVALID_ARG, "n must be >= 1");
  if (n > 2147483646LL) return fail(PC_ERR_INVALID_ARG, "n must be <= 2^31-2");
  if (d < 1 || d > kMaxDim) return fail(PC_ERR_INVALID_ARG, "d must be in [1, 2048]");
  if (linkage < 0 || linkage > 3) return fail(PC_ERR_INVALID_ARG, "unknown linkage");
  if (n > 1 && !out) return fail(PC_ERR_INVALID_ARG, "out is NULL");
  if (opt && opt->struct_size != sizeof(pc_options)) return fail(PC_ERR_INVALID_ARG, "pc_options.struct_size");
  if (stats && stats->struct_size != sizeof(pc_stats)) return fail(PC_ERR_INVALID_ARG, "pc_stats.struct_size");
  const int prune = opt ? (opt->prune != 0) : 1;
  int cache_slots = opt ? opt->cache_slots : -1;
  if (cache_slots < 0) cache_slots = linkage == kAverage ? 64 : 0;
  if (centroid_link(linkage)) cache_slots = 0;  // Ward / avg-2 values cost less than a probe
  const int elem = opt ? opt->precision : PC_PREC_FP16_REFINE;
  if (elem < PC_PREC_FP16_REFINE || elem > PC_PREC_FP32) return fail(PC_ERR_INVALID_ARG, "unknown precision");
  if (!points_on_device) {
    for (int64_t i = 0; i < n * (int64_t)d; ++i)
      if (!std::isfinite(points[i])) return fail(PC_ERR_NONFINITE_INPUT, "non-finite coordinate");
  }
  int expected = 0;
  if (!ctx->busy.compare_exchange_strong(expected, 1)) return fail(PC_ERR_BUSY, "context in use");
  struct Release {
    pc_context *c;
    ~Release() { c->busy.store(0); }
  } release{ctx};

  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  if (stats) {
    uint32_t ss = stats->struct_size;
    memset(stats, 0, sizeof(*stats));
    stats->struct_size = ss;
  }
  if (n == 1) {
    g_err.clear();
    return PC_OK;
  }

  ctx->over_budget = false;
  State S;
  memset(&S, 0, sizeof(S));
  const size_t need = layout(S, nullptr, n, d, linkage, !points_on_device, elem);
  // allocation-free call: every buffer is a window of the scratch array
  Bufs fixed;
  struct Restore {
    pc_context *c;
    ~Restore() { c->cur = &c->own; }
  } restore{ctx};
  unsigned long long fixed_cache = 0;
  if (noalloc) {
    if (!ctx->scratch)
      return fail(PC_ERR_DEVICE, std::string("no scratch address for this device: ") +
                                     hipGetErrorString(ctx->scratch_error));
    pc_status st = carve_scratch((char *)ctx->scratch, need, n, d, linkage, cache_slots, fixed, fixed_cache);
    if (st != PC_OK) return st;
    if (!fixed_cache) cache_slots = 0;  // no room for the cache: values are recomputed (same rows)
    ctx->cur = &fixed;
  }
  HIPCHK(grow(ctx, ctx->cur->ws, need));
  float *xstage = nullptr;
  pc_merge *rstage = nullptr;
  layout(S, (char *)ctx->cur->ws.p, n, d, linkage, !points_on_device, elem, &xstage, &rstage);
  S.n = (int)n;
  S.d = d;
  S.linkage = linkage;
  S.prune = prune;
  S.timing = (opt && (opt->timing & PC_TIME_KERNELS)) ? 1 : 0;
  S.phases = (opt && (opt->timing & PC_TIME_PHASES)) ? 1 : 0;
  // Ward and avg-2 at 3 <= d <= 5 search a box tree over Morton-ordered
  // centroids while many clusters are active and the Gram search once at most
  // tree_gram_switch are (at d = 3, where there is no Gram search, the tree
  // throughout); from d = 6 the Gram search alone (measured faster at 8-D).
  // Without the tree: the centroid grid up to d = 5, the Gram search above.
  // Tuning knobs: PC_TREE_MAX_DIM (0 = no tree, at most 8),
  // PC_TREE_GRAM_SWITCH (0 = tree in every round), PC_GRAM_MIN_DIM.
  int tree_max = 5;
  if (const char *e = getenv("PC_TREE_MAX_DIM")) tree_max = std::min(kTreeMaxDim, atoi(e));
  const bool tree_ok = prune && centroid_link(linkage) && d >= 3 && d <= tree_max;
  int gram_min = centroid_link(linkage) && !tree_ok ? 6 : kGramMinDim;
  if (const char *e = getenv("PC_GRAM_MIN_DIM")) gram_min = std::max(kGramMinDim, atoi(e));
  const bool gram_ok = prune && d >= gram_min && d <= kGramMaxDim;
  long long tree_gram_switch = 200000;  // measured on the paper's 1M-point 5-D sets (flat from 150K to 250K)
  if (const char *e = getenv("PC_TREE_GRAM_SWITCH")) tree_gram_switch = atoll(e);
  // the first round's search (tree_ok also fixes the Morton order of the init)
  S.tree = tree_ok ? 1 : 0;
  S.gram = (!tree_ok && gram_ok) ? 1 : 0;
  S.kt = &ctx->ktimer;
  S.kt->begin_call();
  S.rev = ctx->rev;
  S.xin = nullptr;  // set once the device copy of the points is known
  double kms[4] = {0, 0, 0, 0};
  long long klaunch[4] = {0, 0, 0, 0};
  // after a synchronisation: the timed launches so far stand (a redo from
  // here on drops only its own); the times are read at the end of the call
  auto take_times = [&]() {
    if (S.timing) S.kt->commit();
  };
  float *xdev = (float *)points;
  if (!points_on_device) {
    xdev = xstage;
    HIPCHK(hipMemcpyAsync(xdev, points, (size_t)n * d * sizeof(float), hipMemcpyHostToDevice, s));
  }
  pc_merge *dout = out_on_device ? out : rstage;
  S.xin = xdev;

  {
    pc_status st = grow_part(ctx, S, 2LL * n + 64);
    if (st != PC_OK) return st;
  }
  if (centroid_link(linkage) && gram_ok) {
    pc_status st = grow_cand(ctx, S, initial_cap(ctx, ctx->cur->cand, std::max<long long>(1 << 22, 4 * n),
                                                 kCandBytes, 1024));
    if (st != PC_OK) return st;
    if (const char *e = getenv("PC_TEST_CAND_CAP")) S.cand_cap = std::min<long long>(S.cand_cap, atoll(e));
  }
  if (!centroid_link(linkage)) {
    pc_status st = grow_pairs(ctx, S, initial_cap(ctx, ctx->cur->pairs, std::max<long long>(1 << 20, 2 * n),
                                                  kPairBytes, 1024));
    if (st != PC_OK) return st;
    st = grow_tiles(ctx, S, initial_cap(ctx, ctx->cur->tiles, linkage == kAverage ? (1 << 22) : 1,
                                        sizeof(double), 0));
    if (st != PC_OK) return st;
    st = grow_fidx(ctx, S, initial_cap(ctx, ctx->cur->fidx, linkage == kComplete ? std::max<long long>(1 << 22, 4 * n) : 1,
                                       sizeof(int), 0));
    if (st != PC_OK) return st;
    st = grow_cand(ctx, S, initial_cap(ctx, ctx->cur->cand, std::max<long long>(1 << 22, 4 * n), kCandBytes, 1024));
    if (st != PC_OK) return st;
    // test hooks: shrink the candidate record / pair list to exercise their
    // overflow paths (capacities only ever limit, never extend, the buffers)
    if (const char *e = getenv("PC_TEST_CAND_CAP")) S.cand_cap = std::min<long long>(S.cand_cap, atoll(e));
    if (const char *e = getenv("PC_TEST_PAIR_CAP")) S.pair_cap = std::min<long long>(S.pair_cap, atoll(e));
  }

  // cluster-pair cache: two tables (the second receives the live entries at a rebuild)
  int cache_cur = 0;
  long long cache_base = 0;  // inserts counted when the current table was filled
  if (cache_slots > 0) {
    unsigned long long cap = 1ull << 16;
    while (cap < (unsigned long long)n * (unsigned long long)cache_slots && cap < (1ull << 31)) cap <<= 1;
    if (ctx->cur->fixed) cap = std::min(cap, fixed_cache);
    // test hook: a small table exercises rebuilds and full probe windows
    if (const char *e = getenv("PC_TEST_CACHE_CAP")) {
      unsigned long long want = (unsigned long long)atoll(e), c2 = 64;
      while (c2 < want) c2 <<= 1;
      if (c2 < cap) cap = c2;
    }
    for (int i = 0; i < 2; ++i) HIPCHK(grow(ctx, ctx->cur->cache[i], (size_t)cap * 2 * sizeof(unsigned long long)));
    S.cache_mask = cap - 1;
    S.ck = (unsigned long long *)ctx->cur->cache[0].p;
    S.cv = S.ck + cap;
    launch_cache_clear(S, S.ck, S.cv, S.cache_mask, s);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipMemsetAsync(S.cnt, 0, sizeof(Counters), s));
  HIPCHK(hipEventRecord(ctx->ev[0], s));
  if (points_on_device) {
    launch_check_finite(xdev, (long long)n * d, S.cnt, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ctx->hcnt, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (ctx->hcnt->nonfinite) return fail(PC_ERR_NONFINITE_INPUT, "non-finite coordinate");
  }
  launch_init(S, xdev, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(ctx->ev[1], s));

  const bool debug = getenv("PC_DEBUG") != nullptr;
  // tuning knob: cells a thread-per-terminal ring search visits before it
  // hands the terminal to the block search
  S.cell_budget = centroid_link(linkage) ? 24 : 160;  // measured on the 1M 2-D workload
  if (const char *e = getenv("PC_CELL_BUDGET")) S.cell_budget = std::max(1, atoi(e));
  // tuning knob: active clusters at or below which the ring search's first
  // pass runs a wavefront per terminal (0: never)
  // (avg-2: off; its per-item work is too light to pay for combining lanes)
  S.wave_terms = linkage == kAvgSq ? 0 : (linkage == kWard ? 30000 : 60000);  // swept on the 1M 2-D workload
  if (const char *e = getenv("PC_WAVE_TERMS")) S.wave_terms = std::max(0, atoi(e));
  // cells a wavefront searches before handing its terminal to the block search
  S.wave_budget = 640;
  if (const char *e = getenv("PC_WAVE_BUDGET")) S.wave_budget = std::max(1, atoi(e));
  // tuning knob: active clusters at or below which a grid-path round scans
  // them all instead of walking rings (0: never)
  // (complete: 1024 since its late rounds search a wavefront per terminal)
  S.full_scan_max = centroid_link(linkage) ? 2048 : (linkage == kComplete ? 1024 : 4096);  // swept on the 1M 2-D workload
  if (const char *e = getenv("PC_FULL_SCAN_MAX")) S.full_scan_max = std::max(0, atoi(e));
  long long gram_batch = 0;  // terminals per Gram batch (0: all), kept across rounds
  // test hook: small batches exercise the batch loop on small inputs
  if (const char *e = getenv("PC_TEST_GRAM_BATCH")) gram_batch = std::max<long long>(1, atoll(e));
  int nact = (int)n;
  int merges = 0;
  long long rounds = 0, terms = 0, ovfq = 0, gram_terms = 0;
  double ms_nn = 0.0, ms_merge = 0.0, ms_update = 0.0;
  Counters &h = *ctx->hcnt;
  while (nact > 1) {
    if (rounds > n) return fail(PC_ERR_DEVICE, "round loop did not converge");
    if (S.phases) HIPCHK(hipEventRecord(ctx->rev[0], s));
    if (tree_ok) {
      const bool use_tree = !gram_ok || tree_gram_switch <= 0 || nact > tree_gram_switch;
      S.tree = use_tree ? 1 : 0;
      S.gram = use_tree ? 0 : 1;
    }
    bool need_pairs = false;
    S.tb0 = 0;
    S.tb1 = 0x7fffffff;
    launch_round(S, (int)rounds, nact, s, need_pairs);
    HIPCHK(hipGetLastError());
    // evaluate the emitted pairs of the current terminals (tiles), then their keys
    // (too_big: the work exceeds the record limits; nothing was evaluated)
    auto pairs_pipeline = [&](int np, bool &too_big) -> pc_status {
      too_big = false;
      launch_pairs_prefix(S, np, s);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(&h, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      long long work = 0;
      if (np > 0 && (linkage == kComplete ? h.n_chunks * kChunk > 8 * kMaxRecord : h.n_tiles > 4 * kMaxRecord)) {
        too_big = true;
        return PC_OK;
      }
      if (linkage == kComplete) {
        work = np > 0 ? h.n_chunks : 0;
        if (work * kChunk > S.fidx_cap) {
          // headroom for later rounds, within the limit
          const long long want = std::min<long long>(work * kChunk + work * kChunk / 2 + 1024, 8 * kMaxRecord);
          pc_status st = grow_fidx(ctx, S, std::max<long long>(want, work * kChunk));
          if (st != PC_OK) return st;
        }
      } else {
        work = np > 0 ? h.n_tiles : 0;
        if (work > S.tile_cap) {
          const long long want = std::min<long long>(work + work / 2 + 1024, 4 * kMaxRecord);
          pc_status st = grow_tiles(ctx, S, std::max<long long>(want, work));
          if (st != PC_OK) return st;
        }
      }
      launch_pairs(S, (int)rounds, np, work, s);
      HIPCHK(hipGetLastError());
      if (debug) {
        HIPCHK(hipMemcpyAsync(&h, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        fprintf(stderr, "[parchain] round %lld nact %d nterm %d batch [%d,%d) pairs %d work %lld tiles %lld pp %lld\n",
                rounds, nact, h.n_term, S.tb0, S.tb1 == 0x7fffffff ? h.n_term : S.tb1, np, work, h.n_tiles,
                h.point_pairs);
      }
      return PC_OK;
    };
    if (S.gram) {
      // Gram search: terminals in batches, each with a bounded candidate record
      HIPCHK(hipMemcpyAsync(&h, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
        take_times();  // a timing slot may be reused within the round
      const int nterm = h.n_term;
      long long tb = gram_batch > 0 ? std::min<long long>(gram_batch, nterm) : nterm;
      for (int t0 = 0; t0 < nterm;) {
        const int t1 = (int)std::min<long long>(nterm, t0 + tb);
        S.tb0 = t0;
        S.tb1 = t1;
        launch_gram_batch(S, nact, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&h, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        take_times();  // a timing slot may be reused within the round
        if (!h.cand_overflow) {
          // screening and exact values (or claims) of the recorded candidates
          launch_gram_refine(S, (int)std::min<long long>(h.n_cand, S.cand_cap), s);
          HIPCHK(hipGetLastError());
          HIPCHK(hipMemcpyAsync(&h, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
          HIPCHK(hipStreamSynchronize(s));
        take_times();  // a timing slot may be reused within the round
        }
        const bool pover = h.pair_overflow || h.n_pairs > S.pair_cap || h.n_pend > S.pair_cap;
        if (h.cand_overflow || pover) {
          // redo this batch: larger buffers while they stay within the limit,
          // otherwise fewer terminals per batch
          if (S.timing) S.kt->drop();
          launch_cache_unclaim(S, s);
          bool shrink = false;
          // (beyond the record limit or the context's budget: fewer terminals)
          if (h.cand_overflow) {
            const long long want = h.n_cand + h.n_cand / 2 + 1024;
            if (want <= kMaxRecord && fits(ctx, ctx->cur->cand, (size_t)want * kCandBytes + 1024)) {
              pc_status st = grow_cand(ctx, S, want);
              if (st != PC_OK) return st;
            } else {
              shrink = true;
            }
          }
          if (pover) {
            const long long want = std::max<long long>(h.n_pairs, h.n_pend) * 3 / 2 + 1024;
            if (want <= kMaxRecord && fits(ctx, ctx->cur->pairs, (size_t)want * kPairBytes + 1024)) {
              pc_status st = grow_pairs(ctx, S, want);
              if (st != PC_OK) return st;
            } else {
              shrink = true;
            }
          }
          if (shrink) {
            if (t1 - t0 <= 1) return fail(PC_ERR_OUT_OF_MEMORY, "one terminal exceeds the candidate limit");
            tb = std::max<long long>(1, (t1 - t0) / 4);
            gram_batch = tb;
          }
          continue;
        }
        if (centroid_link(linkage)) {
          launch_gram_keys(S, s);
        } else {
          bool too_big = false;
          pc_status st = pairs_pipeline((int)h.n_pairs, too_big);
          if (st != PC_OK) return st;
          if (too_big) {
            // fewer terminals per batch; the claims of this batch are dropped
            if (S.timing) S.kt->drop();
            launch_cache_unclaim(S, s);
            if (t1 - t0 <= 1) return fail(PC_ERR_OUT_OF_MEMORY, "one terminal's pair evaluation exceeds the limits");
            tb = std::max<long long>(1, (t1 - t0) / 4);
            gram_batch = tb;
            continue;
          }
        }
        t0 = t1;
      }
      S.tb0 = 0;
      S.tb1 = 0x7fffffff;
    } else if (need_pairs) {
      HIPCHK(hipMemcpyAsync(&h, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (h.cand_overflow) {
        // this round: emit by re-walking the rings; later rounds: a larger record
        launch_emit_fallback(S, nact, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&h, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        // later rounds: a larger record, if the budget (or a fixed scratch
        // window) allows; otherwise they re-walk too
        const long long want = std::min<long long>(h.n_cand + h.n_cand / 2 + 1024, kMaxRecord);
        if (fits(ctx, ctx->cur->cand, (size_t)want * kCandBytes + 1024)) {
          pc_status st = grow_cand(ctx, S, want);
          if (st != PC_OK) return st;
        }
      }
      if (h.n_pairs > S.pair_cap || h.n_pend > S.pair_cap) {
        if (S.timing) S.kt->drop();  // the round is redone
        launch_cache_unclaim(S, s);
        const long long want = std::max<long long>(h.n_pairs, h.n_pend);
        pc_status st = grow_pairs(ctx, S, std::max<long long>(want, std::min<long long>(want + want / 2 + 1024, kMaxRecord)));
        if (st != PC_OK) return st;
        launch_round(S, (int)rounds, nact, s, need_pairs);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&h, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (h.cand_overflow) {
          launch_emit_fallback(S, nact, s);
          HIPCHK(hipGetLastError());
          HIPCHK(hipMemcpyAsync(&h, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
          HIPCHK(hipStreamSynchronize(s));
        }
        if (h.n_pairs > S.pair_cap || h.n_pend > S.pair_cap) return fail(PC_ERR_DEVICE, "pair list overflow");
      }
      bool too_big = false;
      pc_status st = pairs_pipeline((int)h.n_pairs, too_big);
      if (st != PC_OK) return st;
      if (too_big) return fail(PC_ERR_OUT_OF_MEMORY, "a round's pair evaluation exceeds the record limits");
    }
    if (S.gram) gram_terms += h.n_term;
    if (S.phases) HIPCHK(hipEventRecord(ctx->rev[1], s));
    launch_round_tail(S, (int)rounds, nact, merges, s);  // records rev[2] after the merges (phases)
    HIPCHK(hipGetLastError());
    if (S.phases) HIPCHK(hipEventRecord(ctx->rev[3], s));
    HIPCHK(hipMemcpyAsync(&h, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (S.phases) {
      float a = 0.f, b = 0.f, c = 0.f;
      if (hipEventElapsedTime(&a, ctx->rev[0], ctx->rev[1]) == hipSuccess) ms_nn += a;
      if (hipEventElapsedTime(&b, ctx->rev[1], ctx->rev[2]) == hipSuccess) ms_merge += b;
      if (hipEventElapsedTime(&c, ctx->rev[2], ctx->rev[3]) == hipSuccess) ms_update += c;
    }
    if (h.nonfinite == 2) return fail(PC_ERR_DEVICE, "a terminal found no neighbour");
    if (h.nonfinite == 3) return fail(PC_ERR_DEVICE, "internal index check failed");
    if (h.nonfinite == 4) return fail(PC_ERR_DEVICE, "a claimed cache entry was never filled");
    if (h.scan_err) return fail(PC_ERR_DEVICE, "a prefix scan's look-back gave up");
    if (S.cache_mask && h.cache_inserts - cache_base > (long long)(S.cache_mask + 1) / 2) {
      // rebuild: keep only entries whose two clusters are still alive
      const int nxt = 1 - cache_cur;
      unsigned long long *ok = S.ck, *ov = S.cv;
      S.ck = (unsigned long long *)ctx->cur->cache[nxt].p;
      S.cv = S.ck + (S.cache_mask + 1);
      launch_cache_clear(S, S.ck, S.cv, S.cache_mask, s);
      launch_cache_rebuild(S, ok, ov, S.cache_mask, s);
      HIPCHK(hipGetLastError());
      cache_base = h.cache_inserts;
      cache_cur = nxt;
    }
    take_times();
    if (debug) {
      const double now = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
      static thread_local double last = 0.0;
      fprintf(stderr, "[parchain] round %lld done: nact %d nterm %d merged %d evals %lld pp %lld cand %lld (%.2f ms)\n",
              rounds, nact, h.n_term, h.n_merge, h.cluster_evals, h.point_pairs, h.n_cand, last > 0.0 ? now - last : 0.0);
      last = now;
    }
    if (h.n_merge <= 0) return fail(PC_ERR_DEVICE, "round merged nothing");
    terms += h.n_term;
    ovfq += h.n_ovf;
    merges += h.n_merge;
    nact = h.n_act;
    ++rounds;
  }
  if (merges != n - 1) return fail(PC_ERR_DEVICE, "merge count mismatch");
  HIPCHK(hipEventRecord(ctx->ev[2], s));
  launch_finalize(S, dout, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(ctx->ev[3], s));
  if (!out_on_device)
    HIPCHK(hipMemcpyAsync(out, dout, (size_t)(n - 1) * sizeof(pc_merge), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&h, S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (S.timing) {
    // every timed launch has completed: read the log once
    KTimer &t = *S.kt;
    t.commit();
    for (size_t j = 0; j + 2 < t.kept; j += 3) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, t.pool[t.done[j + 1]], t.pool[t.done[j + 2]]) == hipSuccess) kms[t.done[j]] += ms;
      ++klaunch[t.done[j]];
    }
  }
  if (stats) {
    float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
    hipEventElapsedTime(&t01, ctx->ev[0], ctx->ev[1]);
    hipEventElapsedTime(&t12, ctx->ev[1], ctx->ev[2]);
    hipEventElapsedTime(&t23, ctx->ev[2], ctx->ev[3]);
    hipEventElapsedTime(&t03, ctx->ev[0], ctx->ev[3]);
    stats->rounds = rounds;
    stats->terminals = terms;
    stats->cluster_evals = h.cluster_evals;
    stats->point_pair_evals = h.point_pairs;
    stats->overflow_queries = ovfq;
    stats->ms_init = t01;
    stats->ms_rounds = t12;
    stats->ms_finalize = t23;
    stats->ms_total = t03;
    for (int k = 0; k < 4; ++k) {
      stats->kernel_ms[k] = kms[k];
      stats->kernel_launches[k] = klaunch[k];
    }
    for (int k = 0; k < 4; ++k) stats->candidate_visits[k] = h.visits[k];
    stats->cache_hits = h.cache_hits;
    stats->cache_inserts = h.cache_inserts;
    stats->cache_fail = h.cache_fail;
    stats->cache_derived = h.cache_derived;
    stats->refined = h.refined;
    stats->fp64_fallbacks = h.refined > gram_terms ? h.refined - gram_terms : 0;
    stats->ms_nn = ms_nn;
    stats->ms_merge = ms_merge;
    stats->ms_update = ms_update;
  }
  g_err.clear();
  return PC_OK;
}

pc_status pc_hac(pc_context *ctx, const float *points, int64_t n, int32_t d, int points_on_device,
                 int32_t linkage, const pc_options *opt, pc_merge *out, int out_on_device, void *stream,
                 pc_stats *stats) {
  return hac_impl(ctx, points, n, d, points_on_device, linkage, opt, out, out_on_device, stream, stats, false);
}

pc_status pc_hac_noalloc(pc_context *ctx, const float *points, int64_t n, int32_t d, int32_t linkage,
                         const pc_options *opt, pc_merge *out, void *stream, pc_stats *stats) {
  return hac_impl(ctx, points, n, d, 1, linkage, opt, out, 1, stream, stats, true);
}

}  // extern "C"
