// Device-wide primitives: exclusive scan (the prefix sums behind every
// parallel filter of Alg. 1) and a stable LSD radix sort of (key, value)
// pairs (initial Morton layout and the final row order).
#include "pc_common.hpp"

namespace pc {

namespace {

constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;  // 1024
constexpr int kSortItems = 8;
constexpr int kSortTile = kBlock * kSortItems;  // 2048
constexpr int kNW = kBlock / kWave;             // waves per block

template <class T>
__device__ T block_exclusive_scan(T v, T &total) {
  __shared__ T sw[kNW + 1];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  T x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) sw[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int w = 0; w < kNW; ++w) {
      T t = sw[w];
      sw[w] = acc;
      acc += t;
    }
    sw[kNW] = acc;
  }
  __syncthreads();
  T r = x - v + sw[wid];
  total = sw[kNW];
  __syncthreads();
  return r;
}

template <class T>
__device__ __forceinline__ int scan_len(int nmax, const int *dlen) {
  if (!dlen) return nmax;
  int l = *dlen;
  return l < nmax ? l : nmax;
}

// Single-pass exclusive scan by decoupled look-back. A block takes the next
// ticket (so every block it waits for has started), scans its 1024 items,
// publishes its total (flag 1), adds the totals of the blocks before it until
// it meets a published prefix (flag 2), and publishes its own prefix. One
// wavefront looks back 64 blocks at a time. The status array of the next
// scan is cleared on the way. A look-back that waits beyond kSpinLimit
// windows gives up with the part it has (every output position then stays
// at or below its true value) and raises the error flag.
constexpr unsigned long long kStValue = (1ull << 62) - 1;
constexpr int kSpinLimit = 1 << 22;

template <class T>
__global__ __launch_bounds__(kBlock) void k_scan_lb(const T *in, T *out, int nmax, const int *dlen,
                                                    unsigned long long *st, int *ticket,
                                                    unsigned long long *st_next, int *ticket_next, int cap,
                                                    long long *total64, int *total32, int *err) {
  __shared__ int sbid;
  __shared__ T sprefix;
  if (threadIdx.x == 0) sbid = atomicAdd(ticket, 1);
  __syncthreads();
  const int bid = sbid;
  for (int j = bid * kBlock + threadIdx.x; j < cap; j += gridDim.x * kBlock) st_next[j] = 0ull;
  if (bid == 0 && threadIdx.x == 0) *ticket_next = 0;
  const int len = scan_len<T>(nmax, dlen);
  // blocks past the device length have nothing to scan (the grid is sized
  // for the host's bound); the last live block writes the total
  const int live = len > 0 ? (len + kScanTile - 1) / kScanTile : 1;
  if (bid >= live) return;  // uniform per block
  const long long base = (long long)bid * kScanTile + threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const long long i = base + j;
    v[j] = i < len ? in[i] : (T)0;
    s += v[j];
  }
  T tot;
  const T ex = block_exclusive_scan<T>(s, tot);
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    T prefix = 0;
    if (bid == 0) {
      if (lane == 0)
        __hip_atomic_store(&st[0], (2ull << 62) | (unsigned long long)tot, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (lane == 0)
        __hip_atomic_store(&st[bid], (1ull << 62) | (unsigned long long)tot, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      int top = bid - 1;  // the nearest block not yet added
      int spins = 0;
      while (true) {
        const int idx = top - lane;
        const unsigned long long w =
            idx >= 0 ? __hip_atomic_load(&st[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : (2ull << 62);
        const unsigned long long pm = __ballot((w >> 62) == 2ull);
        const int fp = pm ? __ffsll((long long)pm) - 1 : kWave;  // nearest published prefix
        const unsigned long long need = fp >= kWave - 1 ? ~0ull : ((2ull << fp) - 1ull);
        if (__ballot((w >> 62) == 0ull) & need) {
          // a block in the window has not published yet
          if (++spins > kSpinLimit) {
            if (lane == 0) atomicExch(err, 1);
            break;
          }
          continue;
        }
        T add = lane <= fp ? (T)(w & kStValue) : (T)0;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) add += __shfl_xor(add, o, kWave);
        prefix += add;
        if (fp < kWave) break;
        top -= kWave;
      }
      if (lane == 0)
        __hip_atomic_store(&st[bid], (2ull << 62) | (unsigned long long)(prefix + tot), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      sprefix = prefix;
      if (bid == live - 1) {
        if (total64) *total64 = (long long)(prefix + tot);
        if (total32) *total32 = (int)(prefix + tot);
      }
    }
  }
  __syncthreads();
  T run = ex + sprefix;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const long long i = base + j;
    if (i < len) out[i] = run;
    run += v[j];
  }
}

__global__ void k_zero_words(unsigned long long *p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// ------------------------------------------------------------ radix sort --
__global__ __launch_bounds__(kBlock) void k_radix_hist(const unsigned long long *keys, int n, int shift,
                                                       int *hist, int nb) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kSortTile;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    long long i = base + (long long)j * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(const unsigned long long *kin, const unsigned *vin,
                                                          unsigned long long *kout, unsigned *vout, int n,
                                                          int shift, const int *offs, int nb) {
  __shared__ int run[256];
  __shared__ int wcnt[kNW][256];
  run[threadIdx.x] = offs[threadIdx.x * nb + blockIdx.x];
  const int wid = threadIdx.x / kWave;
  const unsigned long long lt = lanemask_lt();
  const long long base = (long long)blockIdx.x * kSortTile;
  for (int j = 0; j < kSortItems; ++j) {
    const long long i = base + (long long)j * kBlock + threadIdx.x;
    const bool valid = i < n;
    unsigned long long key = 0;
    unsigned val = 0;
    int dig = 256;  // invalid lanes form their own group
    if (valid) {
      key = kin[i];
      val = vin[i];
      dig = (int)((key >> shift) & 255u);
    }
    unsigned long long mask = ~0ull;
#pragma unroll
    for (int b = 0; b < 9; ++b) {
      const bool bit = (dig >> b) & 1;
      const unsigned long long bal = __ballot(bit);
      mask &= bit ? bal : ~bal;
    }
    const int rank = __popcll(mask & lt);
#pragma unroll
    for (int w = 0; w < kNW; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    if (valid && rank == 0) wcnt[wid][dig] = __popcll(mask);
    __syncthreads();
    if (valid) {
      int pre = 0;
      for (int w = 0; w < wid; ++w) pre += wcnt[w][dig];
      const int dst = run[dig] + pre + rank;
      kout[dst] = key;
      vout[dst] = val;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int w = 0; w < kNW; ++w) add += wcnt[w][threadIdx.x];
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

inline int blocks_for(long long n, int tile) { return (int)((n + tile - 1) / tile); }

// Short scans (at most kSingleScan elements): one block walks the tiles in
// order, so a scan costs one launch instead of three (late rounds are short).
constexpr int kSingleScan = 4 * kScanTile;

template <class T>
__global__ __launch_bounds__(kBlock) void k_scan_single(const T *in, T *out, int nmax, const int *dlen,
                                                        long long *total64, int *total32) {
  const int len = scan_len<T>(nmax, dlen);
  T carry = 0;
  for (int b0 = 0; b0 < len; b0 += kScanTile) {
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int i = b0 + threadIdx.x * kScanItems + j;
      v[j] = i < len ? in[i] : (T)0;
      s += v[j];
    }
    T tot;
    const T ex = block_exclusive_scan<T>(s, tot);
    T run = carry + ex;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int i = b0 + threadIdx.x * kScanItems + j;
      if (i < len) out[i] = run;
      run += v[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    if (total64) *total64 = (long long)carry;
    if (total32) *total32 = (int)carry;
  }
}

}  // namespace

void scan_ws_carve(ScanWs &ws, long long *base, long long words, int *err) {
  ws.cap = (int)std::min<long long>((words - 1) / 2, 0x7fffffffLL);
  ws.st[0] = (unsigned long long *)base;
  ws.st[1] = ws.st[0] + ws.cap;
  ws.ticket = (int *)(ws.st[1] + ws.cap);
  ws.turn = 0;
  ws.fresh = 1;
  ws.err = err;
}

// Launches one scan: a single block for short ones, else the look-back scan.
template <class T>
static void scan_exclusive(const T *in, T *out, int nmax, const int *dlen, long long *dtotal64, int *dtotal32,
                           ScanWs &ws, hipStream_t s) {
  if (nmax <= kSingleScan) {
    k_scan_single<T><<<1, kBlock, 0, s>>>(in, out, nmax, dlen, dtotal64, dtotal32);
    return;
  }
  if (ws.fresh) {
    // both status arrays and the tickets start at zero
    k_zero_words<<<64, kBlock, 0, s>>>(ws.st[0], 2LL * ws.cap + 1);
    ws.fresh = 0;
  }
  const int nb = blocks_for(nmax, kScanTile);
  if (nb > ws.cap) {
    // (the workspace is sized for the longest scan; one block is slow but safe)
    k_scan_single<T><<<1, kBlock, 0, s>>>(in, out, nmax, dlen, dtotal64, dtotal32);
    return;
  }
  const int a = ws.turn;
  ws.turn ^= 1;
  k_scan_lb<T><<<nb, kBlock, 0, s>>>(in, out, nmax, dlen, ws.st[a], ws.ticket + a, ws.st[a ^ 1],
                                     ws.ticket + (a ^ 1), ws.cap, dtotal64, dtotal32, ws.err);
}

void scan_exclusive_i32(const int *in, int *out, int nmax, const int *dlen, int *dtotal, ScanWs &ws,
                        hipStream_t s) {
  if (nmax <= 0) {
    if (dtotal) hipMemsetAsync(dtotal, 0, sizeof(int), s);
    return;
  }
  scan_exclusive<int>(in, out, nmax, dlen, nullptr, dtotal, ws, s);
}

void scan_exclusive_i64(const long long *in, long long *out, int nmax, const int *dlen,
                        long long *dtotal, ScanWs &ws, hipStream_t s) {
  if (nmax <= 0) {
    if (dtotal) hipMemsetAsync(dtotal, 0, sizeof(long long), s);
    return;
  }
  scan_exclusive<long long>(in, out, nmax, dlen, dtotal, nullptr, ws, s);
}

int radix_hist_len(int n) { return 256 * blocks_for(n > 0 ? n : 1, kSortTile); }

void radix_sort_pairs(unsigned long long *&k0, unsigned long long *&k1, unsigned *&v0, unsigned *&v1,
                      int n, int bits, int *hist, ScanWs &ws, hipStream_t s) {
  if (n <= 1) return;
  const int nb = blocks_for(n, kSortTile);
  for (int shift = 0; shift < bits; shift += 8) {
    k_radix_hist<<<nb, kBlock, 0, s>>>(k0, n, shift, hist, nb);
    scan_exclusive_i32(hist, hist, 256 * nb, nullptr, nullptr, ws, s);
    k_radix_scatter<<<nb, kBlock, 0, s>>>(k0, v0, k1, v1, n, shift, hist, nb);
    unsigned long long *tk = k0;
    k0 = k1;
    k1 = tk;
    unsigned *tv = v0;
    v0 = v1;
    v1 = tv;
  }
}

}  // namespace pc
