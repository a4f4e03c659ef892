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

template <class T>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const T *in, int nmax, const int *dlen,
                                                        long long *part) {
  const int len = scan_len<T>(nmax, dlen);
  const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  T s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    long long i = base + j;
    if (i < len) s += in[i];
  }
  T tot;
  block_exclusive_scan<T>(s, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = (long long)tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_partials(long long *part, int nb, long long *total64,
                                                          int *total32) {
  long long carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kScanTile) {
    long long v[kScanItems];
    long long s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      int i = b0 + threadIdx.x * kScanItems + j;
      v[j] = (i < nb) ? part[i] : 0;
      s += v[j];
    }
    long long tot;
    long long ex = block_exclusive_scan<long long>(s, tot);
    long long run = carry + ex;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      int i = b0 + threadIdx.x * kScanItems + j;
      if (i < nb) part[i] = run;
      run += v[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    if (total64) *total64 = carry;
    if (total32) *total32 = (int)carry;
  }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_scan_down(const T *in, T *out, int nmax, const int *dlen,
                                                      const long long *part) {
  const int len = scan_len<T>(nmax, dlen);
  const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    long long i = base + j;
    v[j] = (i < len) ? in[i] : (T)0;
    s += v[j];
  }
  T tot;
  T run = block_exclusive_scan<T>(s, tot) + (T)part[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    long long i = base + j;
    if (i < len) out[i] = run;
    run += v[j];
  }
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

void scan_exclusive_i32(const int *in, int *out, int nmax, const int *dlen, int *dtotal,
                        long long *part, hipStream_t s) {
  if (nmax <= 0) {
    if (dtotal) hipMemsetAsync(dtotal, 0, sizeof(int), s);
    return;
  }
  if (nmax <= kSingleScan) {
    k_scan_single<int><<<1, kBlock, 0, s>>>(in, out, nmax, dlen, nullptr, dtotal);
    return;
  }
  const int nb = blocks_for(nmax, kScanTile);
  k_scan_reduce<int><<<nb, kBlock, 0, s>>>(in, nmax, dlen, part);
  k_scan_partials<<<1, kBlock, 0, s>>>(part, nb, nullptr, dtotal);
  k_scan_down<int><<<nb, kBlock, 0, s>>>(in, out, nmax, dlen, part);
}

void scan_exclusive_i64(const long long *in, long long *out, int nmax, const int *dlen,
                        long long *dtotal, long long *part, hipStream_t s) {
  if (nmax <= 0) {
    if (dtotal) hipMemsetAsync(dtotal, 0, sizeof(long long), s);
    return;
  }
  if (nmax <= kSingleScan) {
    k_scan_single<long long><<<1, kBlock, 0, s>>>(in, out, nmax, dlen, dtotal, nullptr);
    return;
  }
  const int nb = blocks_for(nmax, kScanTile);
  k_scan_reduce<long long><<<nb, kBlock, 0, s>>>(in, nmax, dlen, part);
  k_scan_partials<<<1, kBlock, 0, s>>>(part, nb, dtotal, nullptr);
  k_scan_down<long long><<<nb, kBlock, 0, s>>>(in, out, nmax, dlen, part);
}

int radix_hist_len(int n) { return 256 * blocks_for(n > 0 ? n : 1, kSortTile); }

void radix_sort_pairs(unsigned long long *&k0, unsigned long long *&k1, unsigned *&v0, unsigned *&v1,
                      int n, int bits, int *hist, long long *part, hipStream_t s) {
  if (n <= 1) return;
  const int nb = blocks_for(n, kSortTile);
  for (int shift = 0; shift < bits; shift += 8) {
    k_radix_hist<<<nb, kBlock, 0, s>>>(k0, n, shift, hist, nb);
    scan_exclusive_i32(hist, hist, 256 * nb, nullptr, nullptr, part, s);
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
