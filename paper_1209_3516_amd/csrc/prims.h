// Device-wide building blocks of the GPU tree build, traversal and work plan:
// an exclusive prefix sum and a stable least-significant-digit radix sort,
// written for 64-lane waves.  Included by the .hip files that use them.
//
// Scan (reduce, then scan): the input is cut into tiles of kTile items, one
// 256-thread block per tile.  (1) each block reduces its tile into partial[b];
// (2) one block scans the partials in place (exclusive) and writes the grand
// total; (3) each block scans its tile and adds partial[b].  Inputs and
// outputs are functors, so a caller can compute the summands on the fly and
// consume the offsets without staging them: load(i) -> T, store(i, offset,
// value).  T is any type with + and a zero from T{} (integers, or small
// structs of integers); integer sums do not depend on the order, so the
// result is exact and reproducible.
//
// Radix sort: 8-bit digits from begin_bit up to end_bit, one pass per digit,
// each pass (a) a per-tile histogram of the digit, (b) an exclusive scan of
// the histograms in digit-major order (every tile's offset for every digit),
// (c) a stable scatter: each wave of a tile ranks its keys 64 at a time in
// input order (the lanes holding the same digit are found with eight
// ballots; the lowest of them advances the wave's counter of that digit),
// then the waves' counters give every wave its place within the tile.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace fmmlib {
namespace dev {
namespace prims {

constexpr int kThreads = 256;  // 4 waves
constexpr int kItems = 8;      // items per thread
constexpr int kTile = kThreads * kItems;
constexpr int kWaves = kThreads / 64;

inline unsigned tiles_for(int64_t n) { return (unsigned)((n + kTile - 1) / kTile); }

// __shfl_up of any summand: arithmetic types directly, structs 32 bits at a time.
template <typename T>
__device__ __forceinline__ T shfl_up_any(T v, int d) {
  if constexpr (std::is_arithmetic<T>::value) {
    return __shfl_up(v, d);
  } else {
    static_assert(sizeof(T) % 4 == 0, "summand size");
    T r;
    const int32_t *src = reinterpret_cast<const int32_t *>(&v);
    int32_t *dst = reinterpret_cast<int32_t *>(&r);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = __shfl_up(src[k], d);
    return r;
  }
}

// Exclusive scan of one value per thread over a 256-thread block, in thread
// order; *total gets the block's sum.  `sh` holds kWaves + 1 values.
template <typename T>
__device__ __forceinline__ T block_exclusive_any(T v, T *sh, T *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T u = shfl_up_any(incl, d);
    if (lane >= d) incl = incl + u;
  }
  // exclusive within the wave: the inclusive value of the lane below
  T excl = shfl_up_any(incl, 1);
  if (lane == 0) excl = T{};
  if (lane == 63) sh[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run{};
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const T t = sh[w];
      sh[w] = run;
      run = run + t;
    }
    sh[kWaves] = run;
  }
  __syncthreads();
  const T out = sh[wave] + excl;
  *total = sh[kWaves];
  __syncthreads();
  return out;
}

// (1) partial[b] = sum of tile b.
template <typename T, class Load>
__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(int64_t n, Load load, T *partial) {
  __shared__ T sh[kWaves + 1];
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  T s{};
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    if (base + k < n) s = s + load(base + k);
  T tot;
  (void)block_exclusive_any(s, sh, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// (2) exclusive scan of partial[0, nb) in place by one block; *total = sum.
template <typename T>
__global__ __launch_bounds__(kThreads) void scan_partials_kernel(int64_t nb, T *partial, T *total) {
  __shared__ T sh[kWaves + 1];
  T run{};
  for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
    const int64_t b = b0 + threadIdx.x;
    const T v = b < nb ? partial[b] : T{};
    T tot;
    const T ex = block_exclusive_any(v, sh, &tot);
    if (b < nb) partial[b] = run + ex;
    run = run + tot;
  }
  if (total && threadIdx.x == 0) *total = run;
}

// (3) each block scans its tile and adds its partial offset.  With
// nb == 1 and partial == nullptr this is the whole scan of a small input
// (and *total, if given, gets the sum).
template <typename T, class Load, class Store>
__global__ __launch_bounds__(kThreads) void scan_apply_kernel(int64_t n, Load load, Store store,
                                                              const T *partial, T *total) {
  __shared__ T sh[kWaves + 1];
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  T v[kItems];
  T s{};
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    v[k] = base + k < n ? load(base + k) : T{};
    s = s + v[k];
  }
  T tot;
  T off = block_exclusive_any(s, sh, &tot);
  if (partial) off = off + partial[blockIdx.x];
  else if (total && threadIdx.x == 0) *total = tot;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (base + k < n) store(base + k, off, v[k]);
    off = off + v[k];
  }
}

// Bytes of scratch an exclusive scan of n items needs (the tile partials).
template <typename T>
inline size_t scan_scratch_bytes(int64_t n) {
  return (size_t)(n > kTile ? tiles_for(n) : 1) * sizeof(T);
}

// Exclusive scan of load(0..n) into store(i, offset, value); the grand total
// goes to *total_dev (device memory) when it is not null.  partial_dev holds
// scan_scratch_bytes<T>(n) bytes.  Enqueues 1 kernel (n <= kTile) or 3.
template <typename T, class Load, class Store>
hipError_t exclusive_scan(int64_t n, Load load, Store store, T *partial_dev, T *total_dev,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n <= kTile) {
    scan_apply_kernel<T><<<1, kThreads, 0, st>>>(n, load, store, (const T *)nullptr, total_dev);
    return hipGetLastError();
  }
  const unsigned nb = tiles_for(n);
  scan_reduce_kernel<T><<<nb, kThreads, 0, st>>>(n, load, partial_dev);
  scan_partials_kernel<T><<<1, kThreads, 0, st>>>((int64_t)nb, partial_dev, total_dev);
  scan_apply_kernel<T><<<nb, kThreads, 0, st>>>(n, load, store, (const T *)partial_dev,
                                                (T *)nullptr);
  return hipGetLastError();
}

// Plain array loaders and storers.
template <typename T, typename In>
struct LoadArray {
  const In *p;
  __device__ T operator()(int64_t i) const { return T(p[i]); }
};
template <typename T, typename Out>
struct StoreArray {
  Out *p;
  __device__ void operator()(int64_t i, T off, T) const { p[i] = Out(off); }
};

// ----------------------------------------------------------------------------
// Radix sort
// ----------------------------------------------------------------------------
// Lanes of the wave whose digit equals this lane's (among the lanes with
// `in` set): eight ballots.
__device__ __forceinline__ uint64_t digit_peers(int d, bool in) {
  uint64_t peers = __ballot(in);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const uint64_t set = __ballot((d >> bit) & 1);
    peers &= ((d >> bit) & 1) ? set : ~set;
  }
  return peers;
}

// hist[d * nb + b] = number of keys of tile b whose digit is d.  Each wave
// counts 64 keys at a time; the lowest lane of each digit adds its peers.
template <typename K>
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const K *__restrict__ keys, int64_t n,
                                                              int shift, int32_t *__restrict__ hist,
                                                              unsigned nb) {
  __shared__ int32_t cnt[256];
  const int lane = threadIdx.x & 63;
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    const bool in = i < n;
    const int d = in ? (int)((keys[i] >> shift) & 0xff) : 0;
    const uint64_t peers = digit_peers(d, in);
    if (in && __builtin_ctzll(peers | (1ull << 63)) == lane) atomicAdd(&cnt[d], __popcll(peers));
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one digit; with HAS_V the int32 values move with the keys.
// Every key gets its place within the tile (tile order: by digit, then by
// input position); the tile is reordered in LDS and written back in that
// order, so consecutive threads write consecutive places of a digit's run.
template <typename K, bool HAS_V>
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(
    const K *__restrict__ keys, const int32_t *__restrict__ vals, int64_t n, int shift,
    const int32_t *__restrict__ offs, unsigned nb, K *__restrict__ keys_out,
    int32_t *__restrict__ vals_out) {
  __shared__ int32_t cnt[kWaves][256];
  __shared__ int32_t start[256];  // first place of each digit within the tile
  __shared__ int32_t gbase[256];  // first global place of each digit of the tile
  __shared__ K skey[kTile];
  __shared__ int32_t sval[HAS_V ? kTile : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int w = 0; w < kWaves; ++w) cnt[w][threadIdx.x] = 0;
  gbase[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
  __syncthreads();
  // wave w ranks the keys [base, base + 64 kItems) of the tile, 64 at a time
  const int64_t tile0 = (int64_t)blockIdx.x * kTile;
  const int64_t base = tile0 + (int64_t)wave * (64 * kItems);
  const int64_t n_tile = n - tile0 < kTile ? n - tile0 : kTile;
  const uint64_t below = (1ull << lane) - 1ull;
  K key[kItems];
  int32_t val[kItems];
  int rank[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + (int64_t)k * 64 + lane;
    const bool in = i < n;
    key[k] = in ? keys[i] : K(0);
    if constexpr (HAS_V) val[k] = in ? vals[i] : 0;
    const int d = (int)((key[k] >> shift) & 0xff);
    const uint64_t peers = digit_peers(d, in);
    const int before = cnt[wave][d];
    rank[k] = before + __popcll(peers & below);
    if (in && __builtin_ctzll(peers | (1ull << 63)) == lane) cnt[wave][d] = before + __popcll(peers);
  }
  __syncthreads();
  // each wave's first place per digit within the digit's part of the tile,
  // and the tile's digit totals
  int tot;
  {
    const int d = threadIdx.x;
    int run = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const int t = cnt[w][d];
      cnt[w][d] = run;
      run += t;
    }
    tot = run;
  }
  {
    int all;
    const int ex = block_exclusive_any(tot, start, &all);  // (start[] is scratch here)
    start[threadIdx.x] = ex;
  }
  __syncthreads();
  // reorder the tile in LDS
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + (int64_t)k * 64 + lane;
    if (i < n) {
      const int d = (int)((key[k] >> shift) & 0xff);
      const int lp = start[d] + cnt[wave][d] + rank[k];
      skey[lp] = key[k];
      if constexpr (HAS_V) sval[lp] = val[k];
    }
  }
  __syncthreads();
  // write the tile back in place order
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int lp = k * kThreads + threadIdx.x;
    if (lp < n_tile) {
      const K kk = skey[lp];
      const int d = (int)((kk >> shift) & 0xff);
      const int64_t pos = (int64_t)gbase[d] + (lp - start[d]);
      keys_out[pos] = kk;
      if constexpr (HAS_V) vals_out[pos] = sval[lp];
    }
  }
}

// Scratch (bytes) of radix_sort for n keys: the histograms and their scan.
inline size_t radix_scratch_bytes(int64_t n) {
  const size_t h = (size_t)256 * tiles_for(n > 0 ? n : 1);
  return 2 * h * sizeof(int32_t) + scan_scratch_bytes<int32_t>((int64_t)h) + 64;
}

// Stable sort of keys[0, n) (and vals, if not null) by bits [begin_bit,
// end_bit), ping-ponging with keys_alt / vals_alt; *result_in_alt tells
// which buffer holds the result.  n < 2^31.
template <typename K>
hipError_t radix_sort(K *keys, K *keys_alt, int32_t *vals, int32_t *vals_alt, int64_t n,
                      int begin_bit, int end_bit, void *scratch, hipStream_t st,
                      bool *result_in_alt) {
  *result_in_alt = false;
  if (n <= 1 || end_bit <= begin_bit) return hipSuccess;
  const unsigned nb = tiles_for(n);
  const int64_t h = (int64_t)256 * nb;
  int32_t *hist = (int32_t *)scratch;
  int32_t *offs = hist + h;
  int32_t *part = offs + h;
  K *src = keys, *dst = keys_alt;
  int32_t *vs = vals, *vd = vals_alt;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    radix_hist_kernel<K><<<nb, kThreads, 0, st>>>(src, n, shift, hist, nb);
    hipError_t e = exclusive_scan<int32_t>(h, LoadArray<int32_t, int32_t>{hist},
                                           StoreArray<int32_t, int32_t>{offs}, part,
                                           (int32_t *)nullptr, st);
    if (e != hipSuccess) return e;
    if (vals)
      radix_scatter_kernel<K, true><<<nb, kThreads, 0, st>>>(src, vs, n, shift, offs, nb, dst, vd);
    else
      radix_scatter_kernel<K, false><<<nb, kThreads, 0, st>>>(src, nullptr, n, shift, offs, nb,
                                                              dst, nullptr);
    K *tk = src;
    src = dst;
    dst = tk;
    int32_t *tv = vs;
    vs = vd;
    vd = tv;
    *result_in_alt = !*result_in_alt;
  }
  return hipGetLastError();
}

}  // namespace prims
}  // namespace dev
}  // namespace fmmlib
