// Dual tree traversal on the GPU (section 3.3, Algorithms 3 and 4), with the
// same rules as the host traversal (traverse.cpp), so the lists are identical
// bit for bit:
//  * MAC: (theta*theta) * ((dx*dx + dy*dy) + dz*dz) > (B_A + B_B)^2 in FP64
//    (this file is compiled without FMA contraction);
//  * MAC-first or leaf-first; a self pair splits into all child pairs; a
//    pair of distinct cells splits the larger radius (tie: lower number),
//    never a leaf; start at (root, root).
// The traversal is level-synchronous: every pair of the current frontier is
// classified (M2L, P2P or split) independently; exclusive scans place the
// child pairs of the next frontier and the emitted pairs.  The emitted pairs
// are sorted as integer keys (target << kb | source), kb = bits of a cell
// number, which is the canonical CSR order (rows = targets, sources
// ascending); the radix sort looks at the 2 kb low bits only, and the keys
// are 32-bit when 2 kb <= 32.  Scans and sorts are the ones of prims.h.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <memory>
#include <mutex>
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "kernels.h"
#include "prims.h"

namespace fmmlib {
namespace dev {
namespace {

inline hipStream_t S_(void *s) { return reinterpret_cast<hipStream_t>(s); }
inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

enum Action { kActM2L = 0, kActP2P = 1, kActSplitBoth = 2, kActSplitA = 3, kActSplitB = 4 };

__device__ __forceinline__ int classify(int a, int b, const double4 *__restrict__ geo,
                                        const int32_t *__restrict__ n_child, double theta2,
                                        bool leaf_first, int *n_out) {
  const double4 A = geo[a], B = geo[b];
  const bool la = n_child[a] == 0, lb = n_child[b] == 0;
  const double dx = A.x - B.x, dy = A.y - B.y, dz = A.z - B.z;
  const double d2 = (dx * dx + dy * dy) + dz * dz;
  const double s = A.w + B.w;
  const bool mac = theta2 * d2 > s * s;
  *n_out = 0;
  if (!leaf_first && mac) return kActM2L;
  if (la && lb) return kActP2P;
  if (leaf_first && mac) return kActM2L;
  if (a == b) {
    *n_out = n_child[a] * n_child[a];
    return kActSplitBoth;
  }
  bool split_a = A.w > B.w || (A.w == B.w && a < b);
  if (split_a && la) split_a = false;
  if (!split_a && lb) split_a = true;
  *n_out = split_a ? n_child[a] : n_child[b];
  return split_a ? kActSplitA : kActSplitB;
}

// Per frontier pair: child pairs it creates, emitted lists ((M2L << 32) |
// P2P, one of them 1 or both 0) and its action.  The scan of a level sums the
// first two over the frontier (the action field's sum means nothing).
struct PairCount {
  int64_t children;
  uint64_t emit;
  int64_t act;
  __device__ PairCount operator+(const PairCount &o) const {
    return PairCount{children + o.children, emit + o.emit, act + o.act};
  }
};

static_assert(sizeof(PairCount) <= 4 * sizeof(int64_t), "level totals fit the pinned block");

struct ClassifyPair {
  const int2 *frontier;
  const double4 *geo;
  const int32_t *n_child;
  double theta2;
  int leaf_first;
  __device__ PairCount operator()(int64_t i) const {
    const int2 pr = frontier[i];
    int n;
    const int act = classify(pr.x, pr.y, geo, n_child, theta2, leaf_first != 0, &n);
    return PairCount{n, act == kActM2L ? (1ull << 32) : (act == kActP2P ? 1ull : 0ull), act};
  }
};

// Writes the pair's child pairs into the next frontier, or its list entry
// (key target << kb | source), at the offsets the scan gives it.
template <typename K>
struct ExpandPair {
  const int2 *frontier;
  const int32_t *n_child, *child_begin;
  int2 *next;
  K *p2p_keys, *m2l_keys;
  int64_t p2p_base, m2l_base;
  int kb;
  __device__ void operator()(int64_t i, PairCount off, PairCount v) const {
    const int2 pr = frontier[i];
    const int a = pr.x, b = pr.y;
    const K key = ((K)(uint32_t)a << kb) | (K)(uint32_t)b;
    if (v.act == kActM2L) {
      m2l_keys[m2l_base + (int64_t)(off.emit >> 32)] = key;
    } else if (v.act == kActP2P) {
      p2p_keys[p2p_base + (int64_t)(off.emit & 0xffffffffull)] = key;
    } else {
      int2 *out = next + off.children;
      const int n = (int)v.children;
      if (v.act == kActSplitBoth) {
        const int c0 = child_begin[a], nc = n_child[a];
        for (int x = 0; x < nc; ++x)
          for (int y = 0; y < nc; ++y) out[x * nc + y] = make_int2(c0 + x, c0 + y);
      } else if (v.act == kActSplitA) {
        const int c0 = child_begin[a];
        for (int x = 0; x < n; ++x) out[x] = make_int2(c0 + x, b);
      } else {
        const int c0 = child_begin[b];
        for (int y = 0; y < n; ++y) out[y] = make_int2(a, c0 + y);
      }
    }
  }
};

// CSR from sorted keys: row_ptr[r] = first key with target >= r.
template <typename K>
__global__ void csr_rows(int64_t n_rows, const K *__restrict__ keys, int64_t nnz, int kb,
                         int64_t *__restrict__ row_ptr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > n_rows) return;
  // (row n_rows may not fit the key type: every key is below it)
  if (r == n_rows) {
    row_ptr[r] = nnz;
    return;
  }
  const K want = (K)r << kb;
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < want)
      lo = mid + 1;
    else
      hi = mid;
  }
  row_ptr[r] = lo;
}

template <typename K>
__global__ void csr_cols(int64_t nnz, const K *__restrict__ keys, int kb,
                         int32_t *__restrict__ col) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnz) col[i] = (int32_t)(keys[i] & (((K)1 << kb) - 1));
}

// Growable scratch buffer from the device's stream-ordered memory pool:
// hipFreeAsync hands the memory back in stream order, without a device
// synchronisation, and later builds and traversals reuse it from the pool.
struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
  hipStream_t st = nullptr;
  hipError_t reserve(size_t want, hipStream_t s, bool keep) {
    if (want <= bytes) return hipSuccess;
    size_t nb = bytes ? bytes : 1024;
    while (nb < want) nb *= 2;
    void *np = nullptr;
    hipError_t e = hipMallocAsync(&np, nb, s);
    if (e != hipSuccess) return e;
    if (keep && p) {
      e = hipMemcpyAsync(np, p, bytes, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) {
        (void)hipFreeAsync(np, s);
        return e;
      }
    }
    // stream order: the kernels that still read the old buffer come first
    if (p) (void)hipFreeAsync(p, st);
    p = np;
    bytes = nb;
    st = s;
    return hipSuccess;
  }
  ~Buf() {
    if (p) (void)hipFreeAsync(p, st);
  }
};

// A few values that kernels write straight into pinned host memory (mapped
// into the device's address space) and the host reads after a stream
// synchronisation; allocated once per owner.
struct Pinned {
  int64_t *p = nullptr;
  hipError_t get() {
    return p ? hipSuccess : hipHostMalloc((void **)&p, 4 * sizeof(int64_t), hipHostMallocMapped);
  }
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};

// A growable pinned host block that device-to-host copies land in
// asynchronously (a copy to pageable memory is staged and waited for one at
// a time); kept with the build's scratch, so later builds reuse it.
struct PinnedStage {
  void *p = nullptr;
  size_t bytes = 0;
  hipError_t reserve(size_t want) {
    if (want <= bytes) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    const hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e == hipSuccess) bytes = want;
    return e;
  }
  ~PinnedStage() {
    if (p) (void)hipHostFree(p);
  }
};

#define TRY(x)                             \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) return (int)e_;  \
  } while (0)

}  // namespace

int build_stream(void *user, void **out) {
  static std::mutex mu;
  static hipStream_t streams[kMaxDevices] = {};
  static hipEvent_t events[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(mu);
  if (!streams[dev]) {
    // default priority, not synchronised with the legacy null stream
    e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
    if (e != hipSuccess) return (int)e;
    e = hipEventCreateWithFlags(&events[dev], hipEventDisableTiming);
    if (e != hipSuccess) return (int)e;
  }
  e = hipEventRecord(events[dev], S_(user));
  if (e == hipSuccess) e = hipStreamWaitEvent(streams[dev], events[dev], 0);
  if (e != hipSuccess) return (int)e;
  *out = (void *)streams[dev];
  return 0;
}

int keep_pool_memory() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  hipMemPool_t pool;
  e = hipDeviceGetDefaultMemPool(&pool, dev);
  if (e != hipSuccess) return (int)e;
  uint64_t keep = kPoolKeepBytes;
  return (int)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
}

namespace {

template <typename K>
int sort_to_csr(K *keys, int64_t nnz, int64_t n_rows, int kb, hipStream_t st, Buf &alt,
                Buf &temp, int64_t *row_ptr_dev, int32_t *col_dev) {
  if (nnz > 0) {
    TRY(alt.reserve(nnz * sizeof(K), st, false));
    TRY(temp.reserve(prims::radix_scratch_bytes(nnz), st, false));
    bool in_alt = false;
    TRY(prims::radix_sort<K>(keys, (K *)alt.p, nullptr, nullptr, nnz, 0, 2 * kb, temp.p, st,
                             &in_alt));
    const K *sorted = in_alt ? (const K *)alt.p : keys;
    csr_rows<K><<<blocks_for(n_rows + 1, 256), 256, 0, st>>>(n_rows, sorted, nnz, kb, row_ptr_dev);
    csr_cols<K><<<blocks_for(nnz, 256), 256, 0, st>>>(nnz, sorted, kb, col_dev);
  } else {
    TRY(hipMemsetAsync(row_ptr_dev, 0, (n_rows + 1) * sizeof(int64_t), st));
  }
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tree build on the GPU (section 3.3; same rules as tree.cpp, same FP64
// expressions, no FMA contraction):
//   bounding box -> Morton keys -> stable radix sort of (key, index) ->
//   level-by-level split of cells with more than ncrit bodies into their
//   non-empty octants (breadth-first numbering) -> per-cell bounding box
//   centre and radius.
// ---------------------------------------------------------------------------
struct Box {
  double lo[3], hi[3];
  int finite, exact;
};

__global__ void bbox_partial(int64_t n, const double *__restrict__ xyz, Box *__restrict__ out) {
  __shared__ double slo[3][256], shi[3][256];
  __shared__ int sf[256], se[256];
  double lo[3], hi[3];
  int fin = 1, ex = 1;
  for (int d = 0; d < 3; ++d) {
    lo[d] = __builtin_inf();
    hi[d] = -__builtin_inf();
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    for (int d = 0; d < 3; ++d) {
      const double v = xyz[3 * i + d];
      if (!__builtin_isfinite(v)) fin = 0;
      if ((double)(float)v != v) ex = 0;
      lo[d] = v < lo[d] ? v : lo[d];
      hi[d] = v > hi[d] ? v : hi[d];
    }
  const int t = threadIdx.x;
  for (int d = 0; d < 3; ++d) {
    slo[d][t] = lo[d];
    shi[d][t] = hi[d];
  }
  sf[t] = fin;
  se[t] = ex;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      for (int d = 0; d < 3; ++d) {
        slo[d][t] = slo[d][t + h] < slo[d][t] ? slo[d][t + h] : slo[d][t];
        shi[d][t] = shi[d][t + h] > shi[d][t] ? shi[d][t + h] : shi[d][t];
      }
      sf[t] &= sf[t + h];
      se[t] &= se[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    Box b;
    for (int d = 0; d < 3; ++d) {
      b.lo[d] = slo[d][0];
      b.hi[d] = shi[d][0];
    }
    b.finite = sf[0];
    b.exact = se[0];
    out[blockIdx.x] = b;
  }
}

__device__ __forceinline__ uint64_t dilate3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x001f00000000ffffull;
  v = (v | (v << 16)) & 0x001f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__global__ void morton_keys(int64_t n, const double *__restrict__ xyz, double bx, double by,
                            double bz, double width, int degenerate, uint64_t *__restrict__ key,
                            int32_t *__restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  idx[i] = (int32_t)i;
  if (degenerate) {
    key[i] = 0;
    return;
  }
  const double base[3] = {bx, by, bz};
  uint64_t k = 0;
  for (int d = 0; d < 3; ++d) {
    double s = floor((xyz[3 * i + d] - base[d]) / width * 2097152.0);
    s = s < 0.0 ? 0.0 : (s > 2097151.0 ? 2097151.0 : s);
    k |= dilate3((uint64_t)s) << d;
  }
  key[i] = k;
}

__global__ void gather_positions(int64_t n, const double *__restrict__ xyz,
                                 const int32_t *__restrict__ perm, double *__restrict__ pos) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t u = perm[i];
  for (int d = 0; d < 3; ++d) pos[3 * i + d] = xyz[3 * u + d];
}

// Morton-ordered FP64 positions -> (x, y, z, 0) bodies; FP32 rounds to
// nearest, as the host packing does.
__global__ void pack_f32(int64_t n, const double *__restrict__ pos, float4 *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  b[i] = make_float4((float)pos[3 * i], (float)pos[3 * i + 1], (float)pos[3 * i + 2], 0.0f);
}
__global__ void pack_f64(int64_t n, const double *__restrict__ pos, double4 *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  b[i] = make_double4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], 0.0);
}

// Octant boundaries of cell c at level L: bodies [b0, b1) have sorted keys,
// so each octant digit is a contiguous range, found by binary search.
__device__ __forceinline__ int64_t digit_bound(const uint64_t *__restrict__ keys, int64_t lo,
                                               int64_t hi, int shift, int oct) {
  while (lo < hi) {  // first position whose digit > oct
    const int64_t mid = (lo + hi) >> 1;
    if ((int)((keys[mid] >> shift) & 7u) <= oct)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ void count_children(int64_t c0, int64_t c1, int level, int ncrit, int splittable,
                               const uint64_t *__restrict__ keys,
                               const int64_t *__restrict__ body_begin,
                               const int64_t *__restrict__ n_body, int32_t *__restrict__ nch) {
  const int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  int count = 0;
  if (splittable && n_body[c] > ncrit && level < 21) {
    const int shift = 3 * (20 - level);
    int64_t prev = body_begin[c];
    const int64_t end = prev + n_body[c];
    for (int oct = 0; oct < 8; ++oct) {
      const int64_t b = digit_bound(keys, prev, end, shift, oct);
      count += b > prev;
      prev = b;
    }
  }
  nch[c - c0] = count;
}

__global__ void write_children(int64_t c0, int64_t c1, int level, const uint64_t *__restrict__ keys,
                               const int32_t *__restrict__ nch, const int32_t *__restrict__ off,
                               int64_t next_base, int64_t *__restrict__ body_begin,
                               int64_t *__restrict__ n_body, int32_t *__restrict__ lev,
                               int32_t *__restrict__ parent, int32_t *__restrict__ child_begin,
                               int32_t *__restrict__ n_child) {
  const int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  const int k = nch[c - c0];
  n_child[c] = k;
  child_begin[c] = k ? (int32_t)(next_base + off[c - c0]) : 0;
  if (!k) return;
  const int shift = 3 * (20 - level);
  int64_t prev = body_begin[c];
  const int64_t end = prev + n_body[c];
  int64_t out = next_base + off[c - c0];
  for (int oct = 0; oct < 8; ++oct) {
    const int64_t b = digit_bound(keys, prev, end, shift, oct);
    if (b > prev) {
      body_begin[out] = prev;
      n_body[out] = b - prev;
      lev[out] = level + 1;
      parent[out] = (int32_t)c;
      ++out;
    }
    prev = b;
  }
}

// One 256-thread work-group per cell: tight bounding box of its bodies, its
// middle as the centre, and the largest centre-to-body distance.
// Cell geometry in three passes over chunks of at most kGeoChunk bodies of
// one cell (so the root's million bodies are spread over many blocks):
// bounding box, centre = middle of the box, radius = largest centre-to-body
// distance.  Partial minima and maxima of chunks are combined with 64-bit
// integer atomics on an order-preserving encoding of the doubles, which is
// exact and independent of the order, so the result equals the host's.
constexpr int64_t kGeoChunk = 2048;

__device__ __forceinline__ uint64_t order_key(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double order_value(uint64_t k) {
  return __longlong_as_double((long long)((k >> 63) ? (k & 0x7fffffffffffffffull) : ~k));
}

__global__ void geo_chunk_count(int64_t ncells, const int64_t *__restrict__ n_body,
                                int32_t *__restrict__ nchunk) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncells) nchunk[c] = (int32_t)((n_body[c] + kGeoChunk - 1) / kGeoChunk);
}

// chunk table entry: cell | chunk index << 32; also resets the accumulators
__global__ void geo_chunk_fill(int64_t ncells, const int32_t *__restrict__ nchunk,
                               const int32_t *__restrict__ off, uint64_t *__restrict__ tab,
                               uint64_t *__restrict__ acc) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  for (int32_t k = 0; k < nchunk[c]; ++k) tab[off[c] + k] = (uint64_t)c | ((uint64_t)k << 32);
  for (int d = 0; d < 3; ++d) {
    acc[7 * c + d] = ~0ull;     // lo: min of keys
    acc[7 * c + 3 + d] = 0ull;  // hi: max of keys
  }
  acc[7 * c + 6] = 0ull;        // radius bits (non-negative doubles order as integers)
}

template <int PASS>
__global__ __launch_bounds__(256) void geo_chunk(const double *__restrict__ pos,
                                                 const int64_t *__restrict__ body_begin,
                                                 const int64_t *__restrict__ n_body,
                                                 const uint64_t *__restrict__ tab,
                                                 const double4 *__restrict__ geo,
                                                 uint64_t *__restrict__ acc) {
  __shared__ uint64_t red[6][256];
  const uint64_t e = tab[blockIdx.x];
  const int64_t c = (int64_t)(e & 0xffffffffull), k = (int64_t)(e >> 32);
  const int64_t j0 = k * kGeoChunk;
  const int64_t j1 = n_body[c] < j0 + kGeoChunk ? n_body[c] : j0 + kGeoChunk;
  const double *p = pos + 3 * body_begin[c];
  const int t = threadIdx.x;
  if (PASS == 0) {
    uint64_t lo[3] = {~0ull, ~0ull, ~0ull}, hi[3] = {0ull, 0ull, 0ull};
    for (int64_t j = j0 + t; j < j1; j += 256)
      for (int d = 0; d < 3; ++d) {
        const uint64_t v = order_key(p[3 * j + d]);
        lo[d] = v < lo[d] ? v : lo[d];
        hi[d] = v > hi[d] ? v : hi[d];
      }
    for (int d = 0; d < 3; ++d) {
      red[d][t] = lo[d];
      red[3 + d][t] = hi[d];
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (t < h)
        for (int d = 0; d < 3; ++d) {
          red[d][t] = red[d][t + h] < red[d][t] ? red[d][t + h] : red[d][t];
          red[3 + d][t] = red[3 + d][t + h] > red[3 + d][t] ? red[3 + d][t + h] : red[3 + d][t];
        }
      __syncthreads();
    }
    if (t < 3) atomicMin((unsigned long long *)&acc[7 * c + t], (unsigned long long)red[t][0]);
    else if (t < 6)
      atomicMax((unsigned long long *)&acc[7 * c + t], (unsigned long long)red[t][0]);
  } else {
    const double4 g = geo[c];
    double rmax = 0.0;
    for (int64_t j = j0 + t; j < j1; j += 256) {
      const double dx = p[3 * j] - g.x, dy = p[3 * j + 1] - g.y, dz = p[3 * j + 2] - g.z;
      const double r = sqrt((dx * dx + dy * dy) + dz * dz);
      rmax = r > rmax ? r : rmax;
    }
    red[0][t] = (uint64_t)__double_as_longlong(rmax);
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (t < h) red[0][t] = red[0][t + h] > red[0][t] ? red[0][t + h] : red[0][t];
      __syncthreads();
    }
    if (t == 0) atomicMax((unsigned long long *)&acc[7 * c + 6], (unsigned long long)red[0][0]);
  }
}

// PASS 0: centre from the box (radius 0 for now); PASS 1: radius.
template <int PASS>
__global__ void geo_finish(int64_t ncells, const uint64_t *__restrict__ acc,
                           double4 *__restrict__ geo) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  if (PASS == 0) {
    double X[3];
    for (int d = 0; d < 3; ++d)
      X[d] = 0.5 * (order_value(acc[7 * c + d]) + order_value(acc[7 * c + 3 + d]));
    geo[c] = make_double4(X[0], X[1], X[2], 0.0);
  } else {
    geo[c].w = __longlong_as_double((long long)acc[7 * c + 6]);
  }
}

__global__ void narrow_i64(int64_t n, const int64_t *__restrict__ in, int32_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int32_t)in[i];
}

}  // namespace

int dual_traverse_gpu(int64_t n_cells, const double *geo, const int32_t *child_begin,
                      const int32_t *n_child, double theta, bool leaf_first, void *stream,
                      DeviceLists &out) {
  auto now = [] { return std::chrono::steady_clock::now(); };
  const auto t_entry = now();
  if (int rc = keep_pool_memory()) return rc;
  hipStream_t st;
  if (int rc = build_stream(stream, reinterpret_cast<void **>(&st))) return rc;
  const bool log = std::getenv("FMM_LOG") != nullptr;
  const auto t_start = now();
  if (log)
    std::fprintf(stderr, "[fmm] gpu traversal: set-up %.2f ms\n",
                 std::chrono::duration<double, std::milli>(t_start - t_entry).count());
  int n_levels = 0;
  const double theta2 = theta * theta;
  const double4 *g = (const double4 *)geo;
  out = DeviceLists();
  out.n_rows = n_cells;
  // bits of a cell number: keys (target << kb | source) need 2 kb <= 64 bits
  int kb = 1;
  while (kb < 31 && (int64_t(1) << kb) < n_cells) ++kb;
  // Scratch of the previous traversal on this device is reused (freeing
  // large pool blocks costs milliseconds); at most kKeepScratchBytes are
  // kept between calls.
  struct Scratch {
    Buf front[2], part, temp, p2p, m2l, alt;
    Pinned host;  // the level totals, written there by the scan
    size_t bytes() const {
      return front[0].bytes + front[1].bytes + part.bytes + temp.bytes + p2p.bytes + m2l.bytes +
             alt.bytes;
    }
  };
  // (a heap array that is never destroyed: no HIP call at process exit)
  static std::mutex cache_mu;
  static std::unique_ptr<Scratch> *cache = new std::unique_ptr<Scratch>[kMaxDevices];
  int dev = 0;
  TRY(hipGetDevice(&dev));
  std::unique_ptr<Scratch> sc;
  {
    std::lock_guard<std::mutex> guard(cache_mu);
    if (dev >= 0 && dev < kMaxDevices) sc = std::move(cache[dev]);
  }
  if (!sc) sc.reset(new Scratch);
  Buf(&front)[2] = sc->front;
  Buf &part = sc->part, &temp = sc->temp, &p2p = sc->p2p, &m2l = sc->m2l, &alt = sc->alt;
  TRY(sc->host.get());
  // the device's address of the pinned block (the scan's last phase writes there)
  PairCount *level_total = reinterpret_cast<PairCount *>(sc->host.p);
  PairCount *level_total_dev = nullptr;
  TRY(hipHostGetDevicePointer((void **)&level_total_dev, sc->host.p, 0));
  int64_t nf = n_cells > 0 ? 1 : 0, n_p2p = 0, n_m2l = 0;
  TRY(front[0].reserve(sizeof(int2), st, false));
  if (nf) {
    const int2 root = make_int2(0, 0);
    TRY(hipMemcpyAsync(front[0].p, &root, sizeof(int2), hipMemcpyHostToDevice, st));
  }
  // Counts stay below 2^31 (the sort and the list offsets count in 32 bits);
  // FMM_TRAVERSE_LIMIT lowers the limit so that the failure path can be tested.
  int64_t limit = INT32_MAX;
  if (const char *lim = std::getenv("FMM_TRAVERSE_LIMIT")) {
    const long long v = std::atoll(lim);
    if (v > 0 && v < limit) limit = v;
  }
  auto t_front = now();
  // The levels and the sort, for 32-bit or 64-bit keys.
  auto run = [&]<typename K>(K) -> int {
    int cur = 0;
    while (nf > 0) {
      if (nf > limit) return kTraverseTooLarge;
      // classify and count (scan phases 1 and 2; the level's totals land in
      // pinned host memory), then one synchronisation to size the outputs
      const unsigned nb = prims::tiles_for(nf);
      TRY(part.reserve(nb * sizeof(PairCount), st, false));
      const ClassifyPair load{(const int2 *)front[cur].p, g, n_child, theta2, leaf_first ? 1 : 0};
      prims::scan_reduce_kernel<PairCount><<<nb, prims::kThreads, 0, st>>>(nf, load,
                                                                           (PairCount *)part.p);
      prims::scan_partials_kernel<PairCount><<<1, prims::kThreads, 0, st>>>(
          (int64_t)nb, (PairCount *)part.p, level_total_dev);
      TRY(hipGetLastError());
      TRY(hipStreamSynchronize(st));
      const int64_t n_next = level_total->children;
      const uint64_t e_tot = level_total->emit;
      const int64_t add_p2p = (int64_t)(e_tot & 0xffffffffull), add_m2l = (int64_t)(e_tot >> 32);
      if (n_p2p + add_p2p > limit || n_m2l + add_m2l > limit) return kTraverseTooLarge;
      TRY(front[1 - cur].reserve((n_next > 0 ? n_next : 1) * sizeof(int2), st, false));
      TRY(p2p.reserve((n_p2p + add_p2p + 1) * sizeof(K), st, true));
      TRY(m2l.reserve((n_m2l + add_m2l + 1) * sizeof(K), st, true));
      // phase 3: the offsets place the child pairs and the list entries
      const ExpandPair<K> store{(const int2 *)front[cur].p, n_child, child_begin,
                                (int2 *)front[1 - cur].p, (K *)p2p.p, (K *)m2l.p, n_p2p, n_m2l,
                                kb};
      prims::scan_apply_kernel<PairCount><<<nb, prims::kThreads, 0, st>>>(
          nf, load, store, (const PairCount *)part.p, (PairCount *)nullptr);
      TRY(hipGetLastError());
      n_p2p += add_p2p;
      n_m2l += add_m2l;
      nf = n_next;
      cur = 1 - cur;
      ++n_levels;
    }
    t_front = now();
    TRY(hipMalloc((void **)&out.p2p_ptr, (n_cells + 1) * sizeof(int64_t)));
    TRY(hipMalloc((void **)&out.m2l_ptr, (n_cells + 1) * sizeof(int64_t)));
    TRY(hipMalloc((void **)&out.p2p_col, (n_p2p > 0 ? n_p2p : 1) * sizeof(int32_t)));
    TRY(hipMalloc((void **)&out.m2l_col, (n_m2l > 0 ? n_m2l : 1) * sizeof(int32_t)));
    out.p2p_nnz = n_p2p;
    out.m2l_nnz = n_m2l;
    if (int rc = sort_to_csr<K>((K *)p2p.p, n_p2p, n_cells, kb, st, alt, temp, out.p2p_ptr,
                                out.p2p_col))
      return rc;
    if (int rc = sort_to_csr<K>((K *)m2l.p, n_m2l, n_cells, kb, st, alt, temp, out.m2l_ptr,
                                out.m2l_col))
      return rc;
    return 0;
  };
  const int rc_run = 2 * kb <= 32 ? run(uint32_t{}) : run(uint64_t{});
  if (rc_run) return rc_run;
  TRY(hipStreamSynchronize(st));
  const auto t_end = now();
  if (sc->bytes() <= kKeepScratchBytes && dev >= 0 && dev < kMaxDevices) {
    std::lock_guard<std::mutex> guard(cache_mu);
    if (!cache[dev]) cache[dev] = std::move(sc);
  }
  sc.reset();
  if (log) {
    std::fprintf(stderr, "[fmm] gpu traversal: %d steps %.2f ms, sort+csr %.2f ms, scratch release %.2f ms\n", n_levels,
                 std::chrono::duration<double, std::milli>(t_front - t_start).count(),
                 std::chrono::duration<double, std::milli>(t_end - t_front).count(),
                 std::chrono::duration<double, std::milli>(now() - t_end).count());
  }
  return 0;
}


int pack_positions(bool fp64, int64_t n, const double *pos, void *out, void *stream) {
  if (n <= 0) return 0;
  if (fp64)
    pack_f64<<<blocks_for(n, 256), 256, 0, S_(stream)>>>(n, pos, (double4 *)out);
  else
    pack_f32<<<blocks_for(n, 256), 256, 0, S_(stream)>>>(n, pos, (float4 *)out);
  return (int)hipGetLastError();
}

int build_tree_gpu(const double *xyz, int64_t n, int ncrit, void *stream, DeviceTree &out,
                   TreeData &t, std::string &err) {
  if (int rc = keep_pool_memory()) return rc;
  hipStream_t st;
  if (int rc = build_stream(stream, reinterpret_cast<void **>(&st))) return rc;
  out = DeviceTree();
  t = TreeData();
  t.n = n;
  t.ncrit = ncrit;
  if (n == 0) {
    t.level_begin.assign(1, 0);
    return 0;
  }
  // Scratch of the previous build on this device is reused (as the
  // traversal does; freeing large pool blocks costs milliseconds).
  struct TreeScratch {
    Buf boxes, key, idx, key2, idx2, temp, bb, nbd, lv, par, cb, nc, nch, off, gcnt, goff, gtab,
        gacc, part;
    Pinned host;  // scan totals, written there by the scans
    PinnedStage stage;  // the host copy of the cell arrays passes through here
    size_t bytes() const {
      const Buf *all[] = {&boxes, &key, &idx, &key2, &idx2, &temp, &bb, &nbd, &lv,
                          &par, &cb, &nc, &nch, &off, &gcnt, &goff, &gtab, &gacc, &part};
      size_t s = 0;
      for (const Buf *b : all) s += b->bytes;
      return s;
    }
  };
  static std::mutex cache_mu;  // a heap array never destroyed: no HIP call at exit
  static std::unique_ptr<TreeScratch> *cache = new std::unique_ptr<TreeScratch>[kMaxDevices];
  int dev = 0;
  TRY(hipGetDevice(&dev));
  std::unique_ptr<TreeScratch> sc;
  {
    std::lock_guard<std::mutex> guard(cache_mu);
    if (dev >= 0 && dev < kMaxDevices) sc = std::move(cache[dev]);
  }
  if (!sc) sc.reset(new TreeScratch);
  TRY(sc->host.get());
  int64_t *total_dev = nullptr;  // the device's address of the pinned block
  TRY(hipHostGetDevicePointer((void **)&total_dev, sc->host.p, 0));
  // exclusive scan of cnts[0, m) into offs; returns the total to the host
  // (one synchronisation)
  auto scan_i32 = [&](const int32_t *cnts, int32_t *offs, int64_t m, int64_t *res) -> int {
    TRY(sc->part.reserve(prims::scan_scratch_bytes<int64_t>(m), st, false));
    TRY(prims::exclusive_scan<int64_t>(m, prims::LoadArray<int64_t, int32_t>{cnts},
                                       prims::StoreArray<int64_t, int32_t>{offs},
                                       (int64_t *)sc->part.p, total_dev, st));
    TRY(hipStreamSynchronize(st));
    *res = sc->host.p[0];
    return 0;
  };
  auto keep = [&]() {
    if (sc->bytes() <= kKeepScratchBytes && dev >= 0 && dev < kMaxDevices) {
      std::lock_guard<std::mutex> guard(cache_mu);
      if (!cache[dev]) cache[dev] = std::move(sc);
    }
  };
  Buf &boxes = sc->boxes, &key = sc->key, &idx = sc->idx, &key2 = sc->key2, &idx2 = sc->idx2,
      &temp = sc->temp, &bb = sc->bb, &nbd = sc->nbd, &lv = sc->lv, &par = sc->par, &cb = sc->cb,
      &nc = sc->nc, &nch = sc->nch, &off = sc->off;
  // bounding box, finiteness, FP32 representability
  const int nblk = (int)std::min<int64_t>(1024, (n + 255) / 256);
  TRY(boxes.reserve(nblk * sizeof(Box), st, false));
  bbox_partial<<<nblk, 256, 0, st>>>(n, xyz, (Box *)boxes.p);
  TRY(hipGetLastError());
  std::vector<Box> hb(nblk);
  TRY(hipMemcpyAsync(hb.data(), boxes.p, nblk * sizeof(Box), hipMemcpyDeviceToHost, st));
  TRY(hipStreamSynchronize(st));
  double lo[3], hi[3];
  bool finite = true, exact = true;
  for (int d = 0; d < 3; ++d) {
    lo[d] = hb[0].lo[d];
    hi[d] = hb[0].hi[d];
  }
  for (const Box &b : hb) {
    for (int d = 0; d < 3; ++d) {
      lo[d] = b.lo[d] < lo[d] ? b.lo[d] : lo[d];
      hi[d] = b.hi[d] > hi[d] ? b.hi[d] : hi[d];
    }
    finite = finite && b.finite;
    exact = exact && b.exact;
  }
  if (!finite) {
    err = "fmm_tree_build_gpu: positions must be finite";
    return -1;
  }
  t.fp32_exact = exact;
  double h = 0.0;
  for (int d = 0; d < 3; ++d) {
    t.root_center[d] = 0.5 * (lo[d] + hi[d]);
    const double half = 0.5 * (hi[d] - lo[d]);
    h = half > h ? half : h;
  }
  t.root_half = h;
  // keys, stable sort of (key, index)
  TRY(key.reserve(n * 8, st, false));
  TRY(idx.reserve(n * 4, st, false));
  TRY(key2.reserve(n * 8, st, false));
  TRY(idx2.reserve(n * 4, st, false));
  morton_keys<<<blocks_for(n, 256), 256, 0, st>>>(n, xyz, t.root_center[0] - h,
                                                  t.root_center[1] - h, t.root_center[2] - h,
                                                  2.0 * h, h == 0.0, (uint64_t *)key.p,
                                                  (int32_t *)idx.p);
  TRY(hipGetLastError());
  TRY(temp.reserve(prims::radix_scratch_bytes(n), st, false));
  bool in_alt = false;
  TRY(prims::radix_sort<uint64_t>((uint64_t *)key.p, (uint64_t *)key2.p, (int32_t *)idx.p,
                                  (int32_t *)idx2.p, n, 0, 63, temp.p, st, &in_alt));
  const uint64_t *skeys = in_alt ? (const uint64_t *)key2.p : (const uint64_t *)key.p;
  const int32_t *sperm = in_alt ? (const int32_t *)idx2.p : (const int32_t *)idx.p;
  TRY(hipMalloc((void **)&out.perm, n * 4));
  TRY(hipMemcpyAsync(out.perm, sperm, n * 4, hipMemcpyDeviceToDevice, st));
  TRY(hipMalloc((void **)&out.pos, n * 24));
  gather_positions<<<blocks_for(n, 256), 256, 0, st>>>(n, xyz, out.perm, out.pos);
  TRY(hipGetLastError());
  // levels
  size_t cap = 1024;
  auto grow = [&](size_t want) -> hipError_t {
    if (want <= cap && bb.p) return hipSuccess;
    while (cap < want) cap *= 2;
    hipError_t e;
    if ((e = bb.reserve(cap * 8, st, true)) != hipSuccess) return e;
    if ((e = nbd.reserve(cap * 8, st, true)) != hipSuccess) return e;
    if ((e = lv.reserve(cap * 4, st, true)) != hipSuccess) return e;
    if ((e = par.reserve(cap * 4, st, true)) != hipSuccess) return e;
    if ((e = cb.reserve(cap * 4, st, true)) != hipSuccess) return e;
    return nc.reserve(cap * 4, st, true);
  };
  TRY(grow(1));
  {
    const int64_t zero = 0;
    const int32_t izero = 0, mone = -1;
    TRY(hipMemcpyAsync(bb.p, &zero, 8, hipMemcpyHostToDevice, st));
    TRY(hipMemcpyAsync(nbd.p, &n, 8, hipMemcpyHostToDevice, st));
    TRY(hipMemcpyAsync(lv.p, &izero, 4, hipMemcpyHostToDevice, st));
    TRY(hipMemcpyAsync(par.p, &mone, 4, hipMemcpyHostToDevice, st));
    TRY(hipStreamSynchronize(st));
  }
  t.level_begin.assign(1, 0);
  int64_t c0 = 0, c1 = 1;
  int level = 0;
  while (c0 < c1) {
    t.level_begin.push_back(c1);
    const int64_t m = c1 - c0;
    TRY(nch.reserve(m * 4, st, false));
    TRY(off.reserve(m * 4, st, false));
    count_children<<<blocks_for(m, 256), 256, 0, st>>>(c0, c1, level, ncrit, h > 0.0, skeys,
                                                       (const int64_t *)bb.p,
                                                       (const int64_t *)nbd.p, (int32_t *)nch.p);
    TRY(hipGetLastError());
    int64_t added = 0;
    if (int rc = scan_i32((const int32_t *)nch.p, (int32_t *)off.p, m, &added)) return rc;
    TRY(grow(c1 + added));
    write_children<<<blocks_for(m, 256), 256, 0, st>>>(
        c0, c1, level, skeys, (const int32_t *)nch.p, (const int32_t *)off.p, c1,
        (int64_t *)bb.p, (int64_t *)nbd.p, (int32_t *)lv.p, (int32_t *)par.p, (int32_t *)cb.p,
        (int32_t *)nc.p);
    TRY(hipGetLastError());
    c0 = c1;
    c1 = c1 + added;
    if (c0 < c1) ++level;
  }
  const int64_t ncells = c1;
  t.max_level = level;
  t.level_begin.resize(t.max_level + 2);
  t.level_begin[t.max_level + 1] = ncells;
  // geometry
  TRY(hipMalloc((void **)&out.geo, ncells * 32));
  {
    Buf &gcnt = sc->gcnt, &goff = sc->goff, &gtab = sc->gtab, &gacc = sc->gacc;
    TRY(gcnt.reserve(ncells * 4, st, false));
    TRY(goff.reserve(ncells * 4, st, false));
    TRY(gacc.reserve(ncells * 7 * 8, st, false));
    const unsigned gb = blocks_for(ncells, 256);
    geo_chunk_count<<<gb, 256, 0, st>>>(ncells, (const int64_t *)nbd.p, (int32_t *)gcnt.p);
    TRY(hipGetLastError());
    int64_t nchunks = 0;
    if (int rc = scan_i32((const int32_t *)gcnt.p, (int32_t *)goff.p, ncells, &nchunks)) return rc;
    TRY(gtab.reserve(nchunks * 8, st, false));
    geo_chunk_fill<<<gb, 256, 0, st>>>(ncells, (const int32_t *)gcnt.p, (const int32_t *)goff.p,
                                       (uint64_t *)gtab.p, (uint64_t *)gacc.p);
    TRY(hipGetLastError());
    geo_chunk<0><<<(unsigned)nchunks, 256, 0, st>>>(out.pos, (const int64_t *)bb.p,
                                                     (const int64_t *)nbd.p,
                                                     (const uint64_t *)gtab.p,
                                                     (const double4 *)out.geo,
                                                     (uint64_t *)gacc.p);
    TRY(hipGetLastError());
    geo_finish<0><<<gb, 256, 0, st>>>(ncells, (const uint64_t *)gacc.p, (double4 *)out.geo);
    TRY(hipGetLastError());
    geo_chunk<1><<<(unsigned)nchunks, 256, 0, st>>>(out.pos, (const int64_t *)bb.p,
                                                     (const int64_t *)nbd.p,
                                                     (const uint64_t *)gtab.p,
                                                     (const double4 *)out.geo,
                                                     (uint64_t *)gacc.p);
    TRY(hipGetLastError());
    geo_finish<1><<<gb, 256, 0, st>>>(ncells, (const uint64_t *)gacc.p, (double4 *)out.geo);
    TRY(hipGetLastError());
  }
  TRY(hipMalloc((void **)&out.body_begin, ncells * 4));
  TRY(hipMalloc((void **)&out.n_body, ncells * 4));
  narrow_i64<<<blocks_for(ncells, 256), 256, 0, st>>>(ncells, (const int64_t *)bb.p, out.body_begin);
  narrow_i64<<<blocks_for(ncells, 256), 256, 0, st>>>(ncells, (const int64_t *)nbd.p, out.n_body);
  TRY(hipGetLastError());
  for (int32_t **dst : {&out.child_begin, &out.n_child, &out.parent}) TRY(hipMalloc((void **)dst, ncells * 4));
  TRY(hipMemcpyAsync(out.child_begin, cb.p, ncells * 4, hipMemcpyDeviceToDevice, st));
  TRY(hipMemcpyAsync(out.n_child, nc.p, ncells * 4, hipMemcpyDeviceToDevice, st));
  TRY(hipMemcpyAsync(out.parent, par.p, ncells * 4, hipMemcpyDeviceToDevice, st));
  TRY(hipMalloc((void **)&out.keys, n * 8));
  TRY(hipMemcpyAsync(out.keys, skeys, n * 8, hipMemcpyDeviceToDevice, st));
  // host copy of the cell arrays (the per-body arrays stay on the device):
  // seven asynchronous copies into the pinned block, one wait
  t.level.resize(ncells);
  t.parent.resize(ncells);
  t.child_begin.resize(ncells);
  t.n_child.resize(ncells);
  t.body_begin.resize(ncells);
  t.n_body.resize(ncells);
  t.center.resize(3 * ncells);
  t.radius.resize(ncells);
  const size_t nc_ = (size_t)ncells;
  TRY(sc->stage.reserve(nc_ * (4 * 4 + 2 * 8 + 32)));
  char *hs = static_cast<char *>(sc->stage.p);
  int32_t *h_lv = reinterpret_cast<int32_t *>(hs), *h_par = h_lv + nc_, *h_cb = h_par + nc_,
          *h_nc = h_cb + nc_;
  int64_t *h_bb = reinterpret_cast<int64_t *>(hs + 16 * nc_), *h_nbd = h_bb + nc_;
  double *h_geo = reinterpret_cast<double *>(hs + 32 * nc_);
  TRY(hipMemcpyAsync(h_lv, lv.p, nc_ * 4, hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(h_par, par.p, nc_ * 4, hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(h_cb, cb.p, nc_ * 4, hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(h_nc, nc.p, nc_ * 4, hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(h_bb, bb.p, nc_ * 8, hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(h_nbd, nbd.p, nc_ * 8, hipMemcpyDeviceToHost, st));
  TRY(hipMemcpyAsync(h_geo, out.geo, nc_ * 32, hipMemcpyDeviceToHost, st));
  TRY(hipStreamSynchronize(st));
  std::copy(h_lv, h_lv + nc_, t.level.begin());
  std::copy(h_par, h_par + nc_, t.parent.begin());
  std::copy(h_cb, h_cb + nc_, t.child_begin.begin());
  std::copy(h_nc, h_nc + nc_, t.n_child.begin());
  std::copy(h_bb, h_bb + nc_, t.body_begin.begin());
  std::copy(h_nbd, h_nbd + nc_, t.n_body.begin());
  t.n_leaves = 0;
  for (int64_t c = 0; c < ncells; ++c) {
    for (int d = 0; d < 3; ++d) t.center[3 * c + d] = h_geo[4 * c + d];
    t.radius[c] = h_geo[4 * c + 3];
    t.n_leaves += t.n_child[c] == 0;
  }
  out.n = n;
  out.n_cells = ncells;
  keep();  // the stream is idle: the scratch can serve the next build
  return 0;
}

}  // namespace dev
}  // namespace fmmlib
