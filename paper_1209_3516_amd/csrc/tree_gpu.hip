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
// are sorted as 64-bit keys (target << 32 | source), which is the canonical
// CSR order (rows = targets, sources ascending).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <hipcub/hipcub.hpp>
#include <vector>

#include "kernels.h"

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

// counts[i] = number of child pairs; emit[i] = (M2L count << 32) | P2P count.
__global__ void dtt_count(int64_t nf, const int2 *__restrict__ frontier,
                          const double4 *__restrict__ geo, const int32_t *__restrict__ n_child,
                          double theta2, int leaf_first, int64_t *__restrict__ counts,
                          uint64_t *__restrict__ emit) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const int2 pr = frontier[i];
  int n;
  const int act = classify(pr.x, pr.y, geo, n_child, theta2, leaf_first != 0, &n);
  counts[i] = n;
  emit[i] = act == kActM2L ? (1ull << 32) : (act == kActP2P ? 1ull : 0ull);
}

__global__ void dtt_expand(int64_t nf, const int2 *__restrict__ frontier,
                           const double4 *__restrict__ geo, const int32_t *__restrict__ n_child,
                           const int32_t *__restrict__ child_begin, double theta2, int leaf_first,
                           const int64_t *__restrict__ child_off,
                           const uint64_t *__restrict__ emit_off, int2 *__restrict__ next,
                           uint64_t *__restrict__ p2p_keys, int64_t p2p_base,
                           uint64_t *__restrict__ m2l_keys, int64_t m2l_base) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const int2 pr = frontier[i];
  const int a = pr.x, b = pr.y;
  int n;
  const int act = classify(a, b, geo, n_child, theta2, leaf_first != 0, &n);
  const uint64_t key = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
  if (act == kActM2L) {
    m2l_keys[m2l_base + (int64_t)(emit_off[i] >> 32)] = key;
  } else if (act == kActP2P) {
    p2p_keys[p2p_base + (int64_t)(emit_off[i] & 0xffffffffull)] = key;
  } else {
    int2 *out = next + child_off[i];
    if (act == kActSplitBoth) {
      const int c0 = child_begin[a], nc = n_child[a];
      for (int x = 0; x < nc; ++x)
        for (int y = 0; y < nc; ++y) out[x * nc + y] = make_int2(c0 + x, c0 + y);
    } else if (act == kActSplitA) {
      const int c0 = child_begin[a];
      for (int x = 0; x < n; ++x) out[x] = make_int2(c0 + x, b);
    } else {
      const int c0 = child_begin[b];
      for (int y = 0; y < n; ++y) out[y] = make_int2(a, c0 + y);
    }
  }
}

// CSR from sorted keys: row_ptr[r] = first key with target >= r.
__global__ void csr_rows(int64_t n_rows, const uint64_t *__restrict__ keys, int64_t nnz,
                         int64_t *__restrict__ row_ptr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > n_rows) return;
  const uint64_t want = (uint64_t)r << 32;
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

__global__ void csr_cols(int64_t nnz, const uint64_t *__restrict__ keys, int32_t *__restrict__ col) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnz) col[i] = (int32_t)(keys[i] & 0xffffffffull);
}

// Growable device buffer.
struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
  hipError_t reserve(size_t want, hipStream_t st, bool keep) {
    if (want <= bytes) return hipSuccess;
    size_t nb = bytes ? bytes : 1024;
    while (nb < want) nb *= 2;
    void *np = nullptr;
    hipError_t e = hipMalloc(&np, nb);
    if (e != hipSuccess) return e;
    if (keep && p) {
      e = hipMemcpyAsync(np, p, bytes, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return e;
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
    }
    if (p) {
      // earlier kernels on the stream may still read the old buffer
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
      (void)hipFree(p);
    }
    p = np;
    bytes = nb;
    return hipSuccess;
  }
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

#define TRY(x)                             \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) return (int)e_;  \
  } while (0)

int sort_to_csr(uint64_t *keys, int64_t nnz, int64_t n_rows, hipStream_t st, Buf &alt,
                Buf &temp, int64_t *row_ptr_dev, int32_t *col_dev) {
  if (nnz > 0) {
    TRY(alt.reserve(nnz * sizeof(uint64_t), st, false));
    hipcub::DoubleBuffer<uint64_t> db(keys, (uint64_t *)alt.p);
    size_t tb = 0;
    TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, db, (int)nnz, 0, 64, st));
    TRY(temp.reserve(tb, st, false));
    TRY(hipcub::DeviceRadixSort::SortKeys(temp.p, tb, db, (int)nnz, 0, 64, st));
    const uint64_t *sorted = db.Current();
    csr_rows<<<blocks_for(n_rows + 1, 256), 256, 0, st>>>(n_rows, sorted, nnz, row_ptr_dev);
    csr_cols<<<blocks_for(nnz, 256), 256, 0, st>>>(nnz, sorted, col_dev);
  } else {
    TRY(hipMemsetAsync(row_ptr_dev, 0, (n_rows + 1) * sizeof(int64_t), st));
  }
  return (int)hipGetLastError();
}

}  // namespace

int dual_traverse_gpu(int64_t n_cells, const double *geo, const int32_t *child_begin,
                      const int32_t *n_child, double theta, bool leaf_first, void *stream,
                      DeviceLists &out) {
  const hipStream_t st = S_(stream);
  const double theta2 = theta * theta;
  const double4 *g = (const double4 *)geo;
  out = DeviceLists();
  out.n_rows = n_cells;
  Buf front[2], counts, emit, coff, eoff, temp, p2p, m2l, alt;
  int64_t nf = n_cells > 0 ? 1 : 0, n_p2p = 0, n_m2l = 0;
  TRY(front[0].reserve(sizeof(int2), st, false));
  if (nf) {
    const int2 root = make_int2(0, 0);
    TRY(hipMemcpyAsync(front[0].p, &root, sizeof(int2), hipMemcpyHostToDevice, st));
  }
  int cur = 0;
  while (nf > 0) {
    TRY(counts.reserve(nf * sizeof(int64_t), st, false));
    TRY(emit.reserve(nf * sizeof(uint64_t), st, false));
    TRY(coff.reserve(nf * sizeof(int64_t), st, false));
    TRY(eoff.reserve(nf * sizeof(uint64_t), st, false));
    dtt_count<<<blocks_for(nf, 256), 256, 0, st>>>(nf, (const int2 *)front[cur].p, g, n_child,
                                                   theta2, leaf_first, (int64_t *)counts.p,
                                                   (uint64_t *)emit.p);
    TRY(hipGetLastError());
    size_t tb1 = 0, tb2 = 0;
    TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tb1, (int64_t *)counts.p, (int64_t *)coff.p,
                                         (int)nf, st));
    TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, (uint64_t *)emit.p, (uint64_t *)eoff.p,
                                         (int)nf, st));
    TRY(temp.reserve(tb1 > tb2 ? tb1 : tb2, st, false));
    TRY(hipcub::DeviceScan::ExclusiveSum(temp.p, tb1, (int64_t *)counts.p, (int64_t *)coff.p,
                                         (int)nf, st));
    TRY(hipcub::DeviceScan::ExclusiveSum(temp.p, tb2, (uint64_t *)emit.p, (uint64_t *)eoff.p,
                                         (int)nf, st));
    // totals = last offset + last count
    int64_t last_c[2];
    uint64_t last_e[2];
    TRY(hipMemcpyAsync(&last_c[0], (int64_t *)coff.p + nf - 1, sizeof(int64_t),
                       hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(&last_c[1], (int64_t *)counts.p + nf - 1, sizeof(int64_t),
                       hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(&last_e[0], (uint64_t *)eoff.p + nf - 1, sizeof(uint64_t),
                       hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(&last_e[1], (uint64_t *)emit.p + nf - 1, sizeof(uint64_t),
                       hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    const int64_t n_next = last_c[0] + last_c[1];
    const uint64_t e_tot = last_e[0] + last_e[1];
    const int64_t add_p2p = (int64_t)(e_tot & 0xffffffffull), add_m2l = (int64_t)(e_tot >> 32);
    TRY(front[1 - cur].reserve((n_next > 0 ? n_next : 1) * sizeof(int2), st, false));
    TRY(p2p.reserve((n_p2p + add_p2p + 1) * sizeof(uint64_t), st, true));
    TRY(m2l.reserve((n_m2l + add_m2l + 1) * sizeof(uint64_t), st, true));
    dtt_expand<<<blocks_for(nf, 256), 256, 0, st>>>(
        nf, (const int2 *)front[cur].p, g, n_child, child_begin, theta2, leaf_first,
        (const int64_t *)coff.p, (const uint64_t *)eoff.p, (int2 *)front[1 - cur].p,
        (uint64_t *)p2p.p, n_p2p, (uint64_t *)m2l.p, n_m2l);
    TRY(hipGetLastError());
    n_p2p += add_p2p;
    n_m2l += add_m2l;
    nf = n_next;
    cur = 1 - cur;
  }
  TRY(hipMalloc((void **)&out.p2p_ptr, (n_cells + 1) * sizeof(int64_t)));
  TRY(hipMalloc((void **)&out.m2l_ptr, (n_cells + 1) * sizeof(int64_t)));
  TRY(hipMalloc((void **)&out.p2p_col, (n_p2p > 0 ? n_p2p : 1) * sizeof(int32_t)));
  TRY(hipMalloc((void **)&out.m2l_col, (n_m2l > 0 ? n_m2l : 1) * sizeof(int32_t)));
  out.p2p_nnz = n_p2p;
  out.m2l_nnz = n_m2l;
  if (int rc = sort_to_csr((uint64_t *)p2p.p, n_p2p, n_cells, st, alt, temp, out.p2p_ptr,
                           out.p2p_col))
    return rc;
  if (int rc = sort_to_csr((uint64_t *)m2l.p, n_m2l, n_cells, st, alt, temp, out.m2l_ptr,
                           out.m2l_col))
    return rc;
  TRY(hipStreamSynchronize(st));
  return 0;
}

}  // namespace dev
}  // namespace fmmlib
