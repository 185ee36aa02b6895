// Work plan of the P2P kernel built on the device from device CSR lists, with
// the same chunking, run merging, item order and partial-slot layout as the
// host builder, so both give the same plan entry for entry.
//
// One 64-lane wave per leaf walks the leaf's P2P row twice: a counting pass
// (runs, chunks, source bodies, body pairs) and, after prefix sums give every
// leaf its offsets, a writing pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>


#include "kernels.h"
#include "prims.h"

namespace fmmlib {
namespace dev {

namespace {

struct Chunk {
  int32_t run_begin, n_runs, n_src;
  bool self;
};

// Inclusive sum over the 64 lanes of a wave, in lane order.
__device__ __forceinline__ int wave_incl_sum(int v) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(v, d);
    if (lane >= d) v += u;
  }
  return v;
}

__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

// Walk row `a` (leaf with nA bodies) with one 64-lane wave; every lane calls
// this with the same arguments.  The host builder's rule, taken entry by
// entry in row order: an entry extends the current run when its bodies
// follow the previous entry's in memory (neither being the leaf itself), else
// starts a run; the chunk is closed before an entry when its sources would
// pass kP2PChunkSources (the leaf's own bodies count if it is in the chunk)
// or when it would start run kP2PMaxRuns + 1.  Here the row is taken 64
// entries at a time: scans over the lanes give each entry the chunk's
// sources, self flag and runs before it, a ballot finds the first entry that
// closes the chunk, and the scans restart there (a chunk's first entry never
// closes it, so every pass moves forward).  on_run(k, body, prefix) is called
// (by the lanes holding them, in no particular order) for each run k of the
// row; on_chunk(c, chunk) by all lanes for each chunk, in order.  Returns
// the number of chunks; *row_src and *pairs (on every lane) get the row's
// source bodies and body pairs.
template <class OnRun, class OnChunk>
__device__ int walk_row(int32_t a, int64_t nA, const int64_t *__restrict__ ptr,
                        const int32_t *__restrict__ col, const int32_t *__restrict__ body_begin,
                        const int32_t *__restrict__ n_body, int32_t run_base, int32_t *row_runs,
                        int64_t *row_src, int64_t *pairs, OnRun on_run, OnChunk on_chunk) {
  const int lane = threadIdx.x;
  const int64_t e_beg = ptr[a], E = ptr[a + 1] - e_beg;
  int64_t s = 0;                    // first entry of the current chunk (row order)
  int src_acc = 0, runs_acc = 0;    // the chunk's sources and runs before this segment
  bool self_acc = false;            // ... and whether it holds the leaf itself
  int32_t runs_row = 0;             // runs of the row before the current chunk
  int nch = 0;
  bool prev_self = true;            // the entry before the segment (none: no adjacency)
  int64_t prev_end = -1;
  long long my_src = 0, my_pairs = 0;
  for (int64_t seg = 0; seg < E; seg += 64) {
    const int64_t e = seg + lane;
    const bool valid = e < E;
    // lanes past the row's end read entry 0 and the leaf itself (E >= 1 here)
    // and then count as empty
    const int32_t bcol = col[e_beg + (valid ? e : 0)];
    const int32_t b = valid ? bcol : a;
    const int nb = valid ? n_body[b] : 0;
    const int bb = valid ? body_begin[b] : 0;
    const bool self = valid && b == a;
    my_src += nb;
    my_pairs += (long long)nA * nb - (self ? nA : 0);
    const int up_self = __shfl_up(self ? 1 : 0, 1);
    const int up_end = __shfl_up(bb + nb, 1);
    const bool p_self = lane == 0 ? prev_self : up_self != 0;
    const int64_t p_end = lane == 0 ? prev_end : (int64_t)up_end;
    const int last = (int)(E - 1 - seg < 63 ? E - 1 - seg : 63);
    for (;;) {
      const bool in = valid && e >= s;
      const bool adj = in && e > s && !self && !p_self && p_end == (int64_t)bb;
      const bool newrun = in && !self && !adj;
      const int c_src = in && !self ? nb : 0;
      const int i_src = wave_incl_sum(c_src);
      const int i_self = wave_incl_sum(in && self ? 1 : 0);
      const int i_runs = wave_incl_sum(newrun ? 1 : 0);
      const int src_before = src_acc + i_src - c_src;
      const bool self_before = self_acc || i_self - (in && self ? 1 : 0) > 0;
      const int runs_before = runs_acc + i_runs - (newrun ? 1 : 0);
      const bool full =
          in && (((int64_t)src_before + (self_before ? nA : 0) + nb > kP2PChunkSources &&
                  (src_before > 0 || self_before)) ||
                 (!adj && !self && runs_before >= kP2PMaxRuns));
      const unsigned long long fm = __ballot(full);
      const int stop = fm ? __ffsll((long long)fm) - 1 : 64;
      if (newrun && lane < stop) on_run(runs_row + runs_before, bb, src_before);
      if (fm == 0) {  // the chunk goes on past this segment
        src_acc += __shfl(i_src, last);
        self_acc = self_acc || __shfl(i_self, last) > 0;
        runs_acc += __shfl(i_runs, last);
        break;
      }
      const Chunk ch{run_base + runs_row, __shfl(runs_before, stop), __shfl(src_before, stop),
                     __shfl(self_before ? 1 : 0, stop) != 0};
      on_chunk(nch++, ch);
      runs_row += ch.n_runs;
      s = seg + stop;
      src_acc = 0;
      runs_acc = 0;
      self_acc = false;
    }
    prev_self = __shfl(self ? 1 : 0, last) != 0;
    prev_end = __shfl(bb + nb, last);
  }
  if (src_acc > 0 || self_acc || nch == 0) {
    on_chunk(nch++, Chunk{run_base + runs_row, runs_acc, src_acc, self_acc});
    runs_row += runs_acc;
  }
  *row_runs = runs_row;
  *row_src = wave_sum(my_src);
  *pairs = wave_sum(my_pairs);
  return nch;
}

__global__ void leaf_flags(int64_t nc, const int32_t *__restrict__ n_child,
                           int32_t *__restrict__ flag) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nc) flag[c] = n_child[c] == 0;
}

// Per leaf (one 64-lane wave per cell; other cells return): cell, run
// count, item count, partial slots, chunks, row sources and body pairs.
__global__ __launch_bounds__(64) void plan_count(
    int64_t nc, const int32_t *__restrict__ n_child, const int32_t *__restrict__ leaf_of,
    const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
    const int32_t *__restrict__ body_begin, const int32_t *__restrict__ n_body,
    int32_t *__restrict__ leaf_cell, int32_t *__restrict__ nruns, int32_t *__restrict__ nitems,
    int32_t *__restrict__ nparts, int32_t *__restrict__ nchunk, int64_t *__restrict__ lsrc,
    int64_t *__restrict__ lpairs) {
  const int64_t a = blockIdx.x;
  if (a >= nc || n_child[a] != 0) return;
  const int32_t leaf = leaf_of[a];
  const int64_t nA = n_body[a];
  int32_t runs = 0;
  int64_t src, pairs;
  const int nch = walk_row(
      (int32_t)a, nA, ptr, col, body_begin, n_body, 0, &runs, &src, &pairs,
      [&](int32_t, int32_t, int32_t) {}, [&](int, const Chunk &) {});
  if (threadIdx.x != 0) return;
  leaf_cell[leaf] = (int32_t)a;
  nruns[leaf] = runs;
  nitems[leaf] = (int32_t)((nA + 63) / 64) * nch;
  nparts[leaf] = (int32_t)(nch * nA);
  nchunk[leaf] = nch;
  lsrc[leaf] = src;
  lpairs[leaf] = pairs;
}

// totals: [0] max row sources, [1] body pairs, [2] runs, [3] items, [4]
// partial slots.  One block; each thread takes leaves t, t + 1024, ... and
// the block sums in a fixed tree.
__global__ __launch_bounds__(1024) void plan_totals(
    int64_t n_leaves, const int64_t *__restrict__ lsrc, const int64_t *__restrict__ lpairs,
    const int32_t *__restrict__ nruns, const int32_t *__restrict__ nitems,
    const int32_t *__restrict__ nparts, unsigned long long *__restrict__ totals) {
  __shared__ unsigned long long red[5][1024];
  const int t = threadIdx.x;
  unsigned long long v[5] = {0, 0, 0, 0, 0};
  for (int64_t l = t; l < n_leaves; l += 1024) {
    v[0] = v[0] > (unsigned long long)lsrc[l] ? v[0] : (unsigned long long)lsrc[l];
    v[1] += (unsigned long long)lpairs[l];
    v[2] += (unsigned long long)nruns[l];
    v[3] += (unsigned long long)nitems[l];
    v[4] += (unsigned long long)nparts[l];
  }
  for (int k = 0; k < 5; ++k) red[k][t] = v[k];
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (t < h) {
      red[0][t] = red[0][t] > red[0][t + h] ? red[0][t] : red[0][t + h];
      for (int k = 1; k < 5; ++k) red[k][t] += red[k][t + h];
    }
    __syncthreads();
  }
  if (t < 5) totals[t] = red[t][0];
}

// The plan entries of each leaf (one 64-lane wave per leaf), at the offsets
// the counts gave.  Runs and chunks beyond the counted ones are not written.
__global__ __launch_bounds__(64) void plan_write(
    int64_t n_leaves, const int32_t *__restrict__ leaf_cell, const int64_t *__restrict__ ptr,
    const int32_t *__restrict__ col, const int32_t *__restrict__ body_begin,
    const int32_t *__restrict__ n_body, const int32_t *__restrict__ nruns,
    const int32_t *__restrict__ run_off, const int32_t *__restrict__ item_off,
    const int32_t *__restrict__ pbase, const int32_t *__restrict__ nchunk, PlanLayouts layouts,
    P2PItem *__restrict__ items, int32_t *__restrict__ run_body,
    int32_t *__restrict__ run_prefix, int32_t *__restrict__ body_leaf) {
  const int64_t leaf = blockIdx.x;
  if (leaf >= n_leaves) return;
  const int lane = threadIdx.x;
  const int32_t a = leaf_cell[leaf];
  const int64_t nA = n_body[a], bA = body_begin[a];
  const int32_t r0 = run_off[leaf], i0 = item_off[leaf], pb = pbase[leaf], nch = nchunk[leaf];
  const int32_t run_cap = nruns[leaf];
  const int64_t ng = (nA + 63) / 64;
  int32_t runs = 0;
  int64_t src, pairs;
  walk_row(
      a, nA, ptr, col, body_begin, n_body, r0, &runs, &src, &pairs,
      [&](int32_t k, int32_t body, int32_t prefix) {
        if (k < run_cap) {
          run_body[r0 + k] = body;
          run_prefix[r0 + k] = prefix;
        }
      },
      [&](int c, const Chunk &ch) {
        if (c >= nch) return;
        for (int64_t gi = lane; gi < ng; gi += 64) {
          const int64_t g = 64 * gi;
          const int nt = (int)(nA - g < 64 ? nA - g : 64);
          P2PItem it;
          it.tgt_begin = (int32_t)(bA + g);
          it.tgt_cfg = layouts.cfg[nt];
          it.run_begin = ch.run_begin;
          it.n_runs = ch.n_runs;
          it.n_src = ch.n_src;
          it.self_begin = ch.self ? (int32_t)bA : -1;
          it.self_n = ch.self ? (int32_t)nA : 0;
          it.out_off = (int32_t)(pb + (int64_t)c * nA + g);
          items[i0 + gi * nch + c] = it;
        }
      });
  for (int64_t i = bA + lane; i < bA + nA; i += 64) body_leaf[i] = (int32_t)leaf;
}


}  // namespace

#define PTRY(x)                        \
  do {                                 \
    hipError_t e_ = (x);               \
    if (e_ != hipSuccess) {            \
      release();                       \
      return (int)e_;                  \
    }                                  \
  } while (0)

int build_p2p_plan_gpu(int64_t n, int64_t n_cells, int64_t n_leaves, const int32_t *n_child,
                       const int32_t *body_begin, const int32_t *n_body, const int64_t *p2p_ptr,
                       const int32_t *p2p_col, const PlanLayouts &layouts, void *stream,
                       DevicePlan &out) {
  hipStream_t st;
  if (int rc = build_stream(stream, reinterpret_cast<void **>(&st))) return rc;
  out = DevicePlan();
  if (n_cells <= 0 || n_leaves <= 0) return 0;
  int32_t *leaf_flag = nullptr, *leaf_of = nullptr, *nruns = nullptr, *nitems = nullptr,
          *nparts = nullptr, *run_off = nullptr, *item_off = nullptr;
  unsigned long long *totals = nullptr;
  int64_t *lsrc = nullptr, *lpairs = nullptr;
  void *scan_tmp = nullptr;
  // temporaries from the stream-ordered pool, freed in stream order
  auto free_temps = [&]() {
    void *ps[] = {leaf_flag, leaf_of, nruns,  nitems,   nparts, run_off,
                  item_off,  totals,  lsrc,   lpairs,   scan_tmp};
    for (void *p : ps)
      if (p) (void)hipFreeAsync(p, st);
    leaf_flag = leaf_of = nruns = nitems = nparts = run_off = item_off = nullptr;
    totals = nullptr;
    lsrc = lpairs = nullptr;
    scan_tmp = nullptr;
  };
  auto release = [&]() {
    free_temps();
    out.release();
  };
  if (int rc = keep_pool_memory()) return rc;
  const size_t nl = (size_t)n_leaves, nc = (size_t)n_cells;
  PTRY(hipMallocAsync((void **)&leaf_flag, nc * 4, st));
  PTRY(hipMallocAsync((void **)&leaf_of, nc * 4, st));
  PTRY(hipMallocAsync((void **)&nruns, nl * 4, st));
  PTRY(hipMallocAsync((void **)&nitems, nl * 4, st));
  PTRY(hipMallocAsync((void **)&nparts, nl * 4, st));
  PTRY(hipMallocAsync((void **)&run_off, nl * 4, st));
  PTRY(hipMallocAsync((void **)&item_off, nl * 4, st));
  PTRY(hipMallocAsync((void **)&totals, 8 * sizeof(unsigned long long), st));
  PTRY(hipMallocAsync((void **)&lsrc, nl * 8, st));
  PTRY(hipMallocAsync((void **)&lpairs, nl * 8, st));
  PTRY(hipMalloc(&out.leaf_cell, nl * 4));
  PTRY(hipMalloc(&out.leaf_pbase, nl * 4));
  PTRY(hipMalloc(&out.leaf_nchunk, nl * 4));
  PTRY(hipMalloc(&out.body_leaf, (size_t)(n > 0 ? n : 1) * 4));

  // scratch of the scans (tile partials), for the larger of the two lengths
  PTRY(hipMallocAsync(&scan_tmp, prims::scan_scratch_bytes<int64_t>((int64_t)(nc > nl ? nc : nl)),
                      st));
  auto scan = [&](const int32_t *in, int32_t *out_off, size_t m) -> hipError_t {
    return prims::exclusive_scan<int64_t>((int64_t)m, prims::LoadArray<int64_t, int32_t>{in},
                                          prims::StoreArray<int64_t, int32_t>{out_off},
                                          (int64_t *)scan_tmp, (int64_t *)nullptr, st);
  };

  const unsigned bc = (unsigned)((nc + 255) / 256);
  leaf_flags<<<bc, 256, 0, st>>>((int64_t)nc, n_child, leaf_flag);
  PTRY(hipGetLastError());
  PTRY(scan(leaf_flag, leaf_of, nc));
  plan_count<<<(unsigned)nc, 64, 0, st>>>((int64_t)nc, n_child, leaf_of, p2p_ptr, p2p_col,
                                           body_begin, n_body, out.leaf_cell, nruns, nitems,
                                           nparts, out.leaf_nchunk, lsrc, lpairs);
  PTRY(hipGetLastError());
  plan_totals<<<1, 1024, 0, st>>>((int64_t)nl, lsrc, lpairs, nruns, nitems, nparts, totals);
  PTRY(hipGetLastError());
  unsigned long long host_tot[8] = {};
  PTRY(hipMemcpyAsync(host_tot, totals, 5 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                      st));
  PTRY(hipStreamSynchronize(st));
  out.n_leaves = (int64_t)nl;
  out.max_row_sources = (int64_t)host_tot[0];
  out.p2p_pairs = (int64_t)host_tot[1];
  out.n_runs = (int64_t)host_tot[2];
  out.n_items = (int64_t)host_tot[3];
  out.n_partials = (int64_t)host_tot[4];
  // the plan stores run, item and partial-slot offsets as 32-bit integers
  if (out.n_runs > INT32_MAX || out.n_items > INT32_MAX || out.n_partials > INT32_MAX) {
    release();
    return (int)hipErrorInvalidValue;
  }
  PTRY(scan(nruns, run_off, nl));
  PTRY(scan(nitems, item_off, nl));
  PTRY(scan(nparts, out.leaf_pbase, nl));
  PTRY(hipMalloc(&out.items, (size_t)(out.n_items > 0 ? out.n_items : 1) * sizeof(P2PItem)));
  PTRY(hipMalloc(&out.run_body, (size_t)(out.n_runs > 0 ? out.n_runs : 1) * 4));
  PTRY(hipMalloc(&out.run_prefix, (size_t)(out.n_runs > 0 ? out.n_runs : 1) * 4));
  plan_write<<<(unsigned)nl, 64, 0, st>>>((int64_t)nl, out.leaf_cell, p2p_ptr, p2p_col,
                                           body_begin, n_body, nruns, run_off, item_off,
                                           out.leaf_pbase, out.leaf_nchunk, layouts, out.items,
                                           out.run_body, out.run_prefix, out.body_leaf);
  PTRY(hipGetLastError());
  free_temps();
  PTRY(hipStreamSynchronize(st));
  return 0;
}

namespace {

// Estimated work of an item's wave, in units of 16 VALU instructions (at
// most 0xffff): each staged batch of nb sources takes ceil(nb / K) steps
// over the R targets of a lane (about 14 instructions per target, 3 per
// step) and about 90 for staging and the run lookup; the item adds the
// log2(K) levels of its stream merge (16 R each) and a fixed 2500 for its
// set-up, the latency of its first loads and its stores.  The fixed part is
// measured, not counted: with 200 the XCD ranges full of small items (the
// outskirts of a Plummer sphere) ran well past their estimate, and P2P on
// a Plummer sphere of 10^6 bodies took 1.74 ms against 1.56, 1.49 and
// 1.45 ms with 800, 1500 and 2500 (the uniform cube: 1.76-1.77 ms for all).
__device__ __forceinline__ uint32_t p2p_item_cost(const P2PItem &it) {
  const int64_t R = (it.tgt_cfg >> 8) & 0xff, K = (it.tgt_cfg >> 24) & 0xff;
  const int64_t nb = kP2PStageBatch;
  auto phase = [&](int64_t n) -> int64_t {
    if (n <= 0 || K <= 0) return 0;
    const int64_t full = n / nb, part = n - full * nb;
    const int64_t steps = full * ((nb + K - 1) / K) + (part + K - 1) / K;
    return steps * (14 * R + 3) + 90 * (full + (part > 0 ? 1 : 0));
  };
  int64_t levels = 0;
  for (int64_t k = 1; k < K; k <<= 1) ++levels;
  const int64_t u = (phase(it.n_src) + phase(it.self_n) + 16 * R * levels + 2500) >> 4;
  return (uint32_t)(u < 0xffff ? u : 0xffff);
}

// The work of unit i, which balances the XCD ranges, and its rank within a
// range (at most 0xffff; higher ranks start first).  A P2P item: its
// estimated cost, both.
struct P2PItemWork {
  const P2PItem *items;
  __device__ int64_t operator()(int64_t i) const { return p2p_item_cost(items[i]); }
  __device__ uint32_t rank(int64_t i) const { return p2p_item_cost(items[i]); }
};

// An M2L row: one pass of its wave per 64 entries plus one for the row's
// set-up and final sum over the lanes; ranked by its length.
struct M2LRowWork {
  const int64_t *ptr;
  __device__ int64_t operator()(int64_t i) const { return (ptr[i + 1] - ptr[i] + 63) / 64 + 1; }
  __device__ uint32_t rank(int64_t i) const {
    const int64_t len = ptr[i + 1] - ptr[i];
    return (uint32_t)(len < 0xffff ? len : 0xffff);
  }
};

// XCD range of unit i: the eighth of the total work t that holds the middle
// of the unit's work (prefix: exclusive prefix sums of the work).  It does
// not decrease with i, since 2 prefix[i] + w(i) = prefix[i] + prefix[i + 1]
// grows.
template <class Work>
__device__ __forceinline__ int64_t xcd_range(int64_t i, const Work &w,
                                             const int64_t *__restrict__ prefix, int64_t t) {
  const int64_t x = t > 0 ? (8 * (2 * prefix[i] + w(i))) / (2 * t) : 0;
  return x < 7 ? x : 7;
}

// Keys of a balanced order: the XCD range of unit i above its inverted rank.
// As the ranges do not decrease with i, range r holds the units
// [first[r], first[r + 1]) (first[8] = n): each unit whose range differs
// from its predecessor's writes the first[] entries of the ranges between.
template <class Work>
__global__ __launch_bounds__(256) void balanced_order_keys(int64_t n, Work w,
                                                           const int64_t *__restrict__ prefix,
                                                           const int64_t *__restrict__ total,
                                                           uint32_t *__restrict__ keys,
                                                           int32_t *__restrict__ vals,
                                                           int32_t *__restrict__ first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t t = *total;
  const int64_t x = xcd_range(i, w, prefix, t);
  const int64_t xp = i > 0 ? xcd_range(i - 1, w, prefix, t) : -1;
  keys[i] = ((uint32_t)x << 16) | (0xffffu - w.rank(i));
  vals[i] = (int32_t)i;
  for (int64_t r = xp + 1; r <= x; ++r) first[r] = (int32_t)i;
  if (i == n - 1)
    for (int64_t r = x + 1; r <= 8; ++r) first[r] = (int32_t)n;
}

struct RangeStarts {
  int32_t first[8];
};

// order[8 j + x] = the j-th unit of range x (the units sorted by key, so
// range x at sorted positions [first[x], first[x + 1])).
__global__ __launch_bounds__(256) void balanced_order_scatter(int64_t n,
                                                              const uint32_t *__restrict__ keys,
                                                              const int32_t *__restrict__ vals,
                                                              RangeStarts rs,
                                                              int32_t *__restrict__ order) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int x = (int)(keys[k] >> 16);
  order[8 * (k - rs.first[x]) + x] = vals[k];
}

__global__ __launch_bounds__(256) void fill_i32(int64_t n, int32_t v, int32_t *__restrict__ p) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

// One XCD-balanced dispatch order of n units (see dispatch_orders in
// kernels.h): eight contiguous ranges of about equal work, range x for XCD
// x, each by decreasing rank (ties in unit order), interleaved as
// order[8 j + x] with -1 past a range's end.  sort() enqueues the work's
// prefix sums, the keys (and the first unit of each range, into first[0..8])
// and the sort; scatter() the order itself, from first[] read back.
template <class Work>
struct OrderJob {
  int64_t n;
  Work w;
  int64_t *prefix = nullptr, *total = nullptr;
  uint32_t *keys = nullptr, *keys_alt = nullptr;
  int32_t *vals = nullptr, *vals_alt = nullptr;
  void *scratch = nullptr;
  bool in_alt = false;

  hipError_t sort(int32_t *first, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const size_t sb = std::max(prims::radix_scratch_bytes(n), prims::scan_scratch_bytes<int64_t>(n));
    hipError_t e;
    if ((e = hipMallocAsync((void **)&prefix, (size_t)n * 8, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&total, 8, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&keys, (size_t)n * 4, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&keys_alt, (size_t)n * 4, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&vals, (size_t)n * 4, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync((void **)&vals_alt, (size_t)n * 4, st)) != hipSuccess) return e;
    if ((e = hipMallocAsync(&scratch, sb, st)) != hipSuccess) return e;
    e = prims::exclusive_scan<int64_t>(n, w, prims::StoreArray<int64_t, int64_t>{prefix},
                                       (int64_t *)scratch, total, st);
    if (e != hipSuccess) return e;
    balanced_order_keys<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, w, prefix, total, keys,
                                                                      vals, first);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return prims::radix_sort<uint32_t>(keys, keys_alt, vals, vals_alt, n, 0, 19, scratch, st,
                                       &in_alt);
  }

  hipError_t scatter(const int32_t *first, int32_t **order, int64_t *n_order, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    RangeStarts rs;
    int64_t widest = 0;
    for (int x = 0; x < 8; ++x) {
      rs.first[x] = first[x];
      widest = std::max<int64_t>(widest, (int64_t)first[x + 1] - first[x]);
    }
    const int64_t m = 8 * widest;
    hipError_t e = hipMalloc((void **)order, (size_t)m * 4);
    if (e != hipSuccess) return e;
    *n_order = m;
    fill_i32<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(m, -1, *order);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    balanced_order_scatter<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
        n, in_alt ? keys_alt : keys, in_alt ? vals_alt : vals, rs, *order);
    return hipGetLastError();
  }

  void free_temps(hipStream_t st) {
    void *ps[] = {prefix, total, keys, keys_alt, vals, vals_alt, scratch};
    for (void *q : ps)
      if (q) (void)hipFreeAsync(q, st);
  }
};

}  // namespace

int dispatch_orders(DevicePlan &plan, const int64_t *m2l_ptr, int64_t n_cells,
                    int32_t **m2l_order, int64_t *m2l_len, void *stream) {
  if (plan.order) (void)hipFree(plan.order);
  if (*m2l_order) (void)hipFree(*m2l_order);
  plan.order = *m2l_order = nullptr;
  plan.order_len = *m2l_len = 0;
  if (plan.n_items <= 0 && n_cells <= 0) return 0;
  if (int rc = keep_pool_memory()) return rc;
  hipStream_t st;
  if (int rc = build_stream(stream, reinterpret_cast<void **>(&st))) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  OrderJob<P2PItemWork> pj{plan.n_items, P2PItemWork{plan.items}};
  OrderJob<M2LRowWork> mj{n_cells, M2LRowWork{m2l_ptr}};
  int32_t *first = nullptr;  // first unit of each range: P2P [0, 9), M2L [9, 18)
  int32_t host_first[18] = {};
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t r) {
    if (e == hipSuccess) e = r;
    return e == hipSuccess;
  };
  double t_sorted = 0.0;
  if (ok(hipMallocAsync((void **)&first, sizeof(host_first), st))) {
    if (ok(pj.sort(first, st)) && ok(mj.sort(first + 9, st)) &&
        ok(hipMemcpyAsync(host_first, first, sizeof(host_first), hipMemcpyDeviceToHost, st)) &&
        ok(hipStreamSynchronize(st))) {
      t_sorted = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                     .count();
      if (ok(pj.scatter(host_first, &plan.order, &plan.order_len, st)))
        ok(mj.scatter(host_first + 9, m2l_order, m2l_len, st));
    }
  }
  pj.free_temps(st);
  mj.free_temps(st);
  if (first) (void)hipFreeAsync(first, st);
  ok(hipStreamSynchronize(st));
  if (e != hipSuccess) {
    if (plan.order) (void)hipFree(plan.order);
    if (*m2l_order) (void)hipFree(*m2l_order);
    plan.order = *m2l_order = nullptr;
    plan.order_len = *m2l_len = 0;
  } else if (std::getenv("FMM_LOG")) {
    std::fprintf(stderr, "[fmm] dispatch orders: %.2f ms (sorted and counted %.2f ms)\n",
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                     .count(),
                 t_sorted);
  }
  return (int)e;
}

void DevicePlan::release() {
  void *ps[] = {items, order, run_body, run_prefix, leaf_cell, leaf_pbase, leaf_nchunk,
                body_leaf};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  *this = DevicePlan();
}

}  // namespace dev
}  // namespace fmmlib
