// Work plan of the P2P kernel built on the device from device CSR lists, with
// the same chunking, run merging, item order and partial-slot layout as the
// host builder, so both give the same plan entry for entry.
//
// One thread per leaf walks the leaf's P2P row twice: a counting pass (runs,
// chunks, source bodies, body pairs) and, after prefix sums give every leaf
// its offsets, a writing pass.  The walk is sequential (each chunk and run
// depends on the ones before), with the row's entries loaded in batches.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <hipcub/hipcub.hpp>

#include "kernels.h"

namespace fmmlib {
namespace dev {

namespace {

constexpr int kWalkBatch = 8;

struct Chunk {
  int32_t run_begin, n_runs, n_src;
  bool self;
};

// Walk row `a` (leaf with nA bodies starting at bA).  on_run(body, prefix)
// is called for each new run, on_chunk(index, chunk) for each finished chunk.
// Returns the number of chunks; *row_src and *pairs get the source bodies and
// body pairs of the row.
template <class OnRun, class OnChunk>
__device__ int walk_row(int32_t a, int64_t bA, int64_t nA, const int64_t *__restrict__ ptr,
                        const int32_t *__restrict__ col, const int32_t *__restrict__ body_begin,
                        const int32_t *__restrict__ n_body, int32_t run_base, int64_t *row_src,
                        int64_t *pairs, OnRun on_run, OnChunk on_chunk) {
  int nch = 0;
  int32_t runs = 0;  // runs of this row so far
  Chunk cur{run_base, 0, 0, false};
  int64_t last_end = -1;
  int64_t src = 0, pr = 0;
  // Entries are read eight at a time (the column, then the source leaf's
  // bodies), so a long row costs two memory round trips per eight entries
  // rather than per entry; they are then taken in order, as on the host.
  const int64_t e_end = ptr[a + 1];
  for (int64_t e0 = ptr[a]; e0 < e_end; e0 += kWalkBatch) {
    int32_t bq[kWalkBatch];
    int32_t nbq[kWalkBatch], bbq[kWalkBatch];
#pragma unroll
    for (int k = 0; k < kWalkBatch; ++k) bq[k] = e0 + k < e_end ? col[e0 + k] : 0;
#pragma unroll
    for (int k = 0; k < kWalkBatch; ++k) {
      nbq[k] = e0 + k < e_end ? n_body[bq[k]] : 0;
      bbq[k] = e0 + k < e_end ? body_begin[bq[k]] : 0;
    }
#pragma unroll
    for (int k = 0; k < kWalkBatch; ++k) {
      if (e0 + k >= e_end) break;
      const int32_t b = bq[k];
      const int64_t nb = nbq[k], bb = bbq[k];
      src += nb;
      pr += nA * nb - (b == a ? nA : 0);
      const bool contiguous = (b != a) && cur.n_runs > 0 && last_end == bb;
      const bool full = (cur.n_src + (cur.self ? nA : 0) + nb > kP2PChunkSources &&
                         (cur.n_src > 0 || cur.self)) ||
                        (!contiguous && b != a && cur.n_runs >= kP2PMaxRuns);
      if (full) {
        on_chunk(nch++, cur);
        cur = Chunk{run_base + runs, 0, 0, false};
        last_end = -1;
      }
      if (b == a) {
        cur.self = true;
        last_end = -1;
        continue;
      }
      if (cur.n_runs > 0 && last_end == bb) {
        last_end = bb + nb;
      } else {
        on_run(runs, (int32_t)bb, cur.n_src);
        ++runs;
        cur.n_runs++;
        last_end = bb + nb;
      }
      cur.n_src += (int32_t)nb;
    }
  }
  if (cur.n_src > 0 || cur.self || nch == 0) on_chunk(nch++, cur);
  *row_src = src;
  *pairs = pr;
  return nch;
}

__global__ void leaf_flags(int64_t nc, const int32_t *__restrict__ n_child,
                           int32_t *__restrict__ flag) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nc) flag[c] = n_child[c] == 0;
}

// Per leaf: cell, run count, item count, partial slots, chunks; row maxima
// and pair totals by integer atomics (order-independent).
__global__ void plan_count(int64_t nc, const int32_t *__restrict__ n_child,
                           const int32_t *__restrict__ leaf_of, const int64_t *__restrict__ ptr,
                           const int32_t *__restrict__ col, const int32_t *__restrict__ body_begin,
                           const int32_t *__restrict__ n_body, int32_t *__restrict__ leaf_cell,
                           int32_t *__restrict__ nruns, int32_t *__restrict__ nitems,
                           int32_t *__restrict__ nparts, int32_t *__restrict__ nchunk,
                           unsigned long long *__restrict__ totals) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nc || n_child[a] != 0) return;
  const int32_t leaf = leaf_of[a];
  const int64_t nA = n_body[a], bA = body_begin[a];
  int32_t runs = 0;
  int64_t src, pairs;
  const int nch = walk_row(
      (int32_t)a, bA, nA, ptr, col, body_begin, n_body, 0, &src, &pairs,
      [&](int32_t, int32_t, int32_t) { ++runs; }, [&](int, const Chunk &) {});
  leaf_cell[leaf] = (int32_t)a;
  nruns[leaf] = runs;
  nitems[leaf] = (int32_t)((nA + 63) / 64) * nch;
  nparts[leaf] = (int32_t)(nch * nA);
  nchunk[leaf] = nch;
  atomicMax(&totals[0], (unsigned long long)src);
  atomicAdd(&totals[1], (unsigned long long)pairs);
  atomicAdd(&totals[2], (unsigned long long)runs);
  atomicAdd(&totals[3], (unsigned long long)((nA + 63) / 64) * nch);
  atomicAdd(&totals[4], (unsigned long long)nch * nA);
}

__global__ void plan_write(int64_t n_leaves, const int32_t *__restrict__ leaf_cell,
                           const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           const int32_t *__restrict__ body_begin,
                           const int32_t *__restrict__ n_body, const int32_t *__restrict__ run_off,
                           const int32_t *__restrict__ item_off,
                           const int32_t *__restrict__ pbase, const int32_t *__restrict__ nchunk,
                           PlanLayouts layouts, P2PItem *__restrict__ items,
                           int32_t *__restrict__ run_body, int32_t *__restrict__ run_prefix,
                           int32_t *__restrict__ body_leaf) {
  const int64_t leaf = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (leaf >= n_leaves) return;
  const int32_t a = leaf_cell[leaf];
  const int64_t nA = n_body[a], bA = body_begin[a];
  const int32_t r0 = run_off[leaf], i0 = item_off[leaf], pb = pbase[leaf], nch = nchunk[leaf];
  const int64_t ng = (nA + 63) / 64;
  int64_t src, pairs;
  walk_row(
      a, bA, nA, ptr, col, body_begin, n_body, r0, &src, &pairs,
      [&](int32_t k, int32_t body, int32_t prefix) {
        run_body[r0 + k] = body;
        run_prefix[r0 + k] = prefix;
      },
      [&](int c, const Chunk &ch) {
        for (int64_t gi = 0; gi < ng; ++gi) {
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
  for (int64_t i = bA; i < bA + nA; ++i) body_leaf[i] = (int32_t)leaf;
}

__global__ void plan_zero_totals(unsigned long long *__restrict__ totals) {
  if (threadIdx.x < 8) totals[threadIdx.x] = 0;
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
  void *scan_tmp = nullptr;
  // temporaries from the stream-ordered pool, freed in stream order
  auto free_temps = [&]() {
    void *ps[] = {leaf_flag, leaf_of, nruns, nitems, nparts, run_off, item_off, totals, scan_tmp};
    for (void *p : ps)
      if (p) (void)hipFreeAsync(p, st);
    leaf_flag = leaf_of = nruns = nitems = nparts = run_off = item_off = nullptr;
    totals = nullptr;
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
  PTRY(hipMalloc(&out.leaf_cell, nl * 4));
  PTRY(hipMalloc(&out.leaf_pbase, nl * 4));
  PTRY(hipMalloc(&out.leaf_nchunk, nl * 4));
  PTRY(hipMalloc(&out.body_leaf, (size_t)(n > 0 ? n : 1) * 4));

  size_t tb = 0, tb2 = 0;
  PTRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, leaf_flag, leaf_of, (int)nc, st));
  PTRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, nruns, run_off, (int)nl, st));
  tb = tb > tb2 ? tb : tb2;
  PTRY(hipMallocAsync(&scan_tmp, tb > 0 ? tb : 1, st));

  const unsigned bc = (unsigned)((nc + 255) / 256), bl = (unsigned)((nl + 255) / 256);
  leaf_flags<<<bc, 256, 0, st>>>((int64_t)nc, n_child, leaf_flag);
  PTRY(hipGetLastError());
  tb2 = tb;
  PTRY(hipcub::DeviceScan::ExclusiveSum(scan_tmp, tb2, leaf_flag, leaf_of, (int)nc, st));
  // totals: [0] max row sources, [1] body pairs, [2] runs, [3] items, [4] partial
  // slots, all by 64-bit integer atomics
  plan_zero_totals<<<1, 8, 0, st>>>(totals);
  PTRY(hipGetLastError());
  plan_count<<<bc, 256, 0, st>>>((int64_t)nc, n_child, leaf_of, p2p_ptr, p2p_col, body_begin,
                                  n_body, out.leaf_cell, nruns, nitems, nparts, out.leaf_nchunk,
                                  totals);
  PTRY(hipGetLastError());
  unsigned long long host_tot[8] = {};
  PTRY(hipMemcpyAsync(host_tot, totals, sizeof(host_tot), hipMemcpyDeviceToHost, st));
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
  tb2 = tb;
  PTRY(hipcub::DeviceScan::ExclusiveSum(scan_tmp, tb2, nruns, run_off, (int)nl, st));
  tb2 = tb;
  PTRY(hipcub::DeviceScan::ExclusiveSum(scan_tmp, tb2, nitems, item_off, (int)nl, st));
  tb2 = tb;
  PTRY(hipcub::DeviceScan::ExclusiveSum(scan_tmp, tb2, nparts, out.leaf_pbase, (int)nl, st));
  PTRY(hipMalloc(&out.items, (size_t)(out.n_items > 0 ? out.n_items : 1) * sizeof(P2PItem)));
  PTRY(hipMalloc(&out.run_body, (size_t)(out.n_runs > 0 ? out.n_runs : 1) * 4));
  PTRY(hipMalloc(&out.run_prefix, (size_t)(out.n_runs > 0 ? out.n_runs : 1) * 4));
  plan_write<<<bl, 256, 0, st>>>((int64_t)nl, out.leaf_cell, p2p_ptr, p2p_col, body_begin, n_body,
                                 run_off, item_off, out.leaf_pbase, out.leaf_nchunk, layouts,
                                 out.items, out.run_body, out.run_prefix, out.body_leaf);
  PTRY(hipGetLastError());
  free_temps();
  PTRY(hipStreamSynchronize(st));
  return 0;
}

void DevicePlan::release() {
  void *ps[] = {items, run_body, run_prefix, leaf_cell, leaf_pbase, leaf_nchunk, body_leaf};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  *this = DevicePlan();
}

}  // namespace dev
}  // namespace fmmlib
