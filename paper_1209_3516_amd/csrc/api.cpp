// C interface of the GPU FMM library (declared in include/fmm.h).
//
// fmm_tree_build / fmm_traverse run on the host and never touch the GPU; the
// first evaluation on such a (tree, lists) pair uploads the tree, the lists
// and the P2P work plan.  fmm_tree_build_gpu / fmm_traverse_gpu build the
// same tree, lists and plan on the device and keep them there; the host copy
// of device-built lists is made on the first fmm_lists_view.  Device scratch
// is sized per (p, precision).  Every kernel of one evaluation is enqueued on
// the caller's stream with no host synchronisation in between.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fmm.h"
#include "fmm_internal.h"
#include "kernels.h"
#include "shard.h"

namespace {

thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }

std::atomic<uint64_t> g_next_tree_id{1};

// Fault injection for the failure-handling tests: FMM_FAULT_INJECT=launch:K
// makes the K-th kernel launch of every evaluation (counted from 1) report a
// device error instead of launching.
int fault_launch_target() {
  const char *s = std::getenv("FMM_FAULT_INJECT");
  if (!s || std::strncmp(s, "launch:", 7) != 0) return -1;
  return std::atoi(s + 7);
}
thread_local int g_launch_counter = 0;
thread_local int g_alloc_counter = 0;

struct DevTree {
  int device = -1;
  int64_t n = 0, n_cells = 0;
  uint64_t pos_version_32 = ~0ull, pos_version_64 = ~0ull;
  void *b32 = nullptr;  // float4[n]
  void *b64 = nullptr;  // double4[n]
  int32_t *perm = nullptr;
  double *geo = nullptr;  // double4[n_cells]: centre, radius
  int32_t *body_begin = nullptr, *n_body = nullptr, *child_begin = nullptr, *n_child = nullptr,
          *parent = nullptr;
  // trees built on the device: Morton-ordered FP64 positions and keys stay
  // there, and the host copies of perm, keys and positions are made on demand
  double *pos = nullptr;
  uint64_t *keys = nullptr;
  uint64_t pos_dev_version = ~0ull;  // tree positions version that `pos` holds
  bool host_bodies = true;
  void release() {
    void *ptrs[] = {b32, b64, perm, geo, body_begin, n_body, child_begin, n_child, parent, pos,
                    keys};
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
    *this = DevTree();
  }
};

struct DevLists {
  int device = -1;
  bool uploaded = false;  // lists and P2P plan are on the device
  bool host_valid = true;  // ListData holds the CSR lists (else only the device does)
  int64_t *m2l_ptr = nullptr, *p2p_ptr = nullptr;
  int32_t *m2l_col = nullptr, *p2p_col = nullptr;
  // M2L dispatch order for a launch over all cells (m2l_order_len entries)
  int32_t *m2l_order = nullptr;
  int64_t m2l_order_len = 0;
  int64_t p2p_nnz = 0, m2l_nnz = 0;
  // hybrid lists: M2P CSR and the target leaves that have M2P entries
  int64_t *m2p_ptr = nullptr;
  int32_t *m2p_col = nullptr, *m2p_rows = nullptr;
  int64_t n_m2p_rows = 0;
  void *m2p_buf = nullptr;  // [n] (phi, grad) of M2P, Morton order; zero where unused
  fmmlib::dev::DevicePlan plan;
  // host copies for target-range evaluations: chunks and first item per leaf
  std::vector<int32_t> leaf_nchunk_host;
  std::vector<int64_t> leaf_item_host;
  // scratch for one (p, precision, top) configuration
  int p = 0, prec = -1;
  int64_t n_top = -1;
  void *M = nullptr, *L = nullptr, *Lstage = nullptr;
  void *Mr = nullptr;  // multipoles folded for M2L (stride rstride(p))
  double *M64 = nullptr, *L64 = nullptr, *L64stage = nullptr;
  void *part_s = nullptr, *part_c = nullptr;
  void *tmp_phi = nullptr, *tmp_grad = nullptr;
  void *vec4 = nullptr, *tmp_hv = nullptr;  // backward with a gradient upstream
  bool stage_valid = false;
  // batched M2L of box-centred trees: the plan (built on first use) and the
  // derivative table of its vectors for order dtab_p
  bool mfma_ready = false;
  int32_t *mt_cells = nullptr, *mt_goff = nullptr, *mt_gsrc = nullptr;
  int64_t *mt_gbeg = nullptr;
  double *mt_off = nullptr;
  float *mt_dtab = nullptr;
  int mt_dtab_p = 0;
  int64_t mt_n_tiles = 0, mt_n_groups = 0, mt_n_off = 0;
  std::vector<int64_t> mt_level_tile;
  // mutual P2P: its plan (built on first use) and the source-side sums
  bool mp_ready = false;
  fmmlib::P2PItem *mp_items = nullptr;
  int32_t *mp_run_body = nullptr, *mp_run_prefix = nullptr, *mp_run_dst = nullptr;
  int32_t *mp_leaf_pbase = nullptr, *mp_leaf_nchunk = nullptr, *mp_leaf_mbase = nullptr,
          *mp_leaf_nlow = nullptr;
  int64_t mp_n_items = 0, mp_n_partials = 0, mp_n_mslots = 0;
  void *part_m = nullptr;
  int64_t part_slots = 0;  // partial-sum slots part_s and part_c hold
  // near-field stream (forked from / joined into the caller's stream)
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // timing: each timed evaluation records 8 marks on the caller's stream and
  // 2 around P2P into the next of FMM_TIMING_HISTORY sets, so that a run of
  // evaluations can be timed and read afterwards without waiting between
  // them.  ring_count: consecutive timed evaluations held, the last one
  // newest (an evaluation without timing sets it to 0).
  hipEvent_t ev[FMM_TIMING_HISTORY][FMM_NUM_PHASES + 2] = {};
  bool ev_made[FMM_TIMING_HISTORY] = {};
  bool ring_serial[FMM_TIMING_HISTORY] = {};
  int ring_next = 0, ring_count = 0;
  void release_scratch() {
    void *ptrs[] = {M, Mr, L, Lstage, M64, L64, L64stage, part_s, part_c, tmp_phi, tmp_grad,
                    vec4, tmp_hv, m2p_buf};
    for (void *p2 : ptrs)
      if (p2) (void)hipFree(p2);
    M = Mr = L = Lstage = part_s = part_c = tmp_phi = tmp_grad = vec4 = tmp_hv = m2p_buf = nullptr;
    M64 = L64 = L64stage = nullptr;
    p = 0;
    prec = -1;
    n_top = -1;
    part_slots = 0;
    stage_valid = false;
  }
  // the mutual P2P's plan and source-side sums
  void release_mutual() {
    void *ptrs[] = {mp_items,      mp_run_body,    mp_run_prefix, mp_run_dst, mp_leaf_pbase,
                    mp_leaf_nchunk, mp_leaf_mbase, mp_leaf_nlow,  part_m};
    for (void *p2 : ptrs)
      if (p2) (void)hipFree(p2);
    mp_items = nullptr;
    mp_run_body = mp_run_prefix = mp_run_dst = nullptr;
    mp_leaf_pbase = mp_leaf_nchunk = mp_leaf_mbase = mp_leaf_nlow = nullptr;
    part_m = nullptr;
    mp_n_items = mp_n_partials = mp_n_mslots = 0;
    mp_ready = false;
  }
  void release() {
    release_scratch();
    release_mutual();
    plan.release();
    void *ptrs[] = {m2l_ptr, m2l_col, m2l_order, p2p_ptr, p2p_col, m2p_ptr, m2p_col, m2p_rows,
                    mt_cells, mt_goff, mt_gsrc, mt_gbeg, mt_off, mt_dtab};
    for (void *p2 : ptrs)
      if (p2) (void)hipFree(p2);
    for (int k = 0; k < FMM_TIMING_HISTORY; ++k)
      if (ev_made[k])
        for (auto &e : ev[k]) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (side) (void)hipStreamDestroy(side);
    *this = DevLists();
  }
};

}  // namespace

struct fmm_tree {
  fmmlib::TreeData data;
  DevTree dev;
  fmmlib::LeafIndex leaf_ix;  // built on the first target-range call
  bool leaf_ix_valid = false;
};

struct fmm_lists {
  fmmlib::ListData data;
  DevLists dev;
  // P2P work plan of host-built lists, made by the traversal and released
  // once the first evaluation has uploaded it
  fmmlib::P2PPlan host_plan;
};

namespace fmmlib {
void reset_alloc_checkpoints() { g_alloc_counter = 0; }
void alloc_checkpoint() {
  const char *s = std::getenv("FMM_FAULT_INJECT");
  if (!s || std::strncmp(s, "alloc:", 6) != 0) return;
  if (++g_alloc_counter == std::atoi(s + 6)) throw std::bad_alloc();
}
}  // namespace fmmlib

namespace {

int hip_fail(hipError_t e, const char *what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? FMM_ENOMEM : FMM_EDEVICE;
}

#define HIP_TRY(call)                                 \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

#define LAUNCH_TRY(call)                                                        \
  do {                                                                          \
    const int tgt_ = fault_launch_target();                                     \
    if (tgt_ > 0 && ++g_launch_counter == tgt_) {                               \
      set_error(std::string("injected device fault before ") + #call);          \
      return FMM_EDEVICE;                                                       \
    }                                                                           \
    int e_ = (call);                                                            \
    if (e_ != 0) return hip_fail((hipError_t)e_, #call);                        \
  } while (0)

template <typename T>
int dev_upload(T **dst, const T *src, size_t count) {
  // Empty arrays still get a valid (one-element) allocation.
  HIP_TRY(hipMalloc((void **)dst, std::max<size_t>(1, count) * sizeof(T)));
  if (src && count > 0) HIP_TRY(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return FMM_OK;
}

int current_device(int *dev) {
  HIP_TRY(hipGetDevice(dev));
  return FMM_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Host copies of the per-body arrays of a tree built on the device.
int ensure_tree_host_bodies(fmm_tree *t) {
  DevTree &dv = t->dev;
  if (dv.host_bodies) return FMM_OK;
  fmmlib::TreeData &d = t->data;
  const int64_t n = d.n;
  try {
    d.perm.resize(n);
    d.keys.resize(n);
    d.pos.resize(3 * n);
  } catch (const std::bad_alloc &) {
    set_error("out of host memory");
    return FMM_ENOMEM;
  }
  HIP_TRY(hipMemcpy(d.perm.data(), dv.perm, n * 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(d.keys.data(), dv.keys, n * 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(d.pos.data(), dv.pos, n * 24, hipMemcpyDeviceToHost));
  dv.host_bodies = true;
  return FMM_OK;
}

int ensure_tree_device(fmm_tree *t, bool fp64, void *stream) {
  fmmlib::TreeData &d = t->data;
  DevTree &dv = t->dev;
  int dev;
  if (int rc = current_device(&dev)) return rc;
  if (dv.device >= 0 && dv.device != dev) {
    set_error("tree was first used on another device");
    return FMM_ESTATE;
  }
  if (dv.device < 0) {
    dv.device = dev;
    dv.n = d.n;
    dv.n_cells = d.n_cells();
    const int64_t nc = d.n_cells();
    std::vector<double> geo(4 * nc);
    std::vector<int32_t> bb(nc), nb(nc);
    for (int64_t c = 0; c < nc; ++c) {
      for (int k = 0; k < 3; ++k) geo[4 * c + k] = d.center[3 * c + k];
      geo[4 * c + 3] = d.radius[c];
      bb[c] = (int32_t)d.body_begin[c];
      nb[c] = (int32_t)d.n_body[c];
    }
    if (int rc = dev_upload(&dv.perm, d.perm.data(), d.n)) return rc;
    if (int rc = dev_upload(&dv.geo, geo.data(), 4 * nc)) return rc;
    if (int rc = dev_upload(&dv.body_begin, bb.data(), nc)) return rc;
    if (int rc = dev_upload(&dv.n_body, nb.data(), nc)) return rc;
    if (int rc = dev_upload(&dv.child_begin, d.child_begin.data(), nc)) return rc;
    if (int rc = dev_upload(&dv.n_child, d.n_child.data(), nc)) return rc;
    if (int rc = dev_upload(&dv.parent, d.parent.data(), nc)) return rc;
  }
  const bool dev_pos = dv.pos && dv.pos_dev_version == d.pos_version;
  if (dev_pos && ((fp64 && dv.pos_version_64 != d.pos_version) ||
                  (!fp64 && dv.pos_version_32 != d.pos_version))) {
    // pack from the device positions
    void **dst = fp64 ? &dv.b64 : &dv.b32;
    if (!*dst) HIP_TRY(hipMalloc(dst, std::max<int64_t>(1, d.n) * (fp64 ? 32 : 16)));
    HIP_TRY((hipError_t)fmmlib::dev::pack_positions(fp64, d.n, dv.pos, *dst, stream));
    HIP_TRY(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
    (fp64 ? dv.pos_version_64 : dv.pos_version_32) = d.pos_version;
  }
  if ((fp64 && dv.pos_version_64 != d.pos_version) ||
      (!fp64 && dv.pos_version_32 != d.pos_version))
    if (int rc = ensure_tree_host_bodies(t)) return rc;
  if (fp64 && dv.pos_version_64 != d.pos_version) {
    std::vector<double> b(4 * d.n);
    for (int64_t i = 0; i < d.n; ++i) {
      for (int k = 0; k < 3; ++k) b[4 * i + k] = d.pos[3 * i + k];
      b[4 * i + 3] = 0.0;
    }
    if (!dv.b64) HIP_TRY(hipMalloc(&dv.b64, std::max<int64_t>(1, d.n) * 32));
    HIP_TRY(hipMemcpy(dv.b64, b.data(), d.n * 32, hipMemcpyHostToDevice));
    dv.pos_version_64 = d.pos_version;
  }
  if (!fp64 && dv.pos_version_32 != d.pos_version) {
    std::vector<float> b(4 * d.n);
    for (int64_t i = 0; i < d.n; ++i) {
      for (int k = 0; k < 3; ++k) b[4 * i + k] = (float)d.pos[3 * i + k];
      b[4 * i + 3] = 0.0f;
    }
    if (!dv.b32) HIP_TRY(hipMalloc(&dv.b32, std::max<int64_t>(1, d.n) * 16));
    HIP_TRY(hipMemcpy(dv.b32, b.data(), d.n * 16, hipMemcpyHostToDevice));
    dv.pos_version_32 = d.pos_version;
  }
  return FMM_OK;
}

// The lane-layout table of the P2P plan, indexed by target count.
fmmlib::dev::PlanLayouts plan_layouts() {
  fmmlib::dev::PlanLayouts lay{};
  for (int nt = 1; nt <= 64; ++nt) {
    int R, L, K;
    fmmlib::p2p_lane_layout(nt, &R, &L, &K);
    lay.cfg[nt] = nt | (R << 8) | (L << 16) | (K << 24);
  }
  return lay;
}

int ensure_lists_device(fmm_tree *t, fmm_lists *l) {
  DevLists &dv = l->dev;
  if (dv.uploaded) {
    if (dv.device != t->dev.device) {
      set_error("lists were first used on another device");
      return FMM_ESTATE;
    }
    return FMM_OK;
  }
  const auto t0 = std::chrono::steady_clock::now();
  const fmmlib::ListData &ld = l->data;
  const fmmlib::P2PPlan &pl = l->host_plan;
  auto &dp = dv.plan;
  dp.release();
  if (int rc = dev_upload(&dv.m2l_ptr, ld.m2l_ptr.data(), ld.m2l_ptr.size())) return rc;
  if (int rc = dev_upload(&dv.m2l_col, ld.m2l_col.data(), ld.m2l_col.size())) return rc;
  if (!ld.m2p_col.empty()) {
    std::vector<int32_t> rows;
    for (int64_t c = 0; c < ld.n_rows; ++c)
      if (ld.m2p_ptr[c + 1] > ld.m2p_ptr[c]) rows.push_back((int32_t)c);
    if (int rc = dev_upload(&dv.m2p_ptr, ld.m2p_ptr.data(), ld.m2p_ptr.size())) return rc;
    if (int rc = dev_upload(&dv.m2p_col, ld.m2p_col.data(), ld.m2p_col.size())) return rc;
    if (int rc = dev_upload(&dv.m2p_rows, rows.data(), rows.size())) return rc;
    dv.n_m2p_rows = (int64_t)rows.size();
  }
  if (int rc = dev_upload(&dp.items, pl.items.data(), pl.items.size())) return rc;
  if (int rc = dev_upload(&dp.run_body, pl.run_body.data(), pl.run_body.size())) return rc;
  if (int rc = dev_upload(&dp.run_prefix, pl.run_prefix.data(), pl.run_prefix.size())) return rc;
  if (int rc = dev_upload(&dp.leaf_cell, pl.leaf_cell.data(), pl.leaf_cell.size())) return rc;
  if (int rc = dev_upload(&dp.leaf_pbase, pl.leaf_pbase.data(), pl.leaf_pbase.size())) return rc;
  if (int rc = dev_upload(&dp.leaf_nchunk, pl.leaf_nchunk.data(), pl.leaf_nchunk.size()))
    return rc;
  if (int rc = dev_upload(&dp.body_leaf, pl.body_leaf.data(), pl.body_leaf.size())) return rc;
  dp.n_items = (int64_t)pl.items.size();
  dp.n_runs = (int64_t)pl.run_body.size();
  dp.n_leaves = (int64_t)pl.leaf_cell.size();
  dp.n_partials = pl.n_partials;
  dp.max_row_sources = pl.max_row_sources;
  dp.p2p_pairs = ld.p2p_pairs;
  if (int rc = fmmlib::dev::dispatch_orders(dp, dv.m2l_ptr, ld.n_rows, &dv.m2l_order,
                                            &dv.m2l_order_len, nullptr))
    return hip_fail((hipError_t)rc, "dispatch_orders");
  dv.leaf_nchunk_host = pl.leaf_nchunk;
  dv.device = t->dev.device;
  dv.uploaded = true;
  l->host_plan = fmmlib::P2PPlan();  // the device holds it now
  if (std::getenv("FMM_LOG"))
    std::fprintf(stderr, "[fmm] work plan upload: %.2f ms (%lld items, %lld runs)\n",
                 ms_since(t0), (long long)dp.n_items, (long long)dp.n_runs);
  return FMM_OK;
}

// Host copy of lists that were built on the device.
int ensure_lists_host(fmm_lists *l) {
  DevLists &dv = l->dev;
  if (dv.host_valid) return FMM_OK;
  fmmlib::ListData &ld = l->data;
  const int64_t nr = ld.n_rows;
  try {
    ld.p2p_ptr.assign(nr + 1, 0);
    ld.m2l_ptr.assign(nr + 1, 0);
    ld.m2p_ptr.assign(nr + 1, 0);  // the GPU traversal builds no M2P list
    ld.p2p_col.resize(dv.p2p_nnz);
    ld.m2l_col.resize(dv.m2l_nnz);
  } catch (const std::bad_alloc &) {
    set_error("fmm_lists_view: out of host memory");
    return FMM_ENOMEM;
  }
  if (nr > 0) {
    HIP_TRY(hipMemcpy(ld.p2p_ptr.data(), dv.p2p_ptr, (nr + 1) * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ld.m2l_ptr.data(), dv.m2l_ptr, (nr + 1) * 8, hipMemcpyDeviceToHost));
    if (dv.p2p_nnz)
      HIP_TRY(hipMemcpy(ld.p2p_col.data(), dv.p2p_col, dv.p2p_nnz * 4, hipMemcpyDeviceToHost));
    if (dv.m2l_nnz)
      HIP_TRY(hipMemcpy(ld.m2l_col.data(), dv.m2l_col, dv.m2l_nnz * 4, hipMemcpyDeviceToHost));
  }
  dv.host_valid = true;
  return FMM_OK;
}

// The mutual P2P's plan on the device (built on the host on first use from
// the host copy of the lists) and its buffer of source-side sums.
int ensure_mutual(fmm_tree *t, fmm_lists *l) {
  DevLists &dv = l->dev;
  if (dv.mp_ready) return FMM_OK;
  if (int rc = ensure_lists_host(l)) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  fmmlib::P2PMutualPlan plan;
  std::string err;
  if (int rc = fmmlib::build_p2p_mutual_plan(t->data, l->data, plan, err)) {
    set_error(err);
    return rc;
  }
  // on a failure nothing is kept, so a later call starts afresh
  int rc = dev_upload(&dv.mp_items, plan.items.data(), plan.items.size());
  if (!rc) rc = dev_upload(&dv.mp_run_body, plan.run_body.data(), plan.run_body.size());
  if (!rc) rc = dev_upload(&dv.mp_run_prefix, plan.run_prefix.data(), plan.run_prefix.size());
  if (!rc) rc = dev_upload(&dv.mp_run_dst, plan.run_dst.data(), plan.run_dst.size());
  if (!rc) rc = dev_upload(&dv.mp_leaf_pbase, plan.leaf_pbase.data(), plan.leaf_pbase.size());
  if (!rc) rc = dev_upload(&dv.mp_leaf_nchunk, plan.leaf_nchunk.data(), plan.leaf_nchunk.size());
  if (!rc) rc = dev_upload(&dv.mp_leaf_mbase, plan.leaf_mbase.data(), plan.leaf_mbase.size());
  if (!rc) rc = dev_upload(&dv.mp_leaf_nlow, plan.leaf_nlow.data(), plan.leaf_nlow.size());
  if (!rc) {
    const hipError_t e =
        hipMalloc(&dv.part_m, (size_t)std::max<int64_t>(1, plan.n_mslots) * 16);
    if (e != hipSuccess) rc = hip_fail(e, "hipMalloc");
  }
  if (rc) {
    dv.release_mutual();
    return rc;
  }
  dv.mp_n_items = (int64_t)plan.items.size();
  dv.mp_n_partials = plan.n_partials;
  dv.mp_n_mslots = plan.n_mslots;
  dv.mp_ready = true;
  if (std::getenv("FMM_LOG"))
    std::fprintf(stderr,
                 "[fmm] mutual P2P plan: %lld items, %lld runs, %lld source slots, %.1f ms\n",
                 (long long)dv.mp_n_items, (long long)plan.run_body.size(),
                 (long long)plan.n_mslots, ms_since(t0));
  return FMM_OK;
}

// The batched M2L's plan on the device (built on the host on first use from
// the host copy of the lists) and its derivative table for order p.
int ensure_m2l_mfma(fmm_tree *t, fmm_lists *l, int p, void *stream) {
  DevLists &dv = l->dev;
  if (!t->data.box_centres) {
    set_error("FMM_EVAL_M2L_MFMA needs a tree built with FMM_TREE_BOX_CENTRES");
    return FMM_EINVAL;
  }
  if (!dv.mfma_ready) {
    if (int rc = ensure_lists_host(l)) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    fmmlib::M2LTilePlan plan;
    std::string err;
    if (int rc = fmmlib::build_m2l_tile_plan(t->data, l->data, plan, err)) {
      set_error(err);
      return rc;
    }
    // on a failure nothing is kept, so a later call starts afresh
    int rc = dev_upload(&dv.mt_cells, plan.tile_cells.data(), plan.tile_cells.size());
    if (!rc) rc = dev_upload(&dv.mt_gbeg, plan.tile_group_begin.data(), plan.tile_group_begin.size());
    if (!rc) rc = dev_upload(&dv.mt_goff, plan.group_offset.data(), plan.group_offset.size());
    if (!rc) rc = dev_upload(&dv.mt_gsrc, plan.group_src.data(), plan.group_src.size());
    if (!rc) rc = dev_upload(&dv.mt_off, plan.offsets.data(), plan.offsets.size());
    if (rc) {
      void *ps[] = {dv.mt_cells, dv.mt_gbeg, dv.mt_goff, dv.mt_gsrc, dv.mt_off};
      for (void *q : ps)
        if (q) (void)hipFree(q);
      dv.mt_cells = dv.mt_goff = dv.mt_gsrc = nullptr;
      dv.mt_gbeg = nullptr;
      dv.mt_off = nullptr;
      return rc;
    }
    dv.mt_n_tiles = plan.n_tiles;
    dv.mt_n_groups = plan.n_groups;
    dv.mt_n_off = plan.n_offsets;
    dv.mt_level_tile = plan.level_tile_begin;
    dv.mfma_ready = true;
    if (std::getenv("FMM_LOG"))
      std::fprintf(stderr, "[fmm] batched M2L plan: %lld tiles, %lld groups, %lld vectors, %.1f ms\n",
                   (long long)plan.n_tiles, (long long)plan.n_groups, (long long)plan.n_offsets,
                   ms_since(t0));
  }
  if (dv.mt_dtab_p != p) {
    if (dv.mt_dtab) (void)hipFree(dv.mt_dtab);
    dv.mt_dtab = nullptr;
    dv.mt_dtab_p = 0;
    HIP_TRY(hipMalloc((void **)&dv.mt_dtab,
                      std::max<int64_t>(1, dv.mt_n_off) * fmmlib::dev::terms(p) * sizeof(float)));
    HIP_TRY((hipError_t)fmmlib::dev::m2l_offsets(p, dv.mt_n_off, dv.mt_off, dv.mt_dtab, stream));
    dv.mt_dtab_p = p;
  }
  return FMM_OK;
}

// Leaf index of the tree and first P2P work item of every leaf.
int ensure_range_tables(fmm_tree *t, fmm_lists *l) {
  if (!t->leaf_ix_valid) {
    fmmlib::build_leaf_index(t->data, t->leaf_ix);
    t->leaf_ix_valid = true;
  }
  DevLists &dv = l->dev;
  if (!dv.leaf_item_host.empty()) return FMM_OK;
  const auto &ix = t->leaf_ix;
  const int64_t nl = (int64_t)ix.cell.size();
  if (dv.leaf_nchunk_host.size() != (size_t)nl) {
    dv.leaf_nchunk_host.resize(nl);
    if (nl > 0)
      HIP_TRY(hipMemcpy(dv.leaf_nchunk_host.data(), dv.plan.leaf_nchunk, nl * 4,
                        hipMemcpyDeviceToHost));
  }
  // items of one leaf: one per (group of 64 targets, source chunk), in leaf order
  dv.leaf_item_host.assign(nl + 1, 0);
  for (int64_t i = 0; i < nl; ++i)
    dv.leaf_item_host[i + 1] = dv.leaf_item_host[i] +
                               (t->data.n_body[ix.cell[i]] + 63) / 64 * dv.leaf_nchunk_host[i];
  if (dv.leaf_item_host[nl] != dv.plan.n_items) {
    set_error("internal error: P2P work items do not match the leaf table");
    return FMM_EDEVICE;
  }
  return FMM_OK;
}

int64_t top_cells(const fmmlib::TreeData &t, const fmm_eval_opts *o) {
  if (o->precision != FMM_MIXED) return 0;
  int top = o->fp64_top_levels;
  if (top == -1) top = o->p >= 8 ? 3 : -1;
  if (top < 0) return 0;
  top = std::min(top, t.max_level);
  return t.level_begin[top + 1];
}

int ensure_scratch(fmm_tree *t, fmm_lists *l, const fmm_eval_opts *o) {
  DevLists &dv = l->dev;
  const bool fp64 = o->precision == FMM_FP64;
  const int64_t n_top = top_cells(t->data, o);
  const int64_t slots = std::max<int64_t>(
      1, std::max<int64_t>(dv.plan.n_partials, dv.mp_ready ? dv.mp_n_partials : 0));
  if (dv.p == o->p && dv.prec == o->precision && dv.n_top == n_top && dv.part_slots >= slots)
    return FMM_OK;
  dv.release_scratch();
  const int64_t nc = t->data.n_cells(), n = t->data.n;
  const size_t real = fp64 ? 8 : 4;
  const size_t coef = (size_t)nc * fmmlib::dev::stride(o->p);
  HIP_TRY(hipMalloc(&dv.M, coef * real));
  HIP_TRY(hipMalloc(&dv.Mr, (size_t)nc * fmmlib::dev::rstride(o->p) * real));
  HIP_TRY(hipMalloc(&dv.L, coef * real));
  HIP_TRY(hipMalloc(&dv.Lstage, coef * real));
  if (n_top > 0) {
    const size_t tc = (size_t)n_top * fmmlib::dev::stride(o->p);
    HIP_TRY(hipMalloc((void **)&dv.M64, tc * 8));
    HIP_TRY(hipMalloc((void **)&dv.L64, tc * 8));
    HIP_TRY(hipMalloc((void **)&dv.L64stage, tc * 8));
  }
  const size_t np = (size_t)slots;
  HIP_TRY(hipMalloc(&dv.part_s, np * 4 * real));
  if (!fp64) HIP_TRY(hipMalloc(&dv.part_c, np * 4 * real));
  dv.part_slots = slots;
  HIP_TRY(hipMalloc(&dv.tmp_phi, std::max<int64_t>(1, n) * real));
  HIP_TRY(hipMalloc(&dv.tmp_grad, std::max<int64_t>(1, n) * 3 * real));
  HIP_TRY(hipMalloc(&dv.vec4, std::max<int64_t>(1, n) * 4 * real));
  HIP_TRY(hipMalloc(&dv.tmp_hv, std::max<int64_t>(1, n) * 3 * real));
  if (dv.n_m2p_rows > 0) {
    // bodies of leaves without M2P entries are never written: zero once
    HIP_TRY(hipMalloc(&dv.m2p_buf, std::max<int64_t>(1, n) * 4 * real));
    HIP_TRY(hipMemset(dv.m2p_buf, 0, std::max<int64_t>(1, n) * 4 * real));
  }
  dv.p = o->p;
  dv.prec = o->precision;
  dv.n_top = n_top;
  return FMM_OK;
}

int check_opts(const fmm_eval_opts *o) {
  if (!o) {
    set_error("opts is NULL");
    return FMM_EINVAL;
  }
  if (o->p < 1 || o->p > FMM_MAX_P) {
    set_error("p must be in 1..8");
    return FMM_EINVAL;
  }
  if (o->precision != FMM_MIXED && o->precision != FMM_FP64) {
    set_error("precision must be FMM_MIXED or FMM_FP64");
    return FMM_EINVAL;
  }
  if (o->fp64_top_levels < -2 || o->fp64_top_levels > FMM_MAX_LEVEL) {
    set_error("fp64_top_levels must be -2, -1 or 0..21");
    return FMM_EINVAL;
  }
  if (o->flags & ~(FMM_EVAL_TIMING | FMM_EVAL_KEEP_STAGES | FMM_EVAL_SERIAL | FMM_EVAL_M2L_MFMA |
                   FMM_EVAL_MUTUAL_P2P)) {
    set_error("unknown evaluation flags");
    return FMM_EINVAL;
  }
  if ((o->flags & FMM_EVAL_M2L_MFMA) && o->precision != FMM_MIXED) {
    set_error("FMM_EVAL_M2L_MFMA runs in FP32: it needs FMM_MIXED precision");
    return FMM_EINVAL;
  }
  if ((o->flags & FMM_EVAL_MUTUAL_P2P) && o->precision != FMM_MIXED) {
    set_error("FMM_EVAL_MUTUAL_P2P runs in FP32: it needs FMM_MIXED precision");
    return FMM_EINVAL;
  }
  return FMM_OK;
}

int check_pair(const fmm_tree *t, const fmm_lists *l) {
  if (!t || !l) {
    set_error("tree or lists is NULL");
    return FMM_EINVAL;
  }
  if (l->data.tree_id != t->data.id) {
    set_error("lists were built from another tree");
    return FMM_ESTATE;
  }
  return FMM_OK;
}

// Device buffers of one evaluation besides its inputs, outputs, tree and
// lists: multipoles (M, folded Mr), locals L, the FP64 top levels, the P2P
// partial sums, the gathered per-body vectors and the M2P results.
struct EvalScratch {
  void *M = nullptr, *Mr = nullptr, *L = nullptr;
  double *M64 = nullptr, *L64 = nullptr;
  void *part_s = nullptr, *part_c = nullptr;
  void *vec4 = nullptr;
  void *m2p_buf = nullptr;
};

EvalScratch scratch_of(const DevLists &dv) {
  EvalScratch sc;
  sc.M = dv.M;
  sc.Mr = dv.Mr;
  sc.L = dv.L;
  sc.M64 = dv.M64;
  sc.L64 = dv.L64;
  sc.part_s = dv.part_s;
  sc.part_c = dv.part_c;
  sc.vec4 = dv.vec4;
  sc.m2p_buf = dv.m2p_buf;
  return sc;
}

// Enqueue one evaluation; outputs in user order.  mode kCharges: charges q ->
// (phi, grad).  kDipoles: charges q plus dipoles -v_user (v_user [n][3]) ->
// (phi, grad).  kHessVec: charges q; grad receives H[q] v_user.
// rb0 <= rb1 (rb1 >= 0): only the targets of Morton positions [rb0, rb1),
// which start and end on leaf boundaries; rb1 < 0: all targets.
// The tree, lists and plan must be on the device and `sc` sized for
// (p, precision); with fixed_scratch the call creates nothing (no stream,
// no events), so the caller must have excluded timing, kept stages and the
// side stream.
int enqueue_evaluation(fmm_tree *t, fmm_lists *l, const fmm_eval_opts *o, const EvalScratch &sc,
                       bool fixed_scratch, const void *q, void *phi, void *grad, void *stream,
                       int mode, const void *v_user, int64_t rb0, int64_t rb1) {
  namespace D = fmmlib::dev;
  const fmmlib::TreeData &td = t->data;
  const bool fp64 = o->precision == FMM_FP64;
  const bool ranged = rb1 >= 0;
  fmmlib::RangeCells rcells;
  if (ranged) {
    if (int rc = ensure_range_tables(t, l)) return rc;
    fmmlib::range_cells(td, t->leaf_ix, rb0, rb1, rcells);
  }
  DevLists &dv = l->dev;
  DevTree &dt = t->dev;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool timing = (o->flags & FMM_EVAL_TIMING) != 0;
  const bool overlap = (o->flags & FMM_EVAL_SERIAL) == 0 && !fixed_scratch;
  if (fixed_scratch && (timing || (o->flags & FMM_EVAL_KEEP_STAGES))) {
    set_error("internal error: timing or kept stages with a fixed scratch buffer");
    return FMM_EINVAL;
  }
  const int set = dv.ring_next;  // the event set of a timed evaluation
  if (timing && !dv.ev_made[set]) {
    for (auto &e : dv.ev[set]) HIP_TRY(hipEventCreate(&e));
    dv.ev_made[set] = true;
  }
  if (overlap && !dv.side) {
    // default priority, non-blocking with respect to the null stream
    HIP_TRY(hipStreamCreateWithFlags(&dv.side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&dv.fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&dv.join, hipEventDisableTiming));
  }
  // An evaluation that fails part way leaves no timed evaluations held.  The
  // allocation-free path leaves the timings (and kept stages) of the last
  // allocating evaluation as they are.
  const int prev_count = dv.ring_count;
  if (!fixed_scratch) dv.ring_count = 0;
  g_launch_counter = 0;
  auto mark = [&](int k, hipStream_t st) -> int {
    if (timing) HIP_TRY(hipEventRecord(dv.ev[set][k], st));
    return FMM_OK;
  };
  const int p = o->p;
  const int S = D::stride(p);
  void *bodies = fp64 ? dt.b64 : dt.b32;
  const auto &pl = dv.plan;
  const int64_t n_top = top_cells(td, o);
  const int max_level = td.max_level;
  const double *geo = dt.geo;
  const size_t real = fp64 ? 8 : 4;
  // Bodies of different leaves never coincide for a tree built from these
  // positions (equal positions share a key, hence a leaf), nor in FP32 when
  // every position is FP32-representable; otherwise test every pair.
  const bool mask_all = td.moved || (!fp64 && !td.fp32_exact);
  // The FP32 P2P kernel at four waves per SIMD, except for p = 5 and 6: their
  // M2L waves (about 148 registers) start beside P2P only where a finished
  // P2P wave of the three-wave kernel (168) makes room; at p <= 4 M2L is
  // small enough either way, and at p >= 7 it never fits beside P2P.
  const bool p2p_four_waves = o->p <= 4 || o->p >= 7;
  // Mutual P2P: evaluations with charges alone over all targets.
  const bool mutual = (o->flags & FMM_EVAL_MUTUAL_P2P) && mode == D::kCharges && !ranged;
  if (mutual && (fp64 || fixed_scratch || !dv.mp_ready)) {
    set_error("internal error: mutual P2P without its plan");
    return FMM_EINVAL;
  }

  if (int rc = mark(0, s)) return rc;
  LAUNCH_TRY(D::gather_charges(fp64, td.n, dt.perm, q, bodies, stream));
  const void *vec = nullptr;
  if (mode != D::kCharges) {
    LAUNCH_TRY(D::gather_vectors(fp64, td.n, dt.perm, v_user, mode == D::kDipoles ? -1.0 : 1.0,
                                 sc.vec4, stream));
    vec = sc.vec4;
  }
  if (int rc = mark(1, s)) return rc;

  // Near field: independent of the far field until the final combine.
  const hipStream_t ns = overlap ? dv.side : s;
  if (overlap) {
    HIP_TRY(hipEventRecord(dv.fork, s));
    HIP_TRY(hipStreamWaitEvent(ns, dv.fork, 0));
  }
  if (int rc = mark(8, ns)) return rc;
  if (mutual) {
    LAUNCH_TRY(D::p2p_mutual(mask_all, dv.mp_n_items, dv.mp_items, dv.mp_run_body,
                             dv.mp_run_prefix, dv.mp_run_dst, bodies, sc.part_s, sc.part_c,
                             dv.part_m, ns));
  } else if (!ranged) {
    LAUNCH_TRY(D::p2p(fp64, mode, mask_all, p2p_four_waves, pl.n_items, pl.items, pl.order,
                      pl.order_len, pl.run_body, pl.run_prefix, bodies, vec, sc.part_s,
                      sc.part_c, ns));
  } else {
    // the items of the range's leaves: one contiguous run per level
    for (int lev = 0; lev <= max_level; ++lev) {
      const int64_t i0 = dv.leaf_item_host[rcells.leaf_lo[lev]];
      const int64_t i1 = dv.leaf_item_host[rcells.leaf_hi[lev]];
      if (i1 > i0)
        LAUNCH_TRY(D::p2p(fp64, mode, mask_all, p2p_four_waves, i1 - i0, pl.items + i0,
                          nullptr, 0, pl.run_body, pl.run_prefix, bodies, vec, sc.part_s,
                          sc.part_c, ns));
    }
  }
  if (int rc = mark(9, ns)) return rc;
  if (overlap) HIP_TRY(hipEventRecord(dv.join, ns));

  // Far field on the caller's stream.
  LAUNCH_TRY(D::p2m(p, fp64, pl.n_leaves, pl.leaf_cell, dt.body_begin, dt.n_body,
                    geo, bodies, mode == D::kDipoles ? vec : nullptr, sc.M, sc.M64, n_top,
                    td.n, stream));
  if (int rc = mark(2, s)) return rc;
  for (int lev = max_level - 1; lev >= 0; --lev) {
    const int64_t c0 = td.level_begin[lev], c1 = td.level_begin[lev + 1];
    const bool out64 = c1 <= n_top;        // this level is kept in FP64
    const bool child64 = td.level_begin[lev + 2] <= n_top;
    LAUNCH_TRY(D::m2m(p, fp64, c0, c1, dt.child_begin, dt.n_child, geo, sc.M, sc.M64, child64,
                      out64, stream));
  }
  if (int rc = mark(3, s)) return rc;
  {
    // M2L reads the multipoles folded onto their terms of z exponent <= 1.
    LAUNCH_TRY(D::fold_multipoles(p, fp64, td.n_cells(), sc.M, sc.Mr, stream));
    // every cell is an M2L row (one without entries writes zeros); the top
    // n_top cells accumulate in FP64.  A target range takes, level by level,
    // the cells holding its bodies.
    // In an evaluation of all targets, a launch that runs to the last cell
    // takes the cells in the lists' dispatch order (its kernel skips the
    // cells below its range: the FP64 top levels, launched apart, are a
    // small share of the work).
    auto order_for = [&](int64_t, int64_t b) -> const int32_t * {
      return !ranged && b == td.n_cells() ? dv.m2l_order : nullptr;
    };
    auto m2l_cells = [&](int64_t c0, int64_t c1) -> int {
      const int64_t split = std::max(c0, std::min(n_top, c1));
      if (split > c0)
        LAUNCH_TRY(D::m2l(p, fp64, c0, split, dv.m2l_ptr, dv.m2l_col, geo, sc.Mr, sc.L, sc.L64,
                          true, order_for(c0, split), dv.m2l_order_len, stream));
      if (c1 > split)
        LAUNCH_TRY(D::m2l(p, fp64, split, c1, dv.m2l_ptr, dv.m2l_col, geo, sc.Mr, sc.L, sc.L64,
                          false, order_for(split, c1), dv.m2l_order_len, stream));
      return FMM_OK;
    };
    const bool mfma = (o->flags & FMM_EVAL_M2L_MFMA) != 0;
    if (mfma && (ranged || !dv.mfma_ready || dv.mt_dtab_p != p)) {
      set_error("FMM_EVAL_M2L_MFMA: not for target ranges, and the plan must be on the device");
      return FMM_EINVAL;
    }
    if (mfma) {
      // FP64-accumulated top levels entry by entry, the rest batched
      if (n_top > 0) {
        LAUNCH_TRY(D::m2l(p, fp64, 0, n_top, dv.m2l_ptr, dv.m2l_col, geo, sc.Mr, sc.L, sc.L64,
                          true, order_for(0, n_top), dv.m2l_order_len, stream));
      }
      int lev0 = 0;
      while (lev0 <= max_level && td.level_begin[lev0] < n_top) ++lev0;
      LAUNCH_TRY(D::m2l_mfma(p, dv.mt_level_tile[lev0], dv.mt_n_tiles, dv.mt_cells, dv.mt_gbeg,
                             dv.mt_goff, dv.mt_gsrc, dv.mt_dtab, (const float *)sc.Mr,
                             (float *)sc.L, stream));
    } else if (!ranged) {
      if (int rc = m2l_cells(0, td.n_cells())) return rc;
    } else {
      for (int lev = 0; lev <= max_level; ++lev)
        if (int rc = m2l_cells(rcells.cell_lo[lev], rcells.cell_hi[lev])) return rc;
    }
  }
  if (dv.n_m2p_rows > 0)
    LAUNCH_TRY(D::m2p(p, fp64, dv.n_m2p_rows, dv.m2p_rows, dv.m2p_ptr, dv.m2p_col, dt.body_begin,
                      dt.n_body, geo, sc.M, bodies, sc.m2p_buf, stream));
  if (o->flags & FMM_EVAL_KEEP_STAGES) {
    HIP_TRY(hipMemcpyAsync(dv.Lstage, sc.L, (size_t)td.n_cells() * S * real,
                           hipMemcpyDeviceToDevice, s));
    if (n_top > 0)
      HIP_TRY(hipMemcpyAsync(dv.L64stage, sc.L64, (size_t)n_top * S * 8, hipMemcpyDeviceToDevice,
                             s));
    dv.stage_valid = true;
  } else if (!fixed_scratch) {
    dv.stage_valid = false;
  }
  if (int rc = mark(4, s)) return rc;
  for (int lev = 1; lev <= max_level; ++lev) {
    const int64_t c0 = td.level_begin[lev], c1 = td.level_begin[lev + 1];
    const bool parent64 = td.level_begin[lev] <= n_top && n_top > 0;
    const bool child64 = c1 <= n_top;
    const int64_t r0 = ranged ? rcells.cell_lo[lev] : c0, r1 = ranged ? rcells.cell_hi[lev] : c1;
    if (r1 > r0)
      LAUNCH_TRY(D::l2l(p, fp64, r0, r1, dt.parent, geo, sc.L, sc.L64, parent64, child64,
                        stream));
  }
  if (n_top > 0) LAUNCH_TRY(D::copy_top_locals(p, n_top, sc.L64, (float *)sc.L, stream));
  if (int rc = mark(5, s)) return rc;
  if (overlap) HIP_TRY(hipStreamWaitEvent(s, dv.join, 0));
  if (int rc = mark(6, s)) return rc;
  D::MutualSlots ms;
  if (mutual) {
    ms.part_m = dv.part_m;
    ms.leaf_mbase = dv.mp_leaf_mbase;
    ms.leaf_nlow = dv.mp_leaf_nlow;
  }
  LAUNCH_TRY(D::l2p_combine(p, fp64, mode, ranged ? rb0 : 0, ranged ? rb1 : td.n, pl.body_leaf,
                            pl.leaf_cell, mutual ? dv.mp_leaf_pbase : pl.leaf_pbase,
                            mutual ? dv.mp_leaf_nchunk : pl.leaf_nchunk, dt.body_begin, dt.n_body,
                            geo, sc.L, bodies, vec, sc.part_s, sc.part_c, ms,
                            dv.n_m2p_rows > 0 ? sc.m2p_buf : nullptr, dt.perm, phi, grad,
                            stream));
  if (int rc = mark(7, s)) return rc;
  if (timing) {
    dv.ring_serial[set] = !overlap;
    dv.ring_next = (set + 1) % FMM_TIMING_HISTORY;
    dv.ring_count = std::min(prev_count + 1, FMM_TIMING_HISTORY);
  } else if (fixed_scratch) {
    dv.ring_count = prev_count;
  }
  return FMM_OK;
}

// The allocating path: uploads the tree, lists and plan on first use and
// sizes the lists' own scratch for (p, precision).
int evaluate_impl(fmm_tree *t, fmm_lists *l, const fmm_eval_opts *o, const void *q, void *phi,
                  void *grad, void *stream, int mode = fmmlib::dev::kCharges,
                  const void *v_user = nullptr, int64_t rb0 = 0, int64_t rb1 = -1) {
  const bool fp64 = o->precision == FMM_FP64;
  if (int rc = ensure_tree_device(t, fp64, stream)) return rc;
  if (int rc = ensure_lists_device(t, l)) return rc;
  if (o->flags & FMM_EVAL_MUTUAL_P2P)
    if (int rc = ensure_mutual(t, l)) return rc;
  if (int rc = ensure_scratch(t, l, o)) return rc;
  if (o->flags & FMM_EVAL_M2L_MFMA)
    if (int rc = ensure_m2l_mfma(t, l, o->p, stream)) return rc;
  return enqueue_evaluation(t, l, o, scratch_of(l->dev), false, q, phi, grad, stream, mode,
                            v_user, rb0, rb1);
}

// Carves the buffers of one evaluation out of [base, base + cap), each
// aligned to 256 bytes; the bytes needed go to *need (more than cap: nothing
// is carved).
void carve_scratch(const fmmlib::TreeData &td, const DevLists &dv, const fmm_eval_opts *o,
                   char *base, size_t cap, EvalScratch *sc, size_t *need) {
  const bool fp64 = o->precision == FMM_FP64;
  const size_t real = fp64 ? 8 : 4;
  const size_t nc = (size_t)td.n_cells();
  const size_t n_top = (size_t)top_cells(td, o);
  const size_t S = (size_t)fmmlib::dev::stride(o->p);
  const size_t np = (size_t)std::max<int64_t>(1, dv.plan.n_partials);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    const size_t at = off;
    off += (bytes + 255) & ~size_t(255);
    return base + at;
  };
  EvalScratch c;
  c.M = take(nc * S * real);
  c.Mr = take(nc * (size_t)fmmlib::dev::rstride(o->p) * real);
  c.L = take(nc * S * real);
  if (n_top > 0) {
    c.M64 = (double *)take(n_top * S * 8);
    c.L64 = (double *)take(n_top * S * 8);
  }
  c.part_s = take(np * 4 * real);
  if (!fp64) c.part_c = take(np * 4 * real);
  *need = off;
  if (off <= cap) *sc = c;
}

// Library ordering of expansion terms: by degree, then z exponent, then y.
void term_exps(int p, int32_t *e) {
  int t = 0;
  for (int d = 0; d < p; ++d)
    for (int c = 0; c <= d; ++c)
      for (int b = 0; b <= d - c; ++b) {
        e[3 * t] = d - b - c;
        e[3 * t + 1] = b;
        e[3 * t + 2] = c;
        ++t;
      }
}

}  // namespace

extern "C" {

const char *fmm_last_error(void) { return g_error.c_str(); }

int fmm_num_terms(int p) { return (p < 1 || p > FMM_MAX_P) ? -1 : fmmlib::dev::terms(p); }

int fmm_term_exponents(int p, int32_t *exps) {
  if (p < 1 || p > FMM_MAX_P || !exps) {
    set_error("fmm_term_exponents: bad argument");
    return FMM_EINVAL;
  }
  term_exps(p, exps);
  return FMM_OK;
}

int fmm_tree_build(const double *xyz, int64_t n, int ncrit, fmm_tree **out) {
  return fmm_tree_build_ex(xyz, n, ncrit, 0u, out);
}

int fmm_tree_build_ex(const double *xyz, int64_t n, int ncrit, unsigned flags, fmm_tree **out) {
  if (!out || n < 0 || ncrit < 1 || (n > 0 && !xyz)) {
    set_error("fmm_tree_build: need out != NULL, n >= 0, ncrit >= 1, xyz != NULL");
    return FMM_EINVAL;
  }
  if (flags & ~(unsigned)FMM_TREE_BOX_CENTRES) {
    set_error("fmm_tree_build_ex: unknown flags");
    return FMM_EINVAL;
  }
  if (n > (int64_t)INT32_MAX - 1) {
    set_error("fmm_tree_build: n must be below 2^31 - 1");
    return FMM_EINVAL;
  }
  *out = nullptr;
  fmm_tree *t = nullptr;
  fmmlib::reset_alloc_checkpoints();
  try {
    t = new fmm_tree();
    std::string err;
    const bool box = (flags & FMM_TREE_BOX_CENTRES) != 0;
    const int rc = fmmlib::build_tree(xyz, n, ncrit, t->data, err, box);
    t->data.box_centres = box;
    if (rc != FMM_OK) {
      delete t;
      set_error(err);
      return rc;
    }
  } catch (const std::bad_alloc &) {
    delete t;
    set_error("fmm_tree_build: out of host memory");
    return FMM_ENOMEM;
  }
  t->data.id = g_next_tree_id++;
  if (std::getenv("FMM_LOG"))
    std::fprintf(stderr, "[fmm] tree: n=%lld ncrit=%d cells=%lld leaves=%lld depth=%d fp32_exact=%d\n",
                 (long long)n, ncrit, (long long)t->data.n_cells(), (long long)t->data.n_leaves,
                 t->data.max_level, (int)t->data.fp32_exact);
  *out = t;
  return FMM_OK;
}

int fmm_tree_build_gpu(const void *xyz_dev, int64_t n, int ncrit, fmm_tree **out, void *stream) {
  if (!out || n < 0 || ncrit < 1 || (n > 0 && !xyz_dev)) {
    set_error("fmm_tree_build_gpu: need out != NULL, n >= 0, ncrit >= 1, xyz != NULL");
    return FMM_EINVAL;
  }
  if (n > (int64_t)INT32_MAX - 1) {
    set_error("fmm_tree_build_gpu: n must be below 2^31 - 1");
    return FMM_EINVAL;
  }
  *out = nullptr;
  fmm_tree *t = nullptr;
  fmmlib::dev::DeviceTree dtree;
  auto free_dev = [&]() {
    void *ptrs[] = {dtree.perm, dtree.body_begin, dtree.n_body, dtree.child_begin,
                    dtree.n_child, dtree.parent, dtree.geo, dtree.pos, dtree.keys};
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
  };
  try {
    t = new fmm_tree();
    int dev;
    if (int rc = current_device(&dev)) {
      delete t;
      return rc;
    }
    std::string err;
    const int rc = fmmlib::dev::build_tree_gpu((const double *)xyz_dev, n, ncrit, stream, dtree,
                                               t->data, err);
    if (rc != 0) {
      free_dev();
      delete t;
      if (rc == -1) {
        set_error(err);
        return FMM_EINVAL;
      }
      return hip_fail((hipError_t)rc, "build_tree_gpu");
    }
    if (n > 0) {
      // the device arrays serve the evaluation directly
      DevTree &dv = t->dev;
      dv.device = dev;
      dv.n = n;
      dv.n_cells = dtree.n_cells;
      dv.perm = dtree.perm;
      dv.geo = dtree.geo;
      dv.body_begin = dtree.body_begin;
      dv.n_body = dtree.n_body;
      dv.child_begin = dtree.child_begin;
      dv.n_child = dtree.n_child;
      dv.parent = dtree.parent;
      dv.pos = dtree.pos;
      dv.keys = dtree.keys;
      dv.pos_dev_version = t->data.pos_version;
      dv.host_bodies = false;
      dtree = fmmlib::dev::DeviceTree();
      // FP32 bodies for the evaluation, packed on the device
      if (int rc2 = ensure_tree_device(t, false, stream)) {
        fmm_tree_free(t);
        return rc2;
      }
    }
  } catch (const std::bad_alloc &) {
    free_dev();
    delete t;
    set_error("fmm_tree_build_gpu: out of host memory");
    return FMM_ENOMEM;
  }
  t->data.id = g_next_tree_id++;
  *out = t;
  return FMM_OK;
}

int fmm_tree_set_positions(fmm_tree *t, const double *xyz) {
  if (!t || (t->data.n > 0 && !xyz)) {
    set_error("fmm_tree_set_positions: bad argument");
    return FMM_EINVAL;
  }
  fmmlib::TreeData &d = t->data;
  for (int64_t i = 0; i < 3 * d.n; ++i)
    if (!std::isfinite(xyz[i])) {
      set_error("fmm_tree_set_positions: positions must be finite");
      return FMM_EINVAL;
    }
  if (int rc = ensure_tree_host_bodies(t)) return rc;
  for (int64_t i = 0; i < d.n; ++i)
    for (int k = 0; k < 3; ++k) d.pos[3 * i + k] = xyz[3 * (int64_t)d.perm[i] + k];
  // Moved bodies may now coincide with bodies of other leaves: from here on
  // every P2P pair is tested for zero distance.
  d.moved = true;
  d.pos_version++;
  return FMM_OK;
}

int fmm_tree_view(const fmm_tree *t, fmm_tree_view_t *v) {
  if (!t || !v) {
    set_error("fmm_tree_view: NULL argument");
    return FMM_EINVAL;
  }
  if (int rc = ensure_tree_host_bodies(const_cast<fmm_tree *>(t))) return rc;
  const fmmlib::TreeData &d = t->data;
  v->n = d.n;
  v->n_cells = d.n_cells();
  v->n_leaves = d.n_leaves;
  v->max_level = d.max_level;
  v->fp32_exact = d.fp32_exact ? 1 : 0;
  v->perm = d.perm.data();
  v->keys = d.keys.data();
  v->level = d.level.data();
  v->parent = d.parent.data();
  v->child_begin = d.child_begin.data();
  v->n_child = d.n_child.data();
  v->body_begin = d.body_begin.data();
  v->n_body = d.n_body.data();
  v->center = d.center.data();
  v->radius = d.radius.data();
  return FMM_OK;
}

void fmm_tree_free(fmm_tree *t) {
  if (!t) return;
  t->dev.release();
  delete t;
}

}  // extern "C"

namespace {

int traverse_host(const fmm_tree *t, double theta, unsigned flags, int m2p_max, fmm_lists **out,
                  const char *fn) {
  if (!t || !out) {
    set_error(std::string(fn) + ": NULL argument");
    return FMM_EINVAL;
  }
  if (!(theta > 0.0 && theta < 1.0)) {
    set_error(std::string(fn) + ": theta must be in (0, 1)");
    return FMM_EINVAL;
  }
  if (flags & ~(unsigned)FMM_LEAF_FIRST) {
    set_error(std::string(fn) + ": unknown flags");
    return FMM_EINVAL;
  }
  if (m2p_max < 0 || m2p_max > FMM_MAX_M2P) {
    set_error(std::string(fn) + ": m2p_max must be in 0..64");
    return FMM_EINVAL;
  }
  *out = nullptr;
  fmm_lists *l = nullptr;
  fmmlib::reset_alloc_checkpoints();
  try {
    l = new fmm_lists();
    fmmlib::dual_traverse(t->data, theta, (flags & FMM_LEAF_FIRST) != 0, m2p_max, l->data);
    std::string err;
    if (fmmlib::build_p2p_plan(t->data, l->data, l->host_plan, err) != FMM_OK) {
      delete l;
      set_error(std::string(fn) + ": " + err);
      return FMM_EINVAL;
    }
  } catch (const std::bad_alloc &) {
    delete l;
    set_error(std::string(fn) + ": out of host memory");
    return FMM_ENOMEM;
  }
  if (std::getenv("FMM_LOG"))
    std::fprintf(stderr, "[fmm] lists: theta=%g %s p2p=%lld m2l=%lld m2p=%lld pairs=%lld\n",
                 theta, (flags & FMM_LEAF_FIRST) ? "leaf-first" : "mac-first",
                 (long long)l->data.p2p_col.size(), (long long)l->data.m2l_col.size(),
                 (long long)l->data.m2p_col.size(), (long long)l->data.p2p_pairs);
  *out = l;
  return FMM_OK;
}

}  // namespace

extern "C" {

int fmm_traverse(const fmm_tree *t, double theta, unsigned flags, fmm_lists **out) {
  return traverse_host(t, theta, flags, 0, out, "fmm_traverse");
}

int fmm_traverse_hybrid(const fmm_tree *t, double theta, unsigned flags, int m2p_max,
                        fmm_lists **out) {
  return traverse_host(t, theta, flags, m2p_max, out, "fmm_traverse_hybrid");
}

int fmm_traverse_gpu(const fmm_tree *t, double theta, unsigned flags, fmm_lists **out,
                     void *stream) {
  if (!t || !out) {
    set_error("fmm_traverse_gpu: NULL argument");
    return FMM_EINVAL;
  }
  if (!(theta > 0.0 && theta < 1.0)) {
    set_error("fmm_traverse_gpu: theta must be in (0, 1)");
    return FMM_EINVAL;
  }
  if (flags & ~(unsigned)FMM_LEAF_FIRST) {
    set_error("fmm_traverse_gpu: unknown flags");
    return FMM_EINVAL;
  }
  *out = nullptr;
  const auto t_call = std::chrono::steady_clock::now();
  fmm_tree *tt = const_cast<fmm_tree *>(t);
  fmm_lists *l = nullptr;
  fmmlib::dev::DeviceLists dl;
  auto free_dl = [&]() {
    void *ptrs[] = {dl.p2p_ptr, dl.p2p_col, dl.m2l_ptr, dl.m2l_col};
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
  };
  try {
    l = new fmm_lists();
    fmmlib::ListData &ld = l->data;
    const fmmlib::TreeData &td = t->data;
    ld.tree_id = td.id;
    ld.theta = theta;
    ld.flags = flags;
    ld.n_rows = td.n_cells();
    if (td.n_cells() > 0) {
      if (int rc = ensure_tree_device(tt, false, stream)) {
        delete l;
        return rc;
      }
      if (std::getenv("FMM_LOG"))
        std::fprintf(stderr, "[fmm] fmm_traverse_gpu: %.2f ms before the traversal\n",
                     ms_since(t_call));
      const int rc = fmmlib::dev::dual_traverse_gpu(td.n_cells(), tt->dev.geo, tt->dev.child_begin,
                                                    tt->dev.n_child, theta,
                                                    (flags & FMM_LEAF_FIRST) != 0, stream, dl);
      if (std::getenv("FMM_LOG"))
        std::fprintf(stderr, "[fmm] fmm_traverse_gpu: %.2f ms after the traversal\n",
                     ms_since(t_call));
      if (rc == fmmlib::dev::kTraverseTooLarge) {
        free_dl();
        delete l;
        set_error("fmm_traverse_gpu: a list or a traversal level would hold 2^31 or more cell "
                  "pairs; fmm_traverse (host) builds lists of that size");
        return FMM_EINVAL;
      }
      if (rc != 0) {
        free_dl();
        delete l;
        return hip_fail((hipError_t)rc, "dual_traverse_gpu");
      }
    }
    // The lists stay on the device; the P2P plan is built there too.
    DevLists &dv = l->dev;
    dv.p2p_ptr = dl.p2p_ptr;
    dv.p2p_col = dl.p2p_col;
    dv.m2l_ptr = dl.m2l_ptr;
    dv.m2l_col = dl.m2l_col;
    dv.p2p_nnz = dl.p2p_nnz;
    dv.m2l_nnz = dl.m2l_nnz;
    dl = fmmlib::dev::DeviceLists();
    if (td.n_cells() > 0) {
      const auto t_plan = std::chrono::steady_clock::now();
      const int rc = fmmlib::dev::build_p2p_plan_gpu(
          td.n, td.n_cells(), td.n_leaves, tt->dev.n_child, tt->dev.body_begin, tt->dev.n_body,
          dv.p2p_ptr, dv.p2p_col, plan_layouts(), stream, dv.plan);
      if (rc != 0) {
        fmm_lists_free(l);
        return hip_fail((hipError_t)rc, "build_p2p_plan_gpu");
      }
      if (const int rc2 = fmmlib::dev::dispatch_orders(dv.plan, dv.m2l_ptr, td.n_cells(),
                                                       &dv.m2l_order, &dv.m2l_order_len,
                                                       stream)) {
        fmm_lists_free(l);
        return hip_fail((hipError_t)rc2, "dispatch_orders");
      }
      if (std::getenv("FMM_LOG"))
        std::fprintf(stderr, "[fmm] device work plan: %.2f ms (%lld items, %lld runs)\n",
                     ms_since(t_plan), (long long)dv.plan.n_items, (long long)dv.plan.n_runs);
      ld.p2p_pairs = dv.plan.p2p_pairs;
      ld.max_row_sources = dv.plan.max_row_sources;
      dv.host_valid = false;
      dv.uploaded = true;
      dv.device = tt->dev.device;
    } else {
      ld.p2p_ptr.assign(1, 0);
      ld.m2l_ptr.assign(1, 0);
    }
  } catch (const std::bad_alloc &) {
    free_dl();
    if (l) fmm_lists_free(l);
    set_error("fmm_traverse_gpu: out of host memory");
    return FMM_ENOMEM;
  }
  if (std::getenv("FMM_LOG"))
    std::fprintf(stderr, "[fmm] fmm_traverse_gpu: %.2f ms in all\n", ms_since(t_call));
  *out = l;
  return FMM_OK;
}

int fmm_lists_view(const fmm_lists *l, int kind, const int64_t **row_ptr, const int32_t **col,
                   int64_t *nrows, int64_t *nnz) {
  if (!l || !row_ptr || !col || !nrows || !nnz ||
      (kind != FMM_P2P && kind != FMM_M2L && kind != FMM_M2P)) {
    set_error("fmm_lists_view: bad argument");
    return FMM_EINVAL;
  }
  if (int rc = ensure_lists_host(const_cast<fmm_lists *>(l))) return rc;
  const fmmlib::ListData &d = l->data;
  if (kind == FMM_M2P && d.m2p_ptr.empty()) {
    set_error("fmm_lists_view: no M2P list");
    return FMM_ESTATE;
  }
  *row_ptr = kind == FMM_P2P ? d.p2p_ptr.data() : kind == FMM_M2L ? d.m2l_ptr.data()
                                                                  : d.m2p_ptr.data();
  *col = kind == FMM_P2P ? d.p2p_col.data() : kind == FMM_M2L ? d.m2l_col.data()
                                                              : d.m2p_col.data();
  *nrows = d.n_rows;
  *nnz = (int64_t)(kind == FMM_P2P ? d.p2p_col.size()
                                   : kind == FMM_M2L ? d.m2l_col.size() : d.m2p_col.size());
  return FMM_OK;
}

int fmm_lists_stats(const fmm_lists *l, fmm_lists_stats_t *s) {
  if (!l || !s) {
    set_error("fmm_lists_stats: NULL argument");
    return FMM_EINVAL;
  }
  const bool host = l->dev.host_valid;
  s->p2p_entries = host ? (int64_t)l->data.p2p_col.size() : l->dev.p2p_nnz;
  s->m2l_entries = host ? (int64_t)l->data.m2l_col.size() : l->dev.m2l_nnz;
  s->p2p_pairs = l->data.p2p_pairs;
  s->p2p_work_items = l->dev.uploaded ? l->dev.plan.n_items : (int64_t)l->host_plan.items.size();
  s->m2p_entries = (int64_t)l->data.m2p_col.size();
  s->p2p_max_row_sources = l->data.max_row_sources;
  return FMM_OK;
}

int fmm_mutual_plan_stats(const fmm_tree *t, const fmm_lists *l, int64_t *out) {
  if (int rc = check_pair(t, l)) return rc;
  if (!out) {
    set_error("fmm_mutual_plan_stats: out is NULL");
    return FMM_EINVAL;
  }
  try {
    if (int rc = ensure_lists_host(const_cast<fmm_lists *>(l))) return rc;
    fmmlib::P2PMutualPlan plan;
    std::string err;
    if (int rc = fmmlib::build_p2p_mutual_plan(t->data, l->data, plan, err)) {
      set_error(err);
      return rc;
    }
    out[0] = (int64_t)plan.items.size();
    out[1] = (int64_t)plan.run_body.size();
    out[2] = plan.upper_pairs;
    out[3] = plan.self_pairs;
    out[4] = plan.n_mslots;
  } catch (const std::bad_alloc &) {
    set_error("fmm_mutual_plan_stats: out of host memory");
    return FMM_ENOMEM;
  }
  return FMM_OK;
}

int fmm_dispatch_order(const fmm_lists *l, int kind, int32_t *out, int64_t cap, int64_t *len) {
  if (!l || !len || (kind != FMM_P2P && kind != FMM_M2L)) {
    set_error("fmm_dispatch_order: NULL lists or len, or kind is not FMM_P2P or FMM_M2L");
    return FMM_EINVAL;
  }
  const DevLists &dv = l->dev;
  if (!dv.uploaded) {
    set_error("fmm_dispatch_order: the lists are not on a device yet");
    return FMM_ESTATE;
  }
  const int32_t *src = kind == FMM_P2P ? dv.plan.order : dv.m2l_order;
  const int64_t n = !src ? 0 : kind == FMM_P2P ? dv.plan.order_len : dv.m2l_order_len;
  *len = n;
  if (!out) return FMM_OK;
  if (cap < n) {
    set_error("fmm_dispatch_order: cap is smaller than the order's length");
    return FMM_EINVAL;
  }
  if (n > 0) HIP_TRY(hipMemcpy(out, src, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost));
  return FMM_OK;
}

void fmm_lists_free(fmm_lists *l) {
  if (!l) return;
  l->dev.release();
  delete l;
}

int fmm_evaluate(const fmm_tree *t, const fmm_lists *l, const fmm_eval_opts *o, const void *q_dev,
                 void *phi_dev, void *grad_dev, void *stream) {
  if (int rc = check_pair(t, l)) return rc;
  if (int rc = check_opts(o)) return rc;
  if (t->data.n == 0) return FMM_OK;
  if (!q_dev || !phi_dev) {
    set_error("fmm_evaluate: q and phi must not be NULL");
    return FMM_EINVAL;
  }
  try {
    return evaluate_impl(const_cast<fmm_tree *>(t), const_cast<fmm_lists *>(l), o, q_dev, phi_dev,
                         grad_dev, stream);
  } catch (const std::bad_alloc &) {
    set_error("fmm_evaluate: out of host memory");
    return FMM_ENOMEM;
  }
}

int fmm_evaluate_range(const fmm_tree *t, const fmm_lists *l, const fmm_eval_opts *o,
                       int64_t body_begin, int64_t body_end, const void *q_dev, void *phi_dev,
                       void *grad_dev, void *stream) {
  if (int rc = check_pair(t, l)) return rc;
  if (int rc = check_opts(o)) return rc;
  if (!l->data.m2p_col.empty()) {
    set_error("fmm_evaluate_range: hybrid (M2P) lists are not supported");
    return FMM_EINVAL;
  }
  if (o->flags & FMM_EVAL_MUTUAL_P2P) {
    set_error("fmm_evaluate_range: FMM_EVAL_MUTUAL_P2P evaluates every target");
    return FMM_EINVAL;
  }
  fmm_tree *tt = const_cast<fmm_tree *>(t);
  const int64_t n = t->data.n;
  if (body_begin < 0 || body_end < body_begin || body_end > n) {
    set_error("fmm_evaluate_range: need 0 <= body_begin <= body_end <= n");
    return FMM_EINVAL;
  }
  if (n == 0 || body_begin == body_end) return FMM_OK;
  if (!q_dev || !phi_dev) {
    set_error("fmm_evaluate_range: q and phi must not be NULL");
    return FMM_EINVAL;
  }
  try {
    if (!tt->leaf_ix_valid) {
      fmmlib::build_leaf_index(t->data, tt->leaf_ix);
      tt->leaf_ix_valid = true;
    }
    if (!fmmlib::is_leaf_boundary(t->data, t->leaf_ix, body_begin) ||
        !fmmlib::is_leaf_boundary(t->data, t->leaf_ix, body_end)) {
      set_error("fmm_evaluate_range: body_begin and body_end must be leaf boundaries");
      return FMM_EINVAL;
    }
    return evaluate_impl(tt, const_cast<fmm_lists *>(l), o, q_dev, phi_dev, grad_dev, stream,
                         fmmlib::dev::kCharges, nullptr, body_begin, body_end);
  } catch (const std::bad_alloc &) {
    set_error("fmm_evaluate_range: out of host memory");
    return FMM_ENOMEM;
  }
}

int fmm_partition_targets(const fmm_tree *t, const fmm_lists *l, int n_parts, double m2l_weight,
                          int64_t *bounds) {
  if (int rc = check_pair(t, l)) return rc;
  if (n_parts < 1 || !bounds || !(m2l_weight >= 0.0)) {
    set_error("fmm_partition_targets: need n_parts >= 1, bounds != NULL, m2l_weight >= 0");
    return FMM_EINVAL;
  }
  fmm_tree *tt = const_cast<fmm_tree *>(t);
  try {
    if (t->data.n == 0) {
      for (int k = 0; k <= n_parts; ++k) bounds[k] = 0;
      return FMM_OK;
    }
    if (int rc = ensure_lists_host(const_cast<fmm_lists *>(l))) return rc;
    if (!tt->leaf_ix_valid) {
      fmmlib::build_leaf_index(t->data, tt->leaf_ix);
      tt->leaf_ix_valid = true;
    }
    fmmlib::partition_targets(t->data, l->data, t->leaf_ix, n_parts, m2l_weight, bounds);
  } catch (const std::bad_alloc &) {
    set_error("fmm_partition_targets: out of host memory");
    return FMM_ENOMEM;
  }
  return FMM_OK;
}

int fmm_evaluate_backward(const fmm_tree *t, const fmm_lists *l, const fmm_eval_opts *o,
                          const void *q_dev, const void *grad_q_dev, const void *w_dev,
                          const void *v_dev, void *dq_dev, void *dx_dev, void *stream) {
  if (int rc = check_pair(t, l)) return rc;
  if (int rc = check_opts(o)) return rc;
  if (!l->data.m2p_col.empty()) {
    // M2P breaks the symmetry of the far-field operator that the backward uses
    set_error("fmm_evaluate_backward: hybrid (M2P) lists are not supported");
    return FMM_ESTATE;
  }
  if (t->data.n == 0) return FMM_OK;
  if ((!w_dev && !v_dev) || (dx_dev && (!q_dev || !grad_q_dev))) {
    set_error("fmm_evaluate_backward: w or v is required; dx needs q and grad_q");
    return FMM_EINVAL;
  }
  if (!w_dev) {
    set_error("fmm_evaluate_backward: w is required (pass zeros for a loss on grad only)");
    return FMM_EINVAL;
  }
  if (!dq_dev && !dx_dev) return FMM_OK;
  fmm_tree *tt = const_cast<fmm_tree *>(t);
  fmm_lists *ll = const_cast<fmm_lists *>(l);
  namespace D = fmmlib::dev;
  try {
    const bool fp64 = o->precision == FMM_FP64;
    if (int rc = ensure_tree_device(tt, fp64, stream)) return rc;
    if (int rc = ensure_lists_device(tt, ll)) return rc;
    if (int rc = ensure_scratch(tt, ll, o)) return rc;
    DevLists &dv = ll->dev;
    void *phi_w = dq_dev ? dq_dev : dv.tmp_phi;
    void *grad_w = dx_dev ? dv.tmp_grad : nullptr;
    const void *hv = nullptr;
    if (v_dev && dx_dev) {
      // H[q] v at every body (charges q, per-target vectors v)
      if (int rc = evaluate_impl(tt, ll, o, q_dev, nullptr, dv.tmp_hv, stream, D::kHessVec, v_dev))
        return rc;
      hv = dv.tmp_hv;
    }
    // Phi: charges w plus dipoles -v (or charges w alone)
    if (int rc = evaluate_impl(tt, ll, o, w_dev, phi_w, grad_w, stream,
                               v_dev ? D::kDipoles : D::kCharges, v_dev))
      return rc;
    if (dx_dev)
      LAUNCH_TRY(D::backward_combine(fp64, t->data.n, q_dev, w_dev, grad_q_dev, grad_w, hv, dx_dev,
                                     stream));
    return FMM_OK;
  } catch (const std::bad_alloc &) {
    set_error("fmm_evaluate_backward: out of host memory");
    return FMM_ENOMEM;
  }
}

int fmm_direct(const void *xyz_dev, const void *q_dev, int64_t n, const int64_t *targets_dev,
               int64_t m, void *phi_dev, void *grad_dev, void *stream) {
  if (n < 0 || m < 0 || (m > 0 && (!xyz_dev || !q_dev || !targets_dev || !phi_dev))) {
    set_error("fmm_direct: bad argument");
    return FMM_EINVAL;
  }
  if (m > (int64_t)INT32_MAX) {
    set_error("fmm_direct: too many targets");
    return FMM_EINVAL;
  }
  LAUNCH_TRY(fmmlib::dev::direct_sum((const double *)xyz_dev, (const double *)q_dev, n,
                                     targets_dev, m, (double *)phi_dev, (double *)grad_dev,
                                     stream));
  return FMM_OK;
}

namespace {

// Per-phase times (ms) of the timed evaluation whose events are set k.
int set_timings(const DevLists &dv, int k, double *ms) {
  HIP_TRY(hipEventSynchronize(dv.ev[k][7]));
  HIP_TRY(hipEventSynchronize(dv.ev[k][9]));
  // marks: 0 start, 1 after gather, 8/9 around P2P, 2 after P2M, 3 after M2M,
  // 4 after M2L, 5 after L2L, 6 after the join, 7 end.
  const int p2m_from = dv.ring_serial[k] ? 9 : 1;
  const int pairs[FMM_NUM_PHASES][2] = {{0, 1}, {8, 9}, {p2m_from, 2}, {2, 3},
                                        {3, 4}, {4, 5}, {6, 7}, {0, 7}};
  for (int i = 0; i < FMM_NUM_PHASES; ++i) {
    float f = 0.0f;
    HIP_TRY(hipEventElapsedTime(&f, dv.ev[k][pairs[i][0]], dv.ev[k][pairs[i][1]]));
    ms[i] = f;
  }
  return FMM_OK;
}

}  // namespace

int fmm_last_timings(const fmm_lists *l, double *ms) {
  if (!l || !ms) {
    set_error("fmm_last_timings: NULL argument");
    return FMM_EINVAL;
  }
  const DevLists &dv = l->dev;
  if (dv.ring_count < 1) {
    set_error("fmm_last_timings: last evaluation was not timed");
    return FMM_ESTATE;
  }
  return set_timings(dv, (dv.ring_next + FMM_TIMING_HISTORY - 1) % FMM_TIMING_HISTORY, ms);
}

int fmm_mean_timings(const fmm_lists *l, int n, double *ms) {
  if (!l || !ms || n < 1 || n > FMM_TIMING_HISTORY) {
    set_error("fmm_mean_timings: need l, ms != NULL and 1 <= n <= FMM_TIMING_HISTORY");
    return FMM_EINVAL;
  }
  const DevLists &dv = l->dev;
  if (dv.ring_count < n) {
    set_error("fmm_mean_timings: fewer than n timed evaluations in a row are held");
    return FMM_ESTATE;
  }
  for (int i = 0; i < FMM_NUM_PHASES; ++i) ms[i] = 0.0;
  for (int j = 0; j < n; ++j) {
    double one[FMM_NUM_PHASES];
    if (int rc = set_timings(dv, (dv.ring_next + FMM_TIMING_HISTORY - 1 - j) % FMM_TIMING_HISTORY,
                             one))
      return rc;
    for (int i = 0; i < FMM_NUM_PHASES; ++i) ms[i] += one[i];
  }
  for (int i = 0; i < FMM_NUM_PHASES; ++i) ms[i] /= n;
  return FMM_OK;
}

int fmm_copy_expansions(const fmm_lists *l, int kind, double *dst) {
  if (!l || !dst || kind < 0 || kind > 2) {
    set_error("fmm_copy_expansions: bad argument");
    return FMM_EINVAL;
  }
  const DevLists &dv = l->dev;
  if (dv.p == 0) {
    set_error("fmm_copy_expansions: no evaluation yet");
    return FMM_ESTATE;
  }
  if (kind == 1 && !dv.stage_valid) {
    set_error("fmm_copy_expansions: evaluate with FMM_EVAL_KEEP_STAGES first");
    return FMM_ESTATE;
  }
  const int T = fmmlib::dev::terms(dv.p), S = fmmlib::dev::stride(dv.p);
  const int64_t nc = l->data.n_rows;
  const void *src = kind == 0 ? dv.M : (kind == 1 ? dv.Lstage : dv.L);
  const double *src64 = kind == 0 ? dv.M64 : (kind == 1 ? dv.L64stage : dv.L64);
  HIP_TRY(hipDeviceSynchronize());
  if (dv.prec == FMM_FP64) {
    std::vector<double> h((size_t)nc * S);
    HIP_TRY(hipMemcpy(h.data(), src, h.size() * 8, hipMemcpyDeviceToHost));
    for (int64_t c = 0; c < nc; ++c)
      for (int t = 0; t < T; ++t) dst[c * T + t] = h[c * S + t];
  } else {
    std::vector<float> h((size_t)nc * S);
    HIP_TRY(hipMemcpy(h.data(), src, h.size() * 4, hipMemcpyDeviceToHost));
    for (int64_t c = 0; c < nc; ++c)
      for (int t = 0; t < T; ++t) dst[c * T + t] = h[c * S + t];
    if (dv.n_top > 0) {
      std::vector<double> h64((size_t)dv.n_top * S);
      HIP_TRY(hipMemcpy(h64.data(), src64, h64.size() * 8, hipMemcpyDeviceToHost));
      for (int64_t c = 0; c < dv.n_top; ++c)
        for (int t = 0; t < T; ++t) dst[c * T + t] = h64[c * S + t];
    }
  }
  return FMM_OK;
}

}  // extern "C"

namespace fmmlib {

int evaluate_fixed_scratch(const fmm_tree *t, const fmm_lists *l, const fmm_eval_opts *o,
                           const void *q_dev, void *phi_dev, void *grad_dev, void *stream,
                           int (*scratch_address)(void **), size_t scratch_bytes) {
  if (int rc = check_pair(t, l)) return rc;
  if (int rc = check_opts(o)) return rc;
  if (o->flags & ~FMM_EVAL_SERIAL) {
    set_error("fmm_evaluate_noalloc: timing and kept stages need fmm_evaluate");
    return FMM_EINVAL;
  }
  if (!l->data.m2p_col.empty()) {
    set_error("fmm_evaluate_noalloc: hybrid (M2P) lists need fmm_evaluate");
    return FMM_EINVAL;
  }
  if (t->data.n == 0) return FMM_OK;
  if (!q_dev || !phi_dev) {
    set_error("fmm_evaluate_noalloc: q and phi must not be NULL");
    return FMM_EINVAL;
  }
  fmm_tree *tt = const_cast<fmm_tree *>(t);
  fmm_lists *ll = const_cast<fmm_lists *>(l);
  const bool fp64 = o->precision == FMM_FP64;
  const DevTree &dt = t->dev;
  const DevLists &dv = l->dev;
  int dev;
  if (int rc = current_device(&dev)) return rc;
  const uint64_t have = fp64 ? dt.pos_version_64 : dt.pos_version_32;
  if (dt.device != dev || !dv.uploaded || dv.device != dev || have != t->data.pos_version ||
      !(fp64 ? dt.b64 : dt.b32)) {
    set_error("fmm_evaluate_noalloc: the tree, lists and work plan are not on this device for "
              "this precision; one fmm_evaluate with the same precision on this device puts "
              "them there");
    return FMM_ESTATE;
  }
  void *scratch = nullptr;
  if (int rc = scratch_address(&scratch)) return rc;
  EvalScratch sc;
  size_t need = 0;
  carve_scratch(t->data, dv, o, static_cast<char *>(scratch), scratch_bytes, &sc, &need);
  if (need > scratch_bytes) {
    set_error("fmm_evaluate_noalloc: this evaluation needs " + std::to_string(need) +
              " bytes of scratch; the fixed buffer holds " + std::to_string(scratch_bytes));
    return FMM_EINVAL;
  }
  try {
    return enqueue_evaluation(tt, ll, o, sc, true, q_dev, phi_dev, grad_dev, stream,
                              fmmlib::dev::kCharges, nullptr, 0, -1);
  } catch (const std::bad_alloc &) {
    set_error("fmm_evaluate_noalloc: out of host memory");
    return FMM_ENOMEM;
  }
}

void set_last_error(const char *msg) { set_error(msg); }

}  // namespace fmmlib
