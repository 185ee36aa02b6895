// Internal host-side data structures of the GPU FMM library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fmm.h"

namespace fmmlib {

// Octree in Morton order, cells numbered breadth first (section 3.3).
struct TreeData {
  int64_t n = 0;
  int ncrit = 0;
  int max_level = 0;
  int64_t n_leaves = 0;
  bool fp32_exact = true;
  bool moved = false;        // positions replaced after the build
  bool box_centres = false;  // centres of the Morton cubes (built on the host only)
  uint64_t id = 0;           // identifies the tree for lists built from it
  uint64_t pos_version = 0;  // bumped by set_positions
  double root_center[3] = {0, 0, 0};
  double root_half = 0.0;
  std::vector<double> pos;  // [n][3] positions in Morton order
  std::vector<int32_t> perm;
  std::vector<uint64_t> keys;
  std::vector<int32_t> level, parent, child_begin, n_child;
  std::vector<int64_t> body_begin, n_body;
  std::vector<double> center, radius;  // center [n_cells][3]
  std::vector<int64_t> level_begin;    // cells of level L: [level_begin[L], level_begin[L+1])
  int64_t n_cells() const { return (int64_t)level.size(); }
};

// The two interaction lists as CSR, one row per target cell.
struct ListData {
  uint64_t tree_id = 0;
  double theta = 0.0;
  unsigned flags = 0;
  int64_t n_rows = 0;
  std::vector<int64_t> p2p_ptr, m2l_ptr;
  std::vector<int32_t> p2p_col, m2l_col;
  // treecode/FMM hybrid: accepted pairs whose target is a leaf of at most
  // m2p_max bodies (empty when m2p_max == 0)
  int m2p_max = 0;
  std::vector<int64_t> m2p_ptr;
  std::vector<int32_t> m2p_col;
  int64_t p2p_pairs = 0;
  int64_t max_row_sources = 0;
};

// GPU work plan of the P2P kernel.  A work item is one group of at most 64
// target bodies of one leaf against one chunk of that leaf's source leaves.
// Source leaves whose bodies are contiguous in Morton order are merged into
// runs.  The self pair (A, A) is kept out of the runs and handled with a
// zero-distance mask.
struct P2PItem {
  int32_t tgt_begin;  // first target body (Morton position)
  int32_t tgt_cfg;    // n_tgt | R << 8 | L << 16 | K << 24 (lane layout)
  int32_t run_begin;  // first run of this item
  int32_t n_runs;
  int32_t n_src;       // source bodies in the runs
  int32_t self_begin;  // first body of the target leaf if this item holds (A, A)
  int32_t self_n;      // 0 if not
  int32_t out_off;     // partial-sum slot of the item's first target
};

struct P2PPlan {
  std::vector<P2PItem> items;
  std::vector<int32_t> run_body;    // first body of each run
  std::vector<int32_t> run_prefix;  // offset of each run within its item's source list
  // Per leaf (compact numbering in cell order): cell id, first partial slot,
  // number of source chunks.  Body b of leaf a, chunk c uses partial slot
  // leaf_pbase[a] + c * n_body + (b - body_begin).
  std::vector<int32_t> leaf_cell, leaf_pbase, leaf_nchunk;
  std::vector<int32_t> body_leaf;  // Morton body -> compact leaf
  int64_t n_partials = 0;
  int32_t max_row_sources = 0;
};

// Lane layout of a P2P work item with nt targets: K streams of L lanes, each
// lane holding R <= kP2PMaxTargetsPerLane targets (R*L >= nt, K*L <= 64).
// At most six targets per lane keep the FP32 kernel within 128 registers,
// i.e. four waves per SIMD.
constexpr int kP2PMaxTargetsPerLane = 6;
void p2p_lane_layout(int nt, int *R, int *L, int *K);

// Work plan of the mutual P2P kernel (charges only): every unordered pair of
// leaves {A, B} of the symmetric P2P list is evaluated once, in the item of
// the lower-numbered leaf A, which adds the pair's contributions to both
// sides (the mutual interaction the paper names among the falcON techniques
// that exaFMM inherits, section 2).  An item is leaf A (at most 64 bodies)
// against one chunk of its sources: the self pair (A, A), evaluated one-sided
// with a zero-distance mask, and the leaves B > A of its row, one run each.
// Targets of A take the partial-sum slots of the one-sided plan's layout
// (leaf_pbase + chunk * nA + k).  The sums for the bodies of B go to slots of
// their own, leaf by leaf: body k of leaf B receives, from the j-th leaf
// A < B of B's row, slot leaf_mbase[B] + j * nB + k; run_dst of the run of B
// in A's item is leaf_mbase[B] + j * nB.  Item lane layout tgt_cfg = nt |
// R << 8 | TL << 16 | K << 24: lane l holds targets l % TL + TL * r (r < R),
// K = 64 / TL copies of each target.
struct P2PMutualPlan {
  std::vector<P2PItem> items;
  std::vector<int32_t> run_body, run_prefix, run_dst;
  std::vector<int32_t> leaf_pbase, leaf_nchunk;  // compact leaf numbering (cell order)
  std::vector<int32_t> leaf_mbase, leaf_nlow;
  int64_t n_partials = 0;     // target-side slots
  int64_t n_mslots = 0;       // source-side slots
  int64_t upper_pairs = 0;  // body pairs of the leaf pairs A < B, each evaluated once
  int64_t self_pairs = 0;   // ordered body pairs i != j within a leaf
};

// Mutual lane layout for nt <= 64 targets: TL in {1, 2, 4, 8} target lanes per
// ring of 16, R = ceil(nt / TL) <= 8 targets per lane.
void p2p_mutual_layout(int nt, int *R, int *TL);

// FMM_OK, or FMM_EINVAL with `err` set: a leaf of more than 64 bodies, lists
// that are not symmetric, or counts past plan_index_limit().
int build_p2p_mutual_plan(const TreeData &t, const ListData &l, P2PMutualPlan &plan,
                          std::string &err);

constexpr int kP2PMaxRuns = 256;

// Fault injection for failure-handling tests: with FMM_FAULT_INJECT=alloc:K
// the K-th checkpoint of a tree build or traversal (counted from 1 within
// that call) throws std::bad_alloc, as a failed host allocation would.
void alloc_checkpoint();
void reset_alloc_checkpoints();
constexpr int kP2PChunkSources = 8192;

// box_centres: cell centres at the centres of the Morton cubes (else the
// middles of the cells' bounding boxes).
int build_tree(const double *xyz, int64_t n, int ncrit, TreeData &t, std::string &err,
               bool box_centres = false);
void dual_traverse(const TreeData &t, double theta, bool leaf_first, int m2p_max, ListData &l);
// p2p_pairs and max_row_sources of finished lists.
void list_statistics(const TreeData &t, ListData &l);
// The plan stores run, work-item and partial-slot numbers as 32-bit
// integers: the largest count a plan may hold (INT32_MAX; the environment
// variable FMM_PLAN_LIMIT=K lowers it, to test the refusal).
int64_t plan_index_limit();
// Builds the plan of finished lists.  FMM_OK, or FMM_EINVAL with `err` set
// when its runs, work items or partial slots exceed plan_index_limit().
int build_p2p_plan(const TreeData &t, const ListData &l, P2PPlan &plan, std::string &err);

// Batched M2L for box-centred trees: tiles of kM2LTile target cells (one
// level, one octant class), each with groups of entries sharing one
// (source level, translation vector).  Built on the host from the lists.
constexpr int kM2LTile = 16;
struct M2LTilePlan {
  std::vector<int32_t> tile_cells;        // [n_tiles][kM2LTile], -1 = no cell
  std::vector<int64_t> level_tile_begin;  // tiles of level L: [b[L], b[L+1])
  std::vector<int64_t> tile_group_begin;  // [n_tiles + 1]
  std::vector<int32_t> group_offset;      // [n_groups]: index into offsets
  std::vector<int32_t> group_src;         // [n_groups][kM2LTile]: source cell or -1
  std::vector<double> offsets;            // [n_offsets][3]: X_A - X_B
  int64_t n_tiles = 0, n_groups = 0, n_offsets = 0;
};
int build_m2l_tile_plan(const TreeData &t, const ListData &l, M2LTilePlan &plan,
                        std::string &err);

// fmm_evaluate with every device buffer of the evaluation carved out of a
// fixed device buffer of scratch_bytes, whose address on the current device
// scratch_address gives (called after the arguments are checked): no
// allocation, no stream or event creation.  The tree, lists and plan must
// already be on the current device for o->precision (FMM_ESTATE otherwise);
// FMM_EINVAL if the buffer is too small, for timing or kept-stage flags and
// for hybrid lists.
int evaluate_fixed_scratch(const fmm_tree *t, const fmm_lists *l, const fmm_eval_opts *o,
                           const void *q_dev, void *phi_dev, void *grad_dev, void *stream,
                           int (*scratch_address)(void **), size_t scratch_bytes);
// Sets the thread's fmm_last_error message.
void set_last_error(const char *msg);

}  // namespace fmmlib
