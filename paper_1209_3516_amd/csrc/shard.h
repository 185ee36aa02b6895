// Target ranges: the part of one evaluation that belongs to the target
// bodies of a contiguous range of leaves in Morton order (the share of one
// GPU when the targets are split into such ranges), and the weighted
// partition of the leaves into G ranges.
#pragma once

#include <cstdint>
#include <vector>

#include "fmm_internal.h"

namespace fmmlib {

// Host-side index of the leaves of a tree (built once per tree).
struct LeafIndex {
  std::vector<int32_t> rank;    // [n_cells + 1]: number of leaves before cell c
  std::vector<int32_t> cell;    // [n_leaves]: cell of compact leaf l (cell order)
  std::vector<int64_t> starts;  // [n_leaves]: first body of each leaf, ascending
};
void build_leaf_index(const TreeData &t, LeafIndex &ix);

// True if b is the first body of a leaf, or b == n.
bool is_leaf_boundary(const TreeData &t, const LeafIndex &ix, int64_t b);

// For bodies [b0, b1) with both ends on leaf boundaries: per level L, the
// cells of level L holding bodies of the range, [cells[L][0], cells[L][1]),
// and the compact leaf numbers of the leaves among them (contiguous, since
// the cells of one level are in Morton order).
struct RangeCells {
  std::vector<int64_t> cell_lo, cell_hi, leaf_lo, leaf_hi;
};
void range_cells(const TreeData &t, const LeafIndex &ix, int64_t b0, int64_t b1, RangeCells &rc);

// Split the leaves, in Morton order, into G contiguous ranges of about equal
// weight; a leaf weighs its P2P body pairs plus m2l_weight times the M2L
// entries of its row and its share (by bodies) of its ancestors' rows.
// bounds[0..G] are body positions on leaf boundaries, bounds[0] = 0,
// bounds[G] = n, non-decreasing.
void partition_targets(const TreeData &t, const ListData &l, const LeafIndex &ix, int G,
                       double m2l_weight, int64_t *bounds);

}  // namespace fmmlib
