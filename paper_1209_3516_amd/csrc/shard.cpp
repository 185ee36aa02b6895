// Target ranges and their weighted partition (see shard.h).
#include "shard.h"

#include <algorithm>

namespace fmmlib {

void build_leaf_index(const TreeData &t, LeafIndex &ix) {
  const int64_t nc = t.n_cells();
  ix.rank.assign(nc + 1, 0);
  ix.cell.clear();
  for (int64_t c = 0; c < nc; ++c) {
    ix.rank[c + 1] = ix.rank[c] + (t.n_child[c] == 0);
    if (t.n_child[c] == 0) ix.cell.push_back((int32_t)c);
  }
  ix.starts.resize(ix.cell.size());
  for (size_t l = 0; l < ix.cell.size(); ++l) ix.starts[l] = t.body_begin[ix.cell[l]];
  std::sort(ix.starts.begin(), ix.starts.end());
}

bool is_leaf_boundary(const TreeData &t, const LeafIndex &ix, int64_t b) {
  if (b == t.n) return true;
  return std::binary_search(ix.starts.begin(), ix.starts.end(), b);
}

void range_cells(const TreeData &t, const LeafIndex &ix, int64_t b0, int64_t b1, RangeCells &rc) {
  const int levels = t.max_level + 1;
  rc.cell_lo.assign(levels, 0);
  rc.cell_hi.assign(levels, 0);
  rc.leaf_lo.assign(levels, 0);
  rc.leaf_hi.assign(levels, 0);
  for (int L = 0; L < levels; ++L) {
    const int64_t c0 = t.level_begin[L], c1 = t.level_begin[L + 1];
    // cells of one level hold disjoint body ranges in ascending order
    int64_t lo = c0, hi = c1;
    while (lo < hi) {  // first cell ending after b0
      const int64_t m = (lo + hi) / 2;
      if (t.body_begin[m] + t.n_body[m] <= b0) lo = m + 1;
      else hi = m;
    }
    int64_t cl = lo;
    hi = c1;
    while (lo < hi) {  // first cell starting at or after b1
      const int64_t m = (lo + hi) / 2;
      if (t.body_begin[m] < b1) lo = m + 1;
      else hi = m;
    }
    int64_t ch = lo;
    if (b1 <= b0) cl = ch = c0;
    rc.cell_lo[L] = cl;
    rc.cell_hi[L] = ch;
    rc.leaf_lo[L] = ix.rank[cl];
    rc.leaf_hi[L] = ix.rank[ch];
  }
}

void partition_targets(const TreeData &t, const ListData &l, const LeafIndex &ix, int G,
                       double m2l_weight, int64_t *bounds) {
  const int64_t nc = t.n_cells();
  // M2L work per body: a cell's row spread evenly over its bodies, summed
  // down from the root (parents precede children in breadth-first order).
  std::vector<double> share(nc, 0.0);
  for (int64_t c = 0; c < nc; ++c) {
    const double own = (double)(l.m2l_ptr[c + 1] - l.m2l_ptr[c]) / (double)t.n_body[c];
    share[c] = (t.parent[c] >= 0 ? share[t.parent[c]] : 0.0) + own;
  }
  // leaves in Morton order with their weights
  std::vector<std::pair<int64_t, double>> leaves;
  leaves.reserve(ix.cell.size());
  for (int32_t c : ix.cell) {
    double pairs = 0.0;
    for (int64_t e = l.p2p_ptr[c]; e < l.p2p_ptr[c + 1]; ++e) {
      const int32_t b = l.p2p_col[e];
      pairs += (double)t.n_body[c] * (double)(t.n_body[b] - (b == c ? 1 : 0));
    }
    leaves.emplace_back(t.body_begin[c], pairs + m2l_weight * share[c] * (double)t.n_body[c]);
  }
  std::sort(leaves.begin(), leaves.end());
  double total = 0.0;
  for (const auto &lw : leaves) total += lw.second;
  bounds[0] = 0;
  double acc = 0.0;
  size_t i = 0;
  for (int k = 1; k < G; ++k) {
    const double want = total * (double)k / (double)G;
    // end range k-1 after the leaf whose cumulative weight first reaches `want`
    // (or before it, whichever is closer)
    while (i < leaves.size() && acc + leaves[i].second <= want) acc += leaves[i++].second;
    if (i < leaves.size() && (acc + leaves[i].second - want) < (want - acc)) acc += leaves[i++].second;
    bounds[k] = i < leaves.size() ? leaves[i].first : t.n;
    if (bounds[k] < bounds[k - 1]) bounds[k] = bounds[k - 1];
  }
  bounds[G] = t.n;
}

}  // namespace fmmlib
