// Dual tree traversal on the host (section 3.3, Algorithms 3 and 4), emitting
// explicit CSR interaction lists for the GPU kernels.
//
// The paper runs the traversal with tasks and calls the kernels inline; here
// the traversal only records pairs.  It is made total and deterministic:
//  * MAC (section 3.2): (theta*theta) * ((dx*dx + dy*dy) + dz*dz) > (B_A + B_B)^2,
//    FP64, strict, between expansion centres;
//  * MAC-first (default): accepted -> M2L; else both leaves -> P2P.
//    Leaf-first (the order printed in Algorithm 4): both leaves -> P2P; else
//    accepted -> M2L;
//  * otherwise a self pair splits into all child pairs, a pair of distinct
//    cells splits the cell with the larger radius (equal: lower number), and
//    a leaf is never split (the other cell is);
//  * the traversal starts by visiting (root, root);
//  * treecode/FMM hybrid (m2p_max > 0): an accepted pair whose target is a
//    leaf of at most m2p_max bodies goes to the M2P list instead of M2L.
// The set of pairs does not depend on the visiting order, so the frontier is
// processed in parallel and the lists are then put in canonical CSR order
// (rows = target cells, sources ascending).
#include <algorithm>
#include <cstring>

#ifdef _OPENMP
#include <omp.h>
#endif

#include "fmm_internal.h"

namespace fmmlib {

namespace {

struct PairBuf {
  std::vector<int32_t> p2p_a, p2p_b, m2l_a, m2l_b, m2p_a, m2p_b;
};

struct Walker {
  const TreeData &t;
  double theta2;
  bool leaf_first;
  int m2p_max;  // hybrid: accepted pairs with a leaf target of <= m2p_max bodies -> M2P

  bool is_leaf(int32_t c) const { return t.n_child[c] == 0; }

  bool accept(int32_t a, int32_t b) const {
    const double *A = &t.center[3 * (int64_t)a];
    const double *B = &t.center[3 * (int64_t)b];
    const double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    const double s = t.radius[a] + t.radius[b];
    return theta2 * d2 > s * s;
  }

  void accepted(int32_t a, int32_t b, PairBuf &out) const {
    if (is_leaf(a) && t.n_body[a] <= m2p_max) {
      out.m2p_a.push_back(a);
      out.m2p_b.push_back(b);
    } else {
      out.m2l_a.push_back(a);
      out.m2l_b.push_back(b);
    }
  }

  // One step: record the pair, or push the pairs it splits into.
  template <class Push>
  void step(int32_t a, int32_t b, PairBuf &out, Push push) const {
    const bool both_leaves = is_leaf(a) && is_leaf(b);
    if (!leaf_first && accept(a, b)) {
      accepted(a, b, out);
      return;
    }
    if (both_leaves) {
      out.p2p_a.push_back(a);
      out.p2p_b.push_back(b);
      return;
    }
    if (leaf_first && accept(a, b)) {
      accepted(a, b, out);
      return;
    }
    if (a == b) {
      const int32_t c0 = t.child_begin[a], nc = t.n_child[a];
      for (int32_t i = 0; i < nc; ++i)
        for (int32_t j = 0; j < nc; ++j) push(c0 + i, c0 + j);
      return;
    }
    const double ra = t.radius[a], rb = t.radius[b];
    bool split_target = ra > rb || (ra == rb && a < b);
    if (split_target && is_leaf(a)) split_target = false;
    if (!split_target && is_leaf(b)) split_target = true;
    if (split_target) {
      for (int32_t i = 0; i < t.n_child[a]; ++i) push(t.child_begin[a] + i, b);
    } else {
      for (int32_t j = 0; j < t.n_child[b]; ++j) push(a, t.child_begin[b] + j);
    }
  }
};

// kind: 0 P2P, 1 M2L, 2 M2P
void to_csr(const std::vector<PairBuf> &bufs, int kind, int64_t n_rows, std::vector<int64_t> &ptr,
            std::vector<int32_t> &col) {
  auto rows_of = [&](const PairBuf &b) -> const std::vector<int32_t> & {
    return kind == 0 ? b.p2p_a : kind == 1 ? b.m2l_a : b.m2p_a;
  };
  auto cols_of = [&](const PairBuf &b) -> const std::vector<int32_t> & {
    return kind == 0 ? b.p2p_b : kind == 1 ? b.m2l_b : b.m2p_b;
  };
  ptr.assign(n_rows + 1, 0);
  for (const auto &b : bufs) {
    const auto &ra = rows_of(b);
    for (int32_t a : ra) ptr[a + 1]++;
  }
  for (int64_t r = 0; r < n_rows; ++r) ptr[r + 1] += ptr[r];
  col.resize(ptr[n_rows]);
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (const auto &b : bufs) {
    const auto &ra = rows_of(b);
    const auto &rb = cols_of(b);
    for (size_t i = 0; i < ra.size(); ++i) col[fill[ra[i]]++] = rb[i];
  }
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t r = 0; r < n_rows; ++r) std::sort(col.begin() + ptr[r], col.begin() + ptr[r + 1]);
}

}  // namespace

void dual_traverse(const TreeData &t, double theta, bool leaf_first, int m2p_max, ListData &l) {
  l.tree_id = t.id;
  l.theta = theta;
  l.flags = leaf_first ? FMM_LEAF_FIRST : FMM_MAC_FIRST;
  l.n_rows = t.n_cells();
  l.m2p_max = m2p_max;
  Walker w{t, theta * theta, leaf_first, m2p_max};

  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  alloc_checkpoint();
  std::vector<PairBuf> bufs(nthreads + 1);
  if (l.n_rows > 0) {
    // Breadth-first expansion until there is enough independent work.
    std::vector<std::pair<int32_t, int32_t>> frontier{{0, 0}}, next;
    const size_t want = (size_t)256 * nthreads;
    while (!frontier.empty() && frontier.size() < want) {
      next.clear();
      for (auto &pr : frontier)
        w.step(pr.first, pr.second, bufs[nthreads],
               [&](int32_t a, int32_t b) { next.emplace_back(a, b); });
      frontier.swap(next);
    }
    // Depth-first from each frontier pair, one private stack per thread.
#pragma omp parallel
    {
      int tid = 0;
#ifdef _OPENMP
      tid = omp_get_thread_num();
#endif
      std::vector<std::pair<int32_t, int32_t>> stack;
#pragma omp for schedule(dynamic, 1)
      for (int64_t f = 0; f < (int64_t)frontier.size(); ++f) {
        stack.push_back(frontier[f]);
        while (!stack.empty()) {
          auto pr = stack.back();
          stack.pop_back();
          w.step(pr.first, pr.second, bufs[tid],
                 [&](int32_t a, int32_t b) { stack.emplace_back(a, b); });
        }
      }
    }
  }
  alloc_checkpoint();
  to_csr(bufs, 0, l.n_rows, l.p2p_ptr, l.p2p_col);
  alloc_checkpoint();
  to_csr(bufs, 1, l.n_rows, l.m2l_ptr, l.m2l_col);
  to_csr(bufs, 2, l.n_rows, l.m2p_ptr, l.m2p_col);
  list_statistics(t, l);
}

void list_statistics(const TreeData &t, ListData &l) {
  int64_t pairs = 0, max_src = 0;
  for (int64_t a = 0; a < l.n_rows; ++a) {
    int64_t src = 0;
    for (int64_t e = l.p2p_ptr[a]; e < l.p2p_ptr[a + 1]; ++e) {
      const int32_t b = l.p2p_col[e];
      src += t.n_body[b];
      pairs += t.n_body[a] * t.n_body[b] - (a == b ? t.n_body[a] : 0);
    }
    max_src = src > max_src ? src : max_src;
  }
  l.p2p_pairs = pairs;
  l.max_row_sources = max_src;
}

}  // namespace fmmlib
