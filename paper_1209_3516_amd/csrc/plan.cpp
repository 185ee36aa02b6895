// Work plan of the GPU P2P kernel, built once per (tree, lists) on the host.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>

#include "fmm_internal.h"

namespace fmmlib {

int64_t plan_index_limit() {
  int64_t lim = INT32_MAX;
  if (const char *s = std::getenv("FMM_PLAN_LIMIT")) {
    const long long v = std::atoll(s);
    if (v > 0 && v < lim) lim = v;
  }
  return lim;
}

// Lane layout for a work item of nt <= 64 targets on one 64-lane wave:
// K source streams of L lanes; lane (s, u) holds targets u, u+L, ..., u+(R-1)L
// and visits every K-th staged source.  Maximise the useful fraction
// nt*K / (64*R) of lane-pair slots; on ties take the larger R (more targets
// per staged source read).
void p2p_lane_layout(int nt, int *R, int *L, int *K) {
  double best = -1.0;
  int bR = 1, bL = nt, bK = 1;
  for (int r = 1; r <= kP2PMaxTargetsPerLane; ++r) {
    const int l = (nt + r - 1) / r;
    if (l > 64) continue;
    const int k = 64 / l;
    const double eff = (double)nt * k / (64.0 * r);
    if (eff > best + 1e-12 || std::fabs(eff - best) <= 1e-12) {
      best = eff;
      bR = r;
      bL = l;
      bK = k;
    }
  }
  *R = bR;
  *L = bL;
  *K = bK;
}

int build_p2p_plan(const TreeData &t, const ListData &l, P2PPlan &plan, std::string &err) {
  plan = P2PPlan();
  const int64_t limit = plan_index_limit();
  const int64_t nc = t.n_cells();
  plan.body_leaf.assign(t.n, 0);
  int64_t pbase = 0;
  for (int64_t a = 0; a < nc; ++a) {
    if (t.n_child[a] != 0) continue;
    const int32_t leaf = (int32_t)plan.leaf_cell.size();
    const int64_t nA = t.n_body[a], bA = t.body_begin[a];
    for (int64_t i = bA; i < bA + nA; ++i) plan.body_leaf[i] = leaf;

    // Split the row into source chunks of at most kP2PChunkSources bodies and
    // kP2PMaxRuns runs; merge entries with contiguous bodies into runs.
    struct Chunk {
      int32_t run_begin = 0, n_runs = 0, n_src = 0;
      bool self = false;
    };
    std::vector<Chunk> chunks;
    Chunk cur;
    cur.run_begin = (int32_t)plan.run_body.size();
    int64_t last_end = -1;  // body end of the last run of the current chunk
    int64_t row_src = 0;
    for (int64_t e = l.p2p_ptr[a]; e < l.p2p_ptr[a + 1]; ++e) {
      const int32_t b = l.p2p_col[e];
      const int64_t nb = t.n_body[b], bb = t.body_begin[b];
      row_src += nb;
      const bool contiguous = (b != a) && cur.n_runs > 0 && last_end == bb;
      const bool full = (cur.n_src + (cur.self ? nA : 0) + nb > kP2PChunkSources &&
                         (cur.n_src > 0 || cur.self)) ||
                        (!contiguous && b != a && cur.n_runs >= kP2PMaxRuns);
      if (full) {
        chunks.push_back(cur);
        cur = Chunk();
        cur.run_begin = (int32_t)plan.run_body.size();
        last_end = -1;
      }
      if (b == a) {
        cur.self = true;
        last_end = -1;  // the self leaf interrupts a run
        continue;
      }
      if (cur.n_runs > 0 && last_end == bb) {
        last_end = bb + nb;
      } else {
        plan.run_body.push_back((int32_t)bb);
        plan.run_prefix.push_back(cur.n_src);
        cur.n_runs++;
        last_end = bb + nb;
      }
      cur.n_src += (int32_t)nb;
    }
    if (cur.n_src > 0 || cur.self || chunks.empty()) chunks.push_back(cur);
    plan.max_row_sources = std::max<int32_t>(plan.max_row_sources, (int32_t)row_src);

    const int32_t nch = (int32_t)chunks.size();
    plan.leaf_cell.push_back((int32_t)a);
    plan.leaf_pbase.push_back((int32_t)pbase);
    plan.leaf_nchunk.push_back(nch);
    for (int64_t g = 0; g < nA; g += 64) {
      const int nt = (int)std::min<int64_t>(64, nA - g);
      int R, L, K;
      p2p_lane_layout(nt, &R, &L, &K);
      for (int32_t c = 0; c < nch; ++c) {
        P2PItem it;
        it.tgt_begin = (int32_t)(bA + g);
        it.tgt_cfg = nt | (R << 8) | (L << 16) | (K << 24);
        it.run_begin = chunks[c].run_begin;
        it.n_runs = chunks[c].n_runs;
        it.n_src = chunks[c].n_src;
        it.self_begin = chunks[c].self ? (int32_t)bA : -1;
        it.self_n = chunks[c].self ? (int32_t)nA : 0;
        it.out_off = (int32_t)(pbase + (int64_t)c * nA + g);
        plan.items.push_back(it);
      }
    }
    pbase += (int64_t)nch * nA;
    // Offsets are stored in 32 bits: stop before any of them could wrap.
    if (pbase > limit || (int64_t)plan.items.size() > limit ||
        (int64_t)plan.run_body.size() > limit) {
      err = "P2P work plan too large: more than " + std::to_string(limit) +
            " runs, work items or partial slots (32-bit offsets)";
      plan = P2PPlan();
      return FMM_EINVAL;
    }
  }
  plan.n_partials = pbase;
  return FMM_OK;
}

}  // namespace fmmlib

namespace fmmlib {

// One ring step costs about 18 instructions per (target, source) pair and 6
// per lane besides (the rotation of the travelling source sums and the LDS
// address); a ring of 16 sources takes TL steps.  Take the TL with the lowest
// cost TL * (18 R + 6) per 16 sources; ties go to the smaller TL.
void p2p_mutual_layout(int nt, int *R, int *TL) {
  int bR = 8, bT = 8;
  long best = -1;
  for (int tl = 1; tl <= 8; tl *= 2) {
    const int r = (nt + tl - 1) / tl;
    if (r > 8) continue;
    const long cost = (long)tl * (18 * r + 6);
    if (best < 0 || cost < best) {
      best = cost;
      bR = r;
      bT = tl;
    }
  }
  *R = bR;
  *TL = bT;
}

int build_p2p_mutual_plan(const TreeData &t, const ListData &l, P2PMutualPlan &plan,
                          std::string &err) {
  plan = P2PMutualPlan();
  const int64_t limit = plan_index_limit();
  const int64_t nc = t.n_cells();
  auto fail = [&](const std::string &msg) {
    err = msg;
    plan = P2PMutualPlan();
    return FMM_EINVAL;
  };
  // compact leaf numbers (cell order) and, per leaf B, its leaves A < B
  std::vector<int32_t> leaf_of(nc, -1);
  int64_t nl = 0;
  for (int64_t c = 0; c < nc; ++c)
    if (t.n_child[c] == 0) leaf_of[c] = (int32_t)nl++;
  plan.leaf_mbase.assign(nl, 0);
  plan.leaf_nlow.assign(nl, 0);
  int64_t mbase = 0, n_lower = 0;
  for (int64_t b = 0; b < nc; ++b) {
    if (leaf_of[b] < 0) continue;
    if (t.n_body[b] > 64)
      return fail("mutual P2P needs leaves of at most 64 bodies (a leaf holds " +
                  std::to_string(t.n_body[b]) + ")");
    int32_t low = 0;
    for (int64_t e = l.p2p_ptr[b]; e < l.p2p_ptr[b + 1]; ++e) {
      if (e > l.p2p_ptr[b] && l.p2p_col[e] <= l.p2p_col[e - 1])
        return fail("mutual P2P needs P2P rows in ascending source order");
      if (l.p2p_col[e] < b) ++low;
    }
    plan.leaf_mbase[leaf_of[b]] = (int32_t)std::min<int64_t>(mbase, INT32_MAX);
    plan.leaf_nlow[leaf_of[b]] = low;
    mbase += (int64_t)low * t.n_body[b];
    n_lower += low;
  }
  if (mbase > limit) return fail("mutual P2P plan too large: more than " +
                                 std::to_string(limit) + " source-side slots");
  plan.n_mslots = mbase;

  int64_t pbase = 0, n_upper = 0;
  for (int64_t a = 0; a < nc; ++a) {
    if (leaf_of[a] < 0) continue;
    const int64_t nA = t.n_body[a], bA = t.body_begin[a];
    struct Chunk {
      int32_t run_begin = 0, n_runs = 0, n_src = 0;
      bool self = false;
    };
    std::vector<Chunk> chunks;
    Chunk cur;
    cur.run_begin = (int32_t)plan.run_body.size();
    for (int64_t e = l.p2p_ptr[a]; e < l.p2p_ptr[a + 1]; ++e) {
      const int32_t b = l.p2p_col[e];
      if (b < a) continue;  // evaluated in b's item
      const int64_t nb = t.n_body[b];
      if (b == a) {
        cur.self = true;  // first of the row's entries b >= a (ascending)
        continue;
      }
      plan.upper_pairs += nA * nb;
      // b's row holds a among its leaves below b, at rank j (ascending order)
      const int64_t r0 = l.p2p_ptr[b], r1 = l.p2p_ptr[b + 1];
      const int32_t *pos = std::lower_bound(l.p2p_col.data() + r0, l.p2p_col.data() + r1, (int32_t)a);
      if (pos == l.p2p_col.data() + r1 || *pos != a)
        return fail("mutual P2P needs symmetric P2P lists");
      const int64_t j = pos - (l.p2p_col.data() + r0);
      ++n_upper;
      const bool full = (cur.n_src + (cur.self ? nA : 0) + nb > kP2PChunkSources &&
                         (cur.n_src > 0 || cur.self)) ||
                        cur.n_runs >= kP2PMaxRuns;
      if (full) {
        chunks.push_back(cur);
        cur = Chunk();
        cur.run_begin = (int32_t)plan.run_body.size();
      }
      plan.run_body.push_back((int32_t)t.body_begin[b]);
      plan.run_prefix.push_back(cur.n_src);
      plan.run_dst.push_back((int32_t)(plan.leaf_mbase[leaf_of[b]] + j * nb));
      cur.n_runs++;
      cur.n_src += (int32_t)nb;
    }
    if (cur.n_src > 0 || cur.self || chunks.empty()) chunks.push_back(cur);
    for (const Chunk &ch : chunks)
      if (ch.self) plan.self_pairs += nA * (nA - 1);

    const int32_t nch = (int32_t)chunks.size();
    plan.leaf_pbase.push_back((int32_t)pbase);
    plan.leaf_nchunk.push_back(nch);
    int R, TL;
    p2p_mutual_layout((int)nA, &R, &TL);
    for (int32_t c = 0; c < nch; ++c) {
      P2PItem it;
      it.tgt_begin = (int32_t)bA;
      it.tgt_cfg = (int32_t)nA | (R << 8) | (TL << 16) | ((64 / TL) << 24);
      it.run_begin = chunks[c].run_begin;
      it.n_runs = chunks[c].n_runs;
      it.n_src = chunks[c].n_src;
      it.self_begin = chunks[c].self ? (int32_t)bA : -1;
      it.self_n = chunks[c].self ? (int32_t)nA : 0;
      it.out_off = (int32_t)(pbase + (int64_t)c * nA);
      plan.items.push_back(it);
    }
    pbase += (int64_t)nch * nA;
    if (pbase > limit || (int64_t)plan.items.size() > limit ||
        (int64_t)plan.run_body.size() > limit)
      return fail("mutual P2P plan too large: more than " + std::to_string(limit) +
                  " runs, work items or partial slots (32-bit offsets)");
  }
  // every leaf below B in B's row must have B above it in its own row
  if (n_upper != n_lower) return fail("mutual P2P needs symmetric P2P lists");
  plan.n_partials = pbase;
  return FMM_OK;
}

}  // namespace fmmlib
