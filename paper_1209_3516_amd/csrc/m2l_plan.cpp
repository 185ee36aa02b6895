// Work plan of the batched M2L for box-centred trees (host).
//
// With expansion centres at the centres of the Morton cubes, the translation
// vector R = X_A - X_B of an M2L entry is an integer multiple of u = h / 2^Lf
// (half the side of the finer of the two cubes, Lf its level): in units of u
// a level-L cell with integer coordinate i sits at (2i + 1) 2^(Lf - L).  So
// R, and with it the translation operator K(R), repeats across the tree (the
// reuse of the paper's section 2 on translation operators, and the geometric
// centre of its Table 3).  The plan groups the entries so that one K(R) is
// applied to several source multipoles at once:
//  * tiles: 16 target cells of one level and one octant class (the same
//    position within their parents), in cell order; in the interior of a
//    uniform tree such cells have the same set of vectors R;
//  * groups: within a tile, the entries with one (source level, R), sorted by
//    that key; a group holds the source cell of each of the 16 targets (or
//    -1) and the index of its vector in the table of distinct vectors.
// Every cell of the tree is in exactly one tile (cells without entries get a
// tile row with no groups, so their locals are written as zeros).
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "fmm_internal.h"

namespace fmmlib {

namespace {

struct OffsetKey {
  int32_t la, lb;
  int64_t rx, ry, rz;
  bool operator<(const OffsetKey &o) const {
    return std::tie(la, lb, rx, ry, rz) < std::tie(o.la, o.lb, o.rx, o.ry, o.rz);
  }
  bool operator==(const OffsetKey &o) const {
    return la == o.la && lb == o.lb && rx == o.rx && ry == o.ry && rz == o.rz;
  }
};

struct OffsetHash {
  size_t operator()(const OffsetKey &k) const {
    uint64_t h = (uint64_t)k.la * 0x9E3779B97F4A7C15ull ^ (uint64_t)k.lb * 0xC2B2AE3D27D4EB4Full;
    h ^= (uint64_t)k.rx + 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.ry + 0x27D4EB2F165667C5ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.rz + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

// Integer coordinate along axis d of the level-L cell holding `key`.
inline int64_t cell_coord(uint64_t key, int L, int d) {
  int64_t v = 0;
  for (int b = 0; b < L; ++b) v |= (int64_t)((key >> (3 * (21 - L + b) + d)) & 1ull) << b;
  return v;
}

}  // namespace

int build_m2l_tile_plan(const TreeData &t, const ListData &l, M2LTilePlan &plan,
                        std::string &err) {
  plan = M2LTilePlan();
  if (!t.box_centres) {
    err = "the batched M2L needs a tree with box centres (FMM_TREE_BOX_CENTRES)";
    return FMM_EINVAL;
  }
  const int64_t nc = t.n_cells();
  if (nc == 0 || t.keys.size() != (size_t)t.n) {
    if (nc == 0) return FMM_OK;
    err = "the batched M2L plan needs the tree's keys on the host";
    return FMM_EINVAL;
  }
  // tiles: level-major, octant class, then cell order
  std::vector<std::vector<int32_t>> cls((size_t)(t.max_level + 1) * 8);
  for (int64_t c = 0; c < nc; ++c) {
    const int L = t.level[c];
    const int oct = L == 0 ? 0 : (int)((t.keys[t.body_begin[c]] >> (3 * (21 - L))) & 7ull);
    cls[(size_t)L * 8 + oct].push_back((int32_t)c);
  }
  plan.level_tile_begin.assign(t.max_level + 2, 0);
  for (int L = 0; L <= t.max_level; ++L) {
    for (int o = 0; o < 8; ++o) {
      const auto &v = cls[(size_t)L * 8 + o];
      for (size_t i = 0; i < v.size(); i += kM2LTile) {
        for (int j = 0; j < kM2LTile; ++j)
          plan.tile_cells.push_back(i + j < v.size() ? v[i + j] : -1);
      }
    }
    plan.level_tile_begin[L + 1] = (int64_t)(plan.tile_cells.size() / kM2LTile);
  }
  const int64_t nt = (int64_t)(plan.tile_cells.size() / kM2LTile);
  plan.n_tiles = nt;
  // per cell: integer coordinates
  std::vector<int64_t> coord(3 * nc);
  for (int64_t c = 0; c < nc; ++c)
    for (int d = 0; d < 3; ++d) coord[3 * c + d] = cell_coord(t.keys[t.body_begin[c]], t.level[c], d);
  auto key_of = [&](int32_t a, int32_t b) {
    const int la = t.level[a], lb = t.level[b];
    const int lf = std::max(la, lb);
    OffsetKey k{la, lb, 0, 0, 0};
    int64_t r[3];
    for (int d = 0; d < 3; ++d)
      r[d] = (2 * coord[3 * a + d] + 1) * (int64_t(1) << (lf - la)) -
             (2 * coord[3 * b + d] + 1) * (int64_t(1) << (lf - lb));
    k.rx = r[0];
    k.ry = r[1];
    k.rz = r[2];
    return k;
  };
  // groups of each tile (in parallel), then one table of distinct vectors
  struct Entry {
    OffsetKey key;
    int32_t j, src;
  };
  std::vector<std::vector<OffsetKey>> tile_keys(nt);
  std::vector<std::vector<int32_t>> tile_src(nt);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t ti = 0; ti < nt; ++ti) {
    std::vector<Entry> es;
    for (int j = 0; j < kM2LTile; ++j) {
      const int32_t a = plan.tile_cells[ti * kM2LTile + j];
      if (a < 0) continue;
      for (int64_t e = l.m2l_ptr[a]; e < l.m2l_ptr[a + 1]; ++e)
        es.push_back(Entry{key_of(a, l.m2l_col[e]), j, l.m2l_col[e]});
    }
    std::sort(es.begin(), es.end(), [](const Entry &x, const Entry &y) {
      return x.key < y.key || (x.key == y.key && x.j < y.j);
    });
    auto &ks = tile_keys[ti];
    auto &ss = tile_src[ti];
    for (size_t i = 0; i < es.size();) {
      size_t k = i;
      ks.push_back(es[i].key);
      const size_t g = ss.size();
      ss.resize(g + kM2LTile, -1);
      while (k < es.size() && es[k].key == es[i].key) {
        ss[g + es[k].j] = es[k].src;
        ++k;
      }
      i = k;
    }
  }
  std::unordered_map<OffsetKey, int32_t, OffsetHash> index;
  plan.tile_group_begin.assign(nt + 1, 0);
  for (int64_t ti = 0; ti < nt; ++ti)
    plan.tile_group_begin[ti + 1] = plan.tile_group_begin[ti] + (int64_t)tile_keys[ti].size();
  const int64_t ng = plan.tile_group_begin[nt];
  plan.n_groups = ng;
  plan.group_offset.resize(ng);
  plan.group_src.resize(ng * kM2LTile);
  for (int64_t ti = 0; ti < nt; ++ti) {
    const int64_t g0 = plan.tile_group_begin[ti];
    for (size_t g = 0; g < tile_keys[ti].size(); ++g) {
      const OffsetKey &k = tile_keys[ti][g];
      auto it = index.find(k);
      if (it == index.end()) {
        it = index.emplace(k, (int32_t)(plan.offsets.size() / 3)).first;
        // the vector in length units: R_units * h / 2^Lf
        const double u = std::ldexp(t.root_half, -std::max(k.la, k.lb));
        plan.offsets.push_back((double)k.rx * u);
        plan.offsets.push_back((double)k.ry * u);
        plan.offsets.push_back((double)k.rz * u);
      }
      plan.group_offset[g0 + g] = it->second;
    }
    std::copy(tile_src[ti].begin(), tile_src[ti].end(),
              plan.group_src.begin() + g0 * kM2LTile);
    std::vector<OffsetKey>().swap(tile_keys[ti]);
    std::vector<int32_t>().swap(tile_src[ti]);
  }
  plan.n_offsets = (int64_t)(plan.offsets.size() / 3);
  if (ng > INT32_MAX || plan.n_offsets > INT32_MAX) {
    err = "batched M2L plan too large";
    plan = M2LTilePlan();
    return FMM_EINVAL;
  }
  return FMM_OK;
}

}  // namespace fmmlib
