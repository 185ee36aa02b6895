// Morton-key octree on the host (section 3.3; Table 3: Morton keys and a
// linked tree; ncrit bodies per leaf).
//
// Readings where the paper is silent (the same rules as the C interface states):
//  * root cube: centre (lo+hi)/2, half-width h = max_d (hi_d - lo_d)/2;
//  * integer coordinate floor((x_d - (c_d - h)) / (2h) * 2^21) clamped to
//    [0, 2^21 - 1]; x in the lowest bit of each key triplet;
//  * stable sort by key (ties keep user order);
//  * a cell at level < 21 with more than ncrit bodies gets one child per
//    non-empty octant, in octant order; breadth-first numbering;
//  * expansion centre = middle of the tight bounding box of the cell's bodies
//    (rectangular cells), or with box centres the centre of the cell's cube
//    of the Morton subdivision of the root cube, (c_d - h) + (i_d + 1/2) 2h/2^L;
//    radius = largest centre-to-body distance.
// Compiled without FMA contraction so that keys, centres and radii are the
// same bit for bit as any other code following these rules.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>

#include "fmm_internal.h"

namespace fmmlib {

namespace {

// Spread the low 21 bits of v so that bit b lands on bit 3b.
inline uint64_t dilate3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x001f00000000ffffull;
  v = (v | (v << 16)) & 0x001f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

// LSD radix sort of (key, index) by key, 8 bits per pass; stable, so equal
// keys keep ascending index order.
void radix_sort_pairs(std::vector<uint64_t> &key, std::vector<int32_t> &idx) {
  const size_t n = key.size();
  std::vector<uint64_t> k2(n);
  std::vector<int32_t> i2(n);
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 8 * pass;
    size_t count[257] = {0};
    for (size_t i = 0; i < n; ++i) count[((key[i] >> shift) & 0xff) + 1]++;
    bool trivial = false;
    for (int b = 1; b <= 256; ++b)
      if (count[b] == n) trivial = true;
    if (trivial) continue;
    for (int b = 0; b < 256; ++b) count[b + 1] += count[b];
    for (size_t i = 0; i < n; ++i) {
      size_t dst = count[(key[i] >> shift) & 0xff]++;
      k2[dst] = key[i];
      i2[dst] = idx[i];
    }
    key.swap(k2);
    idx.swap(i2);
  }
}

}  // namespace

int build_tree(const double *xyz, int64_t n, int ncrit, TreeData &t, std::string &err,
               bool box_centres) {
  t.n = n;
  t.ncrit = ncrit;
  if (n == 0) {
    t.level_begin.assign(1, 0);
    return FMM_OK;
  }
  bool finite = true;
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(xyz[i])) finite = false;
  if (!finite) {
    err = "fmm_tree_build: positions must be finite";
    return FMM_EINVAL;
  }
  double lo[3] = {xyz[0], xyz[1], xyz[2]}, hi[3] = {xyz[0], xyz[1], xyz[2]};
  bool exact = true;
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      const double v = xyz[3 * i + d];
      lo[d] = v < lo[d] ? v : lo[d];
      hi[d] = v > hi[d] ? v : hi[d];
      if ((double)(float)v != v) exact = false;
    }
  t.fp32_exact = exact;
  double h = 0.0;
  for (int d = 0; d < 3; ++d) {
    t.root_center[d] = 0.5 * (lo[d] + hi[d]);
    const double half = 0.5 * (hi[d] - lo[d]);
    h = half > h ? half : h;
  }
  t.root_half = h;

  alloc_checkpoint();
  std::vector<uint64_t> key(n, 0);
  std::vector<int32_t> idx(n);
  const double base[3] = {t.root_center[0] - h, t.root_center[1] - h, t.root_center[2] - h};
  const double width = 2.0 * h;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    idx[i] = (int32_t)i;
    if (h == 0.0) continue;
    uint64_t k = 0;
    for (int d = 0; d < 3; ++d) {
      double s = std::floor((xyz[3 * i + d] - base[d]) / width * 2097152.0);
      s = s < 0.0 ? 0.0 : (s > 2097151.0 ? 2097151.0 : s);
      k |= dilate3((uint64_t)s) << d;
    }
    key[i] = k;
  }
  alloc_checkpoint();
  radix_sort_pairs(key, idx);
  t.perm = idx;
  t.keys = key;
  t.pos.resize(3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) t.pos[3 * i + d] = xyz[3 * (int64_t)idx[i] + d];

  alloc_checkpoint();
  // Level by level: the children of the level-L cells, in parent order,
  // form level L+1.  Within a cell the keys are sorted, so the bodies of one
  // octant are a contiguous range found by binary search on the octant digit.
  t.level.assign(1, 0);
  t.parent.assign(1, -1);
  t.child_begin.assign(1, 0);
  t.n_child.assign(1, 0);
  t.body_begin.assign(1, 0);
  t.n_body.assign(1, n);
  t.level_begin.assign(1, 0);
  int64_t lev_lo = 0, lev_hi = 1;
  int lev = 0;
  while (lev_lo < lev_hi) {
    t.level_begin.push_back(lev_hi);
    for (int64_t c = lev_lo; c < lev_hi; ++c) {
      if (h == 0.0 || t.n_body[c] <= ncrit || lev >= FMM_MAX_LEVEL) continue;
      const int shift = 3 * (FMM_MAX_LEVEL - 1 - lev);
      auto digit_of = [&](uint64_t k) { return (int)((k >> shift) & 7u); };
      const uint64_t *first = t.keys.data() + t.body_begin[c];
      const uint64_t *last = first + t.n_body[c];
      t.child_begin[c] = (int32_t)t.level.size();
      int nchild = 0;
      const uint64_t *cur = first;
      for (int oct = 0; oct < 8 && cur < last; ++oct) {
        const uint64_t *end =
            std::partition_point(cur, last, [&](uint64_t k) { return digit_of(k) <= oct; });
        if (end == cur) continue;
        t.level.push_back(lev + 1);
        t.parent.push_back((int32_t)c);
        t.child_begin.push_back(0);
        t.n_child.push_back(0);
        t.body_begin.push_back(cur - t.keys.data());
        t.n_body.push_back(end - cur);
        ++nchild;
        cur = end;
      }
      t.n_child[c] = nchild;
    }
    lev_lo = lev_hi;
    lev_hi = (int64_t)t.level.size();
    if (lev_lo < lev_hi) ++lev;
  }
  // level_begin has one entry per level plus a final end marker.
  t.max_level = lev;
  t.level_begin.resize(t.max_level + 2);
  t.level_begin[t.max_level + 1] = t.n_cells();

  const int64_t nc = t.n_cells();
  t.n_leaves = 0;
  for (int64_t c = 0; c < nc; ++c) t.n_leaves += t.n_child[c] == 0;

  // Geometry, deepest level first: a leaf takes the bounding box of its
  // bodies, a parent the union of its children's boxes (min/max are exact).
  alloc_checkpoint();
  std::vector<double> blo(3 * nc), bhi(3 * nc);
  for (int L = t.max_level; L >= 0; --L) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = t.level_begin[L]; c < t.level_begin[L + 1]; ++c) {
      double l3[3], h3[3];
      if (t.n_child[c] == 0) {
        const double *p = &t.pos[3 * t.body_begin[c]];
        for (int d = 0; d < 3; ++d) l3[d] = h3[d] = p[d];
        for (int64_t j = 1; j < t.n_body[c]; ++j)
          for (int d = 0; d < 3; ++d) {
            const double v = p[3 * j + d];
            l3[d] = v < l3[d] ? v : l3[d];
            h3[d] = v > h3[d] ? v : h3[d];
          }
      } else {
        const int64_t c0 = t.child_begin[c];
        for (int d = 0; d < 3; ++d) {
          l3[d] = blo[3 * c0 + d];
          h3[d] = bhi[3 * c0 + d];
        }
        for (int64_t k = c0 + 1; k < c0 + t.n_child[c]; ++k)
          for (int d = 0; d < 3; ++d) {
            l3[d] = blo[3 * k + d] < l3[d] ? blo[3 * k + d] : l3[d];
            h3[d] = bhi[3 * k + d] > h3[d] ? bhi[3 * k + d] : h3[d];
          }
      }
      for (int d = 0; d < 3; ++d) {
        blo[3 * c + d] = l3[d];
        bhi[3 * c + d] = h3[d];
      }
    }
  }
  t.center.resize(3 * nc);
  t.radius.resize(nc);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t c = 0; c < nc; ++c) {
    double X[3];
    for (int d = 0; d < 3; ++d) X[d] = 0.5 * (blo[3 * c + d] + bhi[3 * c + d]);
    if (box_centres && t.root_half > 0.0) {
      const int L = t.level[c];
      const uint64_t key = t.keys[t.body_begin[c]];
      const double w = (2.0 * t.root_half) / (double)(1ull << L);
      for (int d = 0; d < 3; ++d) {
        uint64_t i = 0;  // the cell's integer coordinate: the top L bits of the body's
        for (int b = 0; b < L; ++b) i |= ((key >> (3 * (21 - L + b) + d)) & 1ull) << b;
        X[d] = (t.root_center[d] - t.root_half) + ((double)i + 0.5) * w;
      }
    }
    double rmax = 0.0;
    const double *p = &t.pos[3 * t.body_begin[c]];
    for (int64_t j = 0; j < t.n_body[c]; ++j) {
      const double dx = p[3 * j] - X[0], dy = p[3 * j + 1] - X[1], dz = p[3 * j + 2] - X[2];
      const double r = std::sqrt((dx * dx + dy * dy) + dz * dz);
      rmax = r > rmax ? r : rmax;
    }
    for (int d = 0; d < 3; ++d) t.center[3 * c + d] = X[d];
    t.radius[c] = rmax;
  }
  return FMM_OK;
}

}  // namespace fmmlib
