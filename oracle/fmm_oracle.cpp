// Oracle: plain, slow, FP64 CPU implementation of the dual-tree-traversal
// Cartesian-Taylor fast multipole method for the 3-D Laplace kernel.
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// CPU-baseline leg of the benchmark load this library.  The GPU library is a
// separate code base and never links, includes or calls anything from here.
//
// Paper: R. Yokota, "An FMM Based on Dual Tree Traversal for Many-core
// Architectures" (arXiv:1209.3516).  The paper gives no formulas for the
// expansions; what is written here is the textbook Cartesian Taylor FMM that
// its section 3.1 (Table 2, "Cartesian Taylor") names, with the readings
// listed beside each function.  Everything is FP64 with plain loops; the only
// parallelism is "omp parallel for" over independent targets.
//
// Build: g++ -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math), so
// that the tree and the multipole acceptance test are reproducible bit for bit.

#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Multi-indices n = (nx, ny, nz) with |n| <= p-1.  Order p keeps the degrees
// 0..p-1, so the error of an accepted pair falls as theta^p (section 3.2).
// Terms are listed by degree, and within a degree by decreasing nx, then
// decreasing ny.
// ---------------------------------------------------------------------------
struct Terms {
  int p = 0;
  std::vector<int> ex, ey, ez;
  std::vector<double> fact;  // nx! ny! nz!
  std::vector<int> lookup;   // (a, b, c) -> term number, -1 outside the set

  explicit Terms(int order) : p(order) {
    lookup.assign(p * p * p, -1);
    for (int deg = 0; deg < p; ++deg)
      for (int a = deg; a >= 0; --a)
        for (int b = deg - a; b >= 0; --b) {
          int c = deg - a - b;
          lookup[(a * p + b) * p + c] = (int)ex.size();
          ex.push_back(a);
          ey.push_back(b);
          ez.push_back(c);
          fact.push_back(factorial(a) * factorial(b) * factorial(c));
        }
  }
  int count() const { return (int)ex.size(); }
  int degree(int t) const { return ex[t] + ey[t] + ez[t]; }
  int index(int a, int b, int c) const {
    if (a < 0 || b < 0 || c < 0 || a + b + c > p - 1) return -1;
    return lookup[(a * p + b) * p + c];
  }
  static double factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
  }
};

double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

// d^n / n! for the three components of d.
double scaled_monomial(const Terms &T, int t, const double d[3]) {
  return ipow(d[0], T.ex[t]) * ipow(d[1], T.ey[t]) * ipow(d[2], T.ez[t]) / T.fact[t];
}

// Derivatives D^m G(R) of G(R) = 1/|R| for |m| <= p-1.  Uses the recurrence
// for the Taylor coefficients a_m = D^m G / m!:
//   |m| |R|^2 a_m = -(2|m|-1) sum_d R_d a_{m-e_d} - (|m|-1) sum_d a_{m-2e_d}
// (terms with a negative index are absent), then D^m G = m! a_m.
void derivatives(const Terms &T, const double R[3], double *D) {
  const int n = T.count();
  std::vector<double> a(n, 0.0);
  const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  a[0] = 1.0 / std::sqrt(r2);
  for (int t = 1; t < n; ++t) {
    const int m[3] = {T.ex[t], T.ey[t], T.ez[t]};
    const int k = T.degree(t);
    double s1 = 0.0, s2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      int m1[3] = {m[0], m[1], m[2]};
      m1[d] -= 1;
      int i1 = T.index(m1[0], m1[1], m1[2]);
      if (i1 >= 0) s1 += R[d] * a[i1];
      int m2[3] = {m[0], m[1], m[2]};
      m2[d] -= 2;
      int i2 = T.index(m2[0], m2[1], m2[2]);
      if (i2 >= 0) s2 += a[i2];
    }
    a[t] = (-(2.0 * k - 1.0) * s1 - (k - 1.0) * s2) / (k * r2);
  }
  for (int t = 0; t < n; ++t) D[t] = T.fact[t] * a[t];
}

// P2M: M_n(B) = sum_j q_j (X_B - x_j)^n / n!
void p2m(const Terms &T, const double X[3], const double *x, const double *y,
         const double *z, const double *q, int64_t nb, double *M) {
  for (int t = 0; t < T.count(); ++t) M[t] = 0.0;
  for (int64_t j = 0; j < nb; ++j) {
    const double d[3] = {X[0] - x[j], X[1] - y[j], X[2] - z[j]};
    for (int t = 0; t < T.count(); ++t) M[t] += q[j] * scaled_monomial(T, t, d);
  }
}

// M2M: M_n(P) += sum_{m <= n} M_m(c) (X_P - X_c)^(n-m) / (n-m)!
void m2m(const Terms &T, const double XP[3], const double Xc[3], const double *Mc, double *MP) {
  const double d[3] = {XP[0] - Xc[0], XP[1] - Xc[1], XP[2] - Xc[2]};
  for (int n = 0; n < T.count(); ++n)
    for (int m = 0; m < T.count(); ++m) {
      int k = T.index(T.ex[n] - T.ex[m], T.ey[n] - T.ey[m], T.ez[n] - T.ez[m]);
      if (k < 0) continue;
      MP[n] += Mc[m] * scaled_monomial(T, k, d);
    }
}

// M2L: L_k(A) += sum_{|n| + |k| <= p-1} M_n(B) D^(n+k) G(X_A - X_B)
void m2l(const Terms &T, const double XA[3], const double XB[3], const double *M, double *L) {
  const double R[3] = {XA[0] - XB[0], XA[1] - XB[1], XA[2] - XB[2]};
  std::vector<double> D(T.count());
  derivatives(T, R, D.data());
  for (int k = 0; k < T.count(); ++k)
    for (int n = 0; n < T.count(); ++n) {
      int s = T.index(T.ex[n] + T.ex[k], T.ey[n] + T.ey[k], T.ez[n] + T.ez[k]);
      if (s < 0) continue;
      L[k] += M[n] * D[s];
    }
}

// L2L: L_k(c) += sum_{m >= k} L_m(P) (X_c - X_P)^(m-k) / (m-k)!
void l2l(const Terms &T, const double XP[3], const double Xc[3], const double *LP, double *Lc) {
  const double d[3] = {Xc[0] - XP[0], Xc[1] - XP[1], Xc[2] - XP[2]};
  for (int k = 0; k < T.count(); ++k)
    for (int m = 0; m < T.count(); ++m) {
      int s = T.index(T.ex[m] - T.ex[k], T.ey[m] - T.ey[k], T.ez[m] - T.ez[k]);
      if (s < 0) continue;
      Lc[k] += LP[m] * scaled_monomial(T, s, d);
    }
}

// L2P: phi(y) = sum_k L_k (y - X_A)^k / k!,
//      d phi / d y_d = sum_{k_d >= 1} L_k (y - X_A)^(k - e_d) / (k - e_d)!
void l2p(const Terms &T, const double XA[3], const double *L, const double y[3],
         double *phi, double g[3]) {
  const double d[3] = {y[0] - XA[0], y[1] - XA[1], y[2] - XA[2]};
  double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int k = 0; k < T.count(); ++k) {
    f += L[k] * scaled_monomial(T, k, d);
    int ix = T.index(T.ex[k] - 1, T.ey[k], T.ez[k]);
    int iy = T.index(T.ex[k], T.ey[k] - 1, T.ez[k]);
    int iz = T.index(T.ex[k], T.ey[k], T.ez[k] - 1);
    if (ix >= 0) gx += L[k] * scaled_monomial(T, ix, d);
    if (iy >= 0) gy += L[k] * scaled_monomial(T, iy, d);
    if (iz >= 0) gz += L[k] * scaled_monomial(T, iz, d);
  }
  *phi += f;
  g[0] += gx;
  g[1] += gy;
  g[2] += gz;
}

// M2P (the treecode's evaluation of a multipole at a body, Algorithm 1):
// Taylor's theorem for G(y - x_j) about y - X_B gives
//   phi(y)         = sum_{|n| <= p-1} M_n(B) D^n G(y - X_B),
//   d phi / d y_d  = sum_{|n| <= p-1} M_n(B) D^(n+e_d) G(y - X_B),
// so the gradient needs derivatives up to degree p (a set of order p+1).
void m2p(const Terms &T, const double XB[3], const double *M, const double y[3], double *phi,
         double g[3]) {
  const Terms T1(T.p + 1);
  const double R[3] = {y[0] - XB[0], y[1] - XB[1], y[2] - XB[2]};
  std::vector<double> D(T1.count());
  derivatives(T1, R, D.data());
  double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int n = 0; n < T.count(); ++n) {
    f += M[n] * D[T1.index(T.ex[n], T.ey[n], T.ez[n])];
    gx += M[n] * D[T1.index(T.ex[n] + 1, T.ey[n], T.ez[n])];
    gy += M[n] * D[T1.index(T.ex[n], T.ey[n] + 1, T.ez[n])];
    gz += M[n] * D[T1.index(T.ex[n], T.ey[n], T.ez[n] + 1)];
  }
  *phi += f;
  g[0] += gx;
  g[1] += gy;
  g[2] += gz;
}

// P2P for one target point: phi += q_j / r, grad += q_j (x_j - x_i) / r^3,
// pairs at zero distance contribute nothing (this also drops the self term).
void p2p_point(const double xi[3], const double *x, const double *y, const double *z,
               const double *q, int64_t nb, double *phi, double g[3]) {
  for (int64_t j = 0; j < nb; ++j) {
    const double dx = x[j] - xi[0], dy = y[j] - xi[1], dz = z[j] - xi[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) continue;
    const double r = std::sqrt(r2);
    const double inv_r = 1.0 / r;
    const double inv_r3 = inv_r / r2;
    *phi += q[j] * inv_r;
    g[0] += q[j] * dx * inv_r3;
    g[1] += q[j] * dy * inv_r3;
    g[2] += q[j] * dz * inv_r3;
  }
}

// Sources that also carry a dipole moment s (used by the backward of a loss
// on the gradient).  A dipole s at x_j has the potential s . grad_y G(y - x_j)
// = s . (x_j - y) / |y - x_j|^3; in the multipole expansion about X_B it
// contributes M_n += sum_d s_d (X_B - x_j)^(n - e_d) / (n - e_d)!.
void p2m_dipole(const Terms &T, const double X[3], const double *x, const double *y,
                const double *z, const double *s, int64_t nb, double *M) {
  for (int64_t j = 0; j < nb; ++j) {
    const double d[3] = {X[0] - x[j], X[1] - y[j], X[2] - z[j]};
    for (int t = 0; t < T.count(); ++t)
      for (int a = 0; a < 3; ++a) {
        int e[3] = {T.ex[t], T.ey[t], T.ez[t]};
        e[a] -= 1;
        const int l = T.index(e[0], e[1], e[2]);
        if (l >= 0) M[t] += s[3 * j + a] * scaled_monomial(T, l, d);
      }
  }
}

// Hessian of the local expansion at y, applied to the vector v:
// (H v)_a = sum_b v_b sum_{k >= e_a + e_b} L_k (y - X_A)^(k - e_a - e_b) / (k - e_a - e_b)!
void l2p_hessian(const Terms &T, const double XA[3], const double *L, const double y[3],
                 const double v[3], double hv[3]) {
  const double d[3] = {y[0] - XA[0], y[1] - XA[1], y[2] - XA[2]};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double h = 0.0;
      for (int k = 0; k < T.count(); ++k) {
        int e[3] = {T.ex[k], T.ey[k], T.ez[k]};
        e[a] -= 1;
        e[b] -= 1;
        const int l = T.index(e[0], e[1], e[2]);
        if (l >= 0) h += L[k] * scaled_monomial(T, l, d);
      }
      hv[a] += h * v[b];
    }
}

// Direct interaction of sources (charges q, optional dipoles s) with one
// target: potential, gradient, and optionally the Hessian of the charge
// field applied to v (Hessian of 1/|r| is (3 r r^T - r^2 I) / r^5).
void p2p_general_point(const double xi[3], const double *x, const double *y, const double *z,
                       const double *q, const double *s, int64_t nb, const double *v,
                       double *phi, double g[3], double hv[3]) {
  for (int64_t j = 0; j < nb; ++j) {
    const double d[3] = {x[j] - xi[0], y[j] - xi[1], z[j] - xi[2]};
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) continue;
    const double r = std::sqrt(r2);
    const double inv3 = 1.0 / (r2 * r);
    const double inv5 = inv3 / r2;
    *phi += q[j] / r;
    for (int a = 0; a < 3; ++a) g[a] += q[j] * d[a] * inv3;
    if (s) {
      const double *sj = &s[3 * j];
      const double sd = sj[0] * d[0] + sj[1] * d[1] + sj[2] * d[2];
      *phi += sd * inv3;
      for (int a = 0; a < 3; ++a) g[a] += -sj[a] * inv3 + 3.0 * sd * d[a] * inv5;
    }
    if (v && hv) {
      const double dv = d[0] * v[0] + d[1] * v[1] + d[2] * v[2];
      for (int a = 0; a < 3; ++a) hv[a] += q[j] * (3.0 * dv * d[a] - r2 * v[a]) * inv5;
    }
  }
}

// ---------------------------------------------------------------------------
// Tree: bounding cube, 21-bit-per-axis Morton keys, stable sort, split every
// cell holding more than ncrit bodies (section 3.3 and Table 3: Morton keys,
// a linked tree, ncrit bodies per leaf).  Readings where the paper is silent:
//  * root cube: centre c = (lo+hi)/2, half-width h = max_d (hi_d - lo_d)/2;
//  * integer coordinate i_d = floor((x_d - (c_d - h)) / (2h) * 2^21), clamped
//    to [0, 2^21-1]; bit b of i_x, i_y, i_z goes to key bit 3b, 3b+1, 3b+2;
//  * a cell at level L < 21 with more than ncrit bodies gets one child per
//    non-empty octant (octant = key digit of level L+1), in octant order;
//  * cells are numbered breadth first, so the children of a cell are
//    contiguous; h == 0 (all bodies coincide) gives a single leaf.
// Cell geometry (rectangular cells, section 3.3): the expansion centre is the
// midpoint of the tight bounding box of the cell's bodies, the radius is the
// largest distance from that centre to one of its bodies.
// ---------------------------------------------------------------------------
struct Cell {
  int level, parent, child_begin, n_child;
  int64_t body_begin, n_body;
  double X[3], B;
};

struct Tree {
  int64_t n = 0;
  int ncrit = 0;
  std::vector<double> xs, ys, zs;  // sorted positions
  std::vector<int32_t> perm;       // sorted position -> user index
  std::vector<uint64_t> keys;      // sorted keys
  std::vector<Cell> cells;
};

uint64_t spread_bits(uint64_t v) {
  uint64_t out = 0;
  for (int b = 0; b < 21; ++b) out |= ((v >> b) & 1ull) << (3 * b);
  return out;
}

// Cell geometry.  Default (reading R6): the centre is the middle of the tight
// bounding box of the cell's bodies.  With `box` (reading R6b, the geometric
// centre of the cell in the paper's comparison of treecode and FMM, Table 3):
// the centre of the cell's cube, the cube of side 2h / 2^L of the Morton
// subdivision of the root cube that holds its key prefix, at
// (c - h) + (i + 1/2) (2h / 2^L) per axis with i the cell's integer
// coordinate.  Either way the radius is the largest distance from the
// centre to a body of the cell.
double box_centre(double c, double h, int level, uint64_t coord) {
  const double w = (2.0 * h) / (double)(1ull << level);
  return (c - h) + ((double)coord + 0.5) * w;
}

// Integer coordinate along axis d of the level-L cell that holds `key`.
uint64_t cell_coord(uint64_t key, int level, int d) {
  uint64_t v = 0;
  for (int b = 0; b < level; ++b) v |= ((key >> (3 * (20 - level + 1 + b) + d)) & 1ull) << b;
  return v;
}

void build_tree(const double *xyz, int64_t n, int ncrit, Tree &tr, bool box = false) {
  tr.n = n;
  tr.ncrit = ncrit;
  tr.cells.clear();
  if (n == 0) return;
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) lo[d] = hi[d] = xyz[d];
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], xyz[3 * i + d]);
      hi[d] = std::max(hi[d], xyz[3 * i + d]);
    }
  double c[3], h = 0.0;
  for (int d = 0; d < 3; ++d) {
    c[d] = 0.5 * (lo[d] + hi[d]);
    h = std::max(h, 0.5 * (hi[d] - lo[d]));
  }
  std::vector<uint64_t> key(n, 0);
  if (h > 0.0) {
    for (int64_t i = 0; i < n; ++i) {
      uint64_t k = 0;
      for (int d = 0; d < 3; ++d) {
        double t = (xyz[3 * i + d] - (c[d] - h)) / (2.0 * h) * 2097152.0;
        double f = std::floor(t);
        if (f < 0.0) f = 0.0;
        if (f > 2097151.0) f = 2097151.0;
        k |= spread_bits((uint64_t)f) << d;
      }
      key[i] = k;
    }
  }
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  tr.perm = order;
  tr.xs.resize(n);
  tr.ys.resize(n);
  tr.zs.resize(n);
  tr.keys.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    tr.xs[i] = xyz[3 * order[i] + 0];
    tr.ys[i] = xyz[3 * order[i] + 1];
    tr.zs[i] = xyz[3 * order[i] + 2];
    tr.keys[i] = key[order[i]];
  }
  tr.cells.push_back(Cell{0, -1, 0, 0, 0, n, {0, 0, 0}, 0});
  // FIFO over the growing cell array: every level-L cell is appended before
  // any level-(L+1) cell, which is breadth-first numbering.
  for (size_t ci = 0; ci < tr.cells.size(); ++ci) {
    Cell cell = tr.cells[ci];
    if (h == 0.0 || cell.n_body <= ncrit || cell.level >= 21) continue;
    const int shift = 3 * (20 - cell.level);
    int first_child = (int)tr.cells.size();
    int nchild = 0;
    int64_t j = cell.body_begin, end = cell.body_begin + cell.n_body;
    while (j < end) {
      uint64_t digit = (tr.keys[j] >> shift) & 7ull;
      int64_t k = j;
      while (k < end && ((tr.keys[k] >> shift) & 7ull) == digit) ++k;
      tr.cells.push_back(Cell{cell.level + 1, (int)ci, 0, 0, j, k - j, {0, 0, 0}, 0});
      ++nchild;
      j = k;
    }
    tr.cells[ci].child_begin = first_child;
    tr.cells[ci].n_child = nchild;
  }
  for (auto &cell : tr.cells) {
    double blo[3], bhi[3];
    int64_t b0 = cell.body_begin;
    blo[0] = bhi[0] = tr.xs[b0];
    blo[1] = bhi[1] = tr.ys[b0];
    blo[2] = bhi[2] = tr.zs[b0];
    for (int64_t j = b0; j < b0 + cell.n_body; ++j) {
      blo[0] = std::min(blo[0], tr.xs[j]);
      bhi[0] = std::max(bhi[0], tr.xs[j]);
      blo[1] = std::min(blo[1], tr.ys[j]);
      bhi[1] = std::max(bhi[1], tr.ys[j]);
      blo[2] = std::min(blo[2], tr.zs[j]);
      bhi[2] = std::max(bhi[2], tr.zs[j]);
    }
    for (int d = 0; d < 3; ++d) cell.X[d] = 0.5 * (blo[d] + bhi[d]);
    if (box && h > 0.0)
      for (int d = 0; d < 3; ++d)
        cell.X[d] = box_centre(c[d], h, cell.level, cell_coord(tr.keys[b0], cell.level, d));
    double B = 0.0;
    for (int64_t j = b0; j < b0 + cell.n_body; ++j) {
      double dx = tr.xs[j] - cell.X[0], dy = tr.ys[j] - cell.X[1], dz = tr.zs[j] - cell.X[2];
      B = std::max(B, std::sqrt((dx * dx + dy * dy) + dz * dz));
    }
    cell.B = B;
  }
}

// ---------------------------------------------------------------------------
// Dual tree traversal (section 3.3, Algorithms 3 and 4).  Readings:
//  * MAC (section 3.2): the pair is well separated iff
//      (theta*theta) * ((dx*dx + dy*dy) + dz*dz) > (B_A + B_B)^2
//    with d the distance between expansion centres (strict, FP64).
//  * default order "MAC first": M2L if accepted, else P2P if both are leaves;
//    "leaf first" (the order printed in Algorithm 4) tests the leaves first.
//  * otherwise a self pair (A,A) splits into all pairs of children; a pair of
//    distinct cells splits the one with the larger radius (equal radii: the
//    one with the lower number); a leaf is never split, the other cell is.
//  * the traversal starts by visiting (root, root), so a single-leaf tree
//    gives P2P(root, root).
// The resulting lists are symmetric: (A,B) is present iff (B,A) is.
// ---------------------------------------------------------------------------
struct Lists {
  int64_t n_rows = 0;
  std::vector<int64_t> p2p_ptr, m2l_ptr, m2p_ptr;
  std::vector<int32_t> p2p_col, m2l_col, m2p_col;
};

// The traversal of Algorithms 3 and 4.  With m2p_max > 0 it is the
// treecode/FMM hybrid: an accepted pair whose target is a leaf of at most
// m2p_max bodies is evaluated by M2P at those bodies instead of M2L.
struct Traversal {
  const Tree &tr;
  double theta;
  bool leaf_first;
  int m2p_max;
  std::vector<std::pair<int32_t, int32_t>> p2p, m2l, m2p;
  // Restricted traversal (empty = the whole one): wanted[c] marks the cells on
  // the paths from the root to chosen leaves.  Every pair that visit(a, b)
  // produces has its target inside a's subtree, so skipping the visits whose
  // target cell is off those paths drops exactly the rows of the other
  // targets and leaves the rows of the marked cells as they are.
  std::vector<char> wanted;

  void accepted(int a, int b) {
    if (leaf(a) && tr.cells[a].n_body <= m2p_max) m2p.emplace_back(a, b);
    else m2l.emplace_back(a, b);
  }

  bool leaf(int c) const { return tr.cells[c].n_child == 0; }
  bool mac(int a, int b) const {
    const Cell &A = tr.cells[a], &B = tr.cells[b];
    double dx = A.X[0] - B.X[0], dy = A.X[1] - B.X[1], dz = A.X[2] - B.X[2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double s = A.B + B.B;
    return (theta * theta) * d2 > s * s;
  }
  void visit(int a, int b) {
    if (!wanted.empty() && !wanted[a]) return;
    if (leaf_first) {
      if (leaf(a) && leaf(b)) { p2p.emplace_back(a, b); return; }
      if (mac(a, b)) { accepted(a, b); return; }
    } else {
      if (mac(a, b)) { accepted(a, b); return; }
      if (leaf(a) && leaf(b)) { p2p.emplace_back(a, b); return; }
    }
    const Cell &A = tr.cells[a], &B = tr.cells[b];
    if (a == b) {
      for (int i = 0; i < A.n_child; ++i)
        for (int j = 0; j < A.n_child; ++j) visit(A.child_begin + i, A.child_begin + j);
      return;
    }
    bool split_a = (A.B > B.B) || (A.B == B.B && a < b);
    if (split_a && leaf(a)) split_a = false;
    else if (!split_a && leaf(b)) split_a = true;
    if (split_a)
      for (int i = 0; i < A.n_child; ++i) visit(A.child_begin + i, b);
    else
      for (int j = 0; j < B.n_child; ++j) visit(a, B.child_begin + j);
  }
};

// Canonical CSR: rows are target cells, sources ascend within a row.
void to_csr(std::vector<std::pair<int32_t, int32_t>> &pairs, int64_t n_rows,
            std::vector<int64_t> &ptr, std::vector<int32_t> &col) {
  std::sort(pairs.begin(), pairs.end());
  ptr.assign(n_rows + 1, 0);
  col.resize(pairs.size());
  for (size_t i = 0; i < pairs.size(); ++i) {
    ptr[pairs[i].first + 1] += 1;
    col[i] = pairs[i].second;
  }
  for (int64_t r = 0; r < n_rows; ++r) ptr[r + 1] += ptr[r];
}

void traverse(const Tree &tr, double theta, bool leaf_first, int m2p_max, Lists &ls,
              const int32_t *leaves = nullptr, int64_t n_leaves = 0) {
  ls.n_rows = (int64_t)tr.cells.size();
  Traversal tv{tr, theta, leaf_first, m2p_max, {}, {}, {}, {}};
  if (leaves) {
    tv.wanted.assign(tr.cells.size(), 0);
    for (int64_t k = 0; k < n_leaves; ++k)
      for (int c = leaves[k]; c >= 0; c = tr.cells[c].parent) tv.wanted[c] = 1;
  }
  if (!tr.cells.empty()) tv.visit(0, 0);
  to_csr(tv.p2p, ls.n_rows, ls.p2p_ptr, ls.p2p_col);
  to_csr(tv.m2l, ls.n_rows, ls.m2l_ptr, ls.m2l_col);
  to_csr(tv.m2p, ls.n_rows, ls.m2p_ptr, ls.m2p_col);
}

// Upward pass: P2M on every leaf, then M2M from the deepest level upwards.
void upward_pass(const Tree &tr, const Terms &T, const std::vector<double> &qs,
                 std::vector<double> &M) {
  const int64_t nc = (int64_t)tr.cells.size();
  const int nt = T.count();
  M.assign(nc * nt, 0.0);
  int max_level = 0;
  for (const auto &c : tr.cells) max_level = std::max(max_level, c.level);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t c = 0; c < nc; ++c) {
    const Cell &C = tr.cells[c];
    if (C.n_child != 0) continue;
    int64_t b = C.body_begin;
    p2m(T, C.X, &tr.xs[b], &tr.ys[b], &tr.zs[b], &qs[b], C.n_body, &M[c * nt]);
  }
  for (int lev = max_level - 1; lev >= 0; --lev) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < nc; ++c) {
      const Cell &C = tr.cells[c];
      if (C.level != lev || C.n_child == 0) continue;
      for (int k = 0; k < C.n_child; ++k) {
        int ch = C.child_begin + k;
        m2m(T, C.X, tr.cells[ch].X, &M[ch * nt], &M[c * nt]);
      }
    }
  }
}

// Wall-clock seconds of the phases of the last full evaluation (timing only;
// no effect on the arithmetic): upward pass, M2L, downward pass, L2P (with
// M2P for hybrid lists), P2P.
double g_phase_seconds[5] = {0, 0, 0, 0, 0};

struct PhaseClock {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  void lap(int k) {
    const auto t1 = std::chrono::steady_clock::now();
    g_phase_seconds[k] = std::chrono::duration<double>(t1 - t0).count();
    t0 = t1;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// C interface (for ctypes).  Every function returns 0 on success.
// ---------------------------------------------------------------------------
struct oracle_fmm {
  Tree tree;
  Lists lists;
};

extern "C" {

int oracle_build(const double *xyz, int64_t n, int ncrit, double theta, int leaf_first,
                 oracle_fmm **out) {
  if (n < 0 || ncrit < 1 || !(theta > 0.0)) return -1;
  oracle_fmm *o = new oracle_fmm;
  build_tree(xyz, n, ncrit, o->tree);
  traverse(o->tree, theta, leaf_first != 0, 0, o->lists);
  *out = o;
  return 0;
}

// The treecode/FMM hybrid lists (m2p_max >= 0; 0 gives oracle_build's lists).
int oracle_build_hybrid(const double *xyz, int64_t n, int ncrit, double theta, int leaf_first,
                        int m2p_max, oracle_fmm **out) {
  if (n < 0 || ncrit < 1 || !(theta > 0.0) || m2p_max < 0) return -1;
  oracle_fmm *o = new oracle_fmm;
  build_tree(xyz, n, ncrit, o->tree);
  traverse(o->tree, theta, leaf_first != 0, m2p_max, o->lists);
  *out = o;
  return 0;
}

// The tree alone; oracle_traverse makes the lists.  box != 0: cell centres
// at the centres of the Morton cubes (reading R6b).
int oracle_build_tree(const double *xyz, int64_t n, int ncrit, int box, oracle_fmm **out) {
  if (n < 0 || ncrit < 1) return -1;
  oracle_fmm *o = new oracle_fmm;
  build_tree(xyz, n, ncrit, o->tree, box != 0);
  o->lists = Lists();
  o->lists.n_rows = (int64_t)o->tree.cells.size();
  *out = o;
  return 0;
}

// (Re)make the lists of a tree.  leaves == NULL: the whole traversal, as
// oracle_build.  Otherwise the restricted traversal: only the rows of the
// given leaves and of their ancestors (each row equal to the whole
// traversal's), every other row empty; enough for oracle_evaluate_leaves on
// those leaves at sizes where the whole lists are large.
int oracle_traverse(oracle_fmm *o, double theta, int leaf_first, int m2p_max,
                    const int32_t *leaves, int64_t n_leaves) {
  if (!(theta > 0.0) || m2p_max < 0 || n_leaves < 0) return -1;
  for (int64_t k = 0; leaves && k < n_leaves; ++k)
    if (leaves[k] < 0 || leaves[k] >= (int64_t)o->tree.cells.size()) return -1;
  o->lists = Lists();
  traverse(o->tree, theta, leaf_first != 0, m2p_max, o->lists, leaves, n_leaves);
  return 0;
}

void oracle_free(oracle_fmm *o) { delete o; }

// OpenMP threads for the calls that follow (n <= 0: all processors).
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }

int oracle_get_threads(void) { return omp_get_max_threads(); }

// Phase times of the last oracle_evaluate on this process (seconds): upward
// pass, M2L, downward pass, L2P, P2P.
void oracle_last_phase_seconds(double *out) {
  for (int k = 0; k < 5; ++k) out[k] = g_phase_seconds[k];
}

int64_t oracle_num_cells(const oracle_fmm *o) { return (int64_t)o->tree.cells.size(); }

void oracle_tree(const oracle_fmm *o, int32_t *perm, uint64_t *keys, int32_t *level,
                 int32_t *parent, int32_t *child_begin, int32_t *n_child, int64_t *body_begin,
                 int64_t *n_body, double *center, double *radius) {
  const Tree &t = o->tree;
  for (int64_t i = 0; i < t.n; ++i) {
    perm[i] = t.perm[i];
    keys[i] = t.keys[i];
  }
  for (size_t c = 0; c < t.cells.size(); ++c) {
    level[c] = t.cells[c].level;
    parent[c] = t.cells[c].parent;
    child_begin[c] = t.cells[c].child_begin;
    n_child[c] = t.cells[c].n_child;
    body_begin[c] = t.cells[c].body_begin;
    n_body[c] = t.cells[c].n_body;
    for (int d = 0; d < 3; ++d) center[3 * c + d] = t.cells[c].X[d];
    radius[c] = t.cells[c].B;
  }
}

// kind 0 = P2P, 1 = M2L, 2 = M2P
int64_t oracle_list_nnz(const oracle_fmm *o, int kind) {
  const Lists &l = o->lists;
  return (int64_t)(kind == 0 ? l.p2p_col.size() : kind == 1 ? l.m2l_col.size() : l.m2p_col.size());
}

void oracle_list(const oracle_fmm *o, int kind, int64_t *row_ptr, int32_t *col) {
  const Lists &l = o->lists;
  const auto &p = kind == 0 ? l.p2p_ptr : kind == 1 ? l.m2l_ptr : l.m2p_ptr;
  const auto &c = kind == 0 ? l.p2p_col : kind == 1 ? l.m2l_col : l.m2p_col;
  std::copy(p.begin(), p.end(), row_ptr);
  std::copy(c.begin(), c.end(), col);
}

int oracle_num_terms(int p) { return p * (p + 1) * (p + 2) / 6; }

void oracle_term_exponents(int p, int32_t *abc) {
  Terms T(p);
  for (int t = 0; t < T.count(); ++t) {
    abc[3 * t + 0] = T.ex[t];
    abc[3 * t + 1] = T.ey[t];
    abc[3 * t + 2] = T.ez[t];
  }
}

// Full evaluation with charges q (user order).  Outputs in user order:
// phi[n], grad[n][3].  Optional staged outputs (NULL to skip), in sorted body
// order / cell order: near_phi, near_grad (P2P only), far_phi, far_grad (L2P
// and, for hybrid lists, M2P), M[n_cells][T], L_m2l[n_cells][T] (after M2L, before L2L),
// L_all[n_cells][T] (after L2L).
int oracle_evaluate(const oracle_fmm *o, int p, const double *q, double *phi, double *grad,
                    double *near_phi, double *near_grad, double *far_phi, double *far_grad,
                    double *M_out, double *Lm2l_out, double *L_out) {
  if (p < 1 || p > 16) return -1;
  const Tree &tr = o->tree;
  const Lists &ls = o->lists;
  const int64_t n = tr.n;
  const int64_t nc = (int64_t)tr.cells.size();
  if (n == 0) return 0;
  Terms T(p);
  const int nt = T.count();
  PhaseClock clock;
  std::vector<double> qs(n);
  for (int64_t i = 0; i < n; ++i) qs[i] = q[tr.perm[i]];

  // Upward pass: P2M on leaves, then M2M from the deepest level upwards.
  std::vector<double> M;
  upward_pass(tr, T, qs, M);
  clock.lap(0);
  int max_level = 0;
  for (const auto &c : tr.cells) max_level = std::max(max_level, c.level);
  // M2L over the M2L list, one target row at a time.
  std::vector<double> L(nc * nt, 0.0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < nc; ++a)
    for (int64_t e = ls.m2l_ptr[a]; e < ls.m2l_ptr[a + 1]; ++e) {
      int b = ls.m2l_col[e];
      m2l(T, tr.cells[a].X, tr.cells[b].X, &M[b * nt], &L[a * nt]);
    }
  clock.lap(1);
  if (Lm2l_out) std::copy(L.begin(), L.end(), Lm2l_out);

  // Downward pass: L2L from the root's children downwards.
  for (int lev = 1; lev <= max_level; ++lev) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < nc; ++c) {
      const Cell &C = tr.cells[c];
      if (C.level != lev) continue;
      l2l(T, tr.cells[C.parent].X, C.X, &L[C.parent * nt], &L[c * nt]);
    }
  }
  clock.lap(2);

  // L2P (far field) on every target leaf; the near field (P2P) separately.
  std::vector<double> fphi(n, 0.0), fg(3 * n, 0.0), nphi(n, 0.0), ng(3 * n, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t a = 0; a < nc; ++a) {
    const Cell &A = tr.cells[a];
    if (A.n_child != 0) continue;
    for (int64_t i = A.body_begin; i < A.body_begin + A.n_body; ++i) {
      const double xi[3] = {tr.xs[i], tr.ys[i], tr.zs[i]};
      l2p(T, A.X, &L[a * nt], xi, &fphi[i], &fg[3 * i]);
      for (int64_t e = ls.m2p_ptr[a]; e < ls.m2p_ptr[a + 1]; ++e) {
        const int b = ls.m2p_col[e];
        m2p(T, tr.cells[b].X, &M[b * nt], xi, &fphi[i], &fg[3 * i]);
      }
    }
  }
  clock.lap(3);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t a = 0; a < nc; ++a) {
    const Cell &A = tr.cells[a];
    if (A.n_child != 0) continue;
    for (int64_t i = A.body_begin; i < A.body_begin + A.n_body; ++i) {
      const double xi[3] = {tr.xs[i], tr.ys[i], tr.zs[i]};
      for (int64_t e = ls.p2p_ptr[a]; e < ls.p2p_ptr[a + 1]; ++e) {
        const Cell &B = tr.cells[ls.p2p_col[e]];
        int64_t b = B.body_begin;
        p2p_point(xi, &tr.xs[b], &tr.ys[b], &tr.zs[b], &qs[b], B.n_body, &nphi[i], &ng[3 * i]);
      }
    }
  }
  clock.lap(4);

  for (int64_t i = 0; i < n; ++i) {
    int64_t u = tr.perm[i];
    phi[u] = nphi[i] + fphi[i];
    for (int d = 0; d < 3; ++d) grad[3 * u + d] = ng[3 * i + d] + fg[3 * i + d];
  }
  if (near_phi) std::copy(nphi.begin(), nphi.end(), near_phi);
  if (near_grad) std::copy(ng.begin(), ng.end(), near_grad);
  if (far_phi) std::copy(fphi.begin(), fphi.end(), far_phi);
  if (far_grad) std::copy(fg.begin(), fg.end(), far_grad);
  if (M_out) std::copy(M.begin(), M.end(), M_out);
  if (L_out) std::copy(L.begin(), L.end(), L_out);
  return 0;
}

// O(N) per target direct sum over all n sources (pairs at zero distance are
// skipped), for m target indices.  The plain definition the FMM approximates.
void oracle_direct(const double *xyz, const double *q, int64_t n, const int64_t *targets,
                   int64_t m, double *phi, double *grad) {
  std::vector<double> x(n), y(n), z(n);
  for (int64_t j = 0; j < n; ++j) {
    x[j] = xyz[3 * j];
    y[j] = xyz[3 * j + 1];
    z[j] = xyz[3 * j + 2];
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < m; ++t) {
    const int64_t i = targets[t];
    const double xi[3] = {x[i], y[i], z[i]};
    double f = 0.0, g[3] = {0.0, 0.0, 0.0};
    p2p_point(xi, x.data(), y.data(), z.data(), q, n, &f, g);
    phi[t] = f;
    for (int d = 0; d < 3; ++d) grad[3 * t + d] = g[d];
  }
}

// Single operators, for the tests that pin the expansions.
void oracle_op_derivatives(int p, const double *R, double *D) {
  Terms T(p);
  derivatives(T, R, D);
}
void oracle_op_p2m(int p, const double *X, const double *xyz, const double *q, int64_t nb,
                   double *M) {
  Terms T(p);
  std::vector<double> x(nb), y(nb), z(nb);
  for (int64_t j = 0; j < nb; ++j) {
    x[j] = xyz[3 * j];
    y[j] = xyz[3 * j + 1];
    z[j] = xyz[3 * j + 2];
  }
  p2m(T, X, x.data(), y.data(), z.data(), q, nb, M);
}
void oracle_op_m2m(int p, const double *XP, const double *Xc, const double *Mc, double *MP) {
  Terms T(p);
  m2m(T, XP, Xc, Mc, MP);
}
void oracle_op_m2l(int p, const double *XA, const double *XB, const double *M, double *L) {
  Terms T(p);
  m2l(T, XA, XB, M, L);
}
void oracle_op_m2p(int p, const double *XB, const double *M, const double *y, int64_t m,
                   double *phi, double *grad) {
  Terms T(p);
  for (int64_t i = 0; i < m; ++i) {
    phi[i] = 0.0;
    grad[3 * i] = grad[3 * i + 1] = grad[3 * i + 2] = 0.0;
    m2p(T, XB, M, &y[3 * i], &phi[i], &grad[3 * i]);
  }
}

void oracle_op_l2l(int p, const double *XP, const double *Xc, const double *LP, double *Lc) {
  Terms T(p);
  l2l(T, XP, Xc, LP, Lc);
}
void oracle_op_l2p(int p, const double *XA, const double *L, const double *y, int64_t m,
                   double *phi, double *grad) {
  Terms T(p);
  for (int64_t i = 0; i < m; ++i) {
    phi[i] = 0.0;
    grad[3 * i] = grad[3 * i + 1] = grad[3 * i + 2] = 0.0;
    l2p(T, XA, L, &y[3 * i], &phi[i], &grad[3 * i]);
  }
}

// The same evaluation restricted to the bodies of the given leaves, for
// checks at sizes where the full evaluation is too slow: the upward pass over
// the whole tree, then for each leaf the M2L rows and L2L translations along
// its chain of ancestors, L2P, and its P2P row, in the same order as
// oracle_evaluate (so the results are identical).  Outputs, for the bodies of
// the leaves in the given order (sorted order within a leaf): user index,
// phi, grad[3].  Returns the number of bodies written, or -1.
int64_t oracle_evaluate_leaves(const oracle_fmm *o, int p, const double *q, const int32_t *leaves,
                               int64_t n_leaves, int64_t *user_index, double *phi,
                               double *grad) {
  if (!o->lists.m2p_col.empty()) return -2;  // hybrid lists: oracle_evaluate only
  if (p < 1 || p > 16) return -1;
  const Tree &tr = o->tree;
  const Lists &ls = o->lists;
  const int64_t n = tr.n;
  Terms T(p);
  const int nt = T.count();
  std::vector<double> qs(n);
  for (int64_t i = 0; i < n; ++i) qs[i] = q[tr.perm[i]];
  std::vector<double> M;
  upward_pass(tr, T, qs, M);
  std::vector<int64_t> offset(n_leaves + 1, 0);
  for (int64_t k = 0; k < n_leaves; ++k) {
    const Cell &A = tr.cells[leaves[k]];
    if (A.n_child != 0) return -1;
    offset[k + 1] = offset[k] + A.n_body;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < n_leaves; ++k) {
    const int a = leaves[k];
    std::vector<int> chain;
    for (int c = a; c >= 0; c = tr.cells[c].parent) chain.push_back(c);
    std::vector<double> Lp, Lc(nt, 0.0);
    for (int idx = (int)chain.size() - 1; idx >= 0; --idx) {
      const int c = chain[idx];
      std::fill(Lc.begin(), Lc.end(), 0.0);
      for (int64_t e = ls.m2l_ptr[c]; e < ls.m2l_ptr[c + 1]; ++e) {
        const int b = ls.m2l_col[e];
        m2l(T, tr.cells[c].X, tr.cells[b].X, &M[b * nt], Lc.data());
      }
      if (!Lp.empty()) l2l(T, tr.cells[tr.cells[c].parent].X, tr.cells[c].X, Lp.data(), Lc.data());
      Lp = Lc;
    }
    const Cell &A = tr.cells[a];
    for (int64_t i = A.body_begin; i < A.body_begin + A.n_body; ++i) {
      const double xi[3] = {tr.xs[i], tr.ys[i], tr.zs[i]};
      double fphi = 0.0, fg[3] = {0.0, 0.0, 0.0}, nphi = 0.0, ng[3] = {0.0, 0.0, 0.0};
      l2p(T, A.X, Lp.data(), xi, &fphi, fg);
      for (int64_t e = ls.p2p_ptr[a]; e < ls.p2p_ptr[a + 1]; ++e) {
        const Cell &B = tr.cells[ls.p2p_col[e]];
        int64_t b = B.body_begin;
        p2p_point(xi, &tr.xs[b], &tr.ys[b], &tr.zs[b], &qs[b], B.n_body, &nphi, ng);
      }
      const int64_t out = offset[k] + (i - A.body_begin);
      user_index[out] = tr.perm[i];
      phi[out] = nphi + fphi;
      for (int d = 0; d < 3; ++d) grad[3 * out + d] = ng[d] + fg[d];
    }
  }
  return offset[n_leaves];
}

// Replace the positions (user order) keeping the tree structure, centres,
// radii and lists: the method with its tree frozen, for finite differences.
void oracle_set_positions(oracle_fmm *o, const double *xyz) {
  Tree &t = o->tree;
  for (int64_t i = 0; i < t.n; ++i) {
    t.xs[i] = xyz[3 * (int64_t)t.perm[i] + 0];
    t.ys[i] = xyz[3 * (int64_t)t.perm[i] + 1];
    t.zs[i] = xyz[3 * (int64_t)t.perm[i] + 2];
  }
}

// Evaluation with sources that carry charges q and optionally dipoles s
// ([n][3]), and optionally, at every body i, the Hessian of the charge field
// applied to v_i ([n][3]; needs s == NULL).  Outputs in user order; any may be
// NULL.  The far field uses the same expansions: dipoles enter through P2M,
// the Hessian through second derivatives of the local expansion.
int oracle_evaluate_general(const oracle_fmm *o, int p, const double *q, const double *s,
                            const double *v, double *phi, double *grad, double *hv) {
  if (!o->lists.m2p_col.empty()) return -2;  // hybrid lists: oracle_evaluate only
  if (p < 1 || p > 16 || (s && v)) return -1;
  const Tree &tr = o->tree;
  const Lists &ls = o->lists;
  const int64_t n = tr.n;
  const int64_t nc = (int64_t)tr.cells.size();
  if (n == 0) return 0;
  Terms T(p);
  const int nt = T.count();
  std::vector<double> qs(n), ss(s ? 3 * n : 0), vs(v ? 3 * n : 0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t u = tr.perm[i];
    qs[i] = q[u];
    for (int a = 0; a < 3; ++a) {
      if (s) ss[3 * i + a] = s[3 * u + a];
      if (v) vs[3 * i + a] = v[3 * u + a];
    }
  }
  std::vector<double> M;
  upward_pass(tr, T, qs, M);
  if (s) {
    // dipole moments of the leaves, then shifted upwards like the charges
    std::vector<double> Md(nc * nt, 0.0);
    int max_level = 0;
    for (const auto &c : tr.cells) max_level = std::max(max_level, c.level);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < nc; ++c) {
      const Cell &C = tr.cells[c];
      if (C.n_child != 0) continue;
      int64_t b = C.body_begin;
      p2m_dipole(T, C.X, &tr.xs[b], &tr.ys[b], &tr.zs[b], &ss[3 * b], C.n_body, &Md[c * nt]);
    }
    for (int lev = max_level - 1; lev >= 0; --lev) {
#pragma omp parallel for schedule(dynamic, 16)
      for (int64_t c = 0; c < nc; ++c) {
        const Cell &C = tr.cells[c];
        if (C.level != lev || C.n_child == 0) continue;
        for (int k = 0; k < C.n_child; ++k) {
          int ch = C.child_begin + k;
          m2m(T, C.X, tr.cells[ch].X, &Md[ch * nt], &Md[c * nt]);
        }
      }
    }
    for (int64_t k = 0; k < nc * nt; ++k) M[k] += Md[k];
  }
  std::vector<double> L(nc * nt, 0.0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < nc; ++a)
    for (int64_t e = ls.m2l_ptr[a]; e < ls.m2l_ptr[a + 1]; ++e) {
      int b = ls.m2l_col[e];
      m2l(T, tr.cells[a].X, tr.cells[b].X, &M[b * nt], &L[a * nt]);
    }
  int max_level = 0;
  for (const auto &c : tr.cells) max_level = std::max(max_level, c.level);
  for (int lev = 1; lev <= max_level; ++lev) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < nc; ++c) {
      const Cell &C = tr.cells[c];
      if (C.level != lev) continue;
      l2l(T, tr.cells[C.parent].X, C.X, &L[C.parent * nt], &L[c * nt]);
    }
  }
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t a = 0; a < nc; ++a) {
    const Cell &A = tr.cells[a];
    if (A.n_child != 0) continue;
    for (int64_t i = A.body_begin; i < A.body_begin + A.n_body; ++i) {
      const double xi[3] = {tr.xs[i], tr.ys[i], tr.zs[i]};
      const double *vi = v ? &vs[3 * i] : nullptr;
      double f = 0.0, g[3] = {0, 0, 0}, h[3] = {0, 0, 0};
      l2p(T, A.X, &L[a * nt], xi, &f, g);
      if (vi) l2p_hessian(T, A.X, &L[a * nt], xi, vi, h);
      double nf = 0.0, ng[3] = {0, 0, 0}, nh[3] = {0, 0, 0};
      for (int64_t e = ls.p2p_ptr[a]; e < ls.p2p_ptr[a + 1]; ++e) {
        const Cell &B = tr.cells[ls.p2p_col[e]];
        int64_t b = B.body_begin;
        p2p_general_point(xi, &tr.xs[b], &tr.ys[b], &tr.zs[b], &qs[b], s ? &ss[3 * b] : nullptr,
                          B.n_body, vi, &nf, ng, nh);
      }
      const int64_t u = tr.perm[i];
      if (phi) phi[u] = nf + f;
      for (int d = 0; d < 3; ++d) {
        if (grad) grad[3 * u + d] = ng[d] + g[d];
        if (hv) hv[3 * u + d] = nh[d] + h[d];
      }
    }
  }
  return 0;
}

// Direct sum with charges q and optional dipoles s at the given targets, and
// optionally the Hessian of the charge field applied to v[target].
void oracle_direct_general(const double *xyz, const double *q, const double *s, int64_t n,
                           const int64_t *targets, int64_t m, const double *v, double *phi,
                           double *grad, double *hv) {
  std::vector<double> x(n), y(n), z(n);
  for (int64_t j = 0; j < n; ++j) {
    x[j] = xyz[3 * j];
    y[j] = xyz[3 * j + 1];
    z[j] = xyz[3 * j + 2];
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < m; ++t) {
    const int64_t i = targets[t];
    const double xi[3] = {x[i], y[i], z[i]};
    double f = 0.0, g[3] = {0, 0, 0}, h[3] = {0, 0, 0};
    p2p_general_point(xi, x.data(), y.data(), z.data(), q, s, n, v ? &v[3 * t] : nullptr, &f,
                      g, h);
    phi[t] = f;
    for (int d = 0; d < 3; ++d) {
      grad[3 * t + d] = g[d];
      if (hv) hv[3 * t + d] = h[d];
    }
  }
}

void oracle_op_p2m_dipole(int p, const double *X, const double *xyz, const double *s, int64_t nb,
                          double *M) {
  Terms T(p);
  std::vector<double> x(nb), y(nb), z(nb);
  for (int64_t j = 0; j < nb; ++j) {
    x[j] = xyz[3 * j];
    y[j] = xyz[3 * j + 1];
    z[j] = xyz[3 * j + 2];
  }
  for (int t = 0; t < T.count(); ++t) M[t] = 0.0;
  p2m_dipole(T, X, x.data(), y.data(), z.data(), s, nb, M);
}

void oracle_op_l2p_hessian(int p, const double *XA, const double *L, const double *y,
                           const double *v, int64_t m, double *hv) {
  Terms T(p);
  for (int64_t i = 0; i < m; ++i) {
    hv[3 * i] = hv[3 * i + 1] = hv[3 * i + 2] = 0.0;
    l2p_hessian(T, XA, L, &y[3 * i], &v[3 * i], &hv[3 * i]);
  }
}

}  // extern "C"
