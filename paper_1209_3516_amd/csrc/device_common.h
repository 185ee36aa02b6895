// Shared device-side machinery of the gfx950 kernels: compile-time
// multi-index tables, unrolling helpers, vector types and launch helpers.
// Included by the kernel translation units only.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "kernels.h"

namespace fmmlib {
namespace dev {
namespace {

// ----------------------------------------------------------------------------
// Multi-indices of total degree < P, ordered by degree, then by the z
// exponent, then by the y exponent.
// ----------------------------------------------------------------------------
constexpr int nterms(int p) { return p * (p + 1) * (p + 2) / 6; }
constexpr int pad4(int t) { return (t + 3) & ~3; }

constexpr int term_index(int p, int a, int b, int c) {
  if (a < 0 || b < 0 || c < 0) return -1;
  const int d = a + b + c;
  if (d > p - 1) return -1;
  return d * (d + 1) * (d + 2) / 6 + c * (d + 1) - c * (c - 1) / 2 + b;
}

template <int P>
struct Basis {
  static constexpr int T = nterms(P);
  int ex[T], ey[T], ez[T];
  int lo[T][3];   // term of m - e_d, or -1
  int lo2[T][3];  // term of m - 2 e_d, or -1
  int axis[T];    // an axis with m_axis > 0 (first one), -1 for m = 0
  int par[T];     // term of m - e_axis
  double fact[T];   // m!
  double inv_e[T];  // 1 / m_axis
  constexpr Basis() : ex(), ey(), ez(), lo(), lo2(), axis(), par(), fact(), inv_e() {
    for (int d = 0; d < P; ++d)
      for (int c = 0; c <= d; ++c)
        for (int b = 0; b <= d - c; ++b) {
          const int t = term_index(P, d - b - c, b, c);
          ex[t] = d - b - c;
          ey[t] = b;
          ez[t] = c;
        }
    for (int t = 0; t < T; ++t) {
      const int m[3] = {ex[t], ey[t], ez[t]};
      for (int k = 0; k < 3; ++k) {
        int m1[3] = {m[0], m[1], m[2]};
        m1[k] -= 1;
        lo[t][k] = term_index(P, m1[0], m1[1], m1[2]);
        int m2[3] = {m[0], m[1], m[2]};
        m2[k] -= 2;
        lo2[t][k] = term_index(P, m2[0], m2[1], m2[2]);
      }
      double f = 1.0;
      for (int k = 0; k < 3; ++k)
        for (int i = 2; i <= m[k]; ++i) f *= i;
      fact[t] = f;
      axis[t] = -1;
      par[t] = -1;
      inv_e[t] = 0.0;
      for (int k = 0; k < 3; ++k)
        if (m[k] > 0) {
          axis[t] = k;
          par[t] = lo[t][k];
          inv_e[t] = 1.0 / m[k];
          break;
        }
    }
  }
};
template <int P>
inline constexpr Basis<P> kBasis{};

// ----------------------------------------------------------------------------
// Harmonic reduction of M2L.  G = 1/r is harmonic, so its derivatives obey
// D^{m+2e_x} + D^{m+2e_y} + D^{m+2e_z} = 0; applied j times,
//   D^{(a, b, c+2j)} = (-1)^j sum_{i=0..j} C(j,i) D^{(a+2i, b+2(j-i), c)}.
// In L_k = sum_{|n| <= p-1-|k|} M_n D^{n+k} this gives two exact identities,
// each keeping the degree of the index it rewrites:
//  * source side: the terms with n_z >= 2 fold onto those with n_z <= 1,
//      Mr_(a,b,c) = sum_{j,i} (-1)^j C(j,i) M_(a-2i, b-2(j-i), c+2j),  c <= 1,
//    a multipole of p^2 terms whose M2L is that of M;
//  * target side: L_(a,b,c+2j) = (-1)^j sum_i C(j,i) L_(a+2i, b+2(j-i), c).
// M2L therefore contracts only the p^2 terms of z exponent <= 1 on both
// sides, with derivatives of z exponent <= 2: sum_{a+b <= p-1} (2a+1)(2b+1)
// products per pair (70 / 301 / 876 for p = 4 / 6 / 8, against
// C(p+5, 6) = 84 / 462 / 1716 for the full contraction).
// ----------------------------------------------------------------------------
constexpr int rterms(int p) { return p * p; }

// Reduced terms (z exponent 0 or 1) of degree < p, ordered by degree, then
// by the z exponent, then by the y exponent.
constexpr int rterm_index(int p, int a, int b, int c) {
  if (a < 0 || b < 0 || c < 0 || c > 1) return -1;
  const int d = a + b + c;
  if (d > p - 1) return -1;
  return d * d + c * (d + 1) + b;
}

constexpr int binom(int j, int i) {
  int r = 1;
  for (int t = 1; t <= i; ++t) r = r * (j - i + t) / t;
  return r;
}

// f(t, r, w, first) for every full term t and each reduced term r it pairs
// with in the identities above, with the integer weight w; `first` marks the
// first pair of each t.  Pairs come in ascending t.
template <int P, class F>
__device__ __forceinline__ void harmonic_pairs(F &&f) {
  static_for<nterms(P)>([&](auto I) {
    constexpr int t = decltype(I)::value;
    constexpr int a = kBasis<P>.ex[t], b = kBasis<P>.ey[t], c = kBasis<P>.ez[t];
    constexpr int j = c / 2;
    static_for<j + 1>([&](auto Ii) {
      constexpr int i = decltype(Ii)::value;
      constexpr int r = rterm_index(P, a + 2 * i, b + 2 * (j - i), c % 2);
      constexpr int w = (j % 2 ? -1 : 1) * binom(j, i);
      f(std::integral_constant<int, t>{}, std::integral_constant<int, r>{},
        std::integral_constant<int, w>{}, std::integral_constant<bool, i == 0>{});
    });
  });
}

constexpr int m2l_reduced_count(int p) {
  int c = 0;
  for (int a = 0; a < p; ++a)
    for (int b = 0; a + b < p; ++b) c += (2 * a + 1) * (2 * b + 1);
  return c;
}

// The reduced contraction as (k, n, s): k and n reduced terms, s the full
// term of n + k (z exponent <= 2), for all |n| + |k| <= P-1.  Ordered by
// source term n, so that each group of four consecutive source terms (one
// 16-byte load of a reduced multipole row) is used at once: the entries of
// group g are [gbeg[g], gbeg[g + 1]).  For every target term k the source
// terms come in ascending order.
template <int P>
struct M2LReduced {
  static constexpr int TR = rterms(P);
  static constexpr int N = m2l_reduced_count(P);
  static constexpr int G = (TR + 3) / 4;
  int k[N], n[N], s[N], gbeg[G + 1];
  constexpr M2LReduced() : k(), n(), s(), gbeg() {
    int rx[TR] = {}, ry[TR] = {}, rz[TR] = {};
    for (int d = 0; d < P; ++d)
      for (int c = 0; c <= 1 && c <= d; ++c)
        for (int b = 0; b <= d - c; ++b) {
          const int r = rterm_index(P, d - b - c, b, c);
          rx[r] = d - b - c;
          ry[r] = b;
          rz[r] = c;
        }
    int i = 0;
    for (int g = 0; g < G; ++g) {
      gbeg[g] = i;
      for (int nn = 4 * g; nn < 4 * g + 4 && nn < TR; ++nn)
        for (int kk = 0; kk < TR; ++kk) {
          const int ss = term_index(P, rx[kk] + rx[nn], ry[kk] + ry[nn], rz[kk] + rz[nn]);
          if (ss < 0) continue;
          k[i] = kk;
          n[i] = nn;
          s[i] = ss;
          ++i;
        }
    }
    gbeg[G] = i;
  }
};
template <int P>
inline constexpr M2LReduced<P> kM2LR{};

// (hi, lo, diff): lo <= hi componentwise, diff = term of hi - lo.
constexpr int shift_count(int p) {
  int c = 0;
  for (int d = 0; d < p; ++d)
    for (int z = 0; z <= d; ++z)
      for (int y = 0; y <= d - z; ++y) c += (d - y - z + 1) * (y + 1) * (z + 1);
  return c;
}
template <int P>
struct ShiftTable {
  static constexpr int N = shift_count(P);
  int hi[N], lo[N], diff[N];
  constexpr ShiftTable() : hi(), lo(), diff() {
    constexpr int T = nterms(P);
    Basis<P> B{};
    int i = 0;
    for (int h = 0; h < T; ++h)
      for (int l = 0; l < T; ++l) {
        const int dd = term_index(P, B.ex[h] - B.ex[l], B.ey[h] - B.ey[l], B.ez[h] - B.ez[l]);
        if (dd < 0) continue;
        hi[i] = h;
        lo[i] = l;
        diff[i] = dd;
        ++i;
      }
  }
};
template <int P>
inline constexpr ShiftTable<P> kShift{};

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(static_cast<F &&>(f), std::make_integer_sequence<int, N>{});
}

template <typename Real>
struct Vec;
template <>
struct Vec<float> {
  using V4 = float4;
  static constexpr float kFar = 1.0e18f;
};
template <>
struct Vec<double> {
  using V4 = double4;
  static constexpr double kFar = 1.0e150;
};

__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }

// (d^m / m!) for every term m, built from a lower term times one coordinate.
template <int P, typename Real>
__device__ __forceinline__ void monomials(Real dx, Real dy, Real dz, Real (&mono)[nterms(P)]) {
  mono[0] = Real(1);
  static_for<nterms(P) - 1>([&](auto I) {
    constexpr int t = decltype(I)::value + 1;
    constexpr int ax = kBasis<P>.axis[t];
    constexpr int par = kBasis<P>.par[t];
    const Real d = ax == 0 ? dx : (ax == 1 ? dy : dz);
    mono[t] = mono[par] * (d * Real(kBasis<P>.inv_e[t]));
  });
}

// D^m (1/|R|) for every term m, computed directly (factorials folded into
// compile-time constants).  From the recurrence for a_m = D^m G / m!,
//   D_m = (1/r^2) [ -(2k-1)/k sum_d m_d R_d D_{m-e_d}
//                   -(k-1)/k sum_d m_d (m_d - 1) D_{m-2e_d} ],   k = |m|,
// and, since 1/r is harmonic (sum_d D_{m'+2e_d} = 0), every term with
// m_z >= 2 follows from two terms of the same degree with smaller m_z:
//   D_m = -D_{m-2e_z+2e_x} - D_{m-2e_z+2e_y}.
// With Z2, only the terms of z exponent <= 2 are computed (the others are
// left unset): those are all that the reduced M2L reads.
template <int P, typename Real, bool Z2 = false>
__device__ __forceinline__ void derivatives(Real Rx, Real Ry, Real Rz, Real (&D)[nterms(P)]) {
  constexpr int T = nterms(P);
  const Real r2 = Rx * Rx + Ry * Ry + Rz * Rz;
  const Real inv_r = rsqrt_(r2);
  const Real ir2 = inv_r * inv_r;
  const Real X = Rx * ir2, Y = Ry * ir2, Z = Rz * ir2;
  D[0] = inv_r;
  static_for<T - 1>([&](auto I) {
    constexpr int t = decltype(I)::value + 1;
    constexpr auto &B = kBasis<P>;
    constexpr int mx = B.ex[t], my = B.ey[t], mz = B.ez[t];
    constexpr int k = mx + my + mz;
    if constexpr (Z2 && mz > 2) {
    } else if constexpr (mz >= 2) {
      constexpr int ia = term_index(P, mx + 2, my, mz - 2);
      constexpr int ib = term_index(P, mx, my + 2, mz - 2);
      D[t] = -D[ia] - D[ib];
    } else {
      constexpr double c1 = -(2.0 * k - 1.0) / k;
      Real s1 = Real(0);
      if constexpr (mx >= 1) s1 += Real(c1 * mx) * (X * D[B.lo[t][0]]);
      if constexpr (my >= 1) s1 += Real(c1 * my) * (Y * D[B.lo[t][1]]);
      if constexpr (mz >= 1) s1 += Real(c1 * mz) * (Z * D[B.lo[t][2]]);
      if constexpr (mx >= 2 || my >= 2) {
        constexpr double c2 = -(k - 1.0) / k;
        Real s2 = Real(0);
        if constexpr (mx >= 2) s2 += Real(c2 * mx * (mx - 1)) * D[B.lo2[t][0]];
        if constexpr (my >= 2) s2 += Real(c2 * my * (my - 1)) * D[B.lo2[t][1]];
        D[t] = s1 + ir2 * s2;
      } else {
        D[t] = s1;
      }
    }
  });
}

template <int N, typename Real>
__device__ __forceinline__ void load_row(const Real *__restrict__ src, Real (&dst)[N]) {
  const Real *p = static_cast<const Real *>(__builtin_assume_aligned(src, 16));
  static_for<N>([&](auto I) { dst[decltype(I)::value] = p[decltype(I)::value]; });
}

// Four consecutive values from a 16-byte aligned address.
__device__ __forceinline__ void load4(const float *__restrict__ src, float (&dst)[4]) {
  const float4 v = *static_cast<const float4 *>(__builtin_assume_aligned(src, 16));
  dst[0] = v.x;
  dst[1] = v.y;
  dst[2] = v.z;
  dst[3] = v.w;
}
__device__ __forceinline__ void load4(const double *__restrict__ src, double (&dst)[4]) {
  const double2 *p = static_cast<const double2 *>(__builtin_assume_aligned(src, 16));
  const double2 a = p[0], b = p[1];
  dst[0] = a.x;
  dst[1] = a.y;
  dst[2] = b.x;
  dst[3] = b.y;
}

// Work-group b of G is placed on XCD b % 8; give each XCD a contiguous range
// of the (Morton-ordered) work so that neighbouring work shares that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
  const int64_t x = b & 7, j = b >> 3, full = G >> 3, rem = G & 7;
  return x * full + (x < rem ? x : rem) + j;
}

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }
inline hipStream_t S_(void *s) { return reinterpret_cast<hipStream_t>(s); }


// Run f(std::integral_constant<int, p>) for the runtime order p.
template <class F>
inline int with_p(int p, F &&f) {
  switch (p) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

}  // namespace
}  // namespace dev
}  // namespace fmmlib
