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

// (k, n, s): s = term of n + k, for all |n| + |k| <= P-1.  C(P+5, 6) entries.
constexpr int m2l_count(int p) {
  long r = 1;
  for (int i = 1; i <= 6; ++i) r = r * (p - 1 + i) / i;
  return (int)r;
}
template <int P>
struct M2LTable {
  static constexpr int N = m2l_count(P);
  int k[N], n[N], s[N];
  constexpr M2LTable() : k(), n(), s() {
    constexpr int T = nterms(P);
    Basis<P> B{};
    int i = 0;
    for (int kk = 0; kk < T; ++kk)
      for (int nn = 0; nn < T; ++nn) {
        const int ss = term_index(P, B.ex[kk] + B.ex[nn], B.ey[kk] + B.ey[nn], B.ez[kk] + B.ez[nn]);
        if (ss < 0) continue;
        k[i] = kk;
        n[i] = nn;
        s[i] = ss;
        ++i;
      }
  }
};
template <int P>
inline constexpr M2LTable<P> kM2L{};

// The same contraction ordered by source term n, so that each group of four
// consecutive source terms (one 16-byte load of a multipole row) is used at
// once: the entries of group g are [gbeg[g], gbeg[g + 1]).  For every target
// term k the source terms still come in ascending order, as in M2LTable.
template <int P>
struct M2LTableBySource {
  static constexpr int N = m2l_count(P);
  static constexpr int G = (nterms(P) + 3) / 4;
  int k[N], n[N], s[N], gbeg[G + 1];
  constexpr M2LTableBySource() : k(), n(), s(), gbeg() {
    constexpr int T = nterms(P);
    Basis<P> B{};
    int i = 0;
    for (int g = 0; g < G; ++g) {
      gbeg[g] = i;
      for (int nn = 4 * g; nn < 4 * g + 4 && nn < T; ++nn)
        for (int kk = 0; kk < T; ++kk) {
          const int ss =
              term_index(P, B.ex[kk] + B.ex[nn], B.ey[kk] + B.ey[nn], B.ez[kk] + B.ez[nn]);
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
inline constexpr M2LTableBySource<P> kM2LS{};

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
template <int P, typename Real>
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
    if constexpr (mz >= 2) {
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
