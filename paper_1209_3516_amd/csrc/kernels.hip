// gfx950 kernels of the dual-tree-traversal Laplace FMM.
//
// Expansions are Cartesian Taylor (section 3.1, Table 2) of total degree
// 0..p-1.  Multipoles about a cell centre X_B, locals about X_A:
//   P2M  M_n(B)  = sum_j q_j (X_B - x_j)^n / n!
//   M2M  M_n(P) += sum_{m <= n} M_m(c) (X_P - X_c)^(n-m) / (n-m)!
//   M2L  L_k(A) += sum_{|n|+|k| <= p-1} M_n(B) D^(n+k) G(X_A - X_B),   G = 1/|r|
//   L2L  L_k(c) += sum_{m >= k} L_m(P) (X_c - X_P)^(m-k) / (m-k)!
//   L2P  phi(y)  = sum_k L_k (y - X_A)^k / k!, gradient by differentiating in y
//   P2P  phi_i  += q_j / r,  grad_i += q_j (x_j - x_i) / r^3   (r > 0)
// The derivatives D^m G come from the recurrence for a_m = D^m G / m!:
//   |m| r^2 a_m = -(2|m|-1) sum_d R_d a_{m-e_d} - (|m|-1) sum_d a_{m-2e_d}.
// Translations are computed on the fly per pair rather than loaded as
// precomputed matrices (section 3.1: bytes per flop keep falling).
//
// All index arithmetic over multi-indices is resolved at compile time: the
// kernels are templated on p and every loop over coefficients is unrolled
// through constexpr tables, so coefficients live in registers.
//
// No floating-point atomics anywhere: each output value is produced by one
// thread or one wave in a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cstdint>
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

// D^m (1/|R|) for every term m.
template <int P, typename Real>
__device__ __forceinline__ void derivatives(Real Rx, Real Ry, Real Rz, Real (&D)[nterms(P)]) {
  constexpr int T = nterms(P);
  const Real r2 = Rx * Rx + Ry * Ry + Rz * Rz;
  const Real inv_r = rsqrt_(r2);
  const Real inv_r2 = inv_r * inv_r;
  Real a[T];
  a[0] = inv_r;
  static_for<T - 1>([&](auto I) {
    constexpr int t = decltype(I)::value + 1;
    constexpr auto &B = kBasis<P>;
    constexpr int k = B.ex[t] + B.ey[t] + B.ez[t];
    Real s1 = Real(0);
    if constexpr (B.lo[t][0] >= 0) s1 += Rx * a[B.lo[t][0]];
    if constexpr (B.lo[t][1] >= 0) s1 += Ry * a[B.lo[t][1]];
    if constexpr (B.lo[t][2] >= 0) s1 += Rz * a[B.lo[t][2]];
    constexpr Real c1 = Real(-(2.0 * k - 1.0) / k);
    if constexpr (k >= 2) {
      Real s2 = Real(0);
      if constexpr (B.lo2[t][0] >= 0) s2 += a[B.lo2[t][0]];
      if constexpr (B.lo2[t][1] >= 0) s2 += a[B.lo2[t][1]];
      if constexpr (B.lo2[t][2] >= 0) s2 += a[B.lo2[t][2]];
      constexpr Real c2 = Real(-(k - 1.0) / k);
      a[t] = inv_r2 * (c1 * s1 + c2 * s2);
    } else {
      a[t] = inv_r2 * (c1 * s1);
    }
  });
  static_for<T>([&](auto I) {
    constexpr int t = decltype(I)::value;
    D[t] = a[t] * Real(kBasis<P>.fact[t]);
  });
}

template <int N, typename Real>
__device__ __forceinline__ void load_row(const Real *__restrict__ src, Real (&dst)[N]) {
  const Real *p = static_cast<const Real *>(__builtin_assume_aligned(src, 16));
  static_for<N>([&](auto I) { dst[decltype(I)::value] = p[decltype(I)::value]; });
}

// Work-group b of G is placed on XCD b % 8; give each XCD a contiguous range
// of the (Morton-ordered) work so that neighbouring work shares that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
  const int64_t x = b & 7, j = b >> 3, full = G >> 3, rem = G & 7;
  return x * full + (x < rem ? x : rem) + j;
}

// ----------------------------------------------------------------------------
// Charges into Morton order: bodies[i].w = q[perm[i]].
// ----------------------------------------------------------------------------
template <typename Real>
__global__ void gather_kernel(int64_t n, const int32_t *__restrict__ perm,
                              const Real *__restrict__ q, typename Vec<Real>::V4 *bodies) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) bodies[i].w = q[perm[i]];
}

// ----------------------------------------------------------------------------
// P2P.  One 64-lane wave per work item (<= 64 targets of one leaf x one chunk
// of its source leaves).  Sources are staged through LDS in batches of kNB
// bodies with coalesced 16-byte loads; lane (s, u) keeps R targets in
// registers and reads every K-th staged source (a broadcast among the lanes
// of one stream).  Within a batch each lane sums in plain arithmetic; the
// batch partial is then added with Kahan compensation (FP32), and the K
// streams and the chunks of a row are merged with the same compensation.
// ----------------------------------------------------------------------------
constexpr int kNB = 512;
static_assert(kP2PMaxRuns == 256, "LDS run table size");

template <typename Real, int R, bool KAHAN, bool MASK, typename IndexFn>
__device__ __forceinline__ void p2p_phase(int nsrc, IndexFn body_of,
                                          const typename Vec<Real>::V4 *__restrict__ bodies,
                                          typename Vec<Real>::V4 *src, int s, int K,
                                          const Real (&xi)[R], const Real (&yi)[R],
                                          const Real (&zi)[R], Real (&S)[R][4], Real (&C)[R][4]) {
  using V4 = typename Vec<Real>::V4;
  const int lane = threadIdx.x;
  const Real far = Vec<Real>::kFar;
  for (int off = 0; off < nsrc; off += kNB) {
    const int nb = min(kNB, nsrc - off);
#pragma unroll
    for (int q = 0; q <= kNB / 64; ++q) {
      const int pos = q * 64 + lane;
      V4 v;
      if (pos < nb) {
        v = bodies[body_of(off + pos)];
      } else {
        v.x = far;
        v.y = far;
        v.z = far;
        v.w = Real(0);
      }
      src[pos] = v;
    }
    __syncthreads();
    const int iters = (nb + K - 1) / K;
    Real p[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) p[r][0] = p[r][1] = p[r][2] = p[r][3] = Real(0);
#pragma unroll 2
    for (int j = 0; j < iters; ++j) {
      const V4 sj = src[s + K * j];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const Real dx = sj.x - xi[r], dy = sj.y - yi[r], dz = sj.z - zi[r];
        const Real r2 = dx * dx + dy * dy + dz * dz;
        Real inv = rsqrt_(r2);
        if constexpr (MASK) inv = r2 > Real(0) ? inv : Real(0);
        const Real qr = sj.w * inv;
        const Real qr3 = qr * (inv * inv);
        p[r][0] += qr;
        p[r][1] += qr3 * dx;
        p[r][2] += qr3 * dy;
        p[r][3] += qr3 * dz;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if constexpr (KAHAN) {
          const Real y = p[r][c] - C[r][c];
          const Real t = S[r][c] + y;
          C[r][c] = (t - S[r][c]) - y;
          S[r][c] = t;
        } else {
          S[r][c] += p[r][c];
        }
      }
    __syncthreads();
  }
}

template <typename Real, int R, bool KAHAN, bool MASK_ALL>
__device__ __forceinline__ void p2p_item(const P2PItem &it, const int32_t *__restrict__ run_body,
                                         const int32_t *__restrict__ run_prefix,
                                         const typename Vec<Real>::V4 *__restrict__ bodies,
                                         typename Vec<Real>::V4 *__restrict__ out_s,
                                         typename Vec<Real>::V4 *__restrict__ out_c,
                                         typename Vec<Real>::V4 *src, int32_t *rb, int32_t *rp) {
  using V4 = typename Vec<Real>::V4;
  const int lane = threadIdx.x;
  const int nt = it.tgt_cfg & 0xff;
  const int L = (it.tgt_cfg >> 16) & 0xff;
  const int K = (it.tgt_cfg >> 24) & 0xff;
  int s = lane / L;
  const int u = lane - s * L;
  if (s >= K) s = K - 1;  // spare lanes repeat the last stream; not merged

  Real xi[R], yi[R], zi[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = u + L * r;
    if (t < nt) {
      const V4 b = bodies[it.tgt_begin + t];
      xi[r] = b.x;
      yi[r] = b.y;
      zi[r] = b.z;
    } else {
      xi[r] = yi[r] = zi[r] = -Vec<Real>::kFar;
    }
  }
  Real S[R][4], C[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) S[r][c] = C[r][c] = Real(0);

  if (it.self_n > 0) {
    const int b0 = it.self_begin;
    p2p_phase<Real, R, KAHAN, true>(
        it.self_n, [&](int c) { return b0 + c; }, bodies, src, s, K, xi, yi, zi, S, C);
  }
  if (it.n_src > 0) {
    for (int r = lane; r < it.n_runs; r += 64) {
      rb[r] = run_body[it.run_begin + r];
      rp[r] = run_prefix[it.run_begin + r];
    }
    if (lane == 0) rp[it.n_runs] = it.n_src;
    __syncthreads();
    int ri = 0;
    p2p_phase<Real, R, KAHAN, MASK_ALL>(
        it.n_src,
        [&](int c) {
          while (rp[ri + 1] <= c) ++ri;
          return rb[ri] + (c - rp[ri]);
        },
        bodies, src, s, K, xi, yi, zi, S, C);
  }

  // Merge the K streams (lanes s*L + u) into the lanes of stream 0.
  V4 *red = src;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    red[2 * lane] = V4{S[r][0], S[r][1], S[r][2], S[r][3]};
    red[2 * lane + 1] = V4{C[r][0], C[r][1], C[r][2], C[r][3]};
    __syncthreads();
    if (lane < L) {
      Real s4[4] = {S[r][0], S[r][1], S[r][2], S[r][3]};
      Real c4[4] = {C[r][0], C[r][1], C[r][2], C[r][3]};
      for (int s2 = 1; s2 < K; ++s2) {
        const V4 ps = red[2 * (s2 * L + lane)];
        const V4 pc = red[2 * (s2 * L + lane) + 1];
        const Real vs[4] = {ps.x, ps.y, ps.z, ps.w};
        const Real vc[4] = {pc.x, pc.y, pc.z, pc.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if constexpr (KAHAN) {
            const Real y = (vs[c] - vc[c]) - c4[c];
            const Real t = s4[c] + y;
            c4[c] = (t - s4[c]) - y;
            s4[c] = t;
          } else {
            s4[c] += vs[c];
          }
        }
      }
      const int t = lane + L * r;
      if (t < nt) {
        out_s[it.out_off + t] = V4{s4[0], s4[1], s4[2], s4[3]};
        if constexpr (KAHAN) out_c[it.out_off + t] = V4{c4[0], c4[1], c4[2], c4[3]};
      }
    }
    __syncthreads();
  }
}

template <typename Real, bool KAHAN, bool MASK_ALL>
__global__ __launch_bounds__(64) void p2p_kernel(const P2PItem *__restrict__ items,
                                                 const int32_t *__restrict__ run_body,
                                                 const int32_t *__restrict__ run_prefix,
                                                 const typename Vec<Real>::V4 *__restrict__ bodies,
                                                 typename Vec<Real>::V4 *__restrict__ out_s,
                                                 typename Vec<Real>::V4 *__restrict__ out_c) {
  using V4 = typename Vec<Real>::V4;
  __shared__ V4 src[kNB + 64];
  __shared__ int32_t rb[kP2PMaxRuns];
  __shared__ int32_t rp[kP2PMaxRuns + 1];
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  const P2PItem it = items[w];
  switch ((it.tgt_cfg >> 8) & 0xff) {
#define FMM_P2P_CASE(RR)                                                                          \
  case RR:                                                                                        \
    p2p_item<Real, RR, KAHAN, MASK_ALL>(it, run_body, run_prefix, bodies, out_s, out_c, src, rb, \
                                        rp);                                                      \
    break;
    FMM_P2P_CASE(1)
    FMM_P2P_CASE(2)
    FMM_P2P_CASE(3)
    FMM_P2P_CASE(4)
    FMM_P2P_CASE(5)
    FMM_P2P_CASE(6)
    FMM_P2P_CASE(7)
    FMM_P2P_CASE(8)
#undef FMM_P2P_CASE
    default:
      break;
  }
}

// ----------------------------------------------------------------------------
// P2M: one thread per leaf.
// ----------------------------------------------------------------------------
template <int P, typename Real>
__global__ __launch_bounds__(64) void p2m_kernel(int64_t n_leaves, const int32_t *__restrict__ leaf_cell,
                           const int32_t *__restrict__ body_begin,
                           const int32_t *__restrict__ n_body, const double4 *__restrict__ geo,
                           const typename Vec<Real>::V4 *__restrict__ bodies, Real *__restrict__ M,
                           double *__restrict__ M64, int64_t n_top) {
  constexpr int T = nterms(P), S = pad4(T);
  const int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (li >= n_leaves) return;
  const int c = leaf_cell[li];
  const double4 g = geo[c];
  Real acc[T];
  static_for<T>([&](auto I) { acc[decltype(I)::value] = Real(0); });
  const int b0 = body_begin[c], nb = n_body[c];
  for (int j = 0; j < nb; ++j) {
    const typename Vec<Real>::V4 b = bodies[b0 + j];
    Real mono[T];
    monomials<P, Real>(Real(g.x - (double)b.x), Real(g.y - (double)b.y), Real(g.z - (double)b.z),
                       mono);
    static_for<T>([&](auto I) { acc[decltype(I)::value] += b.w * mono[decltype(I)::value]; });
  }
  static_for<T>([&](auto I) { M[(int64_t)c * S + decltype(I)::value] = acc[decltype(I)::value]; });
  if (c < n_top)
    static_for<T>(
        [&](auto I) { M64[(int64_t)c * S + decltype(I)::value] = (double)acc[decltype(I)::value]; });
}

// ----------------------------------------------------------------------------
// M2M: one thread per parent cell of one level; the parent gathers from its
// contiguous children (no atomics).
// ----------------------------------------------------------------------------
template <int P, typename CT, typename AT>
__global__ __launch_bounds__(64) void m2m_kernel(int64_t c0, int64_t c1, const int32_t *__restrict__ child_begin,
                           const int32_t *__restrict__ n_child, const double4 *__restrict__ geo,
                           const CT *__restrict__ Mchild, AT *__restrict__ Mout,
                           float *__restrict__ Mcopy) {
  constexpr int T = nterms(P), S = pad4(T);
  const int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  const int nch = n_child[c];
  if (nch == 0) return;
  const double4 gp = geo[c];
  AT acc[T];
  static_for<T>([&](auto I) { acc[decltype(I)::value] = AT(0); });
  for (int k = 0; k < nch; ++k) {
    const int ch = child_begin[c] + k;
    const double4 gc = geo[ch];
    AT mono[T];
    monomials<P, AT>(AT(gp.x - gc.x), AT(gp.y - gc.y), AT(gp.z - gc.z), mono);
    CT mc[T];
    load_row<T>(Mchild + (int64_t)ch * S, mc);
    static_for<kShift<P>.N>([&](auto I) {
      constexpr int i = decltype(I)::value;
      acc[kShift<P>.hi[i]] += AT(mc[kShift<P>.lo[i]]) * mono[kShift<P>.diff[i]];
    });
  }
  static_for<T>([&](auto I) { Mout[c * S + decltype(I)::value] = acc[decltype(I)::value]; });
  if (Mcopy)
    static_for<T>([&](auto I) { Mcopy[c * S + decltype(I)::value] = (float)acc[decltype(I)::value]; });
}

// ----------------------------------------------------------------------------
// M2L: one 64-lane wave per target cell with M2L entries; lane l takes the
// entries l, l+64, ... of the row, computes D^m G(X_A - X_B) with the
// recurrence and contracts it with the source multipole.  The 64 lane
// partials are summed in LDS in a fixed order.
// ----------------------------------------------------------------------------
template <int P, typename Real, typename Acc>
__global__ __launch_bounds__(64) void m2l_kernel(int64_t r0, const int32_t *__restrict__ rows,
                                                 const int64_t *__restrict__ ptr,
                                                 const int32_t *__restrict__ col,
                                                 const double4 *__restrict__ geo,
                                                 const Real *__restrict__ M, Acc *__restrict__ Lout) {
  constexpr int T = nterms(P), S = pad4(T);
  __shared__ Acc red[64 * (T + 1)];
  const int lane = threadIdx.x;
  const int A = rows[r0 + xcd_remap(blockIdx.x, gridDim.x)];
  const double4 ga = geo[A];
  Acc acc[T];
  static_for<T>([&](auto I) { acc[decltype(I)::value] = Acc(0); });
  const int64_t e1 = ptr[A + 1];
  if constexpr (T <= 56) {
    // Software pipeline: the centre and multipole of the lane's next entry
    // are loaded while the current entry is computed.
    int64_t e = ptr[A] + lane;
    double4 gb_next = ga;
    Real mb_next[T];
    static_for<T>([&](auto I) { mb_next[decltype(I)::value] = Real(0); });
    if (e < e1) {
      const int B = col[e];
      gb_next = geo[B];
      load_row<T>(M + (int64_t)B * S, mb_next);
    }
    int B2 = (e + 64 < e1) ? col[e + 64] : 0;
    for (; e < e1; e += 64) {
      const double4 gb = gb_next;
      Real mb[T];
      static_for<T>([&](auto I) { mb[decltype(I)::value] = mb_next[decltype(I)::value]; });
      if (e + 64 < e1) {
        gb_next = geo[B2];
        load_row<T>(M + (int64_t)B2 * S, mb_next);
        B2 = (e + 128 < e1) ? col[e + 128] : 0;
      }
      Real D[T];
      derivatives<P, Real>(Real(ga.x - gb.x), Real(ga.y - gb.y), Real(ga.z - gb.z), D);
      static_for<kM2L<P>.N>([&](auto I) {
        constexpr int i = decltype(I)::value;
        acc[kM2L<P>.k[i]] += Acc(mb[kM2L<P>.n[i]] * D[kM2L<P>.s[i]]);
      });
    }
  } else {
    // High orders: registers are the limit, so no prefetch.
    for (int64_t e = ptr[A] + lane; e < e1; e += 64) {
      const int B = col[e];
      const double4 gb = geo[B];
      Real D[T];
      derivatives<P, Real>(Real(ga.x - gb.x), Real(ga.y - gb.y), Real(ga.z - gb.z), D);
      Real mb[T];
      load_row<T>(M + (int64_t)B * S, mb);
      static_for<kM2L<P>.N>([&](auto I) {
        constexpr int i = decltype(I)::value;
        acc[kM2L<P>.k[i]] += Acc(mb[kM2L<P>.n[i]] * D[kM2L<P>.s[i]]);
      });
    }
  }
  static_for<T>([&](auto I) { red[lane * (T + 1) + decltype(I)::value] = acc[decltype(I)::value]; });
  __syncthreads();
  for (int t = lane; t < T; t += 64) {
    Acc sum = Acc(0);
    for (int l = 0; l < 64; ++l) sum += red[l * (T + 1) + t];
    Lout[(int64_t)A * S + t] = sum;
  }
}

// ----------------------------------------------------------------------------
// L2L: one thread per child cell of one level; the child pulls from its
// parent.  PT: parent's storage type, AT: arithmetic type, CT: child's.
// ----------------------------------------------------------------------------
template <int P, typename PT, typename AT, typename CT>
__global__ __launch_bounds__(64) void l2l_kernel(int64_t c0, int64_t c1, const int32_t *__restrict__ parent,
                           const double4 *__restrict__ geo, const PT *__restrict__ Lpar,
                           CT *__restrict__ Lchild) {
  constexpr int T = nterms(P), S = pad4(T);
  const int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  const int pc = parent[c];
  const double4 gc = geo[c], gp = geo[pc];
  AT mono[T];
  monomials<P, AT>(AT(gc.x - gp.x), AT(gc.y - gp.y), AT(gc.z - gp.z), mono);
  PT lp[T];
  load_row<T>(Lpar + (int64_t)pc * S, lp);
  AT add[T];
  static_for<T>([&](auto I) { add[decltype(I)::value] = AT(0); });
  static_for<kShift<P>.N>([&](auto I) {
    constexpr int i = decltype(I)::value;
    add[kShift<P>.lo[i]] += AT(lp[kShift<P>.hi[i]]) * mono[kShift<P>.diff[i]];
  });
  static_for<T>([&](auto I) {
    constexpr int t = decltype(I)::value;
    Lchild[c * S + t] = CT(AT(Lchild[c * S + t]) + add[t]);
  });
}

__global__ void copy_top_kernel(int64_t n, const double *__restrict__ src, float *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

// ----------------------------------------------------------------------------
// L2P + near/far combine + scatter to user order: one thread per body.
// ----------------------------------------------------------------------------
template <int P, typename Real, bool KAHAN>
__global__ __launch_bounds__(256) void l2p_combine_kernel(
    int64_t n, const int32_t *__restrict__ body_leaf, const int32_t *__restrict__ leaf_cell,
    const int32_t *__restrict__ leaf_pbase, const int32_t *__restrict__ leaf_nchunk,
    const int32_t *__restrict__ cell_body_begin, const int32_t *__restrict__ cell_n_body,
    const double4 *__restrict__ geo, const Real *__restrict__ L,
    const typename Vec<Real>::V4 *__restrict__ bodies,
    const typename Vec<Real>::V4 *__restrict__ part_s,
    const typename Vec<Real>::V4 *__restrict__ part_c, const int32_t *__restrict__ perm,
    Real *__restrict__ phi_out, Real *__restrict__ grad_out) {
  using V4 = typename Vec<Real>::V4;
  constexpr int T = nterms(P), S = pad4(T);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = body_leaf[i];
  const int c = leaf_cell[a];
  const V4 b = bodies[i];
  const double4 g = geo[c];
  Real mono[T];
  monomials<P, Real>(Real((double)b.x - g.x), Real((double)b.y - g.y), Real((double)b.z - g.z),
                     mono);
  Real lc[T];
  load_row<T>(L + (int64_t)c * S, lc);
  Real f = Real(0), gx = Real(0), gy = Real(0), gz = Real(0);
  static_for<T>([&](auto I) {
    constexpr int t = decltype(I)::value;
    f += lc[t] * mono[t];
    if constexpr (kBasis<P>.lo[t][0] >= 0) gx += lc[t] * mono[kBasis<P>.lo[t][0]];
    if constexpr (kBasis<P>.lo[t][1] >= 0) gy += lc[t] * mono[kBasis<P>.lo[t][1]];
    if constexpr (kBasis<P>.lo[t][2] >= 0) gz += lc[t] * mono[kBasis<P>.lo[t][2]];
  });
  Real s4[4] = {0, 0, 0, 0}, c4[4] = {0, 0, 0, 0};
  const int nA = cell_n_body[c];
  const int64_t slot0 = (int64_t)leaf_pbase[a] + (i - cell_body_begin[c]);
  const int nch = leaf_nchunk[a];
  for (int ch = 0; ch < nch; ++ch) {
    const V4 ps = part_s[slot0 + (int64_t)ch * nA];
    const Real vs[4] = {ps.x, ps.y, ps.z, ps.w};
    if constexpr (KAHAN) {
      const V4 pc = part_c[slot0 + (int64_t)ch * nA];
      const Real vc[4] = {pc.x, pc.y, pc.z, pc.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const Real y = (vs[k] - vc[k]) - c4[k];
        const Real t = s4[k] + y;
        c4[k] = (t - s4[k]) - y;
        s4[k] = t;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) s4[k] += vs[k];
    }
  }
  const int64_t u = perm[i];
  phi_out[u] = (s4[0] - c4[0]) + f;
  if (grad_out) {
    grad_out[3 * u + 0] = (s4[1] - c4[1]) + gx;
    grad_out[3 * u + 1] = (s4[2] - c4[2]) + gy;
    grad_out[3 * u + 2] = (s4[3] - c4[3]) + gz;
  }
}

// dL/dx = w * grad[q] + q * grad[w], user order.
template <typename Real>
__global__ void backward_combine_kernel(int64_t n, const Real *__restrict__ q,
                                        const Real *__restrict__ w, const Real *__restrict__ gq,
                                        const Real *__restrict__ gw, Real *__restrict__ dx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Real qi = q[i], wi = w[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) dx[3 * i + d] = wi * gq[3 * i + d] + qi * gw[3 * i + d];
}

__global__ void zero_kernel(int64_t n16, int64_t nbytes, uint8_t *p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) {
    if ((i + 1) * 16 <= nbytes) {
      reinterpret_cast<uint4 *>(p)[i] = uint4{0, 0, 0, 0};
    } else {
      for (int64_t k = i * 16; k < nbytes; ++k) p[k] = 0;
    }
  }
}

// FP64 direct sum: one 256-thread work-group per target, fixed-order reduction.
__global__ __launch_bounds__(256) void direct_kernel(const double *__restrict__ xyz,
                                                     const double *__restrict__ q, int64_t n,
                                                     const int64_t *__restrict__ targets,
                                                     double *__restrict__ phi,
                                                     double *__restrict__ grad) {
  __shared__ double red[4][256];
  const int64_t t = blockIdx.x;
  const int64_t i = targets[t];
  if (i < 0 || i >= n) {  // invalid target index: report NaN, read nothing
    if (threadIdx.x == 0) {
      phi[t] = __builtin_nan("");
      if (grad) grad[3 * t] = grad[3 * t + 1] = grad[3 * t + 2] = __builtin_nan("");
    }
    return;
  }
  const double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2];
  double f = 0, gx = 0, gy = 0, gz = 0;
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    const double dx = xyz[3 * j] - xi, dy = xyz[3 * j + 1] - yi, dz = xyz[3 * j + 2] - zi;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) continue;
    const double r = sqrt(r2);
    const double inv = 1.0 / r;
    const double inv3 = inv / r2;
    f += q[j] * inv;
    gx += q[j] * dx * inv3;
    gy += q[j] * dy * inv3;
    gz += q[j] * dz * inv3;
  }
  red[0][threadIdx.x] = f;
  red[1][threadIdx.x] = gx;
  red[2][threadIdx.x] = gy;
  red[3][threadIdx.x] = gz;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    phi[t] = red[0][0];
    if (grad) {
      grad[3 * t] = red[1][0];
      grad[3 * t + 1] = red[2][0];
      grad[3 * t + 2] = red[3][0];
    }
  }
}

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }
inline hipStream_t S_(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

#define FMM_LAUNCH_CHECK() return (int)hipGetLastError()

// Run f(std::integral_constant<int, p>) for the runtime order p.
template <class F>
int with_p(int p, F &&f) {
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

int gather_charges(bool fp64, int64_t n, const int32_t *perm, const void *q_user, void *bodies,
                   void *stream) {
  if (n == 0) return 0;
  if (fp64)
    gather_kernel<double><<<blocks_for(n, 256), 256, 0, S_(stream)>>>(
        n, perm, (const double *)q_user, (double4 *)bodies);
  else
    gather_kernel<float><<<blocks_for(n, 256), 256, 0, S_(stream)>>>(
        n, perm, (const float *)q_user, (float4 *)bodies);
  FMM_LAUNCH_CHECK();
}

int p2p(bool fp64, bool mask_all, int64_t n_items, const P2PItem *items, const int32_t *run_body,
        const int32_t *run_prefix, const void *bodies, void *part_s, void *part_c, void *stream) {
  if (n_items == 0) return 0;
  const unsigned G = (unsigned)n_items;
  if (fp64) {
    if (mask_all)
      p2p_kernel<double, false, true><<<G, 64, 0, S_(stream)>>>(
          items, run_body, run_prefix, (const double4 *)bodies, (double4 *)part_s, nullptr);
    else
      p2p_kernel<double, false, false><<<G, 64, 0, S_(stream)>>>(
          items, run_body, run_prefix, (const double4 *)bodies, (double4 *)part_s, nullptr);
  } else {
    if (mask_all)
      p2p_kernel<float, true, true><<<G, 64, 0, S_(stream)>>>(
          items, run_body, run_prefix, (const float4 *)bodies, (float4 *)part_s, (float4 *)part_c);
    else
      p2p_kernel<float, true, false><<<G, 64, 0, S_(stream)>>>(
          items, run_body, run_prefix, (const float4 *)bodies, (float4 *)part_s, (float4 *)part_c);
  }
  FMM_LAUNCH_CHECK();
}

int p2m(int p, bool fp64, int64_t n_leaves, const int32_t *leaf_cell, const int32_t *cell_body_begin,
        const int32_t *cell_n_body, const double *geo, const void *bodies, void *M, double *M64,
        int64_t n_top, void *stream) {
  if (n_leaves == 0) return 0;
  const unsigned nb = blocks_for(n_leaves, 64);
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    if (fp64)
      p2m_kernel<PP, double><<<nb, 64, 0, S_(stream)>>>(n_leaves, leaf_cell, cell_body_begin,
                                                        cell_n_body, (const double4 *)geo,
                                                        (const double4 *)bodies, (double *)M,
                                                        M64, 0);
    else
      p2m_kernel<PP, float><<<nb, 64, 0, S_(stream)>>>(n_leaves, leaf_cell, cell_body_begin,
                                                       cell_n_body, (const double4 *)geo,
                                                       (const float4 *)bodies, (float *)M, M64,
                                                       n_top);
  });
}

int m2m(int p, bool fp64, int64_t c0, int64_t c1, const int32_t *child_begin,
        const int32_t *n_child, const double *geo, void *M, double *M64, bool child_fp64,
        bool out_fp64, void *stream) {
  if (c1 <= c0) return 0;
  const unsigned nb = blocks_for(c1 - c0, 64);
  const double4 *g = (const double4 *)geo;
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    if (fp64)
      m2m_kernel<PP, double, double><<<nb, 64, 0, S_(stream)>>>(
          c0, c1, child_begin, n_child, g, (const double *)M, (double *)M, nullptr);
    else if (out_fp64 && child_fp64)
      m2m_kernel<PP, double, double><<<nb, 64, 0, S_(stream)>>>(c0, c1, child_begin, n_child, g,
                                                                M64, M64, (float *)M);
    else if (out_fp64)
      m2m_kernel<PP, float, double><<<nb, 64, 0, S_(stream)>>>(
          c0, c1, child_begin, n_child, g, (const float *)M, M64, (float *)M);
    else
      m2m_kernel<PP, float, float><<<nb, 64, 0, S_(stream)>>>(
          c0, c1, child_begin, n_child, g, (const float *)M, (float *)M, nullptr);
  });
}

int m2l(int p, bool fp64, int64_t r0, int64_t r1, const int32_t *rows, const int64_t *ptr,
        const int32_t *col, const double *geo, const void *M, void *L, double *L64,
        bool acc_fp64, void *stream) {
  if (r1 <= r0) return 0;
  const unsigned G = (unsigned)(r1 - r0);
  const double4 *g = (const double4 *)geo;
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    if (fp64)
      m2l_kernel<PP, double, double><<<G, 64, 0, S_(stream)>>>(r0, rows, ptr, col, g,
                                                               (const double *)M, (double *)L);
    else if (acc_fp64)
      m2l_kernel<PP, float, double><<<G, 64, 0, S_(stream)>>>(r0, rows, ptr, col, g,
                                                              (const float *)M, L64);
    else
      m2l_kernel<PP, float, float><<<G, 64, 0, S_(stream)>>>(r0, rows, ptr, col, g,
                                                             (const float *)M, (float *)L);
  });
}

int l2l(int p, bool fp64, int64_t c0, int64_t c1, const int32_t *parent, const double *geo,
        void *L, double *L64, bool parent_fp64, bool child_fp64, void *stream) {
  if (c1 <= c0) return 0;
  const unsigned nb = blocks_for(c1 - c0, 64);
  const double4 *g = (const double4 *)geo;
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    if (fp64)
      l2l_kernel<PP, double, double, double><<<nb, 64, 0, S_(stream)>>>(
          c0, c1, parent, g, (const double *)L, (double *)L);
    else if (parent_fp64 && child_fp64)
      l2l_kernel<PP, double, double, double><<<nb, 64, 0, S_(stream)>>>(c0, c1, parent, g, L64,
                                                                        L64);
    else if (parent_fp64)
      l2l_kernel<PP, double, double, float><<<nb, 64, 0, S_(stream)>>>(c0, c1, parent, g, L64,
                                                                       (float *)L);
    else
      l2l_kernel<PP, float, float, float><<<nb, 64, 0, S_(stream)>>>(
          c0, c1, parent, g, (const float *)L, (float *)L);
  });
}

int copy_top_locals(int p, int64_t n_top, const double *L64, float *L, void *stream) {
  const int64_t n = n_top * stride(p);
  if (n == 0) return 0;
  copy_top_kernel<<<blocks_for(n, 256), 256, 0, S_(stream)>>>(n, L64, L);
  FMM_LAUNCH_CHECK();
}

int l2p_combine(int p, bool fp64, int64_t n, const int32_t *body_leaf, const int32_t *leaf_cell,
                const int32_t *leaf_pbase, const int32_t *leaf_nchunk,
                const int32_t *cell_body_begin, const int32_t *cell_n_body, const double *geo,
                const void *L, const void *bodies, const void *part_s, const void *part_c,
                const int32_t *perm, void *phi, void *grad, void *stream) {
  if (n == 0) return 0;
  const unsigned nb = blocks_for(n, 256);
  const double4 *g = (const double4 *)geo;
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    if (fp64)
      l2p_combine_kernel<PP, double, false><<<nb, 256, 0, S_(stream)>>>(
          n, body_leaf, leaf_cell, leaf_pbase, leaf_nchunk, cell_body_begin, cell_n_body, g,
          (const double *)L, (const double4 *)bodies, (const double4 *)part_s, nullptr, perm,
          (double *)phi, (double *)grad);
    else
      l2p_combine_kernel<PP, float, true><<<nb, 256, 0, S_(stream)>>>(
          n, body_leaf, leaf_cell, leaf_pbase, leaf_nchunk, cell_body_begin, cell_n_body, g,
          (const float *)L, (const float4 *)bodies, (const float4 *)part_s,
          (const float4 *)part_c, perm, (float *)phi, (float *)grad);
  });
}

int backward_combine(bool fp64, int64_t n, const void *q, const void *w, const void *grad_q,
                     const void *grad_w, void *dx, void *stream) {
  if (n == 0) return 0;
  if (fp64)
    backward_combine_kernel<double><<<blocks_for(n, 256), 256, 0, S_(stream)>>>(
        n, (const double *)q, (const double *)w, (const double *)grad_q, (const double *)grad_w,
        (double *)dx);
  else
    backward_combine_kernel<float><<<blocks_for(n, 256), 256, 0, S_(stream)>>>(
        n, (const float *)q, (const float *)w, (const float *)grad_q, (const float *)grad_w,
        (float *)dx);
  FMM_LAUNCH_CHECK();
}

int zero(void *ptr, int64_t bytes, void *stream) {
  if (bytes <= 0) return 0;
  const int64_t n16 = (bytes + 15) / 16;
  zero_kernel<<<blocks_for(n16, 256), 256, 0, S_(stream)>>>(n16, bytes, (uint8_t *)ptr);
  FMM_LAUNCH_CHECK();
}

int direct_sum(const double *xyz, const double *q, int64_t n, const int64_t *targets, int64_t m,
               double *phi, double *grad, void *stream) {
  if (m == 0) return 0;
  direct_kernel<<<(unsigned)m, 256, 0, S_(stream)>>>(xyz, q, n, targets, phi, grad);
  FMM_LAUNCH_CHECK();
}

}  // namespace dev
}  // namespace fmmlib
