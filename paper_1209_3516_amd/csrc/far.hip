// Far-field kernels (P2M, M2M, M2L, L2L, L2P + combine) of the gfx950 FMM.
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
// precomputed matrices (section 3.1: bytes per flop keep falling).  M2L works
// on harmonic-reduced terms: since G is harmonic, the multipole is first
// folded onto its p^2 terms of z exponent <= 1 and only the p^2 local terms
// of z exponent <= 1 are contracted; the others follow exactly (the
// identities are stated with the reduced contraction table).
//
// All index arithmetic over multi-indices is resolved at compile time: the
// kernels are templated on p and every loop over coefficients is unrolled
// through constexpr tables, so coefficients live in registers.
//
// No floating-point atomics anywhere: each output value is produced by one
// thread or one wave in a fixed order, so results are bitwise reproducible.
#include "device_common.h"

namespace fmmlib {
namespace dev {
namespace {

// ----------------------------------------------------------------------------
// P2M: one 64-lane wave per G = 64 / LPL leaves, LPL lanes per leaf (32, or
// 16 when leaves are small).  Bodies are taken LPL at a time: lane j loads
// body j (coalesced), forms its term row w_t = q (X - x)^t / t! for every
// term t (with dipoles s, also sum_d s_d (X - x)^(t - e_d) / (t - e_d)!) and
// stores the row in LDS; then lane t adds column t over the bodies of the
// batch, in body order (terms beyond LPL go round again).  The sums need no
// cross-lane reduction.
// ----------------------------------------------------------------------------
template <int P, typename Real, bool DIP, int LPL>
__global__ __launch_bounds__(64) void p2m_kernel(int64_t n_leaves, const int32_t *__restrict__ leaf_cell,
                           const int32_t *__restrict__ body_begin,
                           const int32_t *__restrict__ n_body, const double4 *__restrict__ geo,
                           const typename Vec<Real>::V4 *__restrict__ bodies,
                           const typename Vec<Real>::V4 *__restrict__ dip, Real *__restrict__ M,
                           double *__restrict__ M64, int64_t n_top) {
  constexpr int T = nterms(P), S = pad4(T);
  constexpr int G = 64 / LPL;              // leaves per block
  constexpr int RS = T + 1;                // LDS row stride (odd: no bank conflicts on reads)
  constexpr int TPL = (T + LPL - 1) / LPL; // terms per lane
  __shared__ Real rows[G][LPL * RS];
  const int grp = threadIdx.x / LPL, j = threadIdx.x % LPL;
  const int64_t li = G * (int64_t)blockIdx.x + grp;
  const bool active = li < n_leaves;
  const int c = active ? leaf_cell[li] : 0;
  const int b0 = active ? body_begin[c] : 0, nb = active ? n_body[c] : 0;
  const double4 g = geo[c];
  Real *row = rows[grp];
  Real acc[TPL];
#pragma unroll
  for (int k = 0; k < TPL; ++k) acc[k] = Real(0);
  // every group runs as many batches as the largest leaf of the block needs
  // (the barrier is block wide)
  int nbmax = nb;
#pragma unroll
  for (int off = LPL; off < 64; off <<= 1) {
    const int o = __shfl_xor(nbmax, off);
    nbmax = o > nbmax ? o : nbmax;
  }
  for (int j0 = 0; j0 < nbmax; j0 += LPL) {
    const int nj = min(LPL, nb - j0);
    if (j < nj) {
      const typename Vec<Real>::V4 b = bodies[b0 + j0 + j];
      Real mono[T];
      monomials<P, Real>(Real(g.x - (double)b.x), Real(g.y - (double)b.y),
                         Real(g.z - (double)b.z), mono);
      typename Vec<Real>::V4 sd;
      if constexpr (DIP) sd = dip[b0 + j0 + j];
      static_for<T>([&](auto I) {
        constexpr int t = decltype(I)::value;
        Real w = b.w * mono[t];
        if constexpr (DIP) {
          if constexpr (kBasis<P>.lo[t][0] >= 0) w += sd.x * mono[kBasis<P>.lo[t][0]];
          if constexpr (kBasis<P>.lo[t][1] >= 0) w += sd.y * mono[kBasis<P>.lo[t][1]];
          if constexpr (kBasis<P>.lo[t][2] >= 0) w += sd.z * mono[kBasis<P>.lo[t][2]];
        }
        row[j * RS + t] = w;
      });
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      const int t = j + LPL * k;
      if (t < T)
        for (int i = 0; i < nj; ++i) acc[k] += row[i * RS + t];
    }
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    const int t = j + LPL * k;
    if (t < T) {
      M[(int64_t)c * S + t] = acc[k];
      if (c < n_top) M64[(int64_t)c * S + t] = (double)acc[k];
    }
  }
}

// ----------------------------------------------------------------------------
// P2M for low orders (at most 20 terms, p <= 4): eight lanes per leaf, eight
// leaves per one-wave block (one-wave blocks find room beside the P2P
// kernel's waves when the two streams overlap), no LDS.  Lane j of a leaf adds the
// term rows of bodies j, j + 8, j + 16, ... in registers (four bodies' loads
// in flight at a time), then the eight lane sums are added by an xor-shuffle
// tree, the same on every lane of the leaf, and lane j stores the terms
// t = j mod 8.
// ----------------------------------------------------------------------------
constexpr int kP2MRegLanes = 8;

template <int P, typename Real, bool DIP>
__global__ __launch_bounds__(64) void p2m_reg_kernel(
    int64_t n_leaves, const int32_t *__restrict__ leaf_cell,
    const int32_t *__restrict__ body_begin, const int32_t *__restrict__ n_body,
    const double4 *__restrict__ geo, const typename Vec<Real>::V4 *__restrict__ bodies,
    const typename Vec<Real>::V4 *__restrict__ dip, Real *__restrict__ M,
    double *__restrict__ M64, int64_t n_top) {
  using V4 = typename Vec<Real>::V4;
  constexpr int T = nterms(P), S = pad4(T), LPL = kP2MRegLanes, U = 4;
  static_assert(T <= 20, "register P2M is for p <= 4");
  const int j = threadIdx.x % LPL;
  const int64_t li = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LPL;
  const bool active = li < n_leaves;
  const int c = active ? leaf_cell[li] : 0;
  const int b0 = active ? body_begin[c] : 0, nb = active ? n_body[c] : 0;
  const double4 g = geo[c];
  Real acc[T];
  static_for<T>([&](auto I) { acc[decltype(I)::value] = Real(0); });
  for (int i0 = 0; i0 < nb; i0 += U * LPL) {
    V4 bv[U], dv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + j + LPL * u;
      if (i < nb) {
        bv[u] = bodies[b0 + i];
        if constexpr (DIP) dv[u] = dip[b0 + i];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + j + LPL * u < nb) {
        const V4 b = bv[u];
        Real mono[T];
        monomials<P, Real>(Real(g.x - (double)b.x), Real(g.y - (double)b.y),
                           Real(g.z - (double)b.z), mono);
        static_for<T>([&](auto I) {
          constexpr int t = decltype(I)::value;
          Real w = b.w * mono[t];
          if constexpr (DIP) {
            if constexpr (kBasis<P>.lo[t][0] >= 0) w += dv[u].x * mono[kBasis<P>.lo[t][0]];
            if constexpr (kBasis<P>.lo[t][1] >= 0) w += dv[u].y * mono[kBasis<P>.lo[t][1]];
            if constexpr (kBasis<P>.lo[t][2] >= 0) w += dv[u].z * mono[kBasis<P>.lo[t][2]];
          }
          acc[t] += w;
        });
      }
    }
  }
  // a + b on one lane, b + a on its partner: every lane ends with the same sums
#pragma unroll
  for (int off = LPL / 2; off >= 1; off >>= 1)
    static_for<T>([&](auto I) {
      constexpr int t = decltype(I)::value;
      acc[t] += __shfl_xor(acc[t], off);
    });
  if (!active) return;
  static_for<T>([&](auto I) {
    constexpr int t = decltype(I)::value;
    if (t % LPL == j) {
      M[(int64_t)c * S + t] = acc[t];
      if (c < n_top) M64[(int64_t)c * S + t] = (double)acc[t];
    }
  });
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
// Harmonic fold of the multipoles for M2L (the identities are stated with
// the reduced contraction table): one thread per cell, Mr[c] = the p^2
// terms of z exponent <= 1, each a signed binomial sum of terms of M[c] of
// the same degree, summed in FP64 and rounded once.
// ----------------------------------------------------------------------------
template <int P, typename Real>
__global__ __launch_bounds__(64) void fold_kernel(int64_t n_cells, const Real *__restrict__ M,
                                                  Real *__restrict__ Mr) {
  constexpr int T = nterms(P), S = pad4(T), TR = rterms(P), SR = pad4(TR);
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  Real m[T];
  load_row<T>(M + c * S, m);
  double acc[TR];
  static_for<TR>([&](auto I) { acc[decltype(I)::value] = 0.0; });
  harmonic_pairs<P>([&](auto t, auto r, auto w, auto) {
    acc[decltype(r)::value] += double(decltype(w)::value) * double(m[decltype(t)::value]);
  });
  static_for<SR>([&](auto I) {
    constexpr int r = decltype(I)::value;
    Mr[c * SR + r] = r < TR ? Real(acc[r < TR ? r : 0]) : Real(0);
  });
}

// ----------------------------------------------------------------------------
// M2L: one 64-lane wave per target cell (a cell without entries writes
// zeros, so L needs no clearing before M2L); lane l takes the
// entries l, l+64, ... of the row, computes D^m G(X_A - X_B) (z exponent
// <= 2) with the recurrence and contracts it with the folded source
// multipole into the p^2 target terms of z exponent <= 1.  These are
// expanded to all target terms, and the 64 lane partials are summed in LDS
// in a fixed order.
// ----------------------------------------------------------------------------
// Terms per round of the final cross-lane sum of M2L.
constexpr int m2l_red_terms(int T) { return T < 64 ? T : 64; }

template <int P, typename Real, typename Acc, int CH = m2l_red_terms(nterms(P)),
          bool STREAM = (rterms(P) > 36)>
__device__ __forceinline__ void m2l_row(int64_t r0, const int64_t *__restrict__ ptr,
                                        const int32_t *__restrict__ col,
                                        const double4 *__restrict__ geo,
                                        const Real *__restrict__ Mr, Acc *__restrict__ Lout,
                                        Acc *__restrict__ red,
                                        const int32_t *__restrict__ order) {
  constexpr int T = nterms(P), S = pad4(T), TR = rterms(P), SR = pad4(TR);
  const int lane = threadIdx.x;
  const int A = order ? order[blockIdx.x] : (int)(r0 + xcd_remap(blockIdx.x, gridDim.x));
  // an ordered launch: padding, or a cell of [0, r0) (left to another launch)
  if (A < r0) return;
  const double4 ga = geo[A];
  Acc acc[TR];
  static_for<TR>([&](auto I) { acc[decltype(I)::value] = Acc(0); });
  const int64_t e1 = ptr[A + 1];
  if constexpr (!STREAM) {
    // Software pipeline with two register buffers: the centre and multipole
    // of the lane's next entry load while the current entry is computed.
    auto contract = [&](const double4 &gb, const Real (&mb)[TR]) {
      Real D[T];
      derivatives<P, Real, true>(Real(ga.x - gb.x), Real(ga.y - gb.y), Real(ga.z - gb.z), D);
      static_for<kM2LR<P>.N>([&](auto I) {
        constexpr int i = decltype(I)::value;
        acc[kM2LR<P>.k[i]] += Acc(mb[kM2LR<P>.n[i]] * D[kM2LR<P>.s[i]]);
      });
    };
    int64_t e = ptr[A] + lane;
    double4 g0 = ga, g1 = ga;
    Real m0[TR], m1[TR];
    if (e < e1) {
      const int B = col[e];
      g0 = geo[B];
      load_row<TR>(Mr + (int64_t)B * SR, m0);
    }
    int Bn = (e + 64 < e1) ? col[e + 64] : 0;
    while (e < e1) {
      if (e + 64 < e1) {
        g1 = geo[Bn];
        load_row<TR>(Mr + (int64_t)Bn * SR, m1);
        Bn = (e + 128 < e1) ? col[e + 128] : 0;
      }
      contract(g0, m0);
      e += 64;
      if (e >= e1) break;
      if (e + 64 < e1) {
        g0 = geo[Bn];
        load_row<TR>(Mr + (int64_t)Bn * SR, m0);
        Bn = (e + 128 < e1) ? col[e + 128] : 0;
      }
      contract(g1, m1);
      e += 64;
    }
  } else {
    // Streamed: the source multipole comes in groups of four
    // terms, each used by all its contraction entries as soon as it arrives.
    // The source cell of the entry after next and the centre of the next
    // entry load while this entry is computed (indices past the row's end
    // are clamped to its last entry); the empty asm at the end of the body
    // keeps the compiler from moving those loads next to their use.
    // (An empty row has no last entry: it skips the loop and writes zeros.)
    const int64_t e0 = ptr[A];
    int64_t e = e0 + lane;
    const int64_t last = e1 > e0 ? e1 - 1 : e0;
    int Bc = 0, Bn = 0;
    Real rx = Real(0), ry = Real(0), rz = Real(0);
    if (e1 > e0) {
      Bc = col[e < last ? e : last];
      Bn = col[e + 64 < last ? e + 64 : last];
      const double4 g0 = geo[Bc];
      rx = Real(ga.x - g0.x);
      ry = Real(ga.y - g0.y);
      rz = Real(ga.z - g0.z);
    }
    for (; e < e1; e += 64) {
      const int B = Bc;
      const Real Rx = rx, Ry = ry, Rz = rz;
      Bc = Bn;
      const double4 gn = geo[Bc];
      Bn = col[e + 128 < last ? e + 128 : last];
      Real D[T];
      derivatives<P, Real, true>(Rx, Ry, Rz, D);
      const Real *mrow = Mr + (int64_t)B * SR;
      static_for<kM2LR<P>.G>([&](auto Gi) {
        constexpr int g = decltype(Gi)::value;
        Real m4[4];
        load4(mrow + 4 * g, m4);
        static_for<kM2LR<P>.gbeg[g + 1] - kM2LR<P>.gbeg[g]>([&](auto J) {
          constexpr int i = kM2LR<P>.gbeg[g] + decltype(J)::value;
          acc[kM2LR<P>.k[i]] += Acc(m4[kM2LR<P>.n[i] - 4 * g] * D[kM2LR<P>.s[i]]);
        });
      });
      rx = Real(ga.x - gn.x);
      ry = Real(ga.y - gn.y);
      rz = Real(ga.z - gn.z);
      asm volatile("" : "+v"(rx), "+v"(ry), "+v"(rz), "+v"(Bc), "+v"(Bn));
    }
  }
  // All target terms from the reduced ones (a linear map, so it commutes
  // with the sum over lanes).
  Acc full[T];
  harmonic_pairs<P>([&](auto t, auto r, auto w, auto first) {
    constexpr int tt = decltype(t)::value, rr = decltype(r)::value, ww = decltype(w)::value;
    Acc v;
    if constexpr (ww == 1) v = acc[rr];
    else if constexpr (ww == -1) v = -acc[rr];
    else v = Acc(ww) * acc[rr];
    if constexpr (decltype(first)::value) full[tt] = v;
    else full[tt] += v;
  });
  // Sum the 64 lane partials of each term in lane order, at most CH terms at
  // a time (so that the LDS buffer does not limit how many waves a CU holds).
  static_for<(T + CH - 1) / CH>([&](auto Ci) {
    constexpr int c0 = decltype(Ci)::value * CH;
    constexpr int nt = T - c0 < CH ? T - c0 : CH;
    if constexpr (c0 > 0) __syncthreads();
    static_for<nt>([&](auto I) {
      constexpr int j = decltype(I)::value;
      red[lane * (CH + 1) + j] = full[c0 + j];
    });
    __syncthreads();
    if (lane < nt) {
      Acc sum = Acc(0);
      for (int l = 0; l < 64; ++l) sum += red[l * (CH + 1) + lane];
      Lout[(int64_t)A * S + c0 + lane] = sum;
    }
  });
}

template <int P, typename Real, typename Acc>
__global__ __launch_bounds__(64) void m2l_kernel(int64_t r0, const int64_t *__restrict__ ptr,
                                                 const int32_t *__restrict__ col,
                                                 const double4 *__restrict__ geo,
                                                 const Real *__restrict__ Mr, Acc *__restrict__ Lout,
                                                 const int32_t *__restrict__ order) {
  __shared__ Acc red[64 * (m2l_red_terms(nterms(P)) + 1)];
  m2l_row<P, Real, Acc>(r0, ptr, col, geo, Mr, Lout, red, order);
}

// The same for high orders in FP32, held to two waves per SIMD (at most 256
// registers per lane) so that one wave's multipole loads overlap the other
// wave's arithmetic.
template <int P, typename Real, typename Acc>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void m2l_kernel_w2(
    int64_t r0, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
    const double4 *__restrict__ geo, const Real *__restrict__ Mr, Acc *__restrict__ Lout,
    const int32_t *__restrict__ order) {
  __shared__ Acc red[64 * (m2l_red_terms(nterms(P)) + 1)];
  m2l_row<P, Real, Acc>(r0, ptr, col, geo, Mr, Lout, red, order);
}

// Middle orders in FP32 at three waves per SIMD (at most 168 registers per
// lane); the cross-lane sum goes 32 terms at a time to fit twelve waves' LDS.
template <int P, typename Real, typename Acc>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 3))) void m2l_kernel_w3(
    int64_t r0, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
    const double4 *__restrict__ geo, const Real *__restrict__ Mr, Acc *__restrict__ Lout,
    const int32_t *__restrict__ order) {
  __shared__ Acc red[64 * (32 + 1)];
  m2l_row<P, Real, Acc, 32, true>(r0, ptr, col, geo, Mr, Lout, red, order);
}

// ----------------------------------------------------------------------------
// M2P (treecode/FMM hybrid): one 64-lane wave per target leaf with M2P
// entries (at most 64 bodies).  The lanes form G = 64 / nA groups of nA lanes;
// lane (g, t) evaluates the entries g, g + G, ... at body t with derivatives
// of 1/r up to degree p; the G partials of a body are summed in group order.
// Output: (phi, grad) per body in Morton order.
// ----------------------------------------------------------------------------
template <int P, typename Real>
__global__ __launch_bounds__(64) void m2p_kernel(const int32_t *__restrict__ rows,
                                                 const int64_t *__restrict__ ptr,
                                                 const int32_t *__restrict__ col,
                                                 const int32_t *__restrict__ cell_body_begin,
                                                 const int32_t *__restrict__ cell_n_body,
                                                 const double4 *__restrict__ geo,
                                                 const Real *__restrict__ M,
                                                 const typename Vec<Real>::V4 *__restrict__ bodies,
                                                 typename Vec<Real>::V4 *__restrict__ out) {
  using V4 = typename Vec<Real>::V4;
  constexpr int T = nterms(P), T1 = nterms(P + 1), S = pad4(T);
  __shared__ V4 red[64];
  const int A = rows[blockIdx.x];
  const int nA = cell_n_body[A];
  const int G = 64 / nA;
  const int lane = threadIdx.x;
  const int g = lane / nA, t = lane - g * nA;
  Real f = Real(0), gx = Real(0), gy = Real(0), gz = Real(0);
  if (g < G) {
    const V4 b = bodies[cell_body_begin[A] + t];
    for (int64_t e = ptr[A] + g; e < ptr[A + 1]; e += G) {
      const int B = col[e];
      const double4 gb = geo[B];
      Real D[T1];
      derivatives<P + 1, Real>(Real((double)b.x - gb.x), Real((double)b.y - gb.y),
                               Real((double)b.z - gb.z), D);
      Real mb[T];
      load_row<T>(M + (int64_t)B * S, mb);
      // terms are ordered by degree, so term n has the same index among the
      // terms of order P + 1
      static_for<T>([&](auto I) {
        constexpr int n = decltype(I)::value;
        constexpr int ex = kBasis<P>.ex[n], ey = kBasis<P>.ey[n], ez = kBasis<P>.ez[n];
        f += mb[n] * D[n];
        gx += mb[n] * D[term_index(P + 1, ex + 1, ey, ez)];
        gy += mb[n] * D[term_index(P + 1, ex, ey + 1, ez)];
        gz += mb[n] * D[term_index(P + 1, ex, ey, ez + 1)];
      });
    }
  }
  V4 v;
  v.x = f;
  v.y = gx;
  v.z = gy;
  v.w = gz;
  red[lane] = v;
  __syncthreads();
  if (lane < nA) {
    Real s[4] = {Real(0), Real(0), Real(0), Real(0)};
    for (int k = 0; k < G; ++k) {
      const V4 r = red[k * nA + lane];
      s[0] += r.x;
      s[1] += r.y;
      s[2] += r.z;
      s[3] += r.w;
    }
    V4 o;
    o.x = s[0];
    o.y = s[1];
    o.z = s[2];
    o.w = s[3];
    out[cell_body_begin[A] + lane] = o;
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
// HESS: the Hessian of the local expansion applied to the body's vector v,
// (H v)_a = sum_b v_b sum_{k >= e_a + e_b} L_k (y - X)^(k-e_a-e_b) / (k-e_a-e_b)!,
// is combined with the P2P Hessian-vector partials and written to grad_out.
// ----------------------------------------------------------------------------
template <int P, typename Real, bool KAHAN, bool HESS>
__global__ __launch_bounds__(256) void l2p_combine_kernel(
    int64_t i0, int64_t i1, const int32_t *__restrict__ body_leaf, const int32_t *__restrict__ leaf_cell,
    const int32_t *__restrict__ leaf_pbase, const int32_t *__restrict__ leaf_nchunk,
    const int32_t *__restrict__ cell_body_begin, const int32_t *__restrict__ cell_n_body,
    const double4 *__restrict__ geo, const Real *__restrict__ L,
    const typename Vec<Real>::V4 *__restrict__ bodies,
    const typename Vec<Real>::V4 *__restrict__ tvec,
    const typename Vec<Real>::V4 *__restrict__ part_s,
    const typename Vec<Real>::V4 *__restrict__ part_c, MutualSlots ms,
    const typename Vec<Real>::V4 *__restrict__ m2p_in, const int32_t *__restrict__ perm,
    Real *__restrict__ phi_out, Real *__restrict__ grad_out) {
  using V4 = typename Vec<Real>::V4;
  constexpr int T = nterms(P), S = pad4(T);
  const int64_t i = i0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= i1) return;
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
  if constexpr (!HESS) {
    static_for<T>([&](auto I) {
      constexpr int t = decltype(I)::value;
      f += lc[t] * mono[t];
      if constexpr (kBasis<P>.lo[t][0] >= 0) gx += lc[t] * mono[kBasis<P>.lo[t][0]];
      if constexpr (kBasis<P>.lo[t][1] >= 0) gy += lc[t] * mono[kBasis<P>.lo[t][1]];
      if constexpr (kBasis<P>.lo[t][2] >= 0) gz += lc[t] * mono[kBasis<P>.lo[t][2]];
    });
  } else {
    // six distinct second derivatives, then H v
    Real h[3][3] = {};
    static_for<T>([&](auto I) {
      constexpr int t = decltype(I)::value;
      static_for<3>([&](auto A) {
        constexpr int a = decltype(A)::value;
        if constexpr (kBasis<P>.lo[t][a] >= 0) {
          static_for<3>([&](auto Bb) {
            constexpr int b2 = decltype(Bb)::value;
            if constexpr (b2 >= a && kBasis<P>.lo[kBasis<P>.lo[t][a]][b2] >= 0)
              h[a][b2] += lc[t] * mono[kBasis<P>.lo[kBasis<P>.lo[t][a]][b2]];
          });
        }
      });
    });
    const typename Vec<Real>::V4 v = tvec[i];
    gx = h[0][0] * v.x + h[0][1] * v.y + h[0][2] * v.z;
    gy = h[0][1] * v.x + h[1][1] * v.y + h[1][2] * v.z;
    gz = h[0][2] * v.x + h[1][2] * v.y + h[2][2] * v.z;
  }
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
  if constexpr (KAHAN) {
    if (ms.part_m) {  // mutual P2P: the sums this body received as a source
      const float4 *pm = static_cast<const float4 *>(ms.part_m);
      const int nl = ms.leaf_nlow[a];
      const int64_t m0 = (int64_t)ms.leaf_mbase[a] + (i - cell_body_begin[c]);
      for (int j = 0; j < nl; ++j) {
        const float4 v = pm[m0 + (int64_t)j * nA];
        const float vs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float y = vs[k] - c4[k];
          const float t = s4[k] + y;
          c4[k] = (t - s4[k]) - y;
          s4[k] = t;
        }
      }
    }
  }
  if (m2p_in) {  // hybrid lists: the M2P part of the far field
    const V4 mp = m2p_in[i];
    f += mp.x;
    gx += mp.y;
    gy += mp.z;
    gz += mp.w;
  }
  const int64_t u = perm[i];
  if (phi_out) phi_out[u] = (s4[0] - c4[0]) + f;
  if (grad_out) {
    grad_out[3 * u + 0] = (s4[1] - c4[1]) + gx;
    grad_out[3 * u + 1] = (s4[2] - c4[2]) + gy;
    grad_out[3 * u + 2] = (s4[3] - c4[3]) + gz;
  }
}

}  // namespace

#define FMM_LAUNCH_CHECK() return (int)hipGetLastError()

int p2m(int p, bool fp64, int64_t n_leaves, const int32_t *leaf_cell, const int32_t *cell_body_begin,
        const int32_t *cell_n_body, const double *geo, const void *bodies, const void *dipoles,
        void *M, double *M64, int64_t n_top, int64_t n_bodies, void *stream) {
  if (n_leaves == 0) return 0;
  const double4 *g = (const double4 *)geo;
  // 16 lanes per leaf when the mean leaf holds at most 16 bodies, else 32
  const bool small = n_bodies <= 16 * n_leaves;
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    if constexpr (nterms(PP) <= 20) {
      const unsigned nbk = blocks_for(n_leaves, 64 / kP2MRegLanes);
      auto reg = [&](auto *b, auto *d, auto *m, int64_t top) {
        using R = std::remove_cv_t<std::remove_pointer_t<decltype(m)>>;
        if (dipoles)
          p2m_reg_kernel<PP, R, true><<<nbk, 64, 0, S_(stream)>>>(
              n_leaves, leaf_cell, cell_body_begin, cell_n_body, g, b, d, m, M64, top);
        else
          p2m_reg_kernel<PP, R, false><<<nbk, 64, 0, S_(stream)>>>(
              n_leaves, leaf_cell, cell_body_begin, cell_n_body, g, b, d, m, M64, top);
      };
      if (fp64)
        reg((const double4 *)bodies, (const double4 *)dipoles, (double *)M, int64_t(0));
      else
        reg((const float4 *)bodies, (const float4 *)dipoles, (float *)M, n_top);
      return;
    }
    auto go = [&](auto LC, auto *b, auto *d, auto *m, int64_t top) {
      constexpr int LPL = decltype(LC)::value;
      using R = std::remove_cv_t<std::remove_pointer_t<decltype(m)>>;
      const unsigned nb = blocks_for(n_leaves, 64 / LPL);
      if (dipoles)
        p2m_kernel<PP, R, true, LPL><<<nb, 64, 0, S_(stream)>>>(
            n_leaves, leaf_cell, cell_body_begin, cell_n_body, g, b, d, m, M64, top);
      else
        p2m_kernel<PP, R, false, LPL><<<nb, 64, 0, S_(stream)>>>(
            n_leaves, leaf_cell, cell_body_begin, cell_n_body, g, b, d, m, M64, top);
    };
    if (fp64) {
      const double4 *b = (const double4 *)bodies, *d = (const double4 *)dipoles;
      if (small) go(std::integral_constant<int, 16>{}, b, d, (double *)M, int64_t(0));
      else go(std::integral_constant<int, 32>{}, b, d, (double *)M, int64_t(0));
    } else {
      const float4 *b = (const float4 *)bodies, *d = (const float4 *)dipoles;
      if (small) go(std::integral_constant<int, 16>{}, b, d, (float *)M, n_top);
      else go(std::integral_constant<int, 32>{}, b, d, (float *)M, n_top);
    }
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

int fold_multipoles(int p, bool fp64, int64_t n_cells, const void *M, void *Mr, void *stream) {
  if (n_cells <= 0) return 0;
  const unsigned nb = blocks_for(n_cells, 64);
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    if (fp64)
      fold_kernel<PP, double><<<nb, 64, 0, S_(stream)>>>(n_cells, (const double *)M, (double *)Mr);
    else
      fold_kernel<PP, float><<<nb, 64, 0, S_(stream)>>>(n_cells, (const float *)M, (float *)Mr);
  });
}

int m2l(int p, bool fp64, int64_t r0, int64_t r1, const int64_t *ptr,
        const int32_t *col, const double *geo, const void *Mr, void *L, double *L64,
        bool acc_fp64, const int32_t *order, int64_t n_order, void *stream) {
  if (r1 <= r0) return 0;
  const unsigned G = (unsigned)(order ? n_order : r1 - r0);
  const double4 *g = (const double4 *)geo;
  const int32_t *o = order;
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    if (fp64)
      m2l_kernel<PP, double, double><<<G, 64, 0, S_(stream)>>>(
          r0, ptr, col, g, (const double *)Mr, (double *)L, o);
    else if (acc_fp64)
      m2l_kernel<PP, float, double><<<G, 64, 0, S_(stream)>>>(r0, ptr, col, g,
                                                              (const float *)Mr, L64, o);
    else if constexpr (rterms(PP) > 36)
      m2l_kernel_w2<PP, float, float><<<G, 64, 0, S_(stream)>>>(r0, ptr, col, g,
                                                                (const float *)Mr, (float *)L, o);
    else if constexpr (PP >= 5)
      m2l_kernel_w3<PP, float, float><<<G, 64, 0, S_(stream)>>>(r0, ptr, col, g,
                                                                (const float *)Mr, (float *)L, o);
    else
      m2l_kernel<PP, float, float><<<G, 64, 0, S_(stream)>>>(r0, ptr, col, g,
                                                             (const float *)Mr, (float *)L, o);
  });
}

int m2p(int p, bool fp64, int64_t n_rows, const int32_t *rows, const int64_t *ptr,
        const int32_t *col, const int32_t *cell_body_begin, const int32_t *cell_n_body,
        const double *geo, const void *M, const void *bodies, void *out, void *stream) {
  if (n_rows <= 0) return 0;
  const unsigned G = (unsigned)n_rows;
  const double4 *g = (const double4 *)geo;
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    if (fp64)
      m2p_kernel<PP, double><<<G, 64, 0, S_(stream)>>>(rows, ptr, col, cell_body_begin,
                                                       cell_n_body, g, (const double *)M,
                                                       (const double4 *)bodies, (double4 *)out);
    else
      m2p_kernel<PP, float><<<G, 64, 0, S_(stream)>>>(rows, ptr, col, cell_body_begin,
                                                      cell_n_body, g, (const float *)M,
                                                      (const float4 *)bodies, (float4 *)out);
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

template <int PP, typename Real, bool HESS>
void launch_l2p(unsigned nb, hipStream_t st, int64_t i0, int64_t i1, const int32_t *body_leaf,
                const int32_t *leaf_cell, const int32_t *leaf_pbase, const int32_t *leaf_nchunk,
                const int32_t *cell_body_begin, const int32_t *cell_n_body, const double4 *g,
                const void *L, const void *bodies, const void *tvec, const void *part_s,
                const void *part_c, MutualSlots ms, const void *m2p_in, const int32_t *perm,
                void *phi, void *grad) {
  using V4 = typename Vec<Real>::V4;
  constexpr bool kahan = std::is_same<Real, float>::value;
  l2p_combine_kernel<PP, Real, kahan, HESS><<<nb, 256, 0, st>>>(
      i0, i1, body_leaf, leaf_cell, leaf_pbase, leaf_nchunk, cell_body_begin, cell_n_body, g,
      (const Real *)L, (const V4 *)bodies, (const V4 *)tvec, (const V4 *)part_s,
      (const V4 *)part_c, ms, (const V4 *)m2p_in, perm, (Real *)phi, (Real *)grad);
}

int l2p_combine(int p, bool fp64, int mode, int64_t i0, int64_t i1, const int32_t *body_leaf,
                const int32_t *leaf_cell, const int32_t *leaf_pbase, const int32_t *leaf_nchunk,
                const int32_t *cell_body_begin, const int32_t *cell_n_body, const double *geo,
                const void *L, const void *bodies, const void *tvec, const void *part_s,
                const void *part_c, MutualSlots ms, const void *m2p_in, const int32_t *perm,
                void *phi, void *grad, void *stream) {
  if (i1 <= i0) return 0;
  if (fp64 && ms.part_m) return (int)hipErrorInvalidValue;  // mutual sums are FP32
  const unsigned nb = blocks_for(i1 - i0, 256);
  const double4 *g = (const double4 *)geo;
  const hipStream_t st = S_(stream);
  const bool hess = mode == kHessVec;
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    if (fp64 && hess)
      launch_l2p<PP, double, true>(nb, st, i0, i1, body_leaf, leaf_cell, leaf_pbase, leaf_nchunk,
                                   cell_body_begin, cell_n_body, g, L, bodies, tvec, part_s,
                                   nullptr, ms, m2p_in, perm, nullptr, grad);
    else if (fp64)
      launch_l2p<PP, double, false>(nb, st, i0, i1, body_leaf, leaf_cell, leaf_pbase, leaf_nchunk,
                                    cell_body_begin, cell_n_body, g, L, bodies, tvec, part_s,
                                    nullptr, ms, m2p_in, perm, phi, grad);
    else if (hess)
      launch_l2p<PP, float, true>(nb, st, i0, i1, body_leaf, leaf_cell, leaf_pbase, leaf_nchunk,
                                  cell_body_begin, cell_n_body, g, L, bodies, tvec, part_s,
                                  part_c, ms, m2p_in, perm, nullptr, grad);
    else
      launch_l2p<PP, float, false>(nb, st, i0, i1, body_leaf, leaf_cell, leaf_pbase, leaf_nchunk,
                                   cell_body_begin, cell_n_body, g, L, bodies, tvec, part_s,
                                   part_c, ms, m2p_in, perm, phi, grad);
  });
}

}  // namespace dev
}  // namespace fmmlib
