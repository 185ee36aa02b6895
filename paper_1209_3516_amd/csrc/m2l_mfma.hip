// Batched M2L on the matrix cores (box-centred trees).
//
// The harmonic-reduced M2L of far.hip is, per entry, L_k += sum_n K(R)_kn M_n
// over the p^2 reduced terms k, n (z exponent <= 1), with K(R)_kn =
// D^(n+k) G(R), G = 1/r, R = X_A - X_B.  For a box-centred tree R repeats, so
// the plan of m2l_plan.cpp groups the entries of 16 target cells by R; then
// one tile of reduced locals Lr[k][j] (k term, j target) takes
//   Lr += K(R) * [M of the 16 sources of the group]
// as a product of a (p^2 x p^2) matrix with a (p^2 x 16) one.  K(R) is zero
// where |n| + |k| > p - 1, so only the 16 x 4 blocks that hold a nonzero term
// are multiplied, each by one v_mfma_f32_16x16x4f32 (A: K block, 16 rows of
// k by 4 columns of n; B: the 4 n-terms of the 16 sources; C: 16 k-rows by
// 16 targets, in FP32).  The derivatives D(R) of every distinct vector are
// computed once, by the table kernel; the group's D(R) row and the folded
// multipoles of its sources are staged in LDS, and each lane gathers its A
// and B elements from there.  After the last group the reduced locals are
// expanded to all terms (the linear map of the harmonic identities) and
// written; a target without entries gets zeros.
#include "device_common.h"

namespace fmmlib {
namespace dev {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// Nonzero (row block, column block) pairs of K for order P and, per pair and
// lane, the full-term index of the D element that lane supplies to the A
// operand (-1: zero).  Operand layout of v_mfma_f32_16x16x4f32: lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; it holds C[4 (l / 16) +
// v][l % 16] in component v of its accumulator.
template <int P>
struct MfmaPairs {
  static constexpr int TR = rterms(P);
  static constexpr int RT = (TR + 15) / 16;  // 16-row blocks of k
  static constexpr int KC = (TR + 3) / 4;    // 4-column blocks of n
  int n;
  int rt[RT * KC], kc[RT * KC];
  short idx[RT * KC][64];
  constexpr MfmaPairs() : n(0), rt(), kc(), idx() {
    int rx[TR] = {}, ry[TR] = {}, rz[TR] = {};
    for (int d = 0; d < P; ++d)
      for (int c = 0; c <= 1 && c <= d; ++c)
        for (int b = 0; b <= d - c; ++b) {
          const int r = rterm_index(P, d - b - c, b, c);
          rx[r] = d - b - c;
          ry[r] = b;
          rz[r] = c;
        }
    for (int r = 0; r < RT; ++r)
      for (int c = 0; c < KC; ++c) {
        short tmp[64] = {};
        bool any = false;
        for (int lane = 0; lane < 64; ++lane) {
          const int k = 16 * r + lane % 16, nn = 4 * c + lane / 16;
          int s = -1;
          if (k < TR && nn < TR) s = term_index(P, rx[k] + rx[nn], ry[k] + ry[nn], rz[k] + rz[nn]);
          tmp[lane] = (short)s;
          any = any || s >= 0;
        }
        if (!any) continue;
        rt[n] = r;
        kc[n] = c;
        for (int lane = 0; lane < 64; ++lane) idx[n][lane] = tmp[lane];
        ++n;
      }
  }
};
template <int P>
inline constexpr MfmaPairs<P> kMfma{};
template <int P>
__device__ const MfmaPairs<P> kMfmaDev = kMfma<P>;

// D^m G(R) for every distinct vector (the terms of z exponent <= 2, with the
// recurrence M2L uses; the others are never read and are stored as zeros):
// one thread each.
template <int P>
__global__ __launch_bounds__(256) void m2l_offsets_kernel(int64_t n_off,
                                                          const double *__restrict__ off,
                                                          float *__restrict__ dtab) {
  constexpr int T = nterms(P);
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_off) return;
  float D[T];
  static_for<T>([&](auto I) { D[decltype(I)::value] = 0.0f; });
  derivatives<P, float, true>((float)off[3 * o], (float)off[3 * o + 1], (float)off[3 * o + 2], D);
  static_for<T>([&](auto I) {
    constexpr int t = decltype(I)::value;
    dtab[o * T + t] = kBasis<P>.ez[t] <= 2 ? D[t] : 0.0f;
  });
}

// Four waves per tile: wave w takes the groups w, w + 4, ... of the tile,
// each with its own LDS staging, and the four partial tiles of locals are
// added in wave order at the end.
constexpr int kMfmaWaves = 4;

template <int P>
__global__ __launch_bounds__(64 * kMfmaWaves) void m2l_mfma_kernel(
    int64_t tile0, const int32_t *__restrict__ tile_cells,
    const int64_t *__restrict__ tile_group_begin, const int32_t *__restrict__ group_offset,
    const int32_t *__restrict__ group_src, const float *__restrict__ dtab,
    const float *__restrict__ Mr, float *__restrict__ L) {
  constexpr int T = nterms(P), S = pad4(T), TR = rterms(P), SR = pad4(TR);
  constexpr int RT = MfmaPairs<P>::RT;
  constexpr int NP = kMfma<P>.n;
  constexpr int MS = SR + 1;                       // LDS row stride of the staged multipoles
  constexpr int DL = (T + 63) / 64;                // D elements per lane
  constexpr int ML = (16 * (SR / 4) + 63) / 64;    // multipole float4 loads per lane
  constexpr int LS = TR + 1;                       // LDS row stride of the reduced locals
  __shared__ float Ds[kMfmaWaves][DL * 64];
  __shared__ float Ms[kMfmaWaves][16 * MS];
  __shared__ float Lf[kMfmaWaves][16 * LS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t tile = tile0 + blockIdx.x;
  const int j = lane % 16, q4 = lane / 16;
  // this lane's D indices for every nonzero block of K
  short aidx[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) aidx[q] = kMfmaDev<P>.idx[q][lane];
  v4f acc[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) acc[r] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  const int64_t g0 = tile_group_begin[tile], g1 = tile_group_begin[tile + 1];
  const int64_t rounds = (g1 - g0 + kMfmaWaves - 1) / kMfmaWaves;
  // one group's D(R) row and source multipoles, held in registers so that
  // the next group's loads are in flight while this group is multiplied
  float dreg[DL];
  float4 mreg[ML];
  auto load_group = [&](int64_t g) {
    const bool in = g < g1;
    const float *drow = dtab + (int64_t)(in ? group_offset[g] : 0) * T;
#pragma unroll
    for (int i = 0; i < DL; ++i) {
      const int t = lane + 64 * i;
      dreg[i] = in && t < T ? drow[t] : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < ML; ++i) {
      const int e = lane + 64 * i;  // (source jj, 4-term column c4)
      const int jj = e / (SR / 4), c4 = e % (SR / 4);
      mreg[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (in && e < 16 * (SR / 4)) {
        const int32_t src = group_src[g * 16 + jj];
        if (src >= 0) mreg[i] = *reinterpret_cast<const float4 *>(Mr + (int64_t)src * SR + 4 * c4);
      }
    }
  };
  float *ds = Ds[wave], *ms = Ms[wave];
  if (rounds > 0) load_group(g0 + wave);
  for (int64_t k = 0; k < rounds; ++k) {
    const int64_t g = g0 + wave + kMfmaWaves * k;
    __syncthreads();  // the previous round's LDS reads are done
#pragma unroll
    for (int i = 0; i < DL; ++i) ds[lane + 64 * i] = dreg[i];
#pragma unroll
    for (int i = 0; i < ML; ++i) {
      const int e = lane + 64 * i;
      if (e < 16 * (SR / 4)) {
        float *m = ms + (e / (SR / 4)) * MS + 4 * (e % (SR / 4));
        m[0] = mreg[i].x;
        m[1] = mreg[i].y;
        m[2] = mreg[i].z;
        m[3] = mreg[i].w;
      }
    }
    __syncthreads();
    if (k + 1 < rounds) load_group(g + kMfmaWaves);
    if (g < g1) {
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int s = aidx[q];
        const float a = s >= 0 ? ds[s] : 0.0f;
        const float b = ms[j * MS + 4 * kMfma<P>.kc[q] + q4];
        acc[kMfma<P>.rt[q]] =
            __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[kMfma<P>.rt[q]], 0, 0, 0);
      }
    }
  }
  // the waves' reduced locals -> LDS, summed in wave order, then expanded to
  // all terms one term at a time (the pairs of the identities come in
  // ascending term)
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = 16 * r + 4 * q4 + v;
      if (k < TR) Lf[wave][j * LS + k] = acc[r][v];
    }
  __syncthreads();
  for (int i = threadIdx.x; i < 16 * LS; i += 64 * kMfmaWaves) {
    float sum = Lf[0][i];
#pragma unroll
    for (int w = 1; w < kMfmaWaves; ++w) sum += Lf[w][i];
    Lf[0][i] = sum;
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    const int32_t cell = tile_cells[tile * 16 + threadIdx.x];
    if (cell >= 0) {
      const float *red = Lf[0] + threadIdx.x * LS;
      float *out = L + (int64_t)cell * S;
      float cur = 0.0f;
      harmonic_pairs<P>([&](auto t, auto r, auto w, auto first) {
        constexpr int tt = decltype(t)::value, rr = decltype(r)::value, ww = decltype(w)::value;
        if constexpr (decltype(first)::value && tt > 0) out[tt - 1] = cur;
        const float v = ww == 1 ? red[rr] : (ww == -1 ? -red[rr] : float(ww) * red[rr]);
        if constexpr (decltype(first)::value) cur = v;
        else cur += v;
      });
      out[T - 1] = cur;
    }
  }
}

}  // namespace

int m2l_offsets(int p, int64_t n_off, const double *off, float *dtab, void *stream) {
  if (n_off <= 0) return 0;
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    m2l_offsets_kernel<PP><<<blocks_for(n_off, 256), 256, 0, S_(stream)>>>(n_off, off, dtab);
  });
}

int m2l_mfma(int p, int64_t tile0, int64_t tile1, const int32_t *tile_cells,
             const int64_t *tile_group_begin, const int32_t *group_offset,
             const int32_t *group_src, const float *dtab, const float *Mr, float *L,
             void *stream) {
  if (tile1 <= tile0) return 0;
  return with_p(p, [&](auto PC) {
    constexpr int PP = decltype(PC)::value;
    m2l_mfma_kernel<PP><<<(unsigned)(tile1 - tile0), 64 * kMfmaWaves, 0, S_(stream)>>>(
        tile0, tile_cells, tile_group_begin, group_offset, group_src, dtab, Mr, L);
  });
}

}  // namespace dev
}  // namespace fmmlib
