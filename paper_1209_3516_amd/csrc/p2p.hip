// P2P (near field) kernel of the gfx950 FMM.
#include "device_common.h"

namespace fmmlib {
namespace dev {
namespace {

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

}  // namespace

#define FMM_LAUNCH_CHECK() return (int)hipGetLastError()

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

}  // namespace dev
}  // namespace fmmlib
