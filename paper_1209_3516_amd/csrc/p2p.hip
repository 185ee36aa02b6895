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
// of one stream).  Each lane sums in plain arithmetic over its share of one
// batch, or of ceil(K/8) consecutive batches when K > 8 (so a plain partial
// covers at least 64 sources when the share is small); that partial is then
// added with Kahan compensation (FP32), and the K streams and the chunks of
// a row are merged with the same compensation.
//
// Modes (compile time):
//   kCharges      sources are charges q: (phi, grad phi)
//   kDipoles      sources carry charges q and dipoles s; a dipole s at x_j
//                 has the potential s . (x_j - y) / |x_j - y|^3: (phi, grad phi)
//   kHessVec      sources are charges; each target i carries a vector v_i and
//                 gets the Hessian of the charge field applied to it,
//                 sum_j q_j (3 (d.v) d - r^2 v) / r^5, d = x_j - x_i: (0, H v)
// The per-target result is always a 4-vector, so the partial-sum layout and
// the merge are shared.
// ----------------------------------------------------------------------------
// Sources staged per batch.  With 384 the LDS of one wave (staged sources
// and run table, about 9 KB) lets a CU hold the sixteen waves (four per
// SIMD) that the FP32 charges kernel's registers allow.
constexpr int kNB = kP2PStageBatch;
static_assert(kNB % 64 == 0, "whole rows of 64 staged positions");

// An LDS pointer in the LDS address space, as global_load_lds takes it.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(3))) void *lds_ptr(T *p) {
  return (__attribute__((address_space(3))) void *)(p);
}

// Value of `v` in the lane whose byte address (4 * lane) is `addr`.
__device__ __forceinline__ float lane_shuffle(float v, int addr) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_shuffle(double v, int addr) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
static_assert(kP2PMaxRuns == 256, "LDS run table size");

// Staged positions of a batch -> source bodies: stage(off, nb, bi) gives
// lane l in bi[q] the body of position off + 64 q + l of the phase's source
// list, or 0 past nb (a lambda, so that the host pass of the compiler, which
// sees p2p_phase's LDS builtins, accepts the call).
constexpr int kStageRows = kNB / 64;

// An item's runs (in LDS): run r starts at position rp[r] and holds bodies
// from rp[r] + delta[r] on, so position c is body c + delta[run of c].  Per
// batch the starts of the runs that begin in it are flagged in a bit mask
// (one bit per staged position, 2 kStageRows words in LDS); lane l of row q
// then counts the flags at or below its position and adds the flags of the
// rows before and the run before the batch: its run, without a search.
// *nxt: the first run that starts at or after position off (0 at first).
__device__ __forceinline__ void stage_runs(const int32_t *rp, const int32_t *delta,
                                           uint32_t *mask, int n_runs, int &nxt, int off, int nb,
                                           int (&bi)[kStageRows]) {
  const int lane = threadIdx.x;
  if (lane < 2 * kStageRows) mask[lane] = 0u;
  __syncthreads();
  const int before = nxt - 1;  // the run of position off - 1 (-1 before the first)
  int cnt;
  do {  // flag up to 64 run starts at a time
    const int r = nxt + lane;
    const int pos = r < n_runs ? rp[r] - off : nb;
    const bool in = pos < nb;
    if (in) atomicOr(&mask[pos >> 5], 1u << (pos & 31));
    cnt = __popcll(__ballot(in));
    nxt += cnt;
  } while (cnt == 64);
  __syncthreads();
  const uint64_t upto_lane = __lanemask_lt() | __lanemask_eq();
  int seen = 0;
#pragma unroll
  for (int q = 0; q < kStageRows; ++q) {
    const uint64_t m = ((uint64_t)mask[2 * q + 1] << 32) | mask[2 * q];
    const int pos = q * 64 + lane;
    const int d = delta[before + seen + __popcll(m & upto_lane)];
    bi[q] = pos < nb ? off + pos + d : 0;
    seen += __popcll(m);
  }
}

template <typename Real, int MODE, int R, bool KAHAN, bool MASK, typename StageFn>
__device__ __forceinline__ void p2p_phase(int nsrc, StageFn stage,
                                          const typename Vec<Real>::V4 *__restrict__ bodies,
                                          const typename Vec<Real>::V4 *__restrict__ dipoles,
                                          typename Vec<Real>::V4 *src,
                                          typename Vec<Real>::V4 *srcd, int s, int K,
                                          const Real (&xi)[R], const Real (&yi)[R],
                                          const Real (&zi)[R], const Real (&vt)[R][3],
                                          Real (&S)[R][4], Real (&C)[R][4]) {
  using V4 = typename Vec<Real>::V4;
  const int lane = threadIdx.x;
  const Real far = Vec<Real>::kFar;
  // The plain partial of a stream is added into (S, C) every `kb` batches, so
  // that it covers at least 64 sources when a stream's share of one batch
  // (kNB / K) is smaller: kb = ceil(64 K / kNB).
  const int kb = (64 * K + kNB - 1) / kNB;
  Real p[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r) p[r][0] = p[r][1] = p[r][2] = p[r][3] = Real(0);
  // Far-away zero-charge bodies for the positions past a batch.  The row
  // after the kNB staged positions never holds a source, so it is padded once.
  auto pad = [&](int slot) {
    V4 fb;
    fb.x = far;
    fb.y = far;
    fb.z = far;
    fb.w = Real(0);
    src[slot] = fb;
    if constexpr (MODE == kDipoles) {
      V4 z;
      z.x = z.y = z.z = z.w = Real(0);
      srcd[slot] = z;
    }
  };
  pad(kNB + lane);
  int batch = 0;
  for (int off = 0; off < nsrc; off += kNB, ++batch) {
    const int nb = min(kNB, nsrc - off);
    // Staging.  FP32 bodies go from global memory straight into LDS
    // (global_load_lds_dwordx4: lane l's 16 bytes land at base + 16 l), all
    // loads of the batch in flight together and no registers held; positions
    // past the batch load body 0 and are then overwritten with far-away
    // zero-charge bodies.  FP64 bodies (32 bytes) are staged through
    // registers, with all indices computed and all loads issued before the
    // stores.
    constexpr int NL = kStageRows;  // positions that can hold sources
    int bi[NL];
    stage(off, nb, bi);
    if constexpr (sizeof(V4) == 16) {
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        __builtin_amdgcn_global_load_lds(static_cast<const void *>(bodies + bi[q]),
                                         lds_ptr(src + q * 64), 16, 0, 0);
        if constexpr (MODE == kDipoles)
          __builtin_amdgcn_global_load_lds(static_cast<const void *>(dipoles + bi[q]),
                                           lds_ptr(srcd + q * 64), 16, 0, 0);
      }
      __builtin_amdgcn_s_waitcnt(0);  // the LDS writes of the loads are done
    } else {
      V4 v[NL];
#pragma unroll
      for (int q = 0; q < NL; ++q) v[q] = bodies[bi[q]];
#pragma unroll
      for (int q = 0; q < NL; ++q) src[q * 64 + lane] = v[q];
      if constexpr (MODE == kDipoles) {
#pragma unroll
        for (int q = 0; q < NL; ++q) v[q] = dipoles[bi[q]];
#pragma unroll
        for (int q = 0; q < NL; ++q) srcd[q * 64 + lane] = v[q];
      }
    }
    if (nb < kNB) {  // a partial batch: pad its rows past nb
#pragma unroll
      for (int q = 0; q < NL; ++q)
        if (q * 64 + lane >= nb) pad(q * 64 + lane);
    }
    __syncthreads();
    const int iters = (nb + K - 1) / K;
#pragma unroll 2
    for (int j = 0; j < iters; ++j) {
      const V4 sj = src[s + K * j];
      V4 dj;
      if constexpr (MODE == kDipoles) dj = srcd[s + K * j];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const Real dx = sj.x - xi[r], dy = sj.y - yi[r], dz = sj.z - zi[r];
        const Real r2 = dx * dx + dy * dy + dz * dz;
        Real inv = rsqrt_(r2);
        if constexpr (MASK) inv = r2 > Real(0) ? inv : Real(0);
        if constexpr (MODE == kCharges) {
          const Real qr = sj.w * inv;
          const Real qr3 = qr * (inv * inv);
          p[r][0] += qr;
          p[r][1] += qr3 * dx;
          p[r][2] += qr3 * dy;
          p[r][3] += qr3 * dz;
        } else if constexpr (MODE == kDipoles) {
          const Real inv2 = inv * inv;
          const Real inv3 = inv * inv2;
          const Real sd3 = (dj.x * dx + dj.y * dy + dj.z * dz) * inv3;
          const Real t = sj.w * inv3 + Real(3) * sd3 * inv2;
          p[r][0] += sj.w * inv + sd3;
          p[r][1] += t * dx - dj.x * inv3;
          p[r][2] += t * dy - dj.y * inv3;
          p[r][3] += t * dz - dj.z * inv3;
        } else {
          // q/r^5 scales (d.v) and r^2 before they meet d and v: a padded
          // source (zero charge, far away) then gives exact zeros, where
          // (3 d.v) d - r^2 v alone would overflow to infinity and 0 * inf
          // would be NaN.
          const Real inv2 = inv * inv;
          const Real q5 = sj.w * (inv * inv2) * inv2;
          const Real a = q5 * (Real(3) * (dx * vt[r][0] + dy * vt[r][1] + dz * vt[r][2]));
          const Real b = q5 * r2;
          p[r][1] += a * dx - b * vt[r][0];
          p[r][2] += a * dy - b * vt[r][1];
          p[r][3] += a * dz - b * vt[r][2];
        }
      }
    }
    if (batch % kb == kb - 1 || off + kNB >= nsrc) {
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
          p[r][c] = Real(0);
        }
    }
    __syncthreads();
  }
}

// Merge the K streams (lanes s*L + u) into the lanes of stream 0 as a tree:
// while more than one stream is left, the upper ceil-half folds into the
// lower part (stream s takes stream s + h), with values moved across lanes by
// ds_bpermute.  log2(K) steps with every lane busy, no LDS buffer.  Stream 0
// then writes target u + L r of the item to slot out_off + u + L r.
template <typename Real, int R, bool KAHAN>
__device__ __forceinline__ void merge_streams_and_store(Real (&S)[R][4], Real (&C)[R][4], int s,
                                                        int K, int L, int nt, int32_t out_off,
                                                        typename Vec<Real>::V4 *__restrict__ out_s,
                                                        typename Vec<Real>::V4 *__restrict__ out_c) {
  using V4 = typename Vec<Real>::V4;
  const int lane = threadIdx.x;
  int kc = K;
  while (kc > 1) {
    const int h = (kc + 1) >> 1;
    const bool take = s < kc - h;
    const int from = (lane + h * L) << 2;  // byte address of the partner lane
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        // Sums and compensations are added separately: a stream's value is
        // S - C, and the log2(K) rounded additions of the tree are the only
        // ones left uncompensated.
        const Real vs = lane_shuffle(S[r][c], from);
        if constexpr (KAHAN) {
          const Real vc = lane_shuffle(C[r][c], from);
          if (take) {
            S[r][c] += vs;
            C[r][c] += vc;
          }
        } else {
          if (take) S[r][c] += vs;
        }
      }
    kc = h;
  }
  if (s == 0 && lane < L) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int t = lane + L * r;
      if (t < nt) {
        out_s[out_off + t] = V4{S[r][0], S[r][1], S[r][2], S[r][3]};
        if constexpr (KAHAN) out_c[out_off + t] = V4{C[r][0], C[r][1], C[r][2], C[r][3]};
      }
    }
  }
}

template <typename Real, int MODE, int R, bool KAHAN, bool MASK_ALL>
__device__ __forceinline__ void p2p_item(const P2PItem &it, const int32_t *__restrict__ run_body,
                                         const int32_t *__restrict__ run_prefix,
                                         const typename Vec<Real>::V4 *__restrict__ bodies,
                                         const typename Vec<Real>::V4 *__restrict__ vec,
                                         typename Vec<Real>::V4 *__restrict__ out_s,
                                         typename Vec<Real>::V4 *__restrict__ out_c,
                                         typename Vec<Real>::V4 *src,
                                         typename Vec<Real>::V4 *srcd, int32_t *delta,
                                         int32_t *rp, uint32_t *mask) {
  using V4 = typename Vec<Real>::V4;
  const int lane = threadIdx.x;
  const int nt = it.tgt_cfg & 0xff;
  const int L = (it.tgt_cfg >> 16) & 0xff;
  const int K = (it.tgt_cfg >> 24) & 0xff;
  int s = lane / L;
  const int u = lane - s * L;
  if (s >= K) s = K - 1;  // spare lanes repeat the last stream; not merged

  Real xi[R], yi[R], zi[R], vt[R][3];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = u + L * r;
    vt[r][0] = vt[r][1] = vt[r][2] = Real(0);
    if (t < nt) {
      const V4 b = bodies[it.tgt_begin + t];
      xi[r] = b.x;
      yi[r] = b.y;
      zi[r] = b.z;
      if constexpr (MODE == kHessVec) {
        const V4 v = vec[it.tgt_begin + t];
        vt[r][0] = v.x;
        vt[r][1] = v.y;
        vt[r][2] = v.z;
      }
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
    p2p_phase<Real, MODE, R, KAHAN, true>(
        it.self_n,
        [&](int off, int nb, int (&bi)[kStageRows]) {
#pragma unroll
          for (int q = 0; q < kStageRows; ++q) {
            const int pos = q * 64 + lane;
            bi[q] = pos < nb ? b0 + off + pos : 0;
          }
        },
        bodies, vec, src, srcd, s, K, xi, yi, zi, vt, S, C);
  }
  if (it.n_src > 0) {
    for (int r = lane; r < it.n_runs; r += 64) {
      const int32_t p0 = run_prefix[it.run_begin + r];
      rp[r] = p0;
      delta[r] = run_body[it.run_begin + r] - p0;
    }
    __syncthreads();
    int nxt = 0;
    const int n_runs = it.n_runs;
    p2p_phase<Real, MODE, R, KAHAN, MASK_ALL>(
        it.n_src,
        [&](int off, int nb, int (&bi)[kStageRows]) {
          stage_runs(rp, delta, mask, n_runs, nxt, off, nb, bi);
        },
        bodies, vec, src, srcd, s, K, xi, yi, zi, vt, S, C);
  }

  merge_streams_and_store<Real, R, KAHAN>(S, C, s, K, L, nt, it.out_off, out_s, out_c);
}

// One work item per wave, dispatched on its lane layout's R.
// vec: per-body dipoles (kDipoles) or per-target vectors (kHessVec), Morton order.
template <typename Real, int MODE, bool KAHAN, bool MASK_ALL, int MAXR>
__device__ __forceinline__ void p2p_wave(const P2PItem *__restrict__ items,
                                         const int32_t *__restrict__ order,
                                         const int32_t *__restrict__ run_body,
                                         const int32_t *__restrict__ run_prefix,
                                         const typename Vec<Real>::V4 *__restrict__ bodies,
                                         const typename Vec<Real>::V4 *__restrict__ vec,
                                         typename Vec<Real>::V4 *__restrict__ out_s,
                                         typename Vec<Real>::V4 *__restrict__ out_c) {
  using V4 = typename Vec<Real>::V4;
  __shared__ V4 src[kNB + 64];
  __shared__ V4 srcd[MODE == kDipoles ? kNB + 64 : 1];
  __shared__ int32_t delta[kP2PMaxRuns];
  __shared__ int32_t rp[kP2PMaxRuns];
  __shared__ uint32_t mask[2 * (kNB / 64)];
  const int64_t w = order ? order[blockIdx.x] : xcd_remap(blockIdx.x, gridDim.x);
  if (w < 0) return;  // padding of an ordered launch
  const P2PItem it = items[w];
  static_assert(kP2PMaxTargetsPerLane <= MAXR && MAXR <= 8, "a case for every R of the plan");
  switch ((it.tgt_cfg >> 8) & 0xff) {
#define FMM_P2P_CASE(RR)                                                                    \
  case RR:                                                                                  \
    if constexpr (RR <= MAXR)                                                               \
      p2p_item<Real, MODE, RR, KAHAN, MASK_ALL>(it, run_body, run_prefix, bodies, vec, out_s, \
                                                out_c, src, srcd, delta, rp, mask);          \
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

// The general kernel: every mode and precision.  Its code has a case for R
// up to 8 (the plan uses at most kP2PMaxTargetsPerLane), which in FP32
// charges mode gives about 168 registers, i.e. three waves per SIMD.
template <typename Real, int MODE, bool KAHAN, bool MASK_ALL>
__global__ __launch_bounds__(64) void p2p_kernel(const P2PItem *__restrict__ items,
                                                 const int32_t *__restrict__ order,
                                                 const int32_t *__restrict__ run_body,
                                                 const int32_t *__restrict__ run_prefix,
                                                 const typename Vec<Real>::V4 *__restrict__ bodies,
                                                 const typename Vec<Real>::V4 *__restrict__ vec,
                                                 typename Vec<Real>::V4 *__restrict__ out_s,
                                                 typename Vec<Real>::V4 *__restrict__ out_c) {
  p2p_wave<Real, MODE, KAHAN, MASK_ALL, 8>(items, order, run_body, run_prefix, bodies, vec,
                                           out_s, out_c);
}

// The FP32 charges kernel held to four waves per SIMD (at most 128
// registers per lane, cases R <= kP2PMaxTargetsPerLane only): with more
// waves in flight each batch's staging latency is better hidden (leaves of
// about ten bodies, whose sources are staged most often per pair, gain
// most).  Its waves leave too few registers for a far-field M2L wave of
// p = 5 or 6 (about 148) to start beside them, so for those orders the
// evaluation takes the general kernel, whose finished waves make room.
template <bool MASK_ALL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void p2p_kernel_w4(
    const P2PItem *__restrict__ items, const int32_t *__restrict__ order,
    const int32_t *__restrict__ run_body, const int32_t *__restrict__ run_prefix,
    const float4 *__restrict__ bodies, float4 *__restrict__ out_s, float4 *__restrict__ out_c) {
  p2p_wave<float, kCharges, true, MASK_ALL, kP2PMaxTargetsPerLane>(
      items, order, run_body, run_prefix, bodies, nullptr, out_s, out_c);
}

template <typename Real, int MODE>
void launch_p2p(bool mask_all, bool four_waves, unsigned G, hipStream_t st, const P2PItem *items,
                const int32_t *order, const int32_t *run_body, const int32_t *run_prefix, const void *bodies,
                const void *vec, void *part_s, void *part_c) {
  using V4 = typename Vec<Real>::V4;
  constexpr bool kahan = std::is_same<Real, float>::value;
  const V4 *b = (const V4 *)bodies;
  const V4 *v = (const V4 *)vec;
  if constexpr (std::is_same<Real, float>::value && MODE == kCharges) {
    if (four_waves) {
      if (mask_all)
        p2p_kernel_w4<true><<<G, 64, 0, st>>>(items, order, run_body, run_prefix, b,
                                              (V4 *)part_s, (V4 *)part_c);
      else
        p2p_kernel_w4<false><<<G, 64, 0, st>>>(items, order, run_body, run_prefix, b,
                                               (V4 *)part_s, (V4 *)part_c);
      return;
    }
  }
  if (mask_all)
    p2p_kernel<Real, MODE, kahan, true><<<G, 64, 0, st>>>(items, order, run_body, run_prefix,
                                                          b, v, (V4 *)part_s, (V4 *)part_c);
  else
    p2p_kernel<Real, MODE, kahan, false><<<G, 64, 0, st>>>(items, order, run_body, run_prefix,
                                                           b, v, (V4 *)part_s, (V4 *)part_c);
}

// ----------------------------------------------------------------------------
// Mutual P2P (charges, FP32).  One wave per item of the mutual plan: leaf A's
// nt <= 64 targets against its self pair (one-sided with the zero-distance
// mask, as above) and against the bodies of the leaves B > A of its row, each
// such pair of bodies evaluated once for both of them.
//
// The wave is four rows of 16 lanes.  Lane l holds targets l % TL + TL r
// (r < R), so a row holds 16 / TL copies of each target slot.  Staged sources
// are taken in rings of 16 (row w takes rings w, w + 4, ...).  At step k < TL
// lane u of a row evaluates its R targets against ring position (u - k) mod
// 16: the terms go into the targets' sums and into one sum that belongs to
// the source and travels with it, one lane up the row after every step (DPP
// row rotation).  The source at ring position q is at lane q + k at step k,
// so in TL steps it meets each target slot once; its finished sum (over all
// of A's targets, plain FP32) is then stored to its slot, and the combine
// adds it in.  The target sums are merged over rows and copies as in the
// one-sided kernel.
// ----------------------------------------------------------------------------

// Value of v in lane (u - 1) mod 16 of the same row of 16 lanes (row_ror:1).
__device__ __forceinline__ float row_rotate_up(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x121, 0xf, 0xf, false));
}

// The terms of one source sj and R targets: the targets' partial sums p gain
// q_j / r and q_j d / r^3 (d = x_j - x_i); (c0, c1, c2, c3) receive the
// source's q_i / r and -q_i d / r^3, summed over the R targets.
template <int R, bool MASK>
__device__ __forceinline__ void mutual_terms(const float4 &sj, const float (&xi)[R],
                                             const float (&yi)[R], const float (&zi)[R],
                                             const float (&qi)[R], float (&p)[R][4], float &c0,
                                             float &c1, float &c2, float &c3) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float dx = sj.x - xi[r], dy = sj.y - yi[r], dz = sj.z - zi[r];
    const float r2 = dx * dx + dy * dy + dz * dz;
    float inv = rsqrt_(r2);
    if constexpr (MASK) inv = r2 > 0.0f ? inv : 0.0f;
    const float inv3 = inv * inv * inv;
    p[r][0] += sj.w * inv;
    const float tq = sj.w * inv3;
    p[r][1] += tq * dx;
    p[r][2] += tq * dy;
    p[r][3] += tq * dz;
    const float ts = qi[r] * inv3;
    if (r == 0) {
      c0 = qi[r] * inv;
      c1 = -(ts * dx);
      c2 = -(ts * dy);
      c3 = -(ts * dz);
    } else {
      c0 += qi[r] * inv;
      c1 -= ts * dx;
      c2 -= ts * dy;
      c3 -= ts * dz;
    }
  }
}

// lookup(c, body, dst): body and source slot of source position c
// (positions only grow within a lane).
template <int R, bool MASK, typename LookupFn>
__device__ __forceinline__ void p2p_mutual_phase(int nsrc, LookupFn lookup,
                                                 const float4 *__restrict__ bodies,
                                                 float4 *__restrict__ part_m, float4 *src,
                                                 int32_t *sdst, int TL, const float (&xi)[R],
                                                 const float (&yi)[R], const float (&zi)[R],
                                                 const float (&qi)[R], float (&S)[R][4],
                                                 float (&C)[R][4]) {
  const int lane = threadIdx.x;
  const int u = lane & 15, row = lane >> 4;
  const float far = Vec<float>::kFar;
  constexpr int NL = kNB / 64;
  // A lane meets TL sources per ring, NL TL per batch: its plain partial is
  // folded into (S, C) once it covers at least 64.
  const int kb = (64 + NL * TL - 1) / (NL * TL);
  float p[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r) p[r][0] = p[r][1] = p[r][2] = p[r][3] = 0.0f;
  int batch = 0;
  for (int off = 0; off < nsrc; off += kNB, ++batch) {
    const int nb = min(kNB, nsrc - off);
    // Staging as in p2p_phase (bodies straight into LDS), plus each
    // position's slot; positions past the batch get far-away zero-charge
    // bodies and no slot.
    int bi[NL], di[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int pos = q * 64 + lane;
      bi[q] = 0;
      di[q] = -1;
      if (pos < nb) lookup(off + pos, bi[q], di[q]);
    }
#pragma unroll
    for (int q = 0; q < NL; ++q)
      __builtin_amdgcn_global_load_lds(static_cast<const void *>(bodies + bi[q]),
                                       lds_ptr(src + q * 64), 16, 0, 0);
#pragma unroll
    for (int q = 0; q < NL; ++q) sdst[q * 64 + lane] = di[q];
    __builtin_amdgcn_s_waitcnt(0);  // the LDS writes of the loads are done
    if (nb < kNB) {
#pragma unroll
      for (int q = 0; q < NL; ++q)
        if (q * 64 + lane >= nb) src[q * 64 + lane] = make_float4(far, far, far, 0.0f);
    }
    __syncthreads();
    const int nring = (nb + 15) >> 4;
    for (int g = row; g < nring; g += 4) {
      const float4 *ring = src + (g << 4);
      float a0, a1, a2, a3;
      mutual_terms<R, MASK>(ring[u], xi, yi, zi, qi, p, a0, a1, a2, a3);
      for (int k = 1; k < TL; ++k) {
        float c0, c1, c2, c3;
        mutual_terms<R, MASK>(ring[(u - k) & 15], xi, yi, zi, qi, p, c0, c1, c2, c3);
        a0 = row_rotate_up(a0) + c0;
        a1 = row_rotate_up(a1) + c1;
        a2 = row_rotate_up(a2) + c2;
        a3 = row_rotate_up(a3) + c3;
      }
      // this lane now holds the sum of ring position u - TL + 1
      const int d = sdst[(g << 4) + ((u - TL + 1) & 15)];
      if (d >= 0) part_m[d] = make_float4(a0, a1, a2, a3);
    }
    if (batch % kb == kb - 1 || off + kNB >= nsrc) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float y = p[r][c] - C[r][c];
          const float t = S[r][c] + y;
          C[r][c] = (t - S[r][c]) - y;
          S[r][c] = t;
          p[r][c] = 0.0f;
        }
    }
    __syncthreads();
  }
}

template <int R, bool MASK_ALL>
__device__ __forceinline__ void p2p_mutual_item(
    const P2PItem &it, const int32_t *__restrict__ run_body,
    const int32_t *__restrict__ run_prefix, const int32_t *__restrict__ run_dst,
    const float4 *__restrict__ bodies, float4 *__restrict__ out_s, float4 *__restrict__ out_c,
    float4 *__restrict__ part_m, float4 *src, int32_t *sdst, int32_t *rb, int32_t *rp,
    int32_t *rd) {
  const int lane = threadIdx.x;
  const int nt = it.tgt_cfg & 0xff;
  const int TL = (it.tgt_cfg >> 16) & 0xff;
  const int K = (it.tgt_cfg >> 24) & 0xff;  // 64 / TL copies of each target
  const int s = lane / TL;
  const int u = lane - s * TL;
  float xi[R], yi[R], zi[R], qi[R], vt[R][3];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = u + TL * r;
    vt[r][0] = vt[r][1] = vt[r][2] = 0.0f;
    if (t < nt) {
      const float4 b = bodies[it.tgt_begin + t];
      xi[r] = b.x;
      yi[r] = b.y;
      zi[r] = b.z;
      qi[r] = b.w;
    } else {
      xi[r] = yi[r] = zi[r] = -Vec<float>::kFar;
      qi[r] = 0.0f;
    }
  }
  float S[R][4], C[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) S[r][c] = C[r][c] = 0.0f;

  if (it.self_n > 0) {
    // copy s of the targets reads every K-th of A's bodies
    const int b0 = it.self_begin;
    p2p_phase<float, kCharges, R, true, true>(
        it.self_n,
        [&](int off, int nb, int (&bi)[kStageRows]) {
#pragma unroll
          for (int q = 0; q < kStageRows; ++q) {
            const int pos = q * 64 + lane;
            bi[q] = pos < nb ? b0 + off + pos : 0;
          }
        },
        bodies, nullptr, src, nullptr, s, K, xi, yi, zi, vt, S, C);
  }
  if (it.n_src > 0) {
    for (int r = lane; r < it.n_runs; r += 64) {
      rb[r] = run_body[it.run_begin + r];
      rp[r] = run_prefix[it.run_begin + r];
      rd[r] = run_dst[it.run_begin + r];
    }
    if (lane < 2) rp[it.n_runs + lane] = it.n_src;
    __syncthreads();
    int ri = 0, run_pos = rp[0], next_pos = rp[1];
    p2p_mutual_phase<R, MASK_ALL>(
        it.n_src,
        [&](int c, int &body, int &dst) {
          while (next_pos <= c) {
            ++ri;
            run_pos = next_pos;
            next_pos = rp[ri + 1];
          }
          body = rb[ri] + (c - run_pos);
          dst = rd[ri] + (c - run_pos);
        },
        bodies, part_m, src, sdst, TL, xi, yi, zi, qi, S, C);
  }
  merge_streams_and_store<float, R, true>(S, C, s, K, TL, nt, it.out_off, out_s, out_c);
}

template <bool MASK_ALL>
__global__ __launch_bounds__(64) void p2p_mutual_kernel(
    const P2PItem *__restrict__ items, const int32_t *__restrict__ run_body,
    const int32_t *__restrict__ run_prefix, const int32_t *__restrict__ run_dst,
    const float4 *__restrict__ bodies, float4 *__restrict__ out_s, float4 *__restrict__ out_c,
    float4 *__restrict__ part_m) {
  __shared__ float4 src[kNB + 64];
  __shared__ int32_t sdst[kNB];
  __shared__ int32_t rb[kP2PMaxRuns];
  __shared__ int32_t rp[kP2PMaxRuns + 2];
  __shared__ int32_t rd[kP2PMaxRuns];
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  const P2PItem it = items[w];
  switch ((it.tgt_cfg >> 8) & 0xff) {
#define FMM_P2PM_CASE(RR)                                                                   \
  case RR:                                                                                  \
    p2p_mutual_item<RR, MASK_ALL>(it, run_body, run_prefix, run_dst, bodies, out_s, out_c, \
                                  part_m, src, sdst, rb, rp, rd);                          \
    break;
    FMM_P2PM_CASE(1)
    FMM_P2PM_CASE(2)
    FMM_P2PM_CASE(3)
    FMM_P2PM_CASE(4)
    FMM_P2PM_CASE(5)
    FMM_P2PM_CASE(6)
    FMM_P2PM_CASE(7)
    FMM_P2PM_CASE(8)
#undef FMM_P2PM_CASE
    default:
      break;
  }
}

}  // namespace

int p2p(bool fp64, int mode, bool mask_all, bool four_waves, int64_t n_items,
        const P2PItem *items, const int32_t *order, int64_t n_order, const int32_t *run_body,
        const int32_t *run_prefix, const void *bodies, const void *vec, void *part_s,
        void *part_c, void *stream) {
  if (n_items == 0) return 0;
  const unsigned G = (unsigned)(order ? n_order : n_items);
  const hipStream_t st = S_(stream);
  auto go = [&](auto real, auto mode_c) {
    using R = decltype(real);
    constexpr int M = decltype(mode_c)::value;
    launch_p2p<R, M>(mask_all, four_waves, G, st, items, order, run_body, run_prefix, bodies,
                     vec, part_s, std::is_same<R, float>::value ? part_c : nullptr);
  };
  using IC = std::integral_constant<int, kCharges>;
  using ID = std::integral_constant<int, kDipoles>;
  using IH = std::integral_constant<int, kHessVec>;
  if (fp64) {
    if (mode == kCharges) go(0.0, IC{});
    else if (mode == kDipoles) go(0.0, ID{});
    else go(0.0, IH{});
  } else {
    if (mode == kCharges) go(0.0f, IC{});
    else if (mode == kDipoles) go(0.0f, ID{});
    else go(0.0f, IH{});
  }
  return (int)hipGetLastError();
}

int p2p_mutual(bool mask_all, int64_t n_items, const P2PItem *items, const int32_t *run_body,
               const int32_t *run_prefix, const int32_t *run_dst, const void *bodies,
               void *part_s, void *part_c, void *part_m, void *stream) {
  if (n_items == 0) return 0;
  const unsigned G = (unsigned)n_items;
  const hipStream_t st = S_(stream);
  const float4 *b = (const float4 *)bodies;
  if (mask_all)
    p2p_mutual_kernel<true><<<G, 64, 0, st>>>(items, run_body, run_prefix, run_dst, b,
                                              (float4 *)part_s, (float4 *)part_c,
                                              (float4 *)part_m);
  else
    p2p_mutual_kernel<false><<<G, 64, 0, st>>>(items, run_body, run_prefix, run_dst, b,
                                               (float4 *)part_s, (float4 *)part_c,
                                               (float4 *)part_m);
  return (int)hipGetLastError();
}

}  // namespace dev
}  // namespace fmmlib
