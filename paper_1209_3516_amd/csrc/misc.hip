// Small kernels of the gfx950 FMM: charge gather, backward combine, FP64
// direct sum.
#include "device_common.h"

namespace fmmlib {
namespace dev {
namespace {

// ----------------------------------------------------------------------------
// Charges into Morton order: bodies[i].w = q[perm[i]].
// ----------------------------------------------------------------------------
template <typename Real>
__global__ void gather_kernel(int64_t n, const int32_t *__restrict__ perm,
                              const Real *__restrict__ q, typename Vec<Real>::V4 *bodies) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) bodies[i].w = q[perm[i]];
}

// Per-body vectors into Morton order: out[i] = sign * v[perm[i]], w = 0.
template <typename Real>
__global__ void gather_vec_kernel(int64_t n, const int32_t *__restrict__ perm,
                                  const Real *__restrict__ v, Real sign,
                                  typename Vec<Real>::V4 *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t u = perm[i];
  typename Vec<Real>::V4 o;
  o.x = sign * v[3 * u];
  o.y = sign * v[3 * u + 1];
  o.z = sign * v[3 * u + 2];
  o.w = Real(0);
  out[i] = o;
}

// dL/dx = w * grad[q] + q * grad[w] (+ H[q] v), user order.
template <typename Real>
__global__ void backward_combine_kernel(int64_t n, const Real *__restrict__ q,
                                        const Real *__restrict__ w, const Real *__restrict__ gq,
                                        const Real *__restrict__ gw, const Real *__restrict__ hv,
                                        Real *__restrict__ dx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Real qi = q[i], wi = w[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    Real v = wi * gq[3 * i + d] + qi * gw[3 * i + d];
    if (hv) v += hv[3 * i + d];
    dx[3 * i + d] = v;
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

}  // namespace

#define FMM_LAUNCH_CHECK() return (int)hipGetLastError()

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

int gather_vectors(bool fp64, int64_t n, const int32_t *perm, const void *v_user, double sign,
                   void *out, void *stream) {
  if (n == 0) return 0;
  if (fp64)
    gather_vec_kernel<double><<<blocks_for(n, 256), 256, 0, S_(stream)>>>(
        n, perm, (const double *)v_user, sign, (double4 *)out);
  else
    gather_vec_kernel<float><<<blocks_for(n, 256), 256, 0, S_(stream)>>>(
        n, perm, (const float *)v_user, (float)sign, (float4 *)out);
  FMM_LAUNCH_CHECK();
}

int backward_combine(bool fp64, int64_t n, const void *q, const void *w, const void *grad_q,
                     const void *grad_w, const void *hv, void *dx, void *stream) {
  if (n == 0) return 0;
  if (fp64)
    backward_combine_kernel<double><<<blocks_for(n, 256), 256, 0, S_(stream)>>>(
        n, (const double *)q, (const double *)w, (const double *)grad_q, (const double *)grad_w,
        (const double *)hv, (double *)dx);
  else
    backward_combine_kernel<float><<<blocks_for(n, 256), 256, 0, S_(stream)>>>(
        n, (const float *)q, (const float *)w, (const float *)grad_q, (const float *)grad_w,
        (const float *)hv, (float *)dx);
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
