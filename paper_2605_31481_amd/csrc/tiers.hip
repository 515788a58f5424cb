// Result tiers of a workspace (the lazily materialised state of Sec. 3.1,
// extended to dynamics results): strided copies between a caller's array and
// a tier, and inverse dynamics from cached tiers,
//   tau = M(q) qdd + b(q, qd),   b = RNEA(q, qd, 0),
// which holds because RNEA is affine in qdd with slope M(q) (the mass matrix
// CRBA computes).  Tiers are instance-minor rows with stride `ld` (the
// workspace's batch capacity).  All three kernels read each tier element once
// and are bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace bard {

// Row k of the K rows is blockIdx.y; lanes run over instances, so both sides
// are read and written in instance-contiguous runs when their instance stride
// is 1.
template <class Real>
__global__ void __launch_bounds__(256) tier_copy_kernel(const Real* __restrict__ src, int64_t s_b, int64_t s_k,
                                                        Real* __restrict__ dst, int64_t d_b, int64_t d_k,
                                                        int64_t B) {
  const int64_t k = blockIdx.y;
  for (int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x; b < B; b += (int64_t)gridDim.x * 256)
    dst[b * d_b + k * d_k] = src[b * s_b + k * s_k];
}

// tau[a] = b[a] + sum_{d = 0..nv-1} M[a][d] qdd[d], summed in that order.
template <class Real>
__global__ void __launch_bounds__(256) tier_matvec_kernel(const Real* __restrict__ Mt, const Real* __restrict__ bt,
                                                          int64_t ld, const Real* __restrict__ qdd, int64_t sq_b,
                                                          int64_t sq_k, Real* __restrict__ tau, int64_t st_b,
                                                          int64_t st_k, int nv, int64_t B) {
  const int a = blockIdx.y;
  for (int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x; b < B; b += (int64_t)gridDim.x * 256) {
    Real acc = bt[(int64_t)a * ld + b];
    const Real* mr = Mt + (int64_t)a * nv * ld + b;
    const Real* qr = qdd + b * sq_b;
    for (int d = 0; d < nv; ++d) acc += mr[(int64_t)d * ld] * qr[(int64_t)d * sq_k];
    tau[b * st_b + (int64_t)a * st_k] = acc;
  }
}

static dim3 tier_grid(int64_t B, int rows) {
  int64_t gx = (B + 255) / 256;
  if (gx > 256) gx = 256;
  return dim3((unsigned)gx, (unsigned)rows);
}

template <class Real>
hipError_t launch_tier_copy(const Real* src, int64_t s_b, int64_t s_k, Real* dst, int64_t d_b, int64_t d_k, int rows,
                            int64_t B, hipStream_t st) {
  if (rows < 1 || rows > 65535 || B < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((tier_copy_kernel<Real>), tier_grid(B, rows), dim3(256), 0, st, src, s_b, s_k, dst, d_b, d_k, B);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_tier_matvec(const Real* Mt, const Real* bt, int64_t ld, const Real* qdd, int64_t sq_b, int64_t sq_k,
                              Real* tau, int64_t st_b, int64_t st_k, int nv, int64_t B, hipStream_t st) {
  if (nv < 1 || nv > 65535 || B < 1 || B > ld) return hipErrorInvalidValue;
  hipLaunchKernelGGL((tier_matvec_kernel<Real>), tier_grid(B, nv), dim3(256), 0, st, Mt, bt, ld, qdd, sq_b, sq_k, tau,
                     st_b, st_k, nv, B);
  return hipGetLastError();
}

template hipError_t launch_tier_copy<float>(const float*, int64_t, int64_t, float*, int64_t, int64_t, int, int64_t,
                                            hipStream_t);
template hipError_t launch_tier_copy<double>(const double*, int64_t, int64_t, double*, int64_t, int64_t, int, int64_t,
                                             hipStream_t);
template hipError_t launch_tier_matvec<float>(const float*, const float*, int64_t, const float*, int64_t, int64_t,
                                              float*, int64_t, int64_t, int, int64_t, hipStream_t);
template hipError_t launch_tier_matvec<double>(const double*, const double*, int64_t, const double*, int64_t, int64_t,
                                               double*, int64_t, int64_t, int, int64_t, hipStream_t);

}  // namespace bard
