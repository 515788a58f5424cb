// Standalone kinematics of one chain: Sec. 3.1 provides FK and Jacobian
// functions for a single root-to-end-effector chain that visit only that
// path and fill no cache.  One lane per instance walks the path with the
// joint transforms of eqs. (4)-(5) and writes the end effector's world pose
// and the Jacobian columns of eq. (7) for the joints on the path; further
// workgroup rows of the same launch store the zero columns of the joints off
// the path, so the instance lanes write only what the path computes.
//
// Columns ([linear; angular], world axes): a revolute joint with world axis
// w through the point p contributes [p x w; w] at the world origin
// (BARD_WORLD) and [w x (p_e - p); w] at the end effector's origin p_e
// (BARD_LOCAL_WORLD_ALIGNED); a prismatic joint [u; 0]; a free root its
// body-frame translation axes [R e_k; 0] and rotation axes as revolute
// columns.  The end-effector point form needs p_e before the first column,
// so that frame walks the path twice (poses only, then columns); the
// arithmetic of the walk is a few hundred operations per body against
// 6 nv output values, so at large batches the kernel is bound by its stores
// and at small ones by the latency of one memory round trip.
#include <hip/hip_runtime.h>

#include "device.h"
#include "launch.h"

namespace bard {

namespace {

constexpr int kPathThreads = 64;  // one wave per workgroup: many workgroups at small batches
constexpr int kZeroCols = 4;      // zero columns per workgroup row
constexpr int kPathCst = 36;      // R0, A, B, t0, axis, d of a body (the first 36 constants)

// World pose of a body from its parent's (Rw, pw), in place; c its
// constants, qv its coordinates (7 for a free root).
template <class Real>
__device__ __forceinline__ void path_step(const Real* c, int jt, const Real* qv, Real* Rw, Real* pw) {
  if (jt == J_FREE) {
    const Real qf[7] = {qv[0], qv[64], qv[128], qv[192], qv[256], qv[320], qv[384]};
    free_root_pose(c, qf, Rw, pw);
    return;
  }
  Real Rpc[9], tpc[3], Rn[9];
  joint_transform(c, qv[0], Rpc, tpc);
  mul33(Rw, Rpc, Rn);
#pragma unroll
  for (int i = 0; i < 3; ++i) pw[i] += Rw[3 * i] * tpc[0] + Rw[3 * i + 1] * tpc[1] + Rw[3 * i + 2] * tpc[2];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rw[k] = Rn[k];
}

template <class Real>
__device__ __forceinline__ void store_col(Real* Jb, int64_t sJ_k, int nv, int col, const Real* lin, const Real* ang) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    Jb[(int64_t)(r * nv + col) * sJ_k] = lin[r];
    Jb[(int64_t)((3 + r) * nv + col) * sJ_k] = ang[r];
  }
}

// The linear part of a rotation column about the point p for the chosen frame.
template <bool LWA, class Real>
__device__ __forceinline__ void rot_lin(const Real* w, const Real* p, const Real* pe, Real* lin) {
  if (LWA) {
    const Real d[3] = {pe[0] - p[0], pe[1] - p[1], pe[2] - p[2]};
    cross3(w, d, lin);
  } else {
    cross3(p, w, lin);
  }
}

// Dynamic LDS: the path's constants (len x 36) and joint types, then each
// lane's path coordinates (nqp x 64, lane-minor).  The constants are read at
// wave-uniform addresses (broadcast); every load of the walk is issued before
// the walk starts, so a workgroup waits for one memory round trip.
template <class Real, bool LWA>
__global__ void __launch_bounds__(kPathThreads) path_kernel(DevModel dm, PathArgs<Real> a) {
  const int tid = threadIdx.x;
  const int64_t b = (int64_t)blockIdx.x * kPathThreads + tid;
  const bool live = b < a.B;
  const int nv = dm.nv;
  if (blockIdx.y > 0) {  // zero columns of the joints off the path
    if (!live) return;
    Real* Jb = a.J + b * a.sJ_b;
    const int c0 = (blockIdx.y - 1) * kZeroCols, c1 = min(c0 + kZeroCols, a.n_zero);
    for (int z = c0; z < c1; ++z)
#pragma unroll
      for (int r = 0; r < 6; ++r) Jb[(int64_t)(r * nv + a.zcol[z]) * a.sJ_k] = Real(0);
    return;
  }
  extern __shared__ __align__(16) unsigned char path_lds[];
  Real* cs = reinterpret_cast<Real*>(path_lds);
  Real* qs = cs + a.len * kPathCst;
  int* jts = reinterpret_cast<int*>(qs + a.nqp * kPathThreads);
  const unsigned char* img = image<Real>(dm);
  const TabLayout tl = tab_layout(dm.n, dm.P, dm.depth, dm.kmax, dm.nv, (int)sizeof(Real));
  const Real* cst = reinterpret_cast<const Real*>(img + tl.cst);
  const I4* meta = reinterpret_cast<const I4*>(img + tl.meta);
  const int64_t bc = live ? b : a.B - 1;
  const Real* qb = a.q + bc * a.sq_b;
  // Loads in batches of kBatch issued before their LDS stores: a loop of
  // load-then-store waits one memory round trip per element.
  constexpr int kBatch = 16;
  for (int k0 = 0; k0 < a.nqp; k0 += kBatch) {
    Real v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) v[j] = qb[(int64_t)a.qsrc[min(k0 + j, a.nqp - 1)] * a.sq_k];
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (k0 + j < a.nqp) qs[(k0 + j) * kPathThreads + tid] = v[j];
  }
  const int ncs = a.len * kPathCst;
  for (int i0 = tid; i0 < ncs; i0 += kBatch * kPathThreads) {
    Real v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int i = min(i0 + j * kPathThreads, ncs - 1), s = i / kPathCst;
      v[j] = cst[a.body[s] * CST + (i - s * kPathCst)];
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (i0 + j * kPathThreads < ncs) cs[i0 + j * kPathThreads] = v[j];
  }
  if (tid < a.len) jts[tid] = meta[a.body[tid]].y;
  __syncthreads();

  Real pe[3] = {Real(0), Real(0), Real(0)};
  Real Rw[9], pw[3];
  auto reset = [&]() {
#pragma unroll
    for (int k = 0; k < 9; ++k) Rw[k] = (k % 4 == 0) ? Real(1) : Real(0);
    pw[0] = pw[1] = pw[2] = Real(0);
  };
  if (LWA && a.J) {  // first walk: the end effector's origin
    reset();
    for (int s = 0, qo = 0; s < a.len; ++s) {
      const int jt = jts[s];
      path_step(cs + s * kPathCst, jt, qs + qo * kPathThreads + tid, Rw, pw);
      qo += jt == J_FREE ? 7 : 1;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) pe[k] = pw[k];
  }
  reset();
  Real* Jb = a.J ? a.J + bc * a.sJ_b : nullptr;
  for (int s = 0, qo = 0; s < a.len; ++s) {
    const Real* c = cs + s * kPathCst;
    const int jt = jts[s];
    path_step(c, jt, qs + qo * kPathThreads + tid, Rw, pw);
    qo += jt == J_FREE ? 7 : 1;
    if (!Jb || !live) continue;
    const int v0 = a.vcol[s];
    const Real zero[3] = {Real(0), Real(0), Real(0)};
    if (jt == J_FREE) {
      for (int e = 0; e < 3; ++e) {
        const Real u[3] = {Rw[e], Rw[3 + e], Rw[6 + e]};
        store_col(Jb, a.sJ_k, nv, v0 + e, u, zero);
        Real lin[3];
        rot_lin<LWA>(u, pw, pe, lin);
        store_col(Jb, a.sJ_k, nv, v0 + 3 + e, lin, u);
      }
      continue;
    }
    const Real* ax = c + C_AX;
    Real u[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) u[i] = Rw[3 * i] * ax[0] + Rw[3 * i + 1] * ax[1] + Rw[3 * i + 2] * ax[2];
    if (jt == J_PRI) {
      store_col(Jb, a.sJ_k, nv, v0, u, zero);
    } else {
      Real lin[3];
      rot_lin<LWA>(u, pw, pe, lin);
      store_col(Jb, a.sJ_k, nv, v0, lin, u);
    }
  }
  if (a.pose && live) {
    Real* po = a.pose + b * a.sp_b;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int k = 0; k < 3; ++k) po[(int64_t)(4 * r + k) * a.sp_k] = Rw[3 * r + k];
      po[(int64_t)(4 * r + 3) * a.sp_k] = pw[r];
    }
  }
}

// ---- lane-parallel form: L = 4 or 16 lanes per instance ----
//
// At small batches one lane per instance leaves most of the device idle and
// the walk's serial chain sets the time.  Here the L lanes of an instance
// each take a segment of `seg` consecutive path bodies: every lane forms its
// joints' transforms (eqs. (4)-(5)) and their product, the lanes combine the
// products by an inclusive scan (log2 L steps of a rigid-transform product
// with the lane 1, 2, 4, ... below), each lane re-composes its segment from
// the pose the scan gives its predecessor and writes its joints' columns;
// the lanes also share the zero columns.  Fewer lanes per instance keep the
// stores of more instances in one wave contiguous (16 instances per wave at
// L = 4); more lanes shorten the serial part on long paths.
constexpr int kParSeg = 4;  // bodies per lane at most (L = 16: paths of up to 64 bodies)

// (Ra, pa) o (Rb, pb) -> (Ro, po): Ro = Ra Rb, po = Ra pb + pa.
template <class Real>
__device__ __forceinline__ void xf_mul(const Real* Ra, const Real* pa, const Real* Rb, const Real* pb, Real* Ro,
                                       Real* po) {
  Real R[9], p[3];
  mul33(Ra, Rb, R);
#pragma unroll
  for (int i = 0; i < 3; ++i) p[i] = Ra[3 * i] * pb[0] + Ra[3 * i + 1] * pb[1] + Ra[3 * i + 2] * pb[2] + pa[i];
#pragma unroll
  for (int k = 0; k < 9; ++k) Ro[k] = R[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) po[k] = p[k];
}

template <class Real>
__device__ __forceinline__ void xf_identity(Real* R, Real* p) {
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? Real(1) : Real(0);
  p[0] = p[1] = p[2] = Real(0);
}

template <class Real, bool LWA, int kParLanes>
__global__ void __launch_bounds__(kPathThreads) path_par_kernel(DevModel dm, PathArgs<Real> a) {
  const int tid = threadIdx.x;
  const int lane = tid & (kParLanes - 1);
  const int64_t b = (int64_t)blockIdx.x * (kPathThreads / kParLanes) + (tid / kParLanes);
  const bool live = b < a.B;
  const int64_t bc = live ? b : a.B - 1;
  const int nv = dm.nv;
  extern __shared__ __align__(16) unsigned char path_lds[];
  Real* cs = reinterpret_cast<Real*>(path_lds);
  int* jts = reinterpret_cast<int*>(cs + a.len * kPathCst);
  int* qis = jts + a.len;
  const unsigned char* img = image<Real>(dm);
  const TabLayout tl = tab_layout(dm.n, dm.P, dm.depth, dm.kmax, dm.nv, (int)sizeof(Real));
  const Real* cst = reinterpret_cast<const Real*>(img + tl.cst);
  const I4* meta = reinterpret_cast<const I4*>(img + tl.meta);
  constexpr int kBatch = 16;
  const int ncs = a.len * kPathCst;
  for (int i0 = tid; i0 < ncs; i0 += kBatch * kPathThreads) {
    Real v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int i = min(i0 + j * kPathThreads, ncs - 1), s = i / kPathCst;
      v[j] = cst[a.body[s] * CST + (i - s * kPathCst)];
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
      if (i0 + j * kPathThreads < ncs) cs[i0 + j * kPathThreads] = v[j];
  }
  if (tid < a.len) {
    const I4 mt = meta[a.body[tid]];
    jts[tid] = mt.y;
    qis[tid] = mt.z;
  }
  __syncthreads();

  // this lane's segment [s0, s1) of the path
  const int s0 = min(lane * a.seg, a.len), s1 = min(s0 + a.seg, a.len);
  const Real* qb = a.q + bc * a.sq_b;
  // coordinates of the segment's joints, all loads issued first
  Real qv[kParSeg][7];
#pragma unroll
  for (int j = 0; j < kParSeg; ++j) {
    const int s = min(s0 + j, a.len - 1);
    const int nq = jts[s] == J_FREE ? 7 : 1;
#pragma unroll
    for (int k = 0; k < 7; ++k) qv[j][k] = qb[(int64_t)(qis[s] + (k < nq ? k : 0)) * a.sq_k];
  }
  // the segment's joint transforms and their product G
  Real TR[kParSeg][9], Tp[kParSeg][3], GR[9], Gp[3];
  xf_identity(GR, Gp);
#pragma unroll
  for (int j = 0; j < kParSeg; ++j) {
    const int s = s0 + j;
    if (s < s1) {
      const Real* c = cs + s * kPathCst;
      if (jts[s] == J_FREE) {
        free_root_pose(c, qv[j], TR[j], Tp[j]);
      } else {
        joint_transform(c, qv[j][0], TR[j], Tp[j]);
      }
      xf_mul(GR, Gp, TR[j], Tp[j], GR, Gp);
    }
  }
  // inclusive scan over the 16 lanes: P_l = G_0 o ... o G_l
#pragma unroll
  for (int d = 1; d < kParLanes; d <<= 1) {
    Real oR[9], op[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) oR[k] = __shfl_up(GR[k], d, kParLanes);
#pragma unroll
    for (int k = 0; k < 3; ++k) op[k] = __shfl_up(Gp[k], d, kParLanes);
    if (lane >= d) xf_mul(oR, op, GR, Gp, GR, Gp);
  }
  // the pose before this segment: the predecessor's product (identity for lane 0)
  Real R[9], pw[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = __shfl_up(GR[k], 1, kParLanes);
#pragma unroll
  for (int k = 0; k < 3; ++k) pw[k] = __shfl_up(Gp[k], 1, kParLanes);
  if (lane == 0) xf_identity(R, pw);
  // the end effector's origin: the product of the lane holding the last body
  const int last = (a.len - 1) / a.seg;
  Real pe[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) pe[k] = __shfl(Gp[k], last, kParLanes);
  Real* Jb = (a.J && live) ? a.J + b * a.sJ_b : nullptr;
  const Real zero[3] = {Real(0), Real(0), Real(0)};
#pragma unroll
  for (int j = 0; j < kParSeg; ++j) {
    const int s = s0 + j;
    if (s >= s1) continue;
    xf_mul(R, pw, TR[j], Tp[j], R, pw);
    if (Jb) {
      const int v0 = a.vcol[s];
      const int jt = jts[s];
      if (jt == J_FREE) {
        for (int e = 0; e < 3; ++e) {
          const Real u[3] = {R[e], R[3 + e], R[6 + e]};
          store_col(Jb, a.sJ_k, nv, v0 + e, u, zero);
          Real lin[3];
          rot_lin<LWA>(u, pw, pe, lin);
          store_col(Jb, a.sJ_k, nv, v0 + 3 + e, lin, u);
        }
      } else {
        const Real* ax = cs + s * kPathCst + C_AX;
        Real u[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) u[i] = R[3 * i] * ax[0] + R[3 * i + 1] * ax[1] + R[3 * i + 2] * ax[2];
        if (jt == J_PRI) {
          store_col(Jb, a.sJ_k, nv, v0, u, zero);
        } else {
          Real lin[3];
          rot_lin<LWA>(u, pw, pe, lin);
          store_col(Jb, a.sJ_k, nv, v0, lin, u);
        }
      }
    }
    if (s == a.len - 1 && a.pose && live) {
      Real* po = a.pose + b * a.sp_b;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int k = 0; k < 3; ++k) po[(int64_t)(4 * r + k) * a.sp_k] = R[3 * r + k];
        po[(int64_t)(4 * r + 3) * a.sp_k] = pw[r];
      }
    }
  }
  if (Jb)  // the zero columns, shared among the lanes
    for (int z = lane; z < a.n_zero; z += kParLanes)
#pragma unroll
      for (int r = 0; r < 6; ++r) Jb[(int64_t)(r * nv + a.zcol[z]) * a.sJ_k] = Real(0);
}

}  // namespace

template <class Real>
hipError_t launch_path(const DevModel& dm, const PathArgs<Real>& pa, bool lwa, bool par, hipStream_t st) {
  if (pa.B < 1 || pa.len < 1 || pa.len > 64 || pa.nqp < 1 || pa.nqp > 72 || (!pa.J && pa.zero_groups) ||
      pa.zero_groups > 32 || pa.n_zero > 4 * pa.zero_groups)
    return hipErrorInvalidValue;
  if (par) {
    // 4 lanes per instance when the path fits 4 segments of kParSeg bodies
    const int L = pa.seg * 4 >= pa.len ? 4 : 16;
    if (pa.seg < 1 || pa.seg > kParSeg || pa.seg * L < pa.len) return hipErrorInvalidValue;
    const int64_t gx = (pa.B + kPathThreads / L - 1) / (kPathThreads / L);
    if (gx > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = (size_t)pa.len * kPathCst * sizeof(Real) + 8 * pa.len;
    const dim3 grid((unsigned)gx), block(kPathThreads);
    if (L == 4 && lwa) hipLaunchKernelGGL((path_par_kernel<Real, true, 4>), grid, block, lds, st, dm, pa);
    else if (L == 4) hipLaunchKernelGGL((path_par_kernel<Real, false, 4>), grid, block, lds, st, dm, pa);
    else if (lwa) hipLaunchKernelGGL((path_par_kernel<Real, true, 16>), grid, block, lds, st, dm, pa);
    else hipLaunchKernelGGL((path_par_kernel<Real, false, 16>), grid, block, lds, st, dm, pa);
    return hipGetLastError();
  }
  const int64_t gx = (pa.B + kPathThreads - 1) / kPathThreads;
  if (gx > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)gx, (unsigned)(1 + pa.zero_groups));
  const size_t lds = ((size_t)pa.len * kPathCst + (size_t)pa.nqp * kPathThreads) * sizeof(Real) + 4 * pa.len;
  if (lwa)
    hipLaunchKernelGGL((path_kernel<Real, true>), grid, dim3(kPathThreads), lds, st, dm, pa);
  else
    hipLaunchKernelGGL((path_kernel<Real, false>), grid, dim3(kPathThreads), lds, st, dm, pa);
  return hipGetLastError();
}

template hipError_t launch_path<float>(const DevModel&, const PathArgs<float>&, bool, bool, hipStream_t);
template hipError_t launch_path<double>(const DevModel&, const PathArgs<double>&, bool, bool, hipStream_t);

}  // namespace bard
