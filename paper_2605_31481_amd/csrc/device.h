// Device helpers shared by the tree, articulated-body and adjoint kernels:
// constants, joint transforms (eqs. (4)-(5)), rigid-body inertia algebra,
// workgroup staging and views of the staged model tables.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.h"
#include "spatial.h"

namespace bard {

template <class Real> __device__ __forceinline__ const unsigned char* image(const DevModel& dm);
template <> __device__ __forceinline__ const unsigned char* image<float>(const DevModel& dm) { return dm.img32; }
template <> __device__ __forceinline__ const unsigned char* image<double>(const DevModel& dm) { return dm.img64; }
template <class Real> __device__ __forceinline__ Real grav(const DevModel& dm, int k);
template <> __device__ __forceinline__ float grav<float>(const DevModel& dm, int k) { return dm.g32[k]; }
template <> __device__ __forceinline__ double grav<double>(const DevModel& dm, int k) { return dm.g64[k]; }

template <class Real>
__device__ __forceinline__ Real xch(Real v, int src_lane) {
  return __shfl(v, src_lane, 64);
}

// Spatial inertia of a body about the frame origin o, in world axes, from its
// parameters about the body origin (m, h, I_O) and its pose (R, p) relative to o:
//   h_w = R h + m p,
//   I_w = R I_O R^T + m (|p|^2 1 - p p^T) + 2 (p . R h) 1 - p (R h)^T - (R h) p^T.
// Output [m, h(3), Ixx, Ixy, Iyy, Ixz, Iyz, Izz].
template <class Real>
__device__ __forceinline__ void world_inertia(const Real* pi, const Real* R, const Real* p, Real* I0) {
  const Real m = pi[0];
  Real hr[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) hr[i] = R[3 * i] * pi[1] + R[3 * i + 1] * pi[2] + R[3 * i + 2] * pi[3];
  const Real Ib[9] = {pi[4], pi[5], pi[7], pi[5], pi[6], pi[8], pi[7], pi[8], pi[9]};
  Real X[9];
  mul33(R, Ib, X);
  // Y = X R^T (symmetric; six entries)
  const Real yxx = X[0] * R[0] + X[1] * R[1] + X[2] * R[2];
  const Real yxy = X[0] * R[3] + X[1] * R[4] + X[2] * R[5];
  const Real yyy = X[3] * R[3] + X[4] * R[4] + X[5] * R[5];
  const Real yxz = X[0] * R[6] + X[1] * R[7] + X[2] * R[8];
  const Real yyz = X[3] * R[6] + X[4] * R[7] + X[5] * R[8];
  const Real yzz = X[6] * R[6] + X[7] * R[7] + X[8] * R[8];
  const Real pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  const Real ph = p[0] * hr[0] + p[1] * hr[1] + p[2] * hr[2];
  const Real dg = m * pp + Real(2) * ph;
  I0[0] = m;
  I0[1] = hr[0] + m * p[0];
  I0[2] = hr[1] + m * p[1];
  I0[3] = hr[2] + m * p[2];
  I0[4] = yxx + dg - p[0] * (m * p[0] + Real(2) * hr[0]);
  I0[5] = yxy - p[0] * (m * p[1] + hr[1]) - hr[0] * p[1];
  I0[6] = yyy + dg - p[1] * (m * p[1] + Real(2) * hr[1]);
  I0[7] = yxz - p[0] * (m * p[2] + hr[2]) - hr[0] * p[2];
  I0[8] = yyz - p[1] * (m * p[2] + hr[2]) - hr[1] * p[2];
  I0[9] = yzz + dg - p[2] * (m * p[2] + Real(2) * hr[2]);
}

__device__ __forceinline__ int tile_index(int xcd_remap) {
  // Consecutive instance tiles go to the same XCD (workgroups are dealt to the
  // 8 XCDs round-robin), so partial cache lines of neighbouring tiles meet in
  // one L2.
  int bid = blockIdx.x;
  if (!xcd_remap) return bid;
  int nb = gridDim.x;
  int per = nb >> 3;
  int full = per << 3;
  if (bid >= full) return bid;
  return (bid & 7) * per + (bid >> 3);
}

// --------------------------------------------------------------------------
// Workgroup staging.
// --------------------------------------------------------------------------
// Copy `bytes` (a multiple of 16) from global to LDS in 16-byte chunks.
__device__ __forceinline__ void copy16(unsigned char* dst, const unsigned char* src, int bytes, int tid, int nt) {
  const int4* s = reinterpret_cast<const int4*>(src);
  int4* d = reinterpret_cast<int4*>(dst);
  const int n16 = bytes >> 4;
#pragma unroll 4
  for (int i = tid; i < n16; i += nt) d[i] = s[i];
}

// K rows of a strided input array (element k of instance b at b*sb + k*sk),
// staged as an LDS tile [K][T].
template <class Real>
struct InRows {
  const Real* src;
  int64_t sb, sk;
  int K;
  Real* dst;
};

// Staging of a workgroup: n0 16-byte chunks of img0 and n1 of img1 (model
// tables, end-effector image) and the input tiles of up to three arrays
// (instances past B repeat the last one).  Every thread issues its global
// loads, from clamped indices so that no branch separates them, before its
// first LDS write: the workgroup waits for one round trip to memory instead
// of one per source.  Threads past the end rewrite the last element with its
// own value.
template <class Real, int LOGT>
__device__ __forceinline__ void stage_tile(const int4* img0, int n0, int4* dst0, const int4* img1, int n1,
                                           int4* dst1, const InRows<Real>& a, const InRows<Real>& b,
                                           const InRows<Real>& c, int64_t tile0, int64_t B, int tid, int nt) {
  constexpr int T = 1 << LOGT;
  const int n16 = n0 + n1;
  const int nin = (a.K + b.K + c.K) * T;
  auto chunk_src = [&](int i) { return i < n0 ? img0 + i : img1 + (i - n0); };
  auto chunk_dst = [&](int i) { return i < n0 ? dst0 + i : dst1 + (i - n0); };
  auto in_src = [&](int i) {
    const int k = i >> LOGT;
    int64_t bi = tile0 + (i & (T - 1));
    if (bi >= B) bi = B - 1;
    if (k < a.K) return a.src + bi * a.sb + (int64_t)k * a.sk;
    if (k < a.K + b.K) return b.src + bi * b.sb + (int64_t)(k - a.K) * b.sk;
    return c.src + bi * c.sb + (int64_t)(k - a.K - b.K) * c.sk;
  };
  auto in_dst = [&](int i) {
    const int k = i >> LOGT;
    if (k < a.K) return a.dst + i;
    if (k < a.K + b.K) return b.dst + (i - a.K * T);
    return c.dst + (i - (a.K + b.K) * T);
  };
  constexpr int CT = 4, CI = 4;  // loads per thread held in registers
  int4 tv[CT];
  Real iv[CI];
#pragma unroll
  for (int j = 0; j < CT; ++j) tv[j] = *chunk_src(min(tid + j * nt, n16 - 1));
#pragma unroll
  for (int j = 0; j < CI; ++j) iv[j] = *in_src(min(tid + j * nt, nin - 1));
#pragma unroll
  for (int j = 0; j < CT; ++j) *chunk_dst(min(tid + j * nt, n16 - 1)) = tv[j];
#pragma unroll
  for (int j = 0; j < CI; ++j) *in_dst(min(tid + j * nt, nin - 1)) = iv[j];
  for (int i = tid + CT * nt; i < n16; i += nt) *chunk_dst(i) = *chunk_src(i);
  for (int i = tid + CI * nt; i < nin; i += nt) *in_dst(i) = *in_src(i);
}

// Free-root pose from [x y z qx qy qz qw]: R = R0 R(quat), position R0 p + t0.
template <class Real>
__device__ __forceinline__ void free_root_pose(const Real* c, const Real* qv, Real* Rw, Real* o) {
  Real qx = qv[3], qy = qv[4], qz = qv[5], qw = qv[6];
  const Real inv = Real(1) / sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
  qx *= inv; qy *= inv; qz *= inv; qw *= inv;
  const Real Rq[9] = {Real(1) - Real(2) * (qy * qy + qz * qz), Real(2) * (qx * qy - qz * qw), Real(2) * (qx * qz + qy * qw),
                      Real(2) * (qx * qy + qz * qw), Real(1) - Real(2) * (qx * qx + qz * qz), Real(2) * (qy * qz - qx * qw),
                      Real(2) * (qx * qz - qy * qw), Real(2) * (qy * qz + qx * qw), Real(1) - Real(2) * (qx * qx + qy * qy)};
  mul33(c + C_R0, Rq, Rw);
#pragma unroll
  for (int i = 0; i < 3; ++i)
    o[i] = c[C_R0 + 3 * i] * qv[0] + c[C_R0 + 3 * i + 1] * qv[1] + c[C_R0 + 3 * i + 2] * qv[2] + c[C_T0 + i];
}

// Joint transform from the Rodrigues constants (eqs. (4)-(5)):
// R_pc = R0 + sin q A + (1 - cos q) B, t_pc = t0 (+ q d for a prismatic joint).
template <class Real>
__device__ __forceinline__ void joint_transform(const Real* c, Real qv, Real* Rpc, Real* tpc) {
  Real sq, cq;
  sincos_r(qv, &sq, &cq);
  const Real omc = Real(1) - cq;
#pragma unroll
  for (int k = 0; k < 9; ++k) Rpc[k] = c[C_R0 + k] + sq * c[C_A + k] + omc * c[C_B + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) tpc[k] = c[C_T0 + k] + qv * c[C_D + k];
}

// Parent pose (Rw, pw) and joint transform (Rpc, tpc) -> body pose, and the
// body's motion subspace s = [u; p x u] (revolute) or [0; u] (prismatic) with
// u = R axis: in the base frame s is the direct Jacobian column of eq. (7).
template <class Real>
__device__ __forceinline__ void compose_joint(const Real* Rpc, const Real* tpc, const Real* ax, bool rev, Real* Rw,
                                              Real* pw, Real* s) {
  Real Rn[9], pn[3];
  mul33(Rw, Rpc, Rn);
#pragma unroll
  for (int i = 0; i < 3; ++i) pn[i] = Rw[3 * i] * tpc[0] + Rw[3 * i + 1] * tpc[1] + Rw[3 * i + 2] * tpc[2] + pw[i];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rw[k] = Rn[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) pw[k] = pn[k];
  Real u[3], pxu[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) u[i] = Rw[3 * i] * ax[0] + Rw[3 * i + 1] * ax[1] + Rw[3 * i + 2] * ax[2];
  cross3(pw, u, pxu);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s[i] = rev ? u[i] : Real(0);
    s[3 + i] = rev ? pxu[i] : u[i];
  }
}

// One joint step: joint transform, then the composed pose and motion subspace.
template <class Real>
__device__ __forceinline__ void joint_step(const Real* c, bool rev, Real qv, Real* Rw, Real* pw, Real* s) {
  Real Rpc[9], tpc[3];
  joint_transform(c, qv, Rpc, tpc);
  compose_joint(Rpc, tpc, c + C_AX, rev, Rw, pw, s);
}

// Index of entry (r, c) of a symmetric 6x6 stored as its upper triangle, row-major (21 entries).
__host__ __device__ __forceinline__ constexpr int sym6(int r, int c) {
  return r <= c ? (r * 6 - (r * (r - 1)) / 2 + (c - r)) : (c * 6 - (c * (c - 1)) / 2 + (r - c));
}

// Views of the staged table image.
template <class Real>
struct Tables {
  const Real* cst;
  const I4* meta;
  const int16_t* sbody;
  const int8_t* ssrc;
  const int8_t* cslot;
  const int* linfo;
  const I4* srec;
  const I4* bm2;
  const int* dlist;
  const int* ulist;
  const int8_t* jump;
  const int8_t* pre;
  const int* mtab;
};

template <class Real>
__device__ __forceinline__ Tables<Real> tables(const unsigned char* base, const DevModel& dm) {
  const TabLayout t = tab_layout(dm.n, dm.P, dm.depth, dm.kmax, dm.nv, (int)sizeof(Real));
  Tables<Real> v;
  v.cst = reinterpret_cast<const Real*>(base + t.cst);
  v.meta = reinterpret_cast<const I4*>(base + t.meta);
  v.sbody = reinterpret_cast<const int16_t*>(base + t.sbody);
  v.ssrc = reinterpret_cast<const int8_t*>(base + t.ssrc);
  v.cslot = reinterpret_cast<const int8_t*>(base + t.cslot);
  v.linfo = reinterpret_cast<const int*>(base + t.linfo);
  v.srec = reinterpret_cast<const I4*>(base + t.srec);
  v.bm2 = reinterpret_cast<const I4*>(base + t.bm2);
  v.dlist = reinterpret_cast<const int*>(base + t.dlist);
  v.ulist = reinterpret_cast<const int*>(base + t.ulist);
  v.jump = reinterpret_cast<const int8_t*>(base + t.jump);
  v.pre = reinterpret_cast<const int8_t*>(base + t.pre);
  v.mtab = reinterpret_cast<const int*>(base + t.mtab);
  return v;
}

}  // namespace bard
