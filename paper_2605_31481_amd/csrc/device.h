// Device helpers shared by the tree, articulated-body and adjoint kernels:
// constants, joint transforms (eqs. (4)-(5)), rigid-body inertia algebra,
// workgroup staging and views of the staged model tables.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.h"

namespace bard {

template <class Real> __device__ __forceinline__ const unsigned char* image(const DevModel& dm);
template <> __device__ __forceinline__ const unsigned char* image<float>(const DevModel& dm) { return dm.img32; }
template <> __device__ __forceinline__ const unsigned char* image<double>(const DevModel& dm) { return dm.img64; }
template <class Real> __device__ __forceinline__ Real grav(const DevModel& dm, int k);
template <> __device__ __forceinline__ float grav<float>(const DevModel& dm, int k) { return dm.g32[k]; }
template <> __device__ __forceinline__ double grav<double>(const DevModel& dm, int k) { return dm.g64[k]; }

// sin and cos of a joint angle.  Cody-Waite reduction x = k pi/2 + r with
// pi/2 split into three parts (computed from pi by Machin's formula) and
// fused multiply-adds, then the Taylor series of sin and cos on |r| <= pi/4
// truncated where the remainder bound |r|^(n+1)/(n+1)! drops below the
// format's unit roundoff (1.7e-9 for FP32 after x^9, 8e-20 for FP64 after
// x^17), then the quadrant k mod 4 selects and signs the pair.  Arguments
// beyond 1e5 rad (where the three-part reduction loses accuracy) fall back to
// the device library.
__device__ __forceinline__ void sincos_r(float x, float* s, float* c) {
  if (fabsf(x) > 1e5f) {
    sincosf(x, s, c);
    return;
  }
  const float k = rintf(x * 0.6366197466850281f);
  float r = fmaf(-k, 1.5707963705062866f, x);
  r = fmaf(-k, -4.371138828673793e-08f, r);
  r = fmaf(-k, -1.7151245100058819e-15f, r);
  const float r2 = r * r;
  float ps = fmaf(r2, 2.7557319223985893e-06f, -0.0001984126984126984f);
  ps = fmaf(r2, ps, 0.008333333333333333f);
  ps = fmaf(r2, ps, -0.16666666666666666f);
  const float sr = fmaf(r * r2, ps, r);
  float pc = fmaf(r2, -2.755731922398589e-07f, 2.48015873015873e-05f);
  pc = fmaf(r2, pc, -0.001388888888888889f);
  pc = fmaf(r2, pc, 0.041666666666666664f);
  pc = fmaf(r2, pc, -0.5f);
  const float cr = fmaf(r2, pc, 1.0f);
  const int q = (int)k;
  float sv = (q & 1) ? cr : sr;
  float cv = (q & 1) ? sr : cr;
  *s = (q & 2) ? -sv : sv;
  *c = ((q + 1) & 2) ? -cv : cv;
}

__device__ __forceinline__ void sincos_r(double x, double* s, double* c) {
  if (fabs(x) > 1e5) {
    sincos(x, s, c);
    return;
  }
  const double k = rint(x * 0.6366197723675814);
  double r = fma(-k, 1.5707963267948966, x);
  r = fma(-k, 6.123233995736766e-17, r);
  r = fma(-k, -1.4973849048591698e-33, r);
  const double r2 = r * r;
  double ps = fma(r2, 2.8114572543455206e-15, -7.647163731819816e-13);
  ps = fma(r2, ps, 1.6059043836821613e-10);
  ps = fma(r2, ps, -2.505210838544172e-08);
  ps = fma(r2, ps, 2.7557319223985893e-06);
  ps = fma(r2, ps, -0.0001984126984126984);
  ps = fma(r2, ps, 0.008333333333333333);
  ps = fma(r2, ps, -0.16666666666666666);
  const double sr = fma(r * r2, ps, r);
  double pc = fma(r2, 1.5619206968586225e-16, -4.779477332387385e-14);
  pc = fma(r2, pc, 1.1470745597729725e-11);
  pc = fma(r2, pc, -2.08767569878681e-09);
  pc = fma(r2, pc, 2.755731922398589e-07);
  pc = fma(r2, pc, -2.48015873015873e-05);
  pc = fma(r2, pc, 0.001388888888888889);
  pc = fma(r2, pc, -0.041666666666666664);
  pc = fma(r2, pc, 0.5);
  const double cr = fma(-r2, pc, 1.0);
  const int q = (int)k;
  double sv = (q & 1) ? cr : sr;
  double cv = (q & 1) ? sr : cr;
  *s = (q & 2) ? -sv : sv;
  *c = ((q + 1) & 2) ? -cv : cv;
}

// Store of a dense output element; streaming stores bypass cache allocation
// for data the kernel never reads back.
template <class Real>
__device__ __forceinline__ void put(Real* p, Real v, bool streaming) {
  if (streaming) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <class Real>
__device__ __forceinline__ Real xch(Real v, int src_lane) {
  return __shfl(v, src_lane, 64);
}

// c = a * b for row-major 3x3.
template <class Real>
__device__ __forceinline__ void mul33(const Real* a, const Real* b, Real* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

template <class Real>
__device__ __forceinline__ void cross3(const Real* a, const Real* b, Real* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Inertia of a body about its own origin in world axes, from its parameters
// about the body origin (m, h, I_O) and its world rotation R:
// [m, R h, R I_O R^T], packed [m, h(3), Ixx, Ixy, Iyy, Ixz, Iyz, Izz].
template <class Real>
__device__ __forceinline__ void rotate_inertia(const Real* pi, const Real* R, Real* Ip) {
  Ip[0] = pi[0];
#pragma unroll
  for (int i = 0; i < 3; ++i) Ip[1 + i] = R[3 * i] * pi[1] + R[3 * i + 1] * pi[2] + R[3 * i + 2] * pi[3];
  const Real Ib[9] = {pi[4], pi[5], pi[7], pi[5], pi[6], pi[8], pi[7], pi[8], pi[9]};
  Real X[9];
  mul33(R, Ib, X);
  Ip[4] = X[0] * R[0] + X[1] * R[1] + X[2] * R[2];
  Ip[5] = X[0] * R[3] + X[1] * R[4] + X[2] * R[5];
  Ip[6] = X[3] * R[3] + X[4] * R[4] + X[5] * R[5];
  Ip[7] = X[0] * R[6] + X[1] * R[7] + X[2] * R[8];
  Ip[8] = X[3] * R[6] + X[4] * R[7] + X[5] * R[8];
  Ip[9] = X[6] * R[6] + X[7] * R[7] + X[8] * R[8];
}

// A rigid-body inertia [m, h, Ibar] about a point x re-expressed about the
// point x - r (r: the old reference point relative to the new one; same axes).
// With c the centre of mass relative to x, the parallel-axis theorem gives
//   h' = h + m r,
//   Ibar' = Ibar + (m r.r + 2 r.h) 1 - m r r^T - r h^T - h r^T.
template <class Real>
__device__ __forceinline__ void shift_inertia(const Real* I, const Real* r, Real* o) {
  const Real m = I[0];
  const Real h[3] = {I[1], I[2], I[3]};
  const Real g[3] = {m * r[0] + h[0], m * r[1] + h[1], m * r[2] + h[2]};
  const Real dg = r[0] * (g[0] + h[0]) + r[1] * (g[1] + h[1]) + r[2] * (g[2] + h[2]);
  o[0] = m;
  o[1] = g[0];
  o[2] = g[1];
  o[3] = g[2];
  o[4] = I[4] + dg - (r[0] * g[0] + h[0] * r[0]);
  o[5] = I[5] - (r[0] * g[1] + h[0] * r[1]);
  o[6] = I[6] + dg - (r[1] * g[1] + h[1] * r[1]);
  o[7] = I[7] - (r[0] * g[2] + h[0] * r[2]);
  o[8] = I[8] - (r[1] * g[2] + h[1] * r[2]);
  o[9] = I[9] + dg - (r[2] * g[2] + h[2] * r[2]);
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

// f = I m for a rigid-body inertia I = [m, h, Ibar] and motion m = [w; u]:
//   f = [Ibar w + h x u; mass u - h x w].
template <class Real>
__device__ __forceinline__ void inertia_mul(const Real* I0, const Real* mv, Real* f) {
  const Real* w = mv;
  const Real* u = mv + 3;
  const Real h[3] = {I0[1], I0[2], I0[3]};
  Real hxu[3], hxw[3];
  cross3(h, u, hxu);
  cross3(h, w, hxw);
  f[0] = I0[4] * w[0] + I0[5] * w[1] + I0[7] * w[2] + hxu[0];
  f[1] = I0[5] * w[0] + I0[6] * w[1] + I0[8] * w[2] + hxu[1];
  f[2] = I0[7] * w[0] + I0[8] * w[1] + I0[9] * w[2] + hxu[2];
  f[3] = I0[0] * u[0] - hxw[0];
  f[4] = I0[0] * u[1] - hxw[1];
  f[5] = I0[0] * u[2] - hxw[2];
}

// Motion cross product a x b = [wa x wb; wa x ub + ua x wb].
template <class Real>
__device__ __forceinline__ void crm(const Real* a, const Real* b, Real* c) {
  Real t0[3], t1[3];
  cross3(a, b, c);
  cross3(a, b + 3, t0);
  cross3(a + 3, b, t1);
#pragma unroll
  for (int k = 0; k < 3; ++k) c[3 + k] = t0[k] + t1[k];
}

// Force cross product v x* f = [w x n + u x f; w x f].
template <class Real>
__device__ __forceinline__ void crf(const Real* v, const Real* f, Real* c) {
  Real t0[3], t1[3];
  cross3(v, f, t0);
  cross3(v + 3, f + 3, t1);
  cross3(v, f + 3, c + 3);
#pragma unroll
  for (int k = 0; k < 3; ++k) c[k] = t0[k] + t1[k];
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
