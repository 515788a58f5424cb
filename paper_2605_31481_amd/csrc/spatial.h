// Spatial-algebra and joint-angle helpers for the device code: sin/cos of a
// joint angle, 3-vector and 3x3 products, rigid-body inertia rotation, shift
// and product, and the motion and force cross products.  Self-contained (HIP
// runtime only), so the kernels the model specialiser generates at run time
// compile against the same definitions as the library's own kernels.
#pragma once

// hipRTC provides the device built-ins itself (and may not see the
// installed headers, e.g. under a profiler's environment)
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

namespace bard {

// sin and cos of a joint angle.  Cody-Waite reduction x = k pi/2 + r with
// pi/2 split into three parts (computed from pi by Machin's formula) and
// fused multiply-adds, then the Taylor series of sin and cos on |r| <= pi/4
// truncated where the remainder bound |r|^(n+1)/(n+1)! drops below the
// format's unit roundoff (1.7e-9 for FP32 after x^9, 8e-20 for FP64 after
// x^17), then the quadrant k mod 4 selects and signs the pair.  Arguments
// beyond 1e5 rad (where the three-part reduction loses accuracy) fall back to
// the device library.
// The large-argument path stays out of line: it is rarely taken and would
// otherwise be inlined at every revolute joint of unrolled code.
struct SinCos32 { float s, c; };
struct SinCos64 { double s, c; };
__device__ __noinline__ SinCos32 sincos_big(float x) {
  SinCos32 r;
  sincosf(x, &r.s, &r.c);
  return r;
}
__device__ __noinline__ SinCos64 sincos_big(double x) {
  SinCos64 r;
  sincos(x, &r.s, &r.c);
  return r;
}

__device__ __forceinline__ void sincos_r(float x, float* s, float* c) {
  if (fabsf(x) > 1e5f) {
    const SinCos32 r = sincos_big(x);
    *s = r.s;
    *c = r.c;
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
    const SinCos64 r = sincos_big(x);
    *s = r.s;
    *c = r.c;
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

}  // namespace bard
