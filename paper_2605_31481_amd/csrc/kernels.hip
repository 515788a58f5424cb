// Batched tree traversals for gfx950 (CDNA4, wave64).
//
// Mapping.  A workgroup owns T consecutive instances.  Inside a wave, each
// instance gets P adjacent lanes ("slots", P = next power of two >= the widest
// tree level); the model compiler assigns every body a slot so that one level
// of the tree (Sec. 3.3, eq. (6)) is one step for all slots at once.  A child
// normally continues in its parent's slot, so per-body link state stays in
// registers; where the tree branches the state is pulled across lanes with
// one bpermute per scalar.  All lanes of a wave execute every level (idle
// slots compute on a dummy body and store nothing), so exchanges never run
// under divergent control flow.
//
// Frame.  Link state is kept in a fixed frame with world axes and its origin
// at the base (the free root's position, or the world origin for a fixed
// base).  In that frame every body's motion subspace s_i is exactly the
// direct Jacobian column of eq. (7), velocities and accelerations propagate
// as v_i = v_p + s_i qd_i and a_i = a_p + s_i qdd_i + v_p x (s_i qd_i), and
// the leaf-to-root sums of forces, composite inertias (CRBA) and articulated
// inertias (ABA) are plain additions: no 6x6 congruence X^T I X is needed
// (the update Sec. 3.5 singles out as the cost of CRBA and ABA).  Putting the
// origin at the base keeps coordinates small for FP32.
//
// Phases.  A: forward sweep over levels (joint transform from the Rodrigues
// constants, eqs. (4)-(5); world pose; s_i; velocities; world inertia; body
// forces).  Back: reverse sweep gathering each body's children
// (tau_i = s_i . F_i, F_i = f_i + sum children F; Ic_i = I_i + sum Ic).
// B: the workgroup writes the dense outputs (M, J) from LDS with lanes over
// instances, so stores of the instance-minor layout coalesce.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace bard {

template <class Real> __device__ __forceinline__ const Real* consts(const DevModel& dm);
template <> __device__ __forceinline__ const float* consts<float>(const DevModel& dm) { return dm.c32; }
template <> __device__ __forceinline__ const double* consts<double>(const DevModel& dm) { return dm.c64; }
template <class Real> __device__ __forceinline__ Real grav(const DevModel& dm, int k);
template <> __device__ __forceinline__ float grav<float>(const DevModel& dm, int k) { return dm.g32[k]; }
template <> __device__ __forceinline__ double grav<double>(const DevModel& dm, int k) { return dm.g64[k]; }

__device__ __forceinline__ void sincos_r(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_r(double x, double* s, double* c) { sincos(x, s, c); }

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
  Real yxx = X[0] * R[0] + X[1] * R[1] + X[2] * R[2];
  Real yxy = X[0] * R[3] + X[1] * R[4] + X[2] * R[5];
  Real yyy = X[3] * R[3] + X[4] * R[4] + X[5] * R[5];
  Real yxz = X[0] * R[6] + X[1] * R[7] + X[2] * R[8];
  Real yyz = X[3] * R[6] + X[4] * R[7] + X[5] * R[8];
  Real yzz = X[6] * R[6] + X[7] * R[7] + X[8] * R[8];
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
// FK / Jacobian / RNEA / CRBA and their fusion (OPS bit mask).
// --------------------------------------------------------------------------
template <class Real, int OPS>
__global__ void __launch_bounds__(256) tree_kernel(DevModel dm, DevEE ee, Args<Real> ar) {
  constexpr bool FK = OPS & OP_FK;
  constexpr bool JAC = OPS & OP_JAC;
  constexpr bool RNEA = OPS & OP_RNEA;
  constexpr bool CRBA = OPS & OP_CRBA;
  constexpr bool VEL = RNEA;
  constexpr bool BACK = RNEA || CRBA;
  constexpr bool NEED_S = JAC || RNEA || CRBA;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  Real* smem = reinterpret_cast<Real*>(smem_raw);

  const int T = 1 << ar.logT;
  const int nv = dm.nv, n = dm.n;
  Real* s_l = smem;                                   // [nv][6][T]
  Real* fc_l = s_l + (NEED_S ? nv * 6 * T : 0);       // [nv][6][T]
  Real* f_l = fc_l + (CRBA ? nv * 6 * T : 0);         // [n][6][T]
  Real* i0_l = f_l + (RNEA ? n * 6 * T : 0);          // [n][10][T]
  Real* o_l = i0_l + (CRBA ? n * 10 * T : 0);         // [3][T]
  Real* pe_l = o_l + 3 * T;                           // [n_ee][3][T]

  const Real* cst = consts<Real>(dm);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int log2P = ar.log2P;      // lanes per instance used by this launch (>= dm.P)
  const int P = dm.P;              // slots in the model's schedule tables
  const int iw = lane >> log2P;
  const int slot_raw = lane & ((1 << log2P) - 1);
  const bool in_sched = slot_raw < P;
  const int slot = in_sched ? slot_raw : 0;
  const int inst = (wave << (6 - log2P)) + iw;
  const int64_t tile = tile_index(ar.xcd_remap);
  const int64_t b = tile * T + inst;
  const bool bvalid = b < ar.B;
  const int64_t bl = bvalid ? b : (ar.B - 1);
  const int lane0 = iw << log2P;

  const Real a0[6] = {Real(0), Real(0), Real(0), -grav<Real>(dm, 0), -grav<Real>(dm, 1), -grav<Real>(dm, 2)};

  // Link state of the last body processed by this slot.
  Real Rw[9], pw[3], v[6], a[6];
  Real o[3] = {Real(0), Real(0), Real(0)};

  auto qin = [&](int k) { return ar.q[bl * ar.sq_b + (int64_t)k * ar.sq_k]; };
  auto qdin = [&](int k) { return ar.qd[bl * ar.sqd_b + (int64_t)k * ar.sqd_k]; };
  auto qddin = [&](int k) { return ar.qdd[bl * ar.sqdd_b + (int64_t)k * ar.sqdd_k]; };
  auto pi_of = [&](int body, int k) -> Real {
    return ar.pi_ovr ? ar.pi_ovr[body * 10 + k] : cst[body * CST + C_PI + k];
  };

  // ---------------- phase A: forward sweep ----------------
  int lstart = 0;
  if (dm.free_root) {
    // Level 0 holds only the free root (body 0); every slot computes it, slot 0 stores.
    const Real* c = cst;
    const bool act = (slot_raw == 0);
    Real qx = qin(3), qy = qin(4), qz = qin(5), qw = qin(6);
    const Real inv = Real(1) / sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
    qx *= inv; qy *= inv; qz *= inv; qw *= inv;
    const Real Rq[9] = {Real(1) - Real(2) * (qy * qy + qz * qz), Real(2) * (qx * qy - qz * qw), Real(2) * (qx * qz + qy * qw),
                        Real(2) * (qx * qy + qz * qw), Real(1) - Real(2) * (qx * qx + qz * qz), Real(2) * (qy * qz - qx * qw),
                        Real(2) * (qx * qz - qy * qw), Real(2) * (qy * qz + qx * qw), Real(1) - Real(2) * (qx * qx + qy * qy)};
    mul33(c + C_R0, Rq, Rw);
    const Real pr[3] = {qin(0), qin(1), qin(2)};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      o[i] = c[C_R0 + 3 * i] * pr[0] + c[C_R0 + 3 * i + 1] * pr[1] + c[C_R0 + 3 * i + 2] * pr[2] + c[C_T0 + i];
      pw[i] = Real(0);
    }
    // s columns: v_k -> [0; R e_k], w_k -> [R e_k; 0]  (base-centred: root at the origin)
    if (NEED_S && act) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          s_l[((k)*6 + i) * T + inst] = Real(0);
          s_l[((k)*6 + 3 + i) * T + inst] = Rw[3 * i + k];
          s_l[((3 + k) * 6 + i) * T + inst] = Rw[3 * i + k];
          s_l[((3 + k) * 6 + 3 + i) * T + inst] = Real(0);
        }
    }
    Real I0[10];
    if (BACK) {
      Real pic[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) pic[k] = pi_of(0, k);
      world_inertia(pic, Rw, pw, I0);
      if (CRBA && act)
#pragma unroll
        for (int k = 0; k < 10; ++k) i0_l[k * T + inst] = I0[k];
    }
    if (VEL) {
      const Real vb[3] = {qdin(0), qdin(1), qdin(2)}, wb[3] = {qdin(3), qdin(4), qdin(5)};
      const Real ab[3] = {qddin(0), qddin(1), qddin(2)}, wdb[3] = {qddin(3), qddin(4), qddin(5)};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        v[i] = Rw[3 * i] * wb[0] + Rw[3 * i + 1] * wb[1] + Rw[3 * i + 2] * wb[2];
        v[3 + i] = Rw[3 * i] * vb[0] + Rw[3 * i + 1] * vb[1] + Rw[3 * i + 2] * vb[2];
        a[i] = a0[i] + Rw[3 * i] * wdb[0] + Rw[3 * i + 1] * wdb[1] + Rw[3 * i + 2] * wdb[2];
        a[3 + i] = a0[3 + i] + Rw[3 * i] * ab[0] + Rw[3 * i + 1] * ab[1] + Rw[3 * i + 2] * ab[2];
      }
      Real Ia[6], Iv[6], vxIv[6], f[6];
      inertia_mul(I0, a, Ia);
      inertia_mul(I0, v, Iv);
      crf(v, Iv, vxIv);
#pragma unroll
      for (int k = 0; k < 6; ++k) f[k] = Ia[k] + vxIv[k];
      if (act)
#pragma unroll
        for (int k = 0; k < 6; ++k) f_l[k * T + inst] = f[k];
    }
    if (act) {
#pragma unroll
      for (int i = 0; i < 3; ++i) o_l[i * T + inst] = o[i];
    }
    if (FK && act && bvalid) {
#pragma unroll
      for (int k = 0; k < 9; ++k) ar.poses[b * ar.sp_b + (int64_t)k * ar.sp_k] = Rw[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) ar.poses[b * ar.sp_b + (int64_t)(9 + k) * ar.sp_k] = o[k];
    }
    if (JAC && ar.frame == 1 && act) {
      for (int e = 0; e < ee.n_ee; ++e)
        if (ee.ee_body[e] == 0)
#pragma unroll
          for (int i = 0; i < 3; ++i) pe_l[(e * 3 + i) * T + inst] = Real(0);
    }
    lstart = 1;
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Rw[k] = (k % 4 == 0) ? Real(1) : Real(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) pw[k] = Real(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      v[k] = Real(0);
      a[k] = a0[k];
    }
    if (slot_raw == 0)
#pragma unroll
      for (int i = 0; i < 3; ++i) o_l[i * T + inst] = Real(0);
  }
  // Every slot of an instance evaluated the root, so o is known in every lane.

  for (int l = lstart; l < dm.depth; ++l) {
    const int body = in_sched ? dm.sched_body[l * P + slot] : -1;
    const bool act = body >= 0;
    const int bb = act ? body : 0;
    if (dm.level_info[2 * l + 1]) {
      const int src = lane0 + (in_sched ? (int)dm.sched_src[l * P + slot] : slot_raw);
#pragma unroll
      for (int k = 0; k < 9; ++k) Rw[k] = xch(Rw[k], src);
#pragma unroll
      for (int k = 0; k < 3; ++k) pw[k] = xch(pw[k], src);
      if (VEL) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          v[k] = xch(v[k], src);
          a[k] = xch(a[k], src);
        }
      }
    }
    const I4 meta = dm.meta[bb];
    if (meta.x < 0) {  // attached to the world (only at level 0 of a fixed base)
#pragma unroll
      for (int k = 0; k < 9; ++k) Rw[k] = (k % 4 == 0) ? Real(1) : Real(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) pw[k] = Real(0);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        v[k] = Real(0);
        a[k] = a0[k];
      }
    }
    const Real* c = cst + bb * CST;
    const bool rev = (meta.y == J_REV);
    const Real qv = qin(meta.z);
    // eqs. (4)-(5): R_pc = R0 + sin q A + (1 - cos q) B ; t_pc = t0 (+ q d for a prismatic joint)
    Real sq, cq;
    sincos_r(qv, &sq, &cq);
    const Real omc = Real(1) - cq;
    Real Rpc[9], tpc[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) Rpc[k] = c[C_R0 + k] + sq * c[C_A + k] + omc * c[C_B + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) tpc[k] = c[C_T0 + k] + qv * c[C_D + k];
    // world pose: R = R_p R_pc, p = R_p t_pc + p_p
    Real Rn[9], pn[3];
    mul33(Rw, Rpc, Rn);
#pragma unroll
    for (int i = 0; i < 3; ++i) pn[i] = Rw[3 * i] * tpc[0] + Rw[3 * i + 1] * tpc[1] + Rw[3 * i + 2] * tpc[2] + pw[i];
#pragma unroll
    for (int k = 0; k < 9; ++k) Rw[k] = Rn[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) pw[k] = pn[k];

    if (FK && act && bvalid) {
      const int64_t base = b * ar.sp_b + (int64_t)(bb * 12) * ar.sp_k;
#pragma unroll
      for (int k = 0; k < 9; ++k) ar.poses[base + (int64_t)k * ar.sp_k] = Rw[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) ar.poses[base + (int64_t)(9 + k) * ar.sp_k] = pw[k] + o[k];
    }
    if (JAC && ar.frame == 1 && act) {
      for (int e = 0; e < ee.n_ee; ++e)
        if (ee.ee_body[e] == bb)
#pragma unroll
          for (int i = 0; i < 3; ++i) pe_l[(e * 3 + i) * T + inst] = pw[i];
    }
    if (!NEED_S) continue;
    // motion subspace in the base frame = direct Jacobian column (eq. (7))
    Real u[3], s[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) u[i] = Rw[3 * i] * c[C_AX] + Rw[3 * i + 1] * c[C_AX + 1] + Rw[3 * i + 2] * c[C_AX + 2];
    Real pxu[3];
    cross3(pw, u, pxu);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      s[i] = rev ? u[i] : Real(0);
      s[3 + i] = rev ? pxu[i] : u[i];
    }
    if (act)
#pragma unroll
      for (int k = 0; k < 6; ++k) s_l[(meta.w * 6 + k) * T + inst] = s[k];
    if (!BACK) continue;
    Real pic[10], I0[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) pic[k] = pi_of(bb, k);
    world_inertia(pic, Rw, pw, I0);
    if (CRBA && act)
#pragma unroll
      for (int k = 0; k < 10; ++k) i0_l[(bb * 10 + k) * T + inst] = I0[k];
    if (VEL) {
      const Real qdv = qdin(meta.w), qddv = qddin(meta.w);
      Real vJ[6], cJ[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) vJ[k] = s[k] * qdv;
      crm(v, vJ, cJ);  // v_parent x (s qd)
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        a[k] = a[k] + s[k] * qddv + cJ[k];
        v[k] = v[k] + vJ[k];
      }
      Real Ia[6], Iv[6], vxIv[6];
      inertia_mul(I0, a, Ia);
      inertia_mul(I0, v, Iv);
      crf(v, Iv, vxIv);
      if (act)
#pragma unroll
        for (int k = 0; k < 6; ++k) f_l[(bb * 6 + k) * T + inst] = Ia[k] + vxIv[k];
    }
  }

  // ---------------- backward sweep: gather children ----------------
  if (BACK) {
    Real F[6], Ic[10];
#pragma unroll
    for (int k = 0; k < 6; ++k) F[k] = Real(0);
#pragma unroll
    for (int k = 0; k < 10; ++k) Ic[k] = Real(0);
    for (int l = dm.depth - 1; l >= 0; --l) {
      const int body = in_sched ? dm.sched_body[l * P + slot] : -1;
      const bool act = body >= 0;
      const int bb = act ? body : 0;
      Real Fn[6], Icn[10];
      if (RNEA)
#pragma unroll
        for (int k = 0; k < 6; ++k) Fn[k] = f_l[(bb * 6 + k) * T + inst];
      if (CRBA)
#pragma unroll
        for (int k = 0; k < 10; ++k) Icn[k] = i0_l[(bb * 10 + k) * T + inst];
      const int K = dm.level_info[2 * l];
      for (int j = 0; j < K; ++j) {
        const int cs = in_sched ? dm.child_slot[(l * P + slot) * dm.kmax + j] : -1;
        const int src = lane0 + (cs >= 0 ? cs : slot_raw);
        if (RNEA)
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            Real x = xch(F[k], src);
            Fn[k] += (cs >= 0) ? x : Real(0);
          }
        if (CRBA)
#pragma unroll
          for (int k = 0; k < 10; ++k) {
            Real x = xch(Ic[k], src);
            Icn[k] += (cs >= 0) ? x : Real(0);
          }
      }
      if (RNEA)
#pragma unroll
        for (int k = 0; k < 6; ++k) F[k] = Fn[k];
      if (CRBA)
#pragma unroll
        for (int k = 0; k < 10; ++k) Ic[k] = Icn[k];
      if (!act) continue;
      const I4 meta = dm.meta[bb];
      const int ndof = (meta.y == J_FREE) ? 6 : 1;
      for (int d = 0; d < ndof; ++d) {
        Real s[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) s[k] = s_l[((meta.w + d) * 6 + k) * T + inst];
        if (RNEA && bvalid) {
          Real t = s[0] * F[0] + s[1] * F[1] + s[2] * F[2] + s[3] * F[3] + s[4] * F[4] + s[5] * F[5];
          ar.tau[b * ar.st_b + (int64_t)(meta.w + d) * ar.st_k] = t;
        }
        if (CRBA) {
          Real fc[6];
          inertia_mul(Ic, s, fc);
#pragma unroll
          for (int k = 0; k < 6; ++k) fc_l[((meta.w + d) * 6 + k) * T + inst] = fc[k];
        }
      }
    }
  }

  if (!(CRBA || JAC)) return;
  __syncthreads();

  // ---------------- phase B: dense outputs, lanes over instances ----------------
  const int nthreads = blockDim.x;
  const int64_t tile0 = tile * T;
  const int Tm = T - 1;
  if (CRBA) {
    const int total = nv * nv * T;
    for (int idx = threadIdx.x; idx < total; idx += nthreads) {
      const int row = idx >> ar.logT;
      const int in = idx & Tm;
      const int64_t bo = tile0 + in;
      if (bo >= ar.B) continue;
      const int e = dm.mtab[row];
      Real val = Real(0);
      if (e >= 0) {
        const int ad = e >> 16, dd = e & 0xffff;
        const Real* sa = s_l + (ad * 6) * T + in;
        const Real* fd = fc_l + (dd * 6) * T + in;
        val = sa[0] * fd[0] + sa[T] * fd[T] + sa[2 * T] * fd[2 * T] + sa[3 * T] * fd[3 * T] +
              sa[4 * T] * fd[4 * T] + sa[5 * T] * fd[5 * T];
      }
      ar.M[bo * ar.sM_b + (int64_t)row * ar.sM_k] = val;
    }
  }
  if (JAC) {
    const int total = ee.n_ee * 6 * nv * T;
    for (int idx = threadIdx.x; idx < total; idx += nthreads) {
      const int row = idx >> ar.logT;
      const int in = idx & Tm;
      const int64_t bo = tile0 + in;
      if (bo >= ar.B) continue;
      const int col = row % nv;
      const int er = row / nv;
      const int r = er % 6;
      const int e = er / 6;
      const int src = ee.jtab[e * nv + col];
      Real val = Real(0);
      if (src >= 0) {
        const Real* s = s_l + (src * 6) * T + in;
        if (r >= 3) {
          val = s[(r - 3) * T];
        } else {
          const int r1 = (r + 1) % 3, r2 = (r + 2) % 3;
          // linear row: v + o x w (world origin) or v + w x p_e (end-effector origin)
          Real x1, x2;
          if (ar.frame == 0) {
            x1 = o_l[r1 * T + in] * s[r2 * T];
            x2 = o_l[r2 * T + in] * s[r1 * T];
          } else {
            x1 = s[r1 * T] * pe_l[(e * 3 + r2) * T + in];
            x2 = s[r2 * T] * pe_l[(e * 3 + r1) * T + in];
          }
          val = s[(3 + r) * T] + (x1 - x2);
        }
      }
      ar.J[bo * ar.sJ_b + (int64_t)row * ar.sJ_k] = val;
    }
  }
}

// --------------------------------------------------------------------------
// ABA: three sweeps in the base frame.
//   1 (root to leaves): pose, s_i, v_i, c_i = v_p x (s_i qd_i), IA_i = I_i,
//                       pA_i = v_i x* I_i v_i.
//   2 (leaves to root): IA_i += sum Ia_c, pA_i += sum pa_c (plain sums in a
//                       common frame); U = IA s, D = s.U, u = tau - s.pA;
//                       Ia = IA - U U^T / D, pa = pA + Ia c + U u / D.
//   3 (root to leaves): a = a_p + c, qdd = (u - U.a) / D, a += s qdd.
// The free root solves its 6x6 articulated system by Cholesky.
// --------------------------------------------------------------------------

// Symmetric 6x6 stored as the upper triangle, row-major (21 entries).
__device__ __forceinline__ constexpr int sym6(int r, int c) {
  return r <= c ? (r * 6 - (r * (r - 1)) / 2 + (c - r)) : (c * 6 - (c * (c - 1)) / 2 + (r - c));
}

template <class Real>
__device__ __forceinline__ void rigid_to_sym(const Real* I0, Real* S) {
  // [Ibar, h^; h^T, m 1]
  const Real hx = I0[1], hy = I0[2], hz = I0[3], m = I0[0];
  S[sym6(0, 0)] = I0[4]; S[sym6(0, 1)] = I0[5]; S[sym6(1, 1)] = I0[6];
  S[sym6(0, 2)] = I0[7]; S[sym6(1, 2)] = I0[8]; S[sym6(2, 2)] = I0[9];
  // top-right block h^ = [[0,-hz,hy],[hz,0,-hx],[-hy,hx,0]]
  S[sym6(0, 3)] = Real(0); S[sym6(0, 4)] = -hz; S[sym6(0, 5)] = hy;
  S[sym6(1, 3)] = hz; S[sym6(1, 4)] = Real(0); S[sym6(1, 5)] = -hx;
  S[sym6(2, 3)] = -hy; S[sym6(2, 4)] = hx; S[sym6(2, 5)] = Real(0);
  S[sym6(3, 3)] = m; S[sym6(3, 4)] = Real(0); S[sym6(3, 5)] = Real(0);
  S[sym6(4, 4)] = m; S[sym6(4, 5)] = Real(0); S[sym6(5, 5)] = m;
}

template <class Real>
__device__ __forceinline__ void sym_mul(const Real* S, const Real* x, Real* y) {
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    Real acc = Real(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) acc += S[sym6(r, c)] * x[c];
    y[r] = acc;
  }
}

template <class Real>
__global__ void __launch_bounds__(256) aba_kernel(DevModel dm, Args<Real> ar) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Real* smem = reinterpret_cast<Real*>(smem_raw);
  const int T = 1 << ar.logT;
  const int n = dm.n;
  // per body: s(6*ndof) is per dof; c(6), IA(21), pA(6), U(6), Dinv(1), u(1) per body
  Real* s_l = smem;                        // [nv][6][T]
  Real* c_l = s_l + dm.nv * 6 * T;         // [n][6][T]
  Real* ia_l = c_l + n * 6 * T;            // [n][21][T]
  Real* pa_l = ia_l + n * 21 * T;          // [n][6][T]
  Real* u_l = pa_l + n * 6 * T;            // [n][8][T] : U(6), 1/D, u

  const Real* cst = consts<Real>(dm);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int log2P = ar.log2P;      // lanes per instance used by this launch (>= dm.P)
  const int P = dm.P;              // slots in the model's schedule tables
  const int iw = lane >> log2P;
  const int slot_raw = lane & ((1 << log2P) - 1);
  const bool in_sched = slot_raw < P;
  const int slot = in_sched ? slot_raw : 0;
  const int inst = (wave << (6 - log2P)) + iw;
  const int64_t tile = tile_index(ar.xcd_remap);
  const int64_t b = tile * T + inst;
  const bool bvalid = b < ar.B;
  const int64_t bl = bvalid ? b : (ar.B - 1);
  const int lane0 = iw << log2P;
  const Real a0[6] = {Real(0), Real(0), Real(0), -grav<Real>(dm, 0), -grav<Real>(dm, 1), -grav<Real>(dm, 2)};

  auto qin = [&](int k) { return ar.q[bl * ar.sq_b + (int64_t)k * ar.sq_k]; };
  auto qdin = [&](int k) { return ar.qd[bl * ar.sqd_b + (int64_t)k * ar.sqd_k]; };
  auto tauin = [&](int k) { return ar.tau_in[bl * ar.sti_b + (int64_t)k * ar.sti_k]; };

  Real Rw[9], pw[3], v[6];
  int lstart = 0;
  if (dm.free_root) {
    const Real* c = cst;
    const bool act = (slot_raw == 0);
    Real qx = qin(3), qy = qin(4), qz = qin(5), qw = qin(6);
    const Real inv = Real(1) / sqrt(qx * qx + qy * qy + qz * qz + qw * qw);
    qx *= inv; qy *= inv; qz *= inv; qw *= inv;
    const Real Rq[9] = {Real(1) - Real(2) * (qy * qy + qz * qz), Real(2) * (qx * qy - qz * qw), Real(2) * (qx * qz + qy * qw),
                        Real(2) * (qx * qy + qz * qw), Real(1) - Real(2) * (qx * qx + qz * qz), Real(2) * (qy * qz - qx * qw),
                        Real(2) * (qx * qz - qy * qw), Real(2) * (qy * qz + qx * qw), Real(1) - Real(2) * (qx * qx + qy * qy)};
    mul33(c + C_R0, Rq, Rw);
#pragma unroll
    for (int i = 0; i < 3; ++i) pw[i] = Real(0);
    const Real vb[3] = {qdin(0), qdin(1), qdin(2)}, wb[3] = {qdin(3), qdin(4), qdin(5)};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      v[i] = Rw[3 * i] * wb[0] + Rw[3 * i + 1] * wb[1] + Rw[3 * i + 2] * wb[2];
      v[3 + i] = Rw[3 * i] * vb[0] + Rw[3 * i + 1] * vb[1] + Rw[3 * i + 2] * vb[2];
    }
    Real pic[10], I0[10], IA[21], Iv[6], pA[6];
#pragma unroll
    for (int k = 0; k < 10; ++k) pic[k] = c[C_PI + k];
    world_inertia(pic, Rw, pw, I0);
    rigid_to_sym(I0, IA);
    inertia_mul(I0, v, Iv);
    crf(v, Iv, pA);
    if (act) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          s_l[((k)*6 + i) * T + inst] = Real(0);
          s_l[((k)*6 + 3 + i) * T + inst] = Rw[3 * i + k];
          s_l[((3 + k) * 6 + i) * T + inst] = Rw[3 * i + k];
          s_l[((3 + k) * 6 + 3 + i) * T + inst] = Real(0);
        }
#pragma unroll
      for (int k = 0; k < 6; ++k) c_l[k * T + inst] = Real(0);
#pragma unroll
      for (int k = 0; k < 21; ++k) ia_l[k * T + inst] = IA[k];
#pragma unroll
      for (int k = 0; k < 6; ++k) pa_l[k * T + inst] = pA[k];
    }
    lstart = 1;
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Rw[k] = (k % 4 == 0) ? Real(1) : Real(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) pw[k] = Real(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = Real(0);
  }

  // ---- sweep 1 ----
  for (int l = lstart; l < dm.depth; ++l) {
    const int body = in_sched ? dm.sched_body[l * P + slot] : -1;
    const bool act = body >= 0;
    const int bb = act ? body : 0;
    if (dm.level_info[2 * l + 1]) {
      const int src = lane0 + (in_sched ? (int)dm.sched_src[l * P + slot] : slot_raw);
#pragma unroll
      for (int k = 0; k < 9; ++k) Rw[k] = xch(Rw[k], src);
#pragma unroll
      for (int k = 0; k < 3; ++k) pw[k] = xch(pw[k], src);
#pragma unroll
      for (int k = 0; k < 6; ++k) v[k] = xch(v[k], src);
    }
    const I4 meta = dm.meta[bb];
    if (meta.x < 0) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Rw[k] = (k % 4 == 0) ? Real(1) : Real(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) pw[k] = Real(0);
#pragma unroll
      for (int k = 0; k < 6; ++k) v[k] = Real(0);
    }
    const Real* c = cst + bb * CST;
    const bool rev = (meta.y == J_REV);
    const Real qv = qin(meta.z);
    Real sq, cq;
    sincos_r(qv, &sq, &cq);
    const Real omc = Real(1) - cq;
    Real Rpc[9], tpc[3], Rn[9], pn[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) Rpc[k] = c[C_R0 + k] + sq * c[C_A + k] + omc * c[C_B + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) tpc[k] = c[C_T0 + k] + qv * c[C_D + k];
    mul33(Rw, Rpc, Rn);
#pragma unroll
    for (int i = 0; i < 3; ++i) pn[i] = Rw[3 * i] * tpc[0] + Rw[3 * i + 1] * tpc[1] + Rw[3 * i + 2] * tpc[2] + pw[i];
#pragma unroll
    for (int k = 0; k < 9; ++k) Rw[k] = Rn[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) pw[k] = pn[k];
    Real u[3], s[6], pxu[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) u[i] = Rw[3 * i] * c[C_AX] + Rw[3 * i + 1] * c[C_AX + 1] + Rw[3 * i + 2] * c[C_AX + 2];
    cross3(pw, u, pxu);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      s[i] = rev ? u[i] : Real(0);
      s[3 + i] = rev ? pxu[i] : u[i];
    }
    const Real qdv = qdin(meta.w);
    Real vJ[6], cJ[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) vJ[k] = s[k] * qdv;
    crm(v, vJ, cJ);
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] += vJ[k];
    Real pic[10], I0[10], IA[21], Iv[6], pA[6];
#pragma unroll
    for (int k = 0; k < 10; ++k) pic[k] = c[C_PI + k];
    world_inertia(pic, Rw, pw, I0);
    rigid_to_sym(I0, IA);
    inertia_mul(I0, v, Iv);
    crf(v, Iv, pA);
    if (act) {
#pragma unroll
      for (int k = 0; k < 6; ++k) s_l[(meta.w * 6 + k) * T + inst] = s[k];
#pragma unroll
      for (int k = 0; k < 6; ++k) c_l[(bb * 6 + k) * T + inst] = cJ[k];
#pragma unroll
      for (int k = 0; k < 21; ++k) ia_l[(bb * 21 + k) * T + inst] = IA[k];
#pragma unroll
      for (int k = 0; k < 6; ++k) pa_l[(bb * 6 + k) * T + inst] = pA[k];
    }
  }

  // ---- sweep 2 ----
  Real Ia[21], pa[6];
#pragma unroll
  for (int k = 0; k < 21; ++k) Ia[k] = Real(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) pa[k] = Real(0);
  Real Lroot[21];   // Cholesky factor of the free root's D (lower, packed by sym6 index)
  Real uroot[6];
  Real Uroot[36];   // U columns of the free root, [dof][6]
  for (int l = dm.depth - 1; l >= 0; --l) {
    const int body = in_sched ? dm.sched_body[l * P + slot] : -1;
    const bool act = body >= 0;
    const int bb = act ? body : 0;
    Real IA[21], pA[6];
#pragma unroll
    for (int k = 0; k < 21; ++k) IA[k] = ia_l[(bb * 21 + k) * T + inst];
#pragma unroll
    for (int k = 0; k < 6; ++k) pA[k] = pa_l[(bb * 6 + k) * T + inst];
    const int K = dm.level_info[2 * l];
    for (int j = 0; j < K; ++j) {
      const int cs = in_sched ? dm.child_slot[(l * P + slot) * dm.kmax + j] : -1;
      const int src = lane0 + (cs >= 0 ? cs : slot_raw);
#pragma unroll
      for (int k = 0; k < 21; ++k) {
        Real x = xch(Ia[k], src);
        IA[k] += (cs >= 0) ? x : Real(0);
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        Real x = xch(pa[k], src);
        pA[k] += (cs >= 0) ? x : Real(0);
      }
    }
    const I4 meta = dm.meta[bb];
    if (dm.free_root && l == 0) {
      // Free root: U = IA S (6 columns), D = S^T IA S, u = tau - S^T pA; keep the Cholesky factor of D.
      Real Dm[21];
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        Real sd[6], Ud[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) sd[k] = s_l[(d * 6 + k) * T + inst];
        sym_mul(IA, sd, Ud);
#pragma unroll
        for (int k = 0; k < 6; ++k) Uroot[d * 6 + k] = Ud[k];
        uroot[d] = tauin(d) - (sd[0] * pA[0] + sd[1] * pA[1] + sd[2] * pA[2] + sd[3] * pA[3] + sd[4] * pA[4] + sd[5] * pA[5]);
      }
#pragma unroll
      for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int cc = r; cc < 6; ++cc) {
          Real acc = Real(0);
#pragma unroll
          for (int k = 0; k < 6; ++k) acc += s_l[(r * 6 + k) * T + inst] * Uroot[cc * 6 + k];
          Dm[sym6(r, cc)] = acc;
        }
      // Cholesky D = L L^T, L packed with index sym6(r, c) for r >= c.
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        Real d = Dm[sym6(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= Lroot[sym6(j, k)] * Lroot[sym6(j, k)];
        const Real ljj = sqrt(d);
        Lroot[sym6(j, j)] = ljj;
        const Real inv = Real(1) / ljj;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
          Real x = Dm[sym6(i, j)];
#pragma unroll
          for (int k = 0; k < j; ++k) x -= Lroot[sym6(i, k)] * Lroot[sym6(j, k)];
          Lroot[sym6(i, j)] = x * inv;
        }
      }
      continue;
    }
    Real s[6], cJ[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] = s_l[(meta.w * 6 + k) * T + inst];
#pragma unroll
    for (int k = 0; k < 6; ++k) cJ[k] = c_l[(bb * 6 + k) * T + inst];
    Real U[6];
    sym_mul(IA, s, U);
    const Real D = s[0] * U[0] + s[1] * U[1] + s[2] * U[2] + s[3] * U[3] + s[4] * U[4] + s[5] * U[5];
    const Real Dinv = Real(1) / D;
    const Real uu = tauin(meta.w) - (s[0] * pA[0] + s[1] * pA[1] + s[2] * pA[2] + s[3] * pA[3] + s[4] * pA[4] + s[5] * pA[5]);
    // Ia = IA - U U^T / D ; pa = pA + Ia c + U u / D
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int cc = r; cc < 6; ++cc) Ia[sym6(r, cc)] = IA[sym6(r, cc)] - U[r] * U[cc] * Dinv;
    Real Iac[6];
    sym_mul(Ia, cJ, Iac);
    const Real uD = uu * Dinv;
#pragma unroll
    for (int k = 0; k < 6; ++k) pa[k] = pA[k] + Iac[k] + U[k] * uD;
    if (act) {
#pragma unroll
      for (int k = 0; k < 6; ++k) u_l[(bb * 8 + k) * T + inst] = U[k];
      u_l[(bb * 8 + 6) * T + inst] = Dinv;
      u_l[(bb * 8 + 7) * T + inst] = uu;
    }
  }

  // ---- sweep 3 ----
  Real acc[6];
  lstart = 0;
  if (dm.free_root) {
    // qdd_root = D^-1 (u - U^T a0)
    Real rhs[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      Real t = uroot[d];
#pragma unroll
      for (int k = 0; k < 6; ++k) t -= Uroot[d * 6 + k] * a0[k];
      rhs[d] = t;
    }
    // forward then backward substitution
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      Real t = rhs[i];
#pragma unroll
      for (int k = 0; k < i; ++k) t -= Lroot[sym6(i, k)] * rhs[k];
      rhs[i] = t / Lroot[sym6(i, i)];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
      Real t = rhs[i];
#pragma unroll
      for (int k = i + 1; k < 6; ++k) t -= Lroot[sym6(k, i)] * rhs[k];
      rhs[i] = t / Lroot[sym6(i, i)];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = a0[k];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[k] += s_l[(d * 6 + k) * T + inst] * rhs[d];
      if (slot_raw == 0 && bvalid) ar.qdd_out[b * ar.sqo_b + (int64_t)d * ar.sqo_k] = rhs[d];
    }
    lstart = 1;
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = a0[k];
  }
  for (int l = lstart; l < dm.depth; ++l) {
    const int body = in_sched ? dm.sched_body[l * P + slot] : -1;
    const bool act = body >= 0;
    const int bb = act ? body : 0;
    if (dm.level_info[2 * l + 1]) {
      const int src = lane0 + (in_sched ? (int)dm.sched_src[l * P + slot] : slot_raw);
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[k] = xch(acc[k], src);
    }
    const I4 meta = dm.meta[bb];
    if (meta.x < 0)
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[k] = a0[k];
    Real s[6], U[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      s[k] = s_l[(meta.w * 6 + k) * T + inst];
      U[k] = u_l[(bb * 8 + k) * T + inst];
      acc[k] += c_l[(bb * 6 + k) * T + inst];
    }
    const Real Dinv = u_l[(bb * 8 + 6) * T + inst];
    const Real uu = u_l[(bb * 8 + 7) * T + inst];
    const Real qddv = (uu - (U[0] * acc[0] + U[1] * acc[1] + U[2] * acc[2] + U[3] * acc[3] + U[4] * acc[4] + U[5] * acc[5])) * Dinv;
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] += s[k] * qddv;
    if (act && bvalid) ar.qdd_out[b * ar.sqo_b + (int64_t)meta.w * ar.sqo_k] = qddv;
  }
}

// --------------------------------------------------------------------------
// Host-visible launchers.
// --------------------------------------------------------------------------
template <class Real, int OPS>
hipError_t launch_tree(const DevModel& dm, const DevEE& ee, const Args<Real>& ar, int grid, int block, size_t lds,
                       hipStream_t st) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)tree_kernel<Real, OPS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((tree_kernel<Real, OPS>), dim3(grid), dim3(block), lds, st, dm, ee, ar);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_aba(const DevModel& dm, const Args<Real>& ar, int grid, int block, size_t lds, hipStream_t st) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)aba_kernel<Real>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((aba_kernel<Real>), dim3(grid), dim3(block), lds, st, dm, ar);
  return hipGetLastError();
}

#define BARD_INST(R)                                                                                              \
  template hipError_t launch_tree<R, OP_FK>(const DevModel&, const DevEE&, const Args<R>&, int, int, size_t,       \
                                             hipStream_t);                                                        \
  template hipError_t launch_tree<R, OP_JAC>(const DevModel&, const DevEE&, const Args<R>&, int, int, size_t,      \
                                              hipStream_t);                                                       \
  template hipError_t launch_tree<R, OP_RNEA>(const DevModel&, const DevEE&, const Args<R>&, int, int, size_t,     \
                                               hipStream_t);                                                      \
  template hipError_t launch_tree<R, OP_CRBA>(const DevModel&, const DevEE&, const Args<R>&, int, int, size_t,     \
                                               hipStream_t);                                                      \
  template hipError_t launch_tree<R, OP_RNEA | OP_CRBA | OP_JAC>(const DevModel&, const DevEE&, const Args<R>&,   \
                                                                 int, int, size_t, hipStream_t);                  \
  template hipError_t launch_aba<R>(const DevModel&, const Args<R>&, int, int, size_t, hipStream_t);

BARD_INST(float)
BARD_INST(double)

}  // namespace bard
