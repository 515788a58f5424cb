// Batched tree traversals for gfx950 (CDNA4, wave64).
//
// Mapping.  A workgroup owns T consecutive instances (T is a compile-time
// power of two so every LDS offset is an immediate).  Inside a wave, each
// instance gets 2^log2P adjacent lanes ("slots", at least the widest tree
// level); the model compiler assigns every body a slot so that one level of
// the tree (Sec. 3.3, eq. (6)) is one step for all slots at once.  A child
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
// the leaf-to-root sums of forces and articulated inertias (ABA) are plain
// additions, and composite inertias (CRBA) need only a parallel-axis shift:
// no 6x6 congruence X^T I X (the update Sec. 3.5 singles out as the cost of
// CRBA and ABA).  Quantities whose size grows with the distance |p| from the
// base are formed about each body's own origin first: the body force from the
// velocity and acceleration moved to the body origin, the composite inertia
// about each joint's origin from the bodies' positions relative to it.  Formed
// about the base origin directly, they would carry terms of order |p|^2 that
// cancel in the torques and mass-matrix entries of distal joints, which FP32
// would then lose.
//
// Phases.  Staging: the workgroup copies the model's table image and its
// input tile into LDS.  Level sweep: joint transform from the Rodrigues
// constants (eqs. (4)-(5)), world pose, s_i, velocity and acceleration.  Body
// phase: inertia about the body origin (world axes) and body force per (body,
// instance).  Subtree phase: the subtree is a contiguous range of preorder
// positions; F_i is the plain sum of the body forces over it and
// tau_i = s_i . F_i; Ic_i is the sum of the bodies' inertias shifted to joint
// i's origin.  Output: every wave writes the dense M and J from LDS with lanes
// over instances, so stores of the instance-minor layout coalesce.  Only the
// level sweep is serial over the tree.
#include <hip/hip_runtime.h>

#include "device.h"

namespace bard {

// --------------------------------------------------------------------------
// Reverse-mode product of CRBA: q_bar_j = d<M_bar, M(q)>/dq_j.
//
// In the base frame M_ad = s_a . Ic_b s_d, with b the deeper of the bodies of
// dofs a and d, so L = <M_bar, M> depends on q through the motion subspaces s
// and the world inertias.  A change of q_j moves the subtree of body j rigidly
// along the screw s_j: riding motion vectors change at the rate s_j x m and
// riding inertias at the rate s_j x* I - I s_j x.  With Sb = (M_bar + M_bar^T)/2,
//   y_d  = sum over dofs a of strict ancestors of body(d) of Sb_ad s_a,
//   z_d  = y_d + 1/2 sum over dofs a of body(d) of Sb_ad s_a,
//   F_a  = Ic_body(a) y_a + sum over dofs d in the subtree of body(a) of Sb_ad Fc_d
//          (the gradient of L with respect to s_a is 2 F_a),
//   Pc_b = sum over dofs d of body b of s_d z_d^T + z_d s_d^T (the gradient of L
//          with respect to Ic_b, a symmetric 6x6),
//   Pa_b = sum of Pc over the strict ancestors of body b,
//   wI(P, I): the 6-vector with s . wI = <P, s x* I - I s x>, equal to
//          -2 [ax(Q11) + ax(Q22); ax(Q21)] for Q = I P (ax: the axial vector of
//          the antisymmetric part of a 3x3 block, times 2),
//   e_b  = wI(Pc_b, Ic_b) + sum over dofs a of body b of 2 s_a x* F_a,
// and q_bar_j = s_j . (wI(Pa_j, Ic_j) + sum over bodies b in the subtree of j of e_b).
// A free root's coordinates get zero: with the root velocity in its own body
// frame, M does not depend on the root's pose.  Every phase is one item per
// (dof or body, instance) with a fixed summation order (deterministic).
// --------------------------------------------------------------------------
template <class Real>
__device__ __forceinline__ void axial_w(const Real* I0, const Real* P, Real* w) {
  // I = [Ibar, hx; -hx, m 1] from [m, h, Ibar]; P symmetric, packed by sym6.
  Real If[6][6], Pf[6][6];
  const Real hx = I0[1], hy = I0[2], hz = I0[3], m = I0[0];
  const Real Ib[9] = {I0[4], I0[5], I0[7], I0[5], I0[6], I0[8], I0[7], I0[8], I0[9]};
  const Real H[9] = {Real(0), -hz, hy, hz, Real(0), -hx, -hy, hx, Real(0)};
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      If[r][c] = Ib[3 * r + c];
      If[r][3 + c] = H[3 * r + c];
      If[3 + r][c] = -H[3 * r + c];
      If[3 + r][3 + c] = (r == c) ? m : Real(0);
    }
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = 0; c < 6; ++c) Pf[r][c] = P[sym6(r, c)];
  auto q = [&](int r, int c) {
    Real acc = Real(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) acc += If[r][k] * Pf[k][c];
    return acc;
  };
  // ax(A) = [A21 - A12, A02 - A20, A10 - A01] of the block at (r0, c0)
  auto ax = [&](int r0, int c0, Real* o) {
    o[0] = q(r0 + 2, c0 + 1) - q(r0 + 1, c0 + 2);
    o[1] = q(r0 + 0, c0 + 2) - q(r0 + 2, c0 + 0);
    o[2] = q(r0 + 1, c0 + 0) - q(r0 + 0, c0 + 1);
  };
  Real a11[3], a22[3], a21[3];
  ax(0, 0, a11);
  ax(3, 3, a22);
  ax(3, 0, a21);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    w[k] = Real(-2) * (a11[k] + a22[k]);
    w[3 + k] = Real(-2) * a21[k];
  }
}

template <class Real, int LOGT>
__device__ __forceinline__ void crba_vjp_phases(const DevModel& dm, const Args<Real>& ar, const Tables<Real>& tb,
                                                unsigned char* smem, const LdsPlan& L, const Real* s_l,
                                                const Real* fc_l, int64_t tile0) {
  constexpr int T = 1 << LOGT;
  constexpr int SD = 6 * T + block_pad(T, sizeof(Real));
  constexpr int SCD = cvjp_dof_rows() * T + block_pad(T, sizeof(Real));   // y 0-5, z 6-11, w_a 12-17
  constexpr int SCB = cvjp_body_rows() * T + block_pad(T, sizeof(Real));  // Ic 0-9, Pc 10-30, e 31-36, t 37-42
  const int n = dm.n, nv = dm.nv;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int in = tid & (T - 1), r0 = tid >> LOGT, rstep = nt >> LOGT;
  const int64_t bo = tile0 + in;
  const bool bok = bo < ar.B;
  const Real* Mb = ar.Mbar + (bok ? bo : ar.B - 1) * ar.sMb_b;  // past the batch: repeat the last instance
  Real* cvd = reinterpret_cast<Real*>(smem + L.cvd);
  Real* cvb = reinterpret_cast<Real*>(smem + L.cvb);
  auto sbar = [&](int a, int d) {
    return Real(0.5) * (Mb[(int64_t)(a * nv + d) * ar.sMb_k] + Mb[(int64_t)(d * nv + a) * ar.sMb_k]);
  };
  auto load6 = [&](const Real* p, Real* v) {
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = p[k * T];
  };
  auto store6 = [&](Real* p, const Real* v) {
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k * T] = v[k];
  };

  // 1. y_d and z_d for every dof (items: bodies, all dofs of a body)
  for (int bb = r0; bb < n; bb += rstep) {
    const I4 m2 = tb.bm2[bb];  // {preorder position, subtree size, first dof, dofs}
    for (int d = m2.z; d < m2.z + m2.w; ++d) {
      Real y[6] = {Real(0), Real(0), Real(0), Real(0), Real(0), Real(0)};
      for (int pb = tb.meta[bb].x; pb >= 0; pb = tb.meta[pb].x) {
        const I4 pm = tb.bm2[pb];
        for (int a = pm.z; a < pm.z + pm.w; ++a) {
          const Real w = sbar(a, d);
          Real sa[6];
          load6(s_l + a * SD + in, sa);
#pragma unroll
          for (int k = 0; k < 6; ++k) y[k] += w * sa[k];
        }
      }
      Real z[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) z[k] = y[k];
      for (int a = m2.z; a < m2.z + m2.w; ++a) {
        const Real w = Real(0.5) * sbar(a, d);
        Real sa[6];
        load6(s_l + a * SD + in, sa);
#pragma unroll
        for (int k = 0; k < 6; ++k) z[k] += w * sa[k];
      }
      store6(cvd + d * SCD + in, y);
      store6(cvd + d * SCD + 6 * T + in, z);
    }
  }
  __syncthreads();

  // 2. per body: w_a = 2 s_a x* F_a for its dofs, and Pc_b
  for (int bb = r0; bb < n; bb += rstep) {
    const I4 m2 = tb.bm2[bb];
    const Real* cb = cvb + m2.x * SCB + in;
    Real Ic[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) Ic[k] = cb[k * T];
    for (int a = m2.z; a < m2.z + m2.w; ++a) {
      Real y[6], F[6];
      load6(cvd + a * SCD + in, y);
      inertia_mul(Ic, y, F);
      for (int p = m2.x; p < m2.x + m2.y; ++p) {  // the subtree, in preorder
        const I4 n2 = tb.bm2[tb.pre[p]];
        for (int d = n2.z; d < n2.z + n2.w; ++d) {
          const Real w = sbar(a, d);
          Real fc[6];
          load6(fc_l + d * SD + in, fc);
#pragma unroll
          for (int k = 0; k < 6; ++k) F[k] += w * fc[k];
        }
      }
      Real sa[6], wa[6];
      load6(s_l + a * SD + in, sa);
      crf(sa, F, wa);
#pragma unroll
      for (int k = 0; k < 6; ++k) wa[k] *= Real(2);
      store6(cvd + a * SCD + 12 * T + in, wa);
    }
    Real P[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) P[k] = Real(0);
    for (int d = m2.z; d < m2.z + m2.w; ++d) {
      Real sd[6], z[6];
      load6(s_l + d * SD + in, sd);
      load6(cvd + d * SCD + 6 * T + in, z);
#pragma unroll
      for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r; c < 6; ++c) P[sym6(r, c)] += sd[r] * z[c] + z[r] * sd[c];
    }
    Real* pc = cvb + m2.x * SCB + 10 * T + in;
#pragma unroll
    for (int k = 0; k < 21; ++k) pc[k * T] = P[k];
  }
  __syncthreads();

  // 3. per body: e_b = wI(Pc_b, Ic_b) + sum of its w_a; t_b = wI(Pa_b, Ic_b)
  for (int bb = r0; bb < n; bb += rstep) {
    const I4 m2 = tb.bm2[bb];
    Real* cb = cvb + m2.x * SCB + in;
    Real Ic[10], P[21], e[6], t[6];
#pragma unroll
    for (int k = 0; k < 10; ++k) Ic[k] = cb[k * T];
#pragma unroll
    for (int k = 0; k < 21; ++k) P[k] = cb[(10 + k) * T];
    axial_w(Ic, P, e);
    for (int a = m2.z; a < m2.z + m2.w; ++a) {
      Real wa[6];
      load6(cvd + a * SCD + 12 * T + in, wa);
#pragma unroll
      for (int k = 0; k < 6; ++k) e[k] += wa[k];
    }
#pragma unroll
    for (int k = 0; k < 21; ++k) P[k] = Real(0);
    for (int pb = tb.meta[bb].x; pb >= 0; pb = tb.meta[pb].x) {
      const Real* pp = cvb + tb.bm2[pb].x * SCB + 10 * T + in;
#pragma unroll
      for (int k = 0; k < 21; ++k) P[k] += pp[k * T];
    }
    axial_w(Ic, P, t);
    store6(cb + 31 * T, e);
    store6(cb + 37 * T, t);
  }
  __syncthreads();

  // 4. q_bar_j = s_j . (t_j + sum of e over the subtree of j); zero for a free root
  if (!bok) return;
  Real* qo = ar.q_bar + bo * ar.sqb_b;
  for (int bb = r0; bb < n; bb += rstep) {
    const I4 meta = tb.meta[bb];
    const I4 m2 = tb.bm2[bb];
    if (meta.y == J_FREE) {
      for (int k = 0; k < 7; ++k) qo[(int64_t)(meta.z + k) * ar.sqb_k] = Real(0);
      continue;
    }
    Real W[6];
    load6(cvb + m2.x * SCB + 37 * T + in, W);
    for (int p = m2.x; p < m2.x + m2.y; ++p) {
      Real e[6];
      load6(cvb + p * SCB + 31 * T + in, e);
#pragma unroll
      for (int k = 0; k < 6; ++k) W[k] += e[k];
    }
    Real sj[6];
    load6(s_l + m2.z * SD + in, sj);
    qo[(int64_t)meta.z * ar.sqb_k] =
        sj[0] * W[0] + sj[1] * W[1] + sj[2] * W[2] + sj[3] * W[3] + sj[4] * W[4] + sj[5] * W[5];
  }
}

// --------------------------------------------------------------------------
// FK / Jacobian / RNEA / CRBA and their fusion (OPS bit mask).
//   1. staging (all waves);
//   2. level sweep (waves [0, WA), T instances x 2^log2P lanes): pose, s_i,
//      and for RNEA the velocity and acceleration, left in per-body LDS blocks;
//   3. body phase (all waves, one (body, instance) item per lane): world
//      inertia I_i and body force f_i = I_i a_i + v_i x* I_i v_i;
//   4. subtree phase (all waves): F_i = sum of f over the subtree and
//      Ic_i = sum of I over the subtree (contiguous preorder ranges), then
//      tau_i = s_i . F_i and Fc_i = Ic_i s_i;
//   5. dense outputs (all waves, lanes over instances).
// The level sweep is the only serial part; phases 3-5 have no cross-lane
// dependencies, and sums are taken in a fixed order (deterministic results).
// --------------------------------------------------------------------------
template <class Real, int OPS, int LOGT>
__device__ __forceinline__ void tree_tile(const DevModel& dm, const DevEE& ee, const Args<Real>& ar,
                                          const int64_t tile) {
  constexpr bool FK = OPS & OP_FK;
  constexpr bool JAC = OPS & OP_JAC;
  constexpr bool RNEA = OPS & OP_RNEA;
  constexpr bool CRBA = OPS & OP_CRBA;
  constexpr bool BIAS = RNEA && (OPS & OP_BIAS);  // also RNEA(q, qd, 0); not on the scan path
  constexpr bool CVJP = CRBA && (OPS & OP_CVJP);   // CRBA's reverse-mode product instead of M
  constexpr bool MOUT = CRBA && !CVJP;             // the dense mass-matrix output
  constexpr bool VEL = RNEA;
  constexpr bool BACK = RNEA || CRBA;
  constexpr bool NEED_S = JAC || RNEA || CRBA;
  constexpr bool NEED_BODY = FK || RNEA || CRBA || (OPS & OP_KIN);
  constexpr int T = 1 << LOGT;
  constexpr int SD = 6 * T + block_pad(T, sizeof(Real));   // per-dof block stride (elements)
  constexpr int SB = body_rows(OPS) * T + block_pad(T, sizeof(Real));  // per-body block stride (elements)
  constexpr int PR = BIAS ? 22 : 16;  // body origin rows after the body phase
  static_assert(PR + 3 <= body_rows(OPS), "body block too small for the origin rows");

  extern __shared__ __align__(16) unsigned char smem[];
  const int nv = dm.nv, n = dm.n;
  const LdsPlan L = lds_plan(0, OPS, n, dm.nq, nv, ee.n_ee, ar.frame, T, (int)sizeof(Real), dm.P, dm.depth,
                             dm.kmax);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t tile0 = tile * T;
  const bool full = tile0 + T <= ar.B;

  // ---------------- 1. staging ----------------
  Real* q_l = reinterpret_cast<Real*>(smem + L.q);
  Real* qd_l = reinterpret_cast<Real*>(smem + L.qd);
  Real* qdd_l = reinterpret_cast<Real*>(smem + L.qdd);
  stage_tile<Real, LOGT>(reinterpret_cast<const int4*>(image<Real>(dm)), L.tab_bytes >> 4,
                         reinterpret_cast<int4*>(smem + L.tab), reinterpret_cast<const int4*>(ee.img),
                         JAC ? ee_image_bytes(ee.n_ee, nv) >> 4 : 0, reinterpret_cast<int4*>(smem + L.ee),
                         InRows<Real>{ar.q, ar.sq_b, ar.sq_k, dm.nq, q_l},
                         InRows<Real>{ar.qd, ar.sqd_b, ar.sqd_k, VEL ? nv : 0, qd_l},
                         InRows<Real>{ar.qdd, ar.sqdd_b, ar.sqdd_k, VEL ? nv : 0, qdd_l}, tile0, ar.B, tid, nt);
  Real* s_l = reinterpret_cast<Real*>(smem + L.s);        // [nv+1] blocks of 6 rows, block nv = 0
  Real* fc_l = reinterpret_cast<Real*>(smem + L.fc);      // [nv+1] blocks of 6 rows, block nv = 0
  Real* body_l = reinterpret_cast<Real*>(smem + L.body);  // [n] blocks of SB, by preorder position
  Real* o_l = reinterpret_cast<Real*>(smem + L.o);        // [3][T]
  Real* pe_l = reinterpret_cast<Real*>(smem + L.pe);      // [n_ee][3][T]
  if (NEED_S)
    for (int i = tid; i < 6 * T; i += nt) s_l[nv * SD + (i >> LOGT) * T + (i & (T - 1))] = Real(0);
  if (CRBA)
    for (int i = tid; i < 6 * T; i += nt) fc_l[nv * SD + (i >> LOGT) * T + (i & (T - 1))] = Real(0);
  // A kinematics-tier hit stages the poses, motion subspaces and base origin
  // computed by an earlier call on the same configurations; the level sweep
  // then only propagates velocities and accelerations (or does not run).
  const bool hit = ar.kin_mode == 2;
  const int64_t kld = ar.kin_ld;
  const int KP = 12 * n, KS = 6 * nv;
  if (hit) {
    const Real* kin = ar.kin;
    if (NEED_BODY)
      for (int i = tid; i < KP * T; i += nt) {
        const int k = i >> LOGT, in = i & (T - 1);
        const int64_t b = (tile0 + in < ar.B) ? tile0 + in : ar.B - 1;
        body_l[(k / 12) * SB + (k % 12) * T + in] = kin[k * kld + b];
      }
    if (NEED_S)
      for (int i = tid; i < KS * T; i += nt) {
        const int k = i >> LOGT, in = i & (T - 1);
        const int64_t b = (tile0 + in < ar.B) ? tile0 + in : ar.B - 1;
        s_l[(k / 6) * SD + (k % 6) * T + in] = kin[(KP + k) * kld + b];
      }
    for (int i = tid; i < 3 * T; i += nt) {
      const int k = i >> LOGT, in = i & (T - 1);
      o_l[k * T + in] = kin[(KP + KS + k) * kld + ((tile0 + in < ar.B) ? tile0 + in : ar.B - 1)];
    }
  }
  __syncthreads();

  const Tables<Real> tb = tables<Real>(smem + L.tab, dm);
  const int* jrow = reinterpret_cast<const int*>(smem + L.ee);
  const int* eeb_l = jrow + lds_align(ee.n_ee * 6 * nv * 4) / 4;
  if (JAC && hit && ar.frame == 1)  // end-effector origins from the staged tier
    for (int i = tid; i < ee.n_ee * 3 * T; i += nt) {
      const int r = i >> LOGT, in = i & (T - 1);
      const int e = r / 3, c = r - 3 * e;
      pe_l[i] = ar.kin[(12 * tb.bm2[eeb_l[e]].x + 9 + c) * kld + ((tile0 + in < ar.B) ? tile0 + in : ar.B - 1)];
    }

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int log2P = ar.log2P;
  const int WA = (T << log2P) >> 6;
  // Deep trees take the kinematics by pointer jumping (all waves, LDS-resident
  // state, ceil(log2(depth)) steps per quantity); others by the level sweep
  // (registers, depth steps, exchanges only where the tree branches).  The
  // model compiler picks the one with fewer steps.
  const bool SCAN = NEED_BODY && dm.use_scan;
  // Structural zeros are stored during the kinematics phase (by every
  // thread in the scan, by the waves the level sweep leaves idle otherwise).
  const bool early_zero = SCAN || nt > WA * 64;

  if (SCAN) {
    // ---------------- 2. kinematics by pointer jumping ----------------
    // A body's pose is the product of the joint transforms on its root path
    // and its velocity and acceleration are sums over that path, so all of
    // them follow in ceil(log2(depth)) steps: at step k every body combines
    // its partial result with that of its ancestor 2^k levels up.  Every
    // (body, instance) item is one thread's work in every step.
    const int inx = tid & (T - 1);
    const int rb = tid >> LOGT, rbs = nt >> LOGT;
    const int JS = dm.jsteps;
    const Real a0[6] = {Real(0), Real(0), Real(0), -grav<Real>(dm, 0), -grav<Real>(dm, 1), -grav<Real>(dm, 2)};
    auto blk = [&](int bb) { return body_l + tb.bm2[bb].x * SB + inx; };
    // six-row per-body scratch for the velocity and acceleration scans: the
    // fc blocks, unused until the subtree phase
    auto scr = [&](int bb) { return fc_l + bb * SD + inx; };
    // The structural zeros of M and J depend on nothing computed here; stored
    // first, they drain while the scans run.
    {
      const int64_t bz = tile0 + inx;
      if (bz < ar.B) {
        if (MOUT) {
          Real* out = ar.M + bz * ar.sM_b;
          const int* mz = tb.mtab + dm.n_mpair;
          for (int k = rb; k < dm.n_mzero; k += rbs) put(&out[(int64_t)mz[k] * ar.sM_k], Real(0), ar.stream_out);
        }
        if (JAC) {
          Real* out = ar.J + bz * ar.sJ_b;
          const int* jz = jrow + ee.n_col;
          for (int k = rb; k < ee.n_zero; k += rbs) put(&out[(int64_t)jz[k] * ar.sJ_k], Real(0), ar.stream_out);
        }
      }
    }
    if (!hit) {
      // joint transforms (eqs. (4)-(5); the free root's from its quaternion),
      // placed so that the last pose step writes rows 0-11
      const int rq = (JS & 1) ? 12 : 0;
      for (int bb = rb; bb < n; bb += rbs) {
        const I4 meta = tb.meta[bb];
        Real R[9], p[3];
        if (meta.y == J_FREE) {
          Real qr[7], o[3];
#pragma unroll
          for (int k = 0; k < 7; ++k) qr[k] = q_l[(meta.z + k) * T + inx];
          free_root_pose(tb.cst + bb * CST, qr, R, o);
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            p[k] = Real(0);
            o_l[k * T + inx] = o[k];
          }
        } else {
          joint_transform(tb.cst + bb * CST, q_l[meta.z * T + inx], R, p);
        }
        Real* br = blk(bb) + rq * T;
#pragma unroll
        for (int k = 0; k < 9; ++k) br[k * T] = R[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) br[(9 + k) * T] = p[k];
      }
      if (!dm.free_root)
        for (int i = tid; i < 3 * T; i += nt) o_l[i] = Real(0);
      __syncthreads();
      // poses: Q_i <- Q_jump(i) Q_i, rows 0-11 and 12-23 taking turns
      for (int st = 0, cur = rq; st < JS; ++st, cur ^= 12) {
        const int8_t* jmp = tb.jump + st * n;
        for (int bb = rb; bb < n; bb += rbs) {
          const Real* sr = blk(bb) + cur * T;
          Real R[9], p[3];
#pragma unroll
          for (int k = 0; k < 9; ++k) R[k] = sr[k * T];
#pragma unroll
          for (int k = 0; k < 3; ++k) p[k] = sr[(9 + k) * T];
          const int j = jmp[bb];
          if (j >= 0) {
            const Real* sa = blk(j) + cur * T;
            Real Ra[9], pa[3], Rn[9], pn[3];
#pragma unroll
            for (int k = 0; k < 9; ++k) Ra[k] = sa[k * T];
#pragma unroll
            for (int k = 0; k < 3; ++k) pa[k] = sa[(9 + k) * T];
            mul33(Ra, R, Rn);
#pragma unroll
            for (int i = 0; i < 3; ++i) pn[i] = Ra[3 * i] * p[0] + Ra[3 * i + 1] * p[1] + Ra[3 * i + 2] * p[2] + pa[i];
#pragma unroll
            for (int k = 0; k < 9; ++k) R[k] = Rn[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) p[k] = pn[k];
          }
          Real* dr = blk(bb) + (cur ^ 12) * T;
#pragma unroll
          for (int k = 0; k < 9; ++k) dr[k * T] = R[k];
#pragma unroll
          for (int k = 0; k < 3; ++k) dr[(9 + k) * T] = p[k];
        }
        __syncthreads();
      }
    }
    // motion subspaces (eq. (7)) unless staged, and the velocity terms s qd;
    // the velocity scan then ends in rows 12-17
    auto vbuf = [&](int which, int bb) { return which ? scr(bb) : blk(bb) + 12 * T; };
    auto abuf = [&](int which, int bb) { return which ? scr(bb) : blk(bb) + 18 * T; };
    // (kernels without an s region, FK alone, stop at the poses)
    if (NEED_S) for (int bb = rb; bb < n; bb += rbs) {
      const I4 meta = tb.meta[bb];
      const bool freej = meta.y == J_FREE;
      const int nd = freej ? 6 : 1;
      Real vs[6] = {Real(0), Real(0), Real(0), Real(0), Real(0), Real(0)};
      if (!hit) {
        const Real* br = blk(bb);
        Real R[9], p[3];
#pragma unroll
        for (int k = 0; k < 9; ++k) R[k] = br[k * T];
#pragma unroll
        for (int k = 0; k < 3; ++k) p[k] = br[(9 + k) * T];
        for (int d = 0; d < nd; ++d) {
          Real sv[6];
          if (freej) {
            // free root (at the base origin): v dofs -> [0; R e_k], w dofs -> [R e_k; 0]
            const int k = d % 3;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              sv[i] = (d >= 3) ? R[3 * i + k] : Real(0);
              sv[3 + i] = (d < 3) ? R[3 * i + k] : Real(0);
            }
          } else {
            const Real* ax = tb.cst + bb * CST + C_AX;
            Real u[3], pxu[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) u[i] = R[3 * i] * ax[0] + R[3 * i + 1] * ax[1] + R[3 * i + 2] * ax[2];
            cross3(p, u, pxu);
            const bool rev = meta.y == J_REV;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              sv[i] = rev ? u[i] : Real(0);
              sv[3 + i] = rev ? pxu[i] : u[i];
            }
          }
          Real* sr = s_l + (meta.w + d) * SD + inx;
#pragma unroll
          for (int k = 0; k < 6; ++k) sr[k * T] = sv[k];
          if (VEL) {
            const Real qdv = qd_l[(meta.w + d) * T + inx];
#pragma unroll
            for (int k = 0; k < 6; ++k) vs[k] += sv[k] * qdv;
          }
        }
      } else if (VEL) {
        for (int d = 0; d < nd; ++d) {
          const Real* sr = s_l + (meta.w + d) * SD + inx;
          const Real qdv = qd_l[(meta.w + d) * T + inx];
#pragma unroll
          for (int k = 0; k < 6; ++k) vs[k] += sr[k * T] * qdv;
        }
      }
      if (VEL) {
        Real* vr = vbuf(JS & 1, bb);
#pragma unroll
        for (int k = 0; k < 6; ++k) vr[k * T] = vs[k];
      }
    }
    if (JAC && ar.frame == 1 && !hit)  // end-effector origins
      for (int i = tid; i < ee.n_ee * 3 * T; i += nt) {
        const int r = i >> LOGT, in = i & (T - 1);
        const int e = r / 3, c = r - 3 * e;
        pe_l[i] = body_l[tb.bm2[eeb_l[e]].x * SB + (9 + c) * T + in];
      }
    if (VEL) {
      __syncthreads();
      // velocities: V_i <- V_i + V_jump(i)
      for (int st = 0, cur = JS & 1; st < JS; ++st, cur ^= 1) {
        const int8_t* jmp = tb.jump + st * n;
        for (int bb = rb; bb < n; bb += rbs) {
          const Real* sr = vbuf(cur, bb);
          Real V[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) V[k] = sr[k * T];
          const int j = jmp[bb];
          if (j >= 0) {
            const Real* sa = vbuf(cur, j);
#pragma unroll
            for (int k = 0; k < 6; ++k) V[k] += sa[k * T];
          }
          Real* dr = vbuf(cur ^ 1, bb);
#pragma unroll
          for (int k = 0; k < 6; ++k) dr[k * T] = V[k];
        }
        __syncthreads();
      }
      // acceleration terms s qdd + v_parent x (s qd), plus a0 at the roots
      for (int bb = rb; bb < n; bb += rbs) {
        const I4 meta = tb.meta[bb];
        const int nd = (meta.y == J_FREE) ? 6 : 1;
        Real vJ[6] = {Real(0), Real(0), Real(0), Real(0), Real(0), Real(0)};
        Real A[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) A[k] = (meta.x < 0) ? a0[k] : Real(0);
        for (int d = 0; d < nd; ++d) {
          const Real* sr = s_l + (meta.w + d) * SD + inx;
          const Real qdv = qd_l[(meta.w + d) * T + inx];
          const Real qddv = qdd_l[(meta.w + d) * T + inx];
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            const Real sk = sr[k * T];
            vJ[k] += sk * qdv;
            A[k] += sk * qddv;
          }
        }
        if (meta.x >= 0) {
          const Real* vp = blk(meta.x) + 12 * T;
          Real v6[6], c6[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) v6[k] = vp[k * T];
          crm(v6, vJ, c6);
#pragma unroll
          for (int k = 0; k < 6; ++k) A[k] += c6[k];
        }
        Real* ar_ = abuf(JS & 1, bb);
#pragma unroll
        for (int k = 0; k < 6; ++k) ar_[k * T] = A[k];
      }
      __syncthreads();
      // accelerations: A_i <- A_i + A_jump(i), ending in rows 18-23
      for (int st = 0, cur = JS & 1; st < JS; ++st, cur ^= 1) {
        const int8_t* jmp = tb.jump + st * n;
        for (int bb = rb; bb < n; bb += rbs) {
          const Real* sr = abuf(cur, bb);
          Real A[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) A[k] = sr[k * T];
          const int j = jmp[bb];
          if (j >= 0) {
            const Real* sa = abuf(cur, j);
#pragma unroll
            for (int k = 0; k < 6; ++k) A[k] += sa[k * T];
          }
          Real* dr = abuf(cur ^ 1, bb);
#pragma unroll
          for (int k = 0; k < 6; ++k) dr[k * T] = A[k];
        }
        __syncthreads();
      }
    }
  } else {

  // Joint transforms (eqs. (4)-(5)) depend on q only, so every wave computes
  // them, one (body, instance) item per thread, into rows 12-23 of the body's
  // block, which the sweep overwrites with v and a after reading them.  The
  // serial sweep is left with the composition of poses.
  constexpr bool PRE = NEED_BODY;
  if (PRE && !hit) {
    const int inx = tid & (T - 1);
    for (int bb = tid >> LOGT; bb < n; bb += nt >> LOGT) {
      const I4 meta = tb.meta[bb];
      if (meta.y == J_FREE) continue;
      Real Rpc[9], tpc[3];
      joint_transform(tb.cst + bb * CST, q_l[meta.z * T + inx], Rpc, tpc);
      Real* br = body_l + tb.bm2[bb].x * SB + inx;
#pragma unroll
      for (int k = 0; k < 9; ++k) br[(12 + k) * T] = Rpc[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) br[(21 + k) * T] = tpc[k];
    }
    __syncthreads();
  }

  // ---------------- 2. level sweep ----------------
  if (wave < WA && !(hit && !VEL)) {
    const int P = dm.P;
    const int iw = lane >> log2P;
    const int slot_raw = lane & ((1 << log2P) - 1);
    const bool in_sched = slot_raw < P;
    const int slot = in_sched ? slot_raw : 0;
    const int inst = (wave << (6 - log2P)) + iw;
    const int lane0 = iw << log2P;
    const Real a0[6] = {Real(0), Real(0), Real(0), -grav<Real>(dm, 0), -grav<Real>(dm, 1), -grav<Real>(dm, 2)};
    const Real* qi_l = q_l + inst;
    const Real* qdi_l = qd_l + inst;
    const Real* qddi_l = qdd_l + inst;

    Real Rw[9], pw[3], v[6], a[6];
    Real ab[6];  // BIAS: the acceleration without the qdd terms
    int lstart = 0;
    auto store_body = [&](int bb) {
      Real* br = body_l + tb.bm2[bb].x * SB + inst;
#pragma unroll
      for (int k = 0; k < 9; ++k) br[k * T] = Rw[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) br[(9 + k) * T] = pw[k];
      if (VEL) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          br[(12 + k) * T] = v[k];
          br[(18 + k) * T] = a[k];
          if (BIAS) br[(24 + k) * T] = ab[k];
        }
      }
    };
    if (dm.free_root) {
      // Level 0 holds only the free root; every slot evaluates it, slot 0 stores.
      const bool act = (slot_raw == 0);
      Real qr[7], o[3];
      if (hit) {
        const Real* rr = body_l + tb.bm2[0].x * SB + inst;
#pragma unroll
        for (int k = 0; k < 9; ++k) Rw[k] = rr[k * T];
      } else {
#pragma unroll
        for (int k = 0; k < 7; ++k) qr[k] = qi_l[k * T];
        free_root_pose(tb.cst, qr, Rw, o);
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) pw[i] = Real(0);
      if (VEL) {
        const Real vb[3] = {qdi_l[0], qdi_l[T], qdi_l[2 * T]};
        const Real wb[3] = {qdi_l[3 * T], qdi_l[4 * T], qdi_l[5 * T]};
        const Real ab_[3] = {qddi_l[0], qddi_l[T], qddi_l[2 * T]};
        const Real wdb[3] = {qddi_l[3 * T], qddi_l[4 * T], qddi_l[5 * T]};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          v[i] = Rw[3 * i] * wb[0] + Rw[3 * i + 1] * wb[1] + Rw[3 * i + 2] * wb[2];
          v[3 + i] = Rw[3 * i] * vb[0] + Rw[3 * i + 1] * vb[1] + Rw[3 * i + 2] * vb[2];
          a[i] = a0[i] + Rw[3 * i] * wdb[0] + Rw[3 * i + 1] * wdb[1] + Rw[3 * i + 2] * wdb[2];
          a[3 + i] = a0[3 + i] + Rw[3 * i] * ab_[0] + Rw[3 * i + 1] * ab_[1] + Rw[3 * i + 2] * ab_[2];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) ab[k] = a0[k];
      }
      if (act && hit) {
        Real* br = body_l + tb.bm2[0].x * SB + inst;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          br[(12 + k) * T] = v[k];
          br[(18 + k) * T] = a[k];
          if (BIAS) br[(24 + k) * T] = ab[k];
        }
      }
      if (act && !hit) {
        if (NEED_S) {
          // s columns: v_k -> [0; R e_k], w_k -> [R e_k; 0] (the root sits at the origin)
          Real* sr = s_l + inst;
#pragma unroll
          for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              sr[k * SD + i * T] = Real(0);
              sr[k * SD + (3 + i) * T] = Rw[3 * i + k];
              sr[(3 + k) * SD + i * T] = Rw[3 * i + k];
              sr[(3 + k) * SD + (3 + i) * T] = Real(0);
            }
        }
        if (NEED_BODY) store_body(0);
#pragma unroll
        for (int i = 0; i < 3; ++i) o_l[i * T + inst] = o[i];
        if (JAC && ar.frame == 1)
          for (int e = 0; e < ee.n_ee; ++e)
            if (eeb_l[e] == 0)
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
        ab[k] = a0[k];
      }
      if (slot_raw == 0 && !hit)
#pragma unroll
        for (int i = 0; i < 3; ++i) o_l[i * T + inst] = Real(0);
    }

    // What a level needs besides the carried link state.  (Loading it one level
    // ahead measured slower: the copies between the two records cost more than
    // the LDS latency they hide.)
    struct LevelIn {
      Real c[PRE ? 15 : 36];  // PRE: R_pc, t_pc, axis; else the constants R0, A, B, t0, axis, d
      Real q, qd, qdd;
      int bb, act, src, rev, vi, pos;
    };
    // The (level, slot) record is read one level ahead, so every load of a
    // step (joint transform, axis, q, qd, qdd) is issued at once, together
    // with the exchange, instead of behind a chain of dependent table reads.
    auto load_level = [&](const I4 rec, LevelIn& L) {
      const int fl = rec.w;
      L.act = in_sched && ((fl >> 16) & 1);
      L.bb = rec.x;
      L.src = lane0 + (in_sched ? ((fl >> 8) & 255) : slot_raw);
      L.rev = (fl >> 17) & 1;
      L.vi = fl & 255;
      L.pos = rec.y;
      L.q = qi_l[rec.z * T];
      if (VEL) {
        L.qd = qdi_l[L.vi * T];
        L.qdd = qddi_l[L.vi * T];
      }
      {
        const Real* c = tb.cst + L.bb * CST;
        if constexpr (PRE) {
          const Real* br = body_l + L.pos * SB + inst;
#pragma unroll
          for (int k = 0; k < 12; ++k) L.c[k] = br[(12 + k) * T];
#pragma unroll
          for (int k = 0; k < 3; ++k) L.c[12 + k] = c[C_AX + k];
        } else {
#pragma unroll
          for (int k = 0; k < 36; ++k) L.c[k] = c[k];
        }
      }
    };
    // Every body attached to the world sits at level 0 (a free root is the only
    // such body when there is one), where all lanes start from the base state
    // set above, so the loop never resets the carried state.
    // v_i = v_parent + s_i qd_i, a_i = a_parent + s_i qdd_i + v_parent x (s_i qd_i)
    auto propagate = [&](const Real* s, Real qdv, Real qddv) {
      Real vJ[6], cJ[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) vJ[k] = s[k] * qdv;
      crm(v, vJ, cJ);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        a[k] = a[k] + s[k] * qddv + cJ[k];
        if (BIAS) ab[k] = ab[k] + cJ[k];
        v[k] = v[k] + vJ[k];
      }
    };
    if (!hit) {
      const I4* srec = tb.srec + slot;
      I4 rnext = I4{0, 0, 0, 0};
      if (lstart < dm.depth) rnext = srec[lstart * P];
      for (int l = lstart; l < dm.depth; ++l) {
        const I4 rec = rnext;
        if (l + 1 < dm.depth) rnext = srec[(l + 1) * P];
        LevelIn cur;
        load_level(rec, cur);
        if ((dm.xmask >> l) & 1) {
          const int src = cur.src;
#pragma unroll
          for (int k = 0; k < 9; ++k) Rw[k] = xch(Rw[k], src);
#pragma unroll
          for (int k = 0; k < 3; ++k) pw[k] = xch(pw[k], src);
          if (VEL) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
              v[k] = xch(v[k], src);
              a[k] = xch(a[k], src);
              if (BIAS) ab[k] = xch(ab[k], src);
            }
          }
        }
        Real s[6];
        if constexpr (PRE) compose_joint(cur.c, cur.c + 9, cur.c + 12, cur.rev != 0, Rw, pw, s);
        else joint_step(cur.c, cur.rev != 0, cur.q, Rw, pw, s);
        if (VEL) propagate(s, cur.qd, cur.qdd);
        if (cur.act) {
          if (NEED_S) {
            Real* sr = s_l + cur.vi * SD + inst;
#pragma unroll
            for (int k = 0; k < 6; ++k) sr[k * T] = s[k];
          }
          if (NEED_BODY) {
            Real* br = body_l + cur.pos * SB + inst;
#pragma unroll
            for (int k = 0; k < 9; ++k) br[k * T] = Rw[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) br[(9 + k) * T] = pw[k];
            if (VEL) {
#pragma unroll
              for (int k = 0; k < 6; ++k) {
                br[(12 + k) * T] = v[k];
                br[(18 + k) * T] = a[k];
                if (BIAS) br[(24 + k) * T] = ab[k];
              }
            }
          }
          if (JAC && ar.frame == 1)
            for (int e = 0; e < ee.n_ee; ++e)
              if (eeb_l[e] == cur.bb)
#pragma unroll
                for (int i = 0; i < 3; ++i) pe_l[(e * 3 + i) * T + inst] = pw[i];
        }
      }
    } else if (VEL) {
      // Workspace hit: poses and s are staged; only v and a propagate.
      const I4* srec = tb.srec + slot;
      for (int l = lstart; l < dm.depth; ++l) {
        const I4 rec = srec[l * P];
        const int vi = rec.w & 255;
        if ((dm.xmask >> l) & 1) {
          const int src = lane0 + (in_sched ? ((rec.w >> 8) & 255) : slot_raw);
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            v[k] = xch(v[k], src);
            a[k] = xch(a[k], src);
            if (BIAS) ab[k] = xch(ab[k], src);
          }
        }
        Real s[6];
        const Real* sr = s_l + vi * SD + inst;
#pragma unroll
        for (int k = 0; k < 6; ++k) s[k] = sr[k * T];
        propagate(s, qdi_l[vi * T], qddi_l[vi * T]);
        if (in_sched && ((rec.w >> 16) & 1)) {
          Real* br = body_l + rec.y * SB + inst;
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            br[(12 + k) * T] = v[k];
            br[(18 + k) * T] = a[k];
            if (BIAS) br[(24 + k) * T] = ab[k];
          }
        }
      }
    }
  } else if (wave >= WA && (MOUT || JAC)) {
    // The structural zeros of M and J depend on nothing the sweep computes:
    // the waves the sweep leaves idle store them meanwhile.
    const int tz = tid - WA * 64, nz = nt - WA * 64;
    const int64_t b = tile0 + (tid & (T - 1));
    if (b < ar.B) {
      const int r0z = tz >> LOGT, rsz = nz >> LOGT;
      if (MOUT) {
        Real* out = ar.M + b * ar.sM_b;
        const int* mz = tb.mtab + dm.n_mpair;
        for (int k = r0z; k < dm.n_mzero; k += rsz) put(&out[(int64_t)mz[k] * ar.sM_k], Real(0), ar.stream_out);
      }
      if (JAC) {
        Real* out = ar.J + b * ar.sJ_b;
        const int* jz = jrow + ee.n_col;
        for (int k = r0z; k < ee.n_zero; k += rsz) put(&out[(int64_t)jz[k] * ar.sJ_k], Real(0), ar.stream_out);
      }
    }
  }

  }

  if (BACK || FK || JAC) __syncthreads();

  // Kinematics-tier store: this launch's poses (by preorder position), motion
  // subspaces and base origin, before the body phase overwrites the poses.
  if (ar.kin_mode == 1) {
    Real* kin = ar.kin;
    if (NEED_BODY)
      for (int i = tid; i < KP * T; i += nt) {
        const int k = i >> LOGT, in = i & (T - 1);
        if (tile0 + in < ar.B) kin[k * kld + tile0 + in] = body_l[(k / 12) * SB + (k % 12) * T + in];
      }
    if (NEED_S)
      for (int i = tid; i < KS * T; i += nt) {
        const int k = i >> LOGT, in = i & (T - 1);
        if (tile0 + in < ar.B) kin[(KP + k) * kld + tile0 + in] = s_l[(k / 6) * SD + (k % 6) * T + in];
      }
    for (int i = tid; i < 3 * T; i += nt) {
      const int k = i >> LOGT, in = i & (T - 1);
      if (tile0 + in < ar.B) kin[(KP + KS + k) * kld + tile0 + in] = o_l[k * T + in];
    }
    __syncthreads();
  }

  // Phases 3-5 give every thread one fixed instance of the tile and stride over
  // items, so output addresses advance by a constant and loads from
  // independent items overlap.
  const int in = tid & (T - 1);
  const int r0 = tid >> LOGT;
  const int rstep = nt >> LOGT;
  const int64_t bo = tile0 + in;
  const bool bok = full || bo < ar.B;

  // Jacobian columns on an end effector's root path: the 6 rows of column c of
  // block e are [v + sgn p x w; w] from s_c = [w; v], with p the world origin
  // relative to the base (o, sgn = +1) or the end-effector origin (p_e,
  // sgn = -1).  They depend on the kinematics only, so when the body phase
  // leaves row groups idle (more row groups than bodies) those store them
  // meanwhile, and the writes overlap the inertia arithmetic.
  auto store_jac_columns = [&](int k0, int kstep) {
    const int NC = ee.n_col;
    const bool world = ar.frame == 0;
    const Real sgn = world ? Real(1) : Real(-1);
    Real* out = ar.J + bo * ar.sJ_b;
    for (int k = k0; k < NC; k += 2 * kstep) {
      Real val[2][6];
      int code[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int kk = k + u * kstep;
        code[u] = (kk < NC) ? jrow[kk] : nv;  // the tail reads the all-zero block
        const Real* s = s_l + (code[u] & 0xff) * SD + in;
        const Real* P = world ? (o_l + in) : (pe_l + (code[u] >> 8) * 3 * T + in);
        const Real w0 = s[0], w1 = s[T], w2 = s[2 * T];
        const Real p0 = P[0], p1 = P[T], p2 = P[2 * T];
        val[u][0] = s[3 * T] + sgn * (p1 * w2 - p2 * w1);
        val[u][1] = s[4 * T] + sgn * (p2 * w0 - p0 * w2);
        val[u][2] = s[5 * T] + sgn * (p0 * w1 - p1 * w0);
        val[u][3] = w0;
        val[u][4] = w1;
        val[u][5] = w2;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
        if (k + u * kstep < NC) {
          const int c = code[u] & 0xff, e = code[u] >> 8;
          Real* o = out + (int64_t)(e * 6 * nv + c) * ar.sJ_k;
#pragma unroll
          for (int r = 0; r < 6; ++r) put(&o[(int64_t)(r * nv) * ar.sJ_k], val[u][r], ar.stream_out);
        }
    }
  };
  const bool jac_early = JAC && BACK && rstep > n;

  // ---------------- 3. body phase: world inertia and body force ----------------
  if (BACK) {
    if (jac_early && r0 >= n && bok) store_jac_columns(r0 - n, rstep - n);
    for (int bb = r0; bb < n; bb += rstep) {
      Real* br = body_l + tb.bm2[bb].x * SB + in;
      Real R[9], p[3], pic[10];
#pragma unroll
      for (int k = 0; k < 9; ++k) R[k] = br[k * T];
#pragma unroll
      for (int k = 0; k < 3; ++k) p[k] = br[(9 + k) * T];
#pragma unroll
      for (int k = 0; k < 10; ++k) pic[k] = ar.pi_ovr ? ar.pi_ovr[bb * 10 + k] : tb.cst[bb * CST + C_PI + k];
      // The block keeps the inertia about the body's own origin (world axes)
      // and that origin: the subtree phase re-expresses composite inertias
      // about each joint from relative positions.  The body force is formed
      // about the body origin too, from the velocity and acceleration moved
      // there (u_p = u_O + w x p), and then moved to the base origin
      // (n_O = n_p + p x f).  Formed about the base origin directly, it would
      // carry terms of order m |p|^2 |dw/dt| that cancel, and FP32 would lose
      // the torques of joints far from the base.
      Real Ip[10];
      rotate_inertia(pic, R, Ip);
      Real f[6], fb[6];
      if (VEL) {
        Real v[6], a[6], Ia[6], Iv[6], vxIv[6], t3[3];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          v[k] = br[(12 + k) * T];
          a[k] = br[(18 + k) * T];
        }
        cross3(v, p, t3);
#pragma unroll
        for (int k = 0; k < 3; ++k) v[3 + k] += t3[k];
        cross3(a, p, t3);
#pragma unroll
        for (int k = 0; k < 3; ++k) a[3 + k] += t3[k];
        inertia_mul(Ip, a, Ia);
        inertia_mul(Ip, v, Iv);
        crf(v, Iv, vxIv);
#pragma unroll
        for (int k = 0; k < 6; ++k) f[k] = Ia[k] + vxIv[k];
        cross3(p, f + 3, t3);
#pragma unroll
        for (int k = 0; k < 3; ++k) f[k] += t3[k];
        if (BIAS) {
          Real abv[6], Iab[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) abv[k] = br[(24 + k) * T];
          cross3(abv, p, t3);
#pragma unroll
          for (int k = 0; k < 3; ++k) abv[3 + k] += t3[k];
          inertia_mul(Ip, abv, Iab);
#pragma unroll
          for (int k = 0; k < 6; ++k) fb[k] = Iab[k] + vxIv[k];
          cross3(p, fb + 3, t3);
#pragma unroll
          for (int k = 0; k < 3; ++k) fb[k] += t3[k];
        }
      }
      // overwrite this body's block in place: rows 0-5 f, rows 6-15 the
      // inertia about the body origin, rows PR-PR+2 that origin, and for BIAS
      // rows 16-21 the bias force (R, p, v, a, ab were read above)
      if (VEL)
#pragma unroll
        for (int k = 0; k < 6; ++k) br[k * T] = f[k];
#pragma unroll
      for (int k = 0; k < 10; ++k) br[(6 + k) * T] = Ip[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) br[(PR + k) * T] = p[k];
      if (BIAS)
#pragma unroll
        for (int k = 0; k < 6; ++k) br[(16 + k) * T] = fb[k];
    }
    __syncthreads();

    // ---------------- 4. subtree phase ----------------
    // A wave takes U = 64 / T work entries at a time (one row group of T lanes
    // each).  Large subtrees come as U entries of one body, each summing a
    // slice of its preorder range; the slices are combined with a butterfly
    // over the row groups, which yields the same bits in every lane.
    {
      constexpr int U = 64 >> LOGT;
      constexpr int ui = 6 - LOGT;
      const int* ul = tb.ulist + ui * 8 * n;
      const int nent = dm.ulen[ui];
      const int rg = (tid >> LOGT) & (U - 1);
      const int nw = nt >> 6;
      for (int base = wave * U; base < nent; base += nw * U) {
        const int code = ul[base + rg];
        const bool valid = code >= 0;
        const int bb = valid ? (code & 0xff) : 0;
        const int part = (code >> 8) & 0xf;
        const int np = valid ? ((code >> 12) & 0xf) : 1;
        const bool split = ((ul[base] >> 12) & 0xf) > 1;  // same for the whole wave
        const I4 m2 = tb.bm2[bb];  // {preorder position, subtree size, v index, dofs}
        // Part p of a split body sums positions p, p + np, p + 2 np, ... of
        // its range, so the row groups of a wave read adjacent blocks (blocks
        // a fixed distance apart would share LDS banks).
        const int c1 = valid ? m2.y : 0;
        Real F[6], Ic[10], Fb[6], pj[3];
#pragma unroll
        for (int k = 0; k < 6; ++k) F[k] = Fb[k] = Real(0);
#pragma unroll
        for (int k = 0; k < 10; ++k) Ic[k] = Real(0);
        // The composite inertia is summed about the subtree root's own origin
        // p_j, each body's term shifted by its position relative to p_j.
        // Taken about the base origin, the sum would carry terms of order
        // m |p|^2 that cancel in s_j . Ic_j s_j, and FP32 would lose the
        // mass-matrix entries of joints far from the base.
        if (CRBA)
#pragma unroll
          for (int k = 0; k < 3; ++k) pj[k] = body_l[m2.x * SB + (PR + k) * T + in];
        const Real* br = body_l + (m2.x + part) * SB + in;
        for (int c = part; c < c1; c += np, br += np * SB) {
          if (RNEA)
#pragma unroll
            for (int k = 0; k < 6; ++k) F[k] += br[k * T];
          if (CRBA) {
            Real Ik[10], d[3], Is[10];
#pragma unroll
            for (int k = 0; k < 10; ++k) Ik[k] = br[(6 + k) * T];
#pragma unroll
            for (int k = 0; k < 3; ++k) d[k] = br[(PR + k) * T] - pj[k];
            shift_inertia(Ik, d, Is);
#pragma unroll
            for (int k = 0; k < 10; ++k) Ic[k] += Is[k];
          }
          if (BIAS)
#pragma unroll
            for (int k = 0; k < 6; ++k) Fb[k] += br[(16 + k) * T];
        }
        if (U > 1 && split) {
#pragma unroll
          for (int sh = T; sh < 64; sh <<= 1) {
            if (RNEA)
#pragma unroll
              for (int k = 0; k < 6; ++k) F[k] += xch(F[k], lane ^ sh);
            if (CRBA)
#pragma unroll
              for (int k = 0; k < 10; ++k) Ic[k] += xch(Ic[k], lane ^ sh);
            if (BIAS)
#pragma unroll
              for (int k = 0; k < 6; ++k) Fb[k] += xch(Fb[k], lane ^ sh);
          }
        }
        if (!valid) continue;
        if (CVJP && part == 0) {
          // the composite inertia Ic_i about the base origin, by preorder
          // position, for the CRBA adjoint
          Real Ico[10];
          shift_inertia(Ic, pj, Ico);
          Real* icr = reinterpret_cast<Real*>(smem + L.cvb) + m2.x * (cvjp_body_rows() * T + block_pad(T, sizeof(Real))) + in;
#pragma unroll
          for (int k = 0; k < 10; ++k) icr[k * T] = Ico[k];
        }
        const bool rev = tb.meta[bb].y == J_REV;
        for (int d = part; d < m2.w; d += np) {
          const Real* sr = s_l + (m2.z + d) * SD + in;
          Real s[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) s[k] = sr[k * T];
          if (RNEA && bok) {
            const Real t = s[0] * F[0] + s[1] * F[1] + s[2] * F[2] + s[3] * F[3] + s[4] * F[4] + s[5] * F[5];
            put(&ar.tau[bo * ar.st_b + (int64_t)(m2.z + d) * ar.st_k], t, ar.stream_out);
            if (BIAS) {
              const Real tb_ = s[0] * Fb[0] + s[1] * Fb[1] + s[2] * Fb[2] + s[3] * Fb[3] + s[4] * Fb[4] + s[5] * Fb[5];
              put(&ar.bias[bo * ar.sb_b + (int64_t)(m2.z + d) * ar.sb_k], tb_, ar.stream_out);
            }
          }
          if (CRBA) {
            // s_j about p_j (a revolute axis passes through p_j: no linear
            // part; prismatic columns are the same about every point, and a
            // free root sits at the base origin), Fc_j = Ic_j s_j about p_j,
            // then moved to the base origin: n_O = n + p_j x f.
            Real sp[6], fcv[6], pxf[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              sp[k] = s[k];
              sp[3 + k] = rev ? Real(0) : s[3 + k];
            }
            inertia_mul(Ic, sp, fcv);
            cross3(pj, fcv + 3, pxf);
            Real* fo = fc_l + (m2.z + d) * SD + in;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              fo[k * T] = fcv[k] + pxf[k];
              fo[(3 + k) * T] = fcv[3 + k];
            }
          }
        }
      }
    }
    if (CRBA) __syncthreads();
  }

  if constexpr (CVJP) {
    crba_vjp_phases<Real, LOGT>(dm, ar, tb, smem, L, s_l, fc_l, tile0);
    return;
  }

  // ---------------- 5. dense outputs, lanes over instances ----------------
  // Compiled lists drive M and J: one entry per non-zero pair or column (LDS
  // reads only for those), then plain stores of the structural zeros.
  if (!bok) return;
  if (FK) {
    const int NR = n * 12;
    Real* out = ar.poses + bo * ar.sp_b;
    for (int row = r0; row < NR; row += rstep) {
      // pose element (r, c) of the 3x4 [R | p]; body rows hold R row-major, then p
      const int bb = row / 12;
      const int k = row - bb * 12;
      const int r = k >> 2, c = k & 3;
      const int src = (c == 3) ? 9 + r : 3 * r + c;
      Real val = body_l[tb.bm2[bb].x * SB + src * T + in];
      if (c == 3) val += o_l[r * T + in];
      put(&out[(int64_t)row * ar.sp_k], val, ar.stream_out);
    }
  }
  if (CRBA) {
    // Related pairs: M[a][d] = M[d][a] = s_a . Fc_d, both triangles from one
    // register (M is bitwise symmetric).  Entries go four at a time so their
    // LDS reads are in flight together; the tail reads the all-zero block and
    // stores nothing.
    const int NP = dm.n_mpair;
    Real* out = ar.M + bo * ar.sM_b;
    const int zcode = (nv << 16) | nv;
    for (int k = r0; k < NP; k += 4 * rstep) {
      Real val[4];
      int code[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = k + u * rstep;
        code[u] = (kk < NP) ? tb.mtab[kk] : zcode;
        const Real* sa = s_l + (code[u] & 0xffff) * SD + in;
        const Real* fd = fc_l + (code[u] >> 16) * SD + in;
        val[u] = sa[0] * fd[0] + sa[T] * fd[T] + sa[2 * T] * fd[2 * T] + sa[3 * T] * fd[3 * T] +
                 sa[4 * T] * fd[4 * T] + sa[5 * T] * fd[5 * T];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (k + u * rstep < NP) {
          const int a = code[u] & 0xffff, d = code[u] >> 16;
          put(&out[(int64_t)(a * nv + d) * ar.sM_k], val[u], ar.stream_out);
          put(&out[(int64_t)(d * nv + a) * ar.sM_k], val[u], ar.stream_out);
        }
    }
    if (!early_zero) {
      const int* mz = tb.mtab + NP;
      for (int k = r0; k < dm.n_mzero; k += rstep) put(&out[(int64_t)mz[k] * ar.sM_k], Real(0), ar.stream_out);
    }
  }
  if (JAC) {
    if (!jac_early) store_jac_columns(r0, rstep);
    if (!early_zero) {
      Real* out = ar.J + bo * ar.sJ_b;
      const int* jz = jrow + ee.n_col;
      for (int k = r0; k < ee.n_zero; k += rstep) put(&out[(int64_t)jz[k] * ar.sJ_k], Real(0), ar.stream_out);
    }
  }
}

// One tree, one tile per workgroup.
template <class Real, int OPS, int LOGT>
__global__ void __launch_bounds__(tree_max_threads(sizeof(Real))) tree_kernel(DevModel dm, DevEE ee, Args<Real> ar) {
  tree_tile<Real, OPS, LOGT>(dm, ee, ar, tile_index(ar.xcd_remap));
}

// Several trees in one launch.  Workgroup b runs the work item
// items[item0 + b] = {model, tile}; the items are sorted longest first, so the
// hardware dispatcher, which hands out workgroups in order as slots free up,
// acts as a longest-processing-time work queue.  Each model's tables, end
// effectors and I/O arguments come from device arrays (uniform loads).
template <class Real, int OPS, int LOGT>
__global__ void __launch_bounds__(tree_max_threads(sizeof(Real))) plan_kernel(PlanPtrs<Real> pp) {
  const int2 it = pp.items[pp.item0 + blockIdx.x];
  tree_tile<Real, OPS, LOGT>(pp.dm[it.x], pp.ee[it.x], pp.args[it.x], it.y);
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

template <class Real>
__device__ __forceinline__ void rigid_to_sym(const Real* I0, Real* S) {
  // [Ibar, h^; h^T, m 1]
  const Real hx = I0[1], hy = I0[2], hz = I0[3], m = I0[0];
  S[sym6(0, 0)] = I0[4]; S[sym6(0, 1)] = I0[5]; S[sym6(1, 1)] = I0[6];
  S[sym6(0, 2)] = I0[7]; S[sym6(1, 2)] = I0[8]; S[sym6(2, 2)] = I0[9];
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

template <class Real, int LOGT>
__global__ void __launch_bounds__(aba_max_threads(sizeof(Real))) aba_kernel(DevModel dm, Args<Real> ar) {
  constexpr int T = 1 << LOGT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nv = dm.nv;
  const LdsPlan L = lds_plan(1, 0, dm.n, dm.nq, nv, 0, 0, T, (int)sizeof(Real), dm.P, dm.depth, dm.kmax);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t tile = tile_index(ar.xcd_remap);
  const int64_t tile0 = tile * T;

  Real* q_l = reinterpret_cast<Real*>(smem + L.q);
  Real* qd_l = reinterpret_cast<Real*>(smem + L.qd);
  Real* t_l = reinterpret_cast<Real*>(smem + L.tin);
  const int4* timg = reinterpret_cast<const int4*>(image<Real>(dm));
  int4* tdst = reinterpret_cast<int4*>(smem + L.tab);
  stage_tile<Real, LOGT>(timg, L.tab_bytes >> 4, tdst, timg, 0, tdst,
                         InRows<Real>{ar.q, ar.sq_b, ar.sq_k, dm.nq, q_l},
                         InRows<Real>{ar.qd, ar.sqd_b, ar.sqd_k, ar.aba_solve ? 0 : nv, qd_l},
                         InRows<Real>{ar.tau_in, ar.sti_b, ar.sti_k, nv, t_l}, tile0, ar.B, tid, nt);
  // solve mode (qdd = M^-1 tau): zero velocities instead of staged ones
  if (ar.aba_solve)
    for (int i = tid; i < nv * T; i += nt) qd_l[i] = Real(0);
  __syncthreads();

  const Tables<Real> tb = tables<Real>(smem + L.tab, dm);
  Real* s_l = reinterpret_cast<Real*>(smem + L.s);    // [nv][6][T]
  Real* c_l = reinterpret_cast<Real*>(smem + L.c);    // [n][6][T]
  Real* ia_l = reinterpret_cast<Real*>(smem + L.ia);  // [n][21][T]
  Real* pa_l = reinterpret_cast<Real*>(smem + L.pa);  // [n][6][T]
  Real* u_l = reinterpret_cast<Real*>(smem + L.u);    // [n][8][T] : U(6), 1/D, u

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int log2P = ar.log2P;
  const int WA = (T << log2P) >> 6;
  if (wave >= WA) return;  // no cross-wave phase follows

  const int P = dm.P;
  const int iw = lane >> log2P;
  const int slot_raw = lane & ((1 << log2P) - 1);
  const bool in_sched = slot_raw < P;
  const int slot = in_sched ? slot_raw : 0;
  const int inst = (wave << (6 - log2P)) + iw;
  const int64_t b = tile0 + inst;
  const bool bvalid = b < ar.B;
  const int lane0 = iw << log2P;
  const Real gs = ar.aba_solve ? Real(0) : Real(1);  // solve mode: no gravity
  const Real a0[6] = {Real(0), Real(0), Real(0), -gs * grav<Real>(dm, 0), -gs * grav<Real>(dm, 1),
                      -gs * grav<Real>(dm, 2)};
  const Real* qi_l = q_l + inst;
  const Real* qdi_l = qd_l + inst;
  const Real* ti_l = t_l + inst;

  Real Rw[9], pw[3], v[6];
  int lstart = 0;
  if (dm.free_root) {
    const bool act = (slot_raw == 0);
    Real qr[7], o[3];
#pragma unroll
    for (int k = 0; k < 7; ++k) qr[k] = qi_l[k * T];
    free_root_pose(tb.cst, qr, Rw, o);
#pragma unroll
    for (int i = 0; i < 3; ++i) pw[i] = Real(0);
    const Real vb[3] = {qdi_l[0], qdi_l[T], qdi_l[2 * T]}, wb[3] = {qdi_l[3 * T], qdi_l[4 * T], qdi_l[5 * T]};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      v[i] = Rw[3 * i] * wb[0] + Rw[3 * i + 1] * wb[1] + Rw[3 * i + 2] * wb[2];
      v[3 + i] = Rw[3 * i] * vb[0] + Rw[3 * i + 1] * vb[1] + Rw[3 * i + 2] * vb[2];
    }
    Real pic[10], I0[10], IA[21], Iv[6], pA[6];
#pragma unroll
    for (int k = 0; k < 10; ++k) pic[k] = tb.cst[C_PI + k];
    world_inertia(pic, Rw, pw, I0);
    rigid_to_sym(I0, IA);
    inertia_mul(I0, v, Iv);
    crf(v, Iv, pA);
    if (act) {
      Real* sr = s_l + inst;
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          sr[(k * 6 + i) * T] = Real(0);
          sr[(k * 6 + 3 + i) * T] = Rw[3 * i + k];
          sr[((3 + k) * 6 + i) * T] = Rw[3 * i + k];
          sr[((3 + k) * 6 + 3 + i) * T] = Real(0);
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
    const int body = in_sched ? tb.sbody[l * P + slot] : -1;
    const bool act = body >= 0;
    const int bb = act ? body : 0;
    if (tb.linfo[2 * l + 1]) {
      const int src = lane0 + (in_sched ? (int)tb.ssrc[l * P + slot] : slot_raw);
#pragma unroll
      for (int k = 0; k < 9; ++k) Rw[k] = xch(Rw[k], src);
#pragma unroll
      for (int k = 0; k < 3; ++k) pw[k] = xch(pw[k], src);
#pragma unroll
      for (int k = 0; k < 6; ++k) v[k] = xch(v[k], src);
    }
    const I4 meta = tb.meta[bb];
    if (meta.x < 0) {
#pragma unroll
      for (int k = 0; k < 9; ++k) Rw[k] = (k % 4 == 0) ? Real(1) : Real(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) pw[k] = Real(0);
#pragma unroll
      for (int k = 0; k < 6; ++k) v[k] = Real(0);
    }
    const Real* c = tb.cst + bb * CST;
    Real s[6];
    joint_step(c, meta.y == J_REV, qi_l[meta.z * T], Rw, pw, s);
    const Real qdv = qdi_l[meta.w * T];
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
      Real* sr = s_l + meta.w * 6 * T + inst;
      Real* cr = c_l + bb * 6 * T + inst;
      Real* ir = ia_l + bb * 21 * T + inst;
      Real* pr = pa_l + bb * 6 * T + inst;
#pragma unroll
      for (int k = 0; k < 6; ++k) sr[k * T] = s[k];
#pragma unroll
      for (int k = 0; k < 6; ++k) cr[k * T] = cJ[k];
#pragma unroll
      for (int k = 0; k < 21; ++k) ir[k * T] = IA[k];
#pragma unroll
      for (int k = 0; k < 6; ++k) pr[k * T] = pA[k];
    }
  }

  // ---- sweep 2 ----
  Real Ia[21], pa[6];
#pragma unroll
  for (int k = 0; k < 21; ++k) Ia[k] = Real(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) pa[k] = Real(0);
  Real Lroot[21];   // Cholesky factor of the free root's D, packed by sym6(r, c), r >= c
  Real uroot[6];
  Real Uroot[36];   // U columns of the free root, [dof][6]
  for (int l = dm.depth - 1; l >= 0; --l) {
    const int body = in_sched ? tb.sbody[l * P + slot] : -1;
    const bool act = body >= 0;
    const int bb = act ? body : 0;
    Real IA[21], pA[6];
    {
      const Real* ir = ia_l + bb * 21 * T + inst;
      const Real* pr = pa_l + bb * 6 * T + inst;
#pragma unroll
      for (int k = 0; k < 21; ++k) IA[k] = ir[k * T];
#pragma unroll
      for (int k = 0; k < 6; ++k) pA[k] = pr[k * T];
    }
    const int K = tb.linfo[2 * l];
    for (int j = 0; j < K; ++j) {
      const int cs = in_sched ? tb.cslot[(l * P + slot) * dm.kmax + j] : -1;
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
    const I4 meta = tb.meta[bb];
    if (dm.free_root && l == 0) {
      // Free root: U = IA S (6 columns), D = S^T IA S, u = tau - S^T pA; factor D = L L^T.
      Real Dm[21];
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        Real sd[6], Ud[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) sd[k] = s_l[(d * 6 + k) * T + inst];
        sym_mul(IA, sd, Ud);
#pragma unroll
        for (int k = 0; k < 6; ++k) Uroot[d * 6 + k] = Ud[k];
        uroot[d] = ti_l[d * T] - (sd[0] * pA[0] + sd[1] * pA[1] + sd[2] * pA[2] + sd[3] * pA[3] + sd[4] * pA[4] +
                                  sd[5] * pA[5]);
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
    {
      const Real* sr = s_l + meta.w * 6 * T + inst;
      const Real* cr = c_l + bb * 6 * T + inst;
#pragma unroll
      for (int k = 0; k < 6; ++k) s[k] = sr[k * T];
#pragma unroll
      for (int k = 0; k < 6; ++k) cJ[k] = cr[k * T];
    }
    Real U[6];
    sym_mul(IA, s, U);
    const Real D = s[0] * U[0] + s[1] * U[1] + s[2] * U[2] + s[3] * U[3] + s[4] * U[4] + s[5] * U[5];
    const Real Dinv = Real(1) / D;
    const Real uu = ti_l[meta.w * T] - (s[0] * pA[0] + s[1] * pA[1] + s[2] * pA[2] + s[3] * pA[3] + s[4] * pA[4] +
                                        s[5] * pA[5]);
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
      Real* ur = u_l + bb * 8 * T + inst;
#pragma unroll
      for (int k = 0; k < 6; ++k) ur[k * T] = U[k];
      ur[6 * T] = Dinv;
      ur[7 * T] = uu;
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
    const int body = in_sched ? tb.sbody[l * P + slot] : -1;
    const bool act = body >= 0;
    const int bb = act ? body : 0;
    if (tb.linfo[2 * l + 1]) {
      const int src = lane0 + (in_sched ? (int)tb.ssrc[l * P + slot] : slot_raw);
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[k] = xch(acc[k], src);
    }
    const I4 meta = tb.meta[bb];
    if (meta.x < 0)
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[k] = a0[k];
    Real s[6], U[6];
    const Real* sr = s_l + meta.w * 6 * T + inst;
    const Real* ur = u_l + bb * 8 * T + inst;
    const Real* cr = c_l + bb * 6 * T + inst;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      s[k] = sr[k * T];
      U[k] = ur[k * T];
      acc[k] += cr[k * T];
    }
    const Real Dinv = ur[6 * T];
    const Real uu = ur[7 * T];
    const Real qddv =
        (uu - (U[0] * acc[0] + U[1] * acc[1] + U[2] * acc[2] + U[3] * acc[3] + U[4] * acc[4] + U[5] * acc[5])) * Dinv;
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] += s[k] * qddv;
    if (act && bvalid) ar.qdd_out[b * ar.sqo_b + (int64_t)meta.w * ar.sqo_k] = qddv;
  }
}

// --------------------------------------------------------------------------
// Host-visible launchers: pick the compile-time tile and launch.
// --------------------------------------------------------------------------
// Allow `lds` bytes of dynamic LDS for `kernel`.  The largest size granted so
// far is remembered per device (one static per kernel instantiation), so
// repeated launches, and launches recorded into a graph, make no further call.
template <class K>
static hipError_t raise_lds(K kernel, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  static size_t granted[BARD_MAX_DEVICES] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= BARD_MAX_DEVICES) dev = 0;
  if (lds <= granted[dev]) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) granted[dev] = lds;
  return e;
}

template <class Real, int OPS, int LOGT>
static hipError_t launch_tree_t(const DevModel& dm, const DevEE& ee, const Args<Real>& ar, int grid, int block,
                                size_t lds, hipStream_t st) {
  hipError_t e = raise_lds(tree_kernel<Real, OPS, LOGT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((tree_kernel<Real, OPS, LOGT>), dim3(grid), dim3(block), lds, st, dm, ee, ar);
  return hipGetLastError();
}

template <class Real, int OPS>
hipError_t launch_tree(const DevModel& dm, const DevEE& ee, const Args<Real>& ar, int grid, int block, size_t lds,
                       hipStream_t st) {
  switch (ar.logT) {
    case 3: return launch_tree_t<Real, OPS, 3>(dm, ee, ar, grid, block, lds, st);
    case 4: return launch_tree_t<Real, OPS, 4>(dm, ee, ar, grid, block, lds, st);
    case 5: return launch_tree_t<Real, OPS, 5>(dm, ee, ar, grid, block, lds, st);
    case 6: return launch_tree_t<Real, OPS, 6>(dm, ee, ar, grid, block, lds, st);
    default: return hipErrorInvalidValue;
  }
}

template <class Real, int OPS, int LOGT>
static hipError_t launch_plan_t(const PlanPtrs<Real>& pp, int grid, int block, size_t lds, hipStream_t st) {
  hipError_t e = raise_lds(plan_kernel<Real, OPS, LOGT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((plan_kernel<Real, OPS, LOGT>), dim3(grid), dim3(block), lds, st, pp);
  return hipGetLastError();
}

template <class Real, int OPS>
hipError_t launch_plan(const PlanPtrs<Real>& pp, int logT, int grid, int block, size_t lds, hipStream_t st) {
  switch (logT) {
    case 3: return launch_plan_t<Real, OPS, 3>(pp, grid, block, lds, st);
    case 4: return launch_plan_t<Real, OPS, 4>(pp, grid, block, lds, st);
    case 5: return launch_plan_t<Real, OPS, 5>(pp, grid, block, lds, st);
    default: return hipErrorInvalidValue;
  }
}

template <class Real, int LOGT>
static hipError_t launch_aba_t(const DevModel& dm, const Args<Real>& ar, int grid, int block, size_t lds,
                               hipStream_t st) {
  hipError_t e = raise_lds(aba_kernel<Real, LOGT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((aba_kernel<Real, LOGT>), dim3(grid), dim3(block), lds, st, dm, ar);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_aba(const DevModel& dm, const Args<Real>& ar, int grid, int block, size_t lds, hipStream_t st) {
  switch (ar.logT) {
    case 3: return launch_aba_t<Real, 3>(dm, ar, grid, block, lds, st);
    case 4: return launch_aba_t<Real, 4>(dm, ar, grid, block, lds, st);
    case 5: return launch_aba_t<Real, 5>(dm, ar, grid, block, lds, st);
    case 6: return launch_aba_t<Real, 6>(dm, ar, grid, block, lds, st);
    default: return hipErrorInvalidValue;
  }
}

#define BARD_INST(R)                                                                                              \
  template hipError_t launch_tree<R, OP_FK>(const DevModel&, const DevEE&, const Args<R>&, int, int, size_t,       \
                                             hipStream_t);                                                        \
  template hipError_t launch_tree<R, OP_JAC>(const DevModel&, const DevEE&, const Args<R>&, int, int, size_t,      \
                                              hipStream_t);                                                       \
  template hipError_t launch_tree<R, OP_JAC | OP_KIN>(const DevModel&, const DevEE&, const Args<R>&, int, int,     \
                                                       size_t, hipStream_t);                                      \
  template hipError_t launch_tree<R, OP_RNEA>(const DevModel&, const DevEE&, const Args<R>&, int, int, size_t,     \
                                               hipStream_t);                                                      \
  template hipError_t launch_tree<R, OP_CRBA>(const DevModel&, const DevEE&, const Args<R>&, int, int, size_t,     \
                                               hipStream_t);                                                      \
  template hipError_t launch_tree<R, OP_RNEA | OP_BIAS>(const DevModel&, const DevEE&, const Args<R>&, int, int,   \
                                                        size_t, hipStream_t);                                     \
  template hipError_t launch_tree<R, OP_RNEA | OP_CRBA | OP_JAC>(const DevModel&, const DevEE&, const Args<R>&,   \
                                                                 int, int, size_t, hipStream_t);                  \
  template hipError_t launch_tree<R, OP_CRBA | OP_CVJP>(const DevModel&, const DevEE&, const Args<R>&, int, int,   \
                                                        size_t, hipStream_t);                                     \
  template hipError_t launch_aba<R>(const DevModel&, const Args<R>&, int, int, size_t, hipStream_t);          \
  template hipError_t launch_plan<R, OP_RNEA>(const PlanPtrs<R>&, int, int, int, size_t, hipStream_t);           \
  template hipError_t launch_plan<R, OP_CRBA>(const PlanPtrs<R>&, int, int, int, size_t, hipStream_t);           \
  template hipError_t launch_plan<R, OP_JAC>(const PlanPtrs<R>&, int, int, int, size_t, hipStream_t);            \
  template hipError_t launch_plan<R, OP_RNEA | OP_CRBA | OP_JAC>(const PlanPtrs<R>&, int, int, int, size_t,      \
                                                                 hipStream_t);

BARD_INST(float)
BARD_INST(double)

}  // namespace bard
