// Reverse-mode products (vector-Jacobian products) of FK and RNEA: the
// gradients Sec. 4.3 takes through RNEA with respect to
// the state and the inertial parameters, and the FK gradient of the
// functional mode.
//
// Base-frame form.  In the frame with world axes and its origin at the base
// (the world origin, or the free root's position), a change dq of a revolute
// or prismatic q_j moves the whole subtree of body j rigidly along the screw s_j (its
// motion subspace, which is the Jacobian column of eq. (7)): every motion
// vector X riding on a body of that subtree changes by dq s_j x X, every
// force vector by dq s_j x* X, every world inertia by the congruence of that
// screw.  Hence dL/dq_j = s_j . W_j, where W_j is the sum over the subtree of
// j of each body's screw sensitivity w_k: the adjoints of the quantities the
// body carries, contracted with their rates under a unit screw.  Every step is
// then a root-to-leaf path sum (carried in the level sweep) or a leaf-to-root
// subtree sum (a contiguous range of preorder positions), the same two
// patterns as the forward kernels; no 6x6 transform and no stored tape.
//
// RNEA adjoint, given tau_bar (f_k = I_k a_k + v_k x* I_k v_k, F_i the
// subtree sum of f, tau_i = s_i . F_i):
//   sweep:    phi_k = phi_parent + tau_bar_k s_k        (= dL/df_k)
//   per body: psi = -v x phi, abar = I phi, h = I v,
//             vbar_own = [h_w x phi_w + h_u x phi_u; h_u x phi_w] + I psi,
//             g = vbar_own + v x* abar,
//             wI = -(phi x* I a + a x* abar + psi x* h + v x* I psi);
//   subtree:  F, Abar = sum abar, G = sum g;
//             vbar = G - v x* Abar, vJbar = vbar - v_parent x* Abar,
//             qd_bar = s . vJbar, qdd_bar = s . Abar,
//             sbar = tau_bar F + qd vJbar + qdd Abar, w = s x* sbar + wI;
//   subtree:  q_bar = s . (sum of w).
// The gradient for the inertial parameters is the adjoint of the two products
// I a and I v (with adjoints phi and psi) mapped back to the body-frame
// parameters, summed over the batch in FP64 in a fixed order.
//
// A free root's coordinates move the whole tree: its rotation by a rotation
// about the base origin, its position by a translation (which leaves RNEA
// unchanged), so their gradients come from the sum over all bodies.
//
// FK adjoint, given (Rbar_k, pbar_k) per body:
//   w_k = [vee(Rbar_k R_k^T) + p_k x pbar_k; pbar_k], q_bar_j = s_j . (sum of w),
// with vee(G) = (G21 - G12, G02 - G20, G10 - G01).
#include <hip/hip_runtime.h>

#include <mutex>

#include "device.h"

namespace bard {

// Subtree sums over the balanced work list (a wave takes U = 64 / T entries,
// one row group of T lanes each; large subtrees come split into U slices that
// a butterfly over the row groups recombines, so every lane of the group ends
// with the same bits).  For every body j: S = sum over j's preorder range of
// rows [R0, R0 + NR) of the per-body blocks, then fn(j, m2, part, S) with
// m2 = {preorder position, subtree size, v index, dofs}.
template <class Real, int NR, int R0, int LOGT, int SB, class Fn>
__device__ __forceinline__ void subtree_sums(const Tables<Real>& tb, const DevModel& dm, const Real* body_l, int tid,
                                             int nt, Fn&& fn) {
  constexpr int T = 1 << LOGT;
  constexpr int U = 64 >> LOGT;
  constexpr int ui = 6 - LOGT;
  const int* ul = tb.ulist + ui * 8 * dm.n;
  const int nent = dm.ulen[ui];
  const int in = tid & (T - 1);
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int rg = (tid >> LOGT) & (U - 1);
  const int nw = nt >> 6;
  for (int base = wave * U; base < nent; base += nw * U) {
    const int code = ul[base + rg];
    const bool valid = code >= 0;
    const int bb = valid ? (code & 0xff) : 0;
    const int part = (code >> 8) & 0xf;
    const int np = valid ? ((code >> 12) & 0xf) : 1;
    const bool split = ((ul[base] >> 12) & 0xf) > 1;  // same for the whole wave
    const I4 m2 = tb.bm2[bb];
    // part p sums positions p, p + np, ... so row groups read adjacent blocks
    const int c1 = valid ? m2.y : 0;
    Real S[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) S[k] = Real(0);
    const Real* br = body_l + (m2.x + part) * SB + R0 * T + in;
    for (int c = part; c < c1; c += np, br += np * SB)
#pragma unroll
      for (int k = 0; k < NR; ++k) S[k] += br[k * T];
    if (U > 1 && split)
#pragma unroll
      for (int sh = T; sh < 64; sh <<= 1)
#pragma unroll
        for (int k = 0; k < NR; ++k) S[k] += xch(S[k], lane ^ sh);
    if (valid) fn(bb, m2, part, S);
  }
}

// Gradient with respect to the body-frame inertial parameters [m, h, I_O]
// (h = m c, I_O about the body origin) of a scalar that depends on the world
// inertia I of the body (about the base origin, from world_inertia) only
// through the products I x1 and I x2, whose adjoints are y1 and y2.  The map
// parameters -> I -> I x is linear, so the gradient is its transpose applied
// to (y1 x1^T + y2 x2^T):
//   world:  mbar = y_u . x_u,  hbar_w = x_u x y_w - x_w x y_u,
//           Gbar = sym(y_w x_w^T)            (summed over both pairs);
//   body:   mbar += hbar_w . p + tr(G) |p|^2 - p^T G p,
//           hbar = R^T (hbar_w + 2 tr(G) p - 2 G p),
//           I_O bar = R^T G R (off-diagonal parameters take twice the entry).
template <class Real>
__device__ __forceinline__ void inertia_param_grad(const Real* R, const Real* p, const Real* x1, const Real* y1,
                                                   const Real* x2, const Real* y2, Real* g) {
  const Real mw = y1[3] * x1[3] + y1[4] * x1[4] + y1[5] * x1[5] + y2[3] * x2[3] + y2[4] * x2[4] + y2[5] * x2[5];
  Real c1[3], c2[3], c3[3], c4[3], hw[3];
  cross3(x1 + 3, y1, c1);
  cross3(x1, y1 + 3, c2);
  cross3(x2 + 3, y2, c3);
  cross3(x2, y2 + 3, c4);
#pragma unroll
  for (int i = 0; i < 3; ++i) hw[i] = c1[i] - c2[i] + c3[i] - c4[i];
  Real G[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      G[3 * i + j] = Real(0.5) * (y1[i] * x1[j] + y1[j] * x1[i] + y2[i] * x2[j] + y2[j] * x2[i]);
  const Real tr = G[0] + G[4] + G[8];
  Real Gp[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Gp[i] = G[3 * i] * p[0] + G[3 * i + 1] * p[1] + G[3 * i + 2] * p[2];
  const Real pp = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  g[0] = mw + hw[0] * p[0] + hw[1] * p[1] + hw[2] * p[2] + tr * pp - (p[0] * Gp[0] + p[1] * Gp[1] + p[2] * Gp[2]);
  Real hr[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) hr[i] = hw[i] + Real(2) * (tr * p[i] - Gp[i]);
#pragma unroll
  for (int j = 0; j < 3; ++j) g[1 + j] = R[j] * hr[0] + R[3 + j] * hr[1] + R[6 + j] * hr[2];
  Real X[9];  // G R
  mul33(G, R, X);
  auto gb = [&](int i, int j) { return R[i] * X[j] + R[3 + i] * X[3 + j] + R[6 + i] * X[6 + j]; };
  g[4] = gb(0, 0);
  g[5] = Real(2) * gb(0, 1);
  g[6] = gb(1, 1);
  g[7] = Real(2) * gb(0, 2);
  g[8] = Real(2) * gb(1, 2);
  g[9] = gb(2, 2);
}

template <class Real>
__device__ __forceinline__ Real dot6(const Real* a, const Real* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3] + a[4] * b[4] + a[5] * b[5];
}

// One workgroup loops over instance tiles tile = blockIdx.x, + gridDim.x, ...
// (a single pass when the launch covers every tile).  Per tile: staging, the
// level sweep (waves [0, WA)), a body phase and one (FK) or two (RNEA) subtree
// phases over all waves.  The inertial-parameter sums of a workgroup
// accumulate in LDS in tile order and are written once at the end.
// FREE: the tree has a free root (a separate instantiation, so fixed-base
// trees keep the single-dof code and its register budget).
template <class Real, bool RNEA, bool FREE, int LOGT>
__global__ void __launch_bounds__(kAdjMaxThreads, sizeof(Real) == 4 ? 4 : 1) adjoint_kernel(DevModel dm,
                                                                                        AdjArgs<Real> ar) {
  constexpr int T = 1 << LOGT;
  constexpr int SD = 6 * T + block_pad(T, sizeof(Real));
  constexpr int SB = adj_rows(RNEA) * T + block_pad(T, sizeof(Real));
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = dm.n, nv = dm.nv;
  const AdjPlan L = adj_plan(RNEA, n, dm.nq, nv, T, (int)sizeof(Real), dm.P, dm.depth, dm.kmax);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6;
  Real* const inbuf[2] = {reinterpret_cast<Real*>(smem + L.in0), reinterpret_cast<Real*>(smem + L.in1)};
  Real* s_l = reinterpret_cast<Real*>(smem + L.s);        // [nv] blocks of 6 rows
  Real* body_l = reinterpret_cast<Real*>(smem + L.body);  // [n] blocks by preorder position
  double* acc_l = reinterpret_cast<double*>(smem + L.acc);

  copy16(smem + L.tab, image<Real>(dm), L.tab_bytes, tid, nt);
  const bool want_pi = RNEA && ar.partial != nullptr;
  if (want_pi)
    for (int i = tid; i < n * 10; i += nt) acc_l[i] = 0.0;
  const Tables<Real> tb = tables<Real>(smem + L.tab, dm);

  const int log2P = ar.log2P;
  const int WA = (T << log2P) >> 6;
  const int in = tid & (T - 1);
  const int r0 = tid >> LOGT;
  const int rstep = nt >> LOGT;

  // Element k of instance b of the concatenated input rows (q, then qd, qdd,
  // tau_bar for RNEA); b is clamped into the batch.
  const int KIN = adj_in_rows(RNEA, dm.nq, nv);
  auto input = [&](int k, int64_t b) -> Real {
    if (b >= ar.B) b = ar.B - 1;
    if (k < dm.nq) return ar.q[b * ar.sq_b + (int64_t)k * ar.sq_k];
    k -= dm.nq;
    if (k < nv) return ar.qd[b * ar.sqd_b + (int64_t)k * ar.sqd_k];
    k -= nv;
    if (k < nv) return ar.qdd[b * ar.sqdd_b + (int64_t)k * ar.sqdd_k];
    return ar.tb_scale * ar.tau_bar[b * ar.stb_b + (int64_t)(k - nv) * ar.stb_k];
  };
  // The next tile's inputs are loaded into registers while this tile's body
  // and subtree phases run, and written to the other input buffer at the end.
  constexpr int PF = 4;
  const bool can_pf = KIN * T <= PF * nt;
  if (blockIdx.x < ar.ntiles)
    for (int i = tid; i < KIN * T; i += nt) inbuf[0][i] = input(i >> LOGT, blockIdx.x * T + (i & (T - 1)));
  int cur = 0;

  for (int64_t tile = blockIdx.x; tile < ar.ntiles; tile += gridDim.x) {
    const int64_t tile0 = tile * T;
    const int64_t bo = tile0 + in;
    const bool bok = bo < ar.B;
    const int64_t nxt = tile + gridDim.x;
    Real* q_l = inbuf[cur];
    Real* qd_l = q_l + dm.nq * T;
    Real* qdd_l = qd_l + nv * T;
    Real* tb_l = qdd_l + nv * T;
    __syncthreads();  // inputs staged; the previous tile's phases are done

    // ---------------- level sweep: pose, s, v, a, phi ----------------
    if (wave < WA) {
      const int P = dm.P;
      const int iw = lane >> log2P;
      const int slot_raw = lane & ((1 << log2P) - 1);
      const bool in_sched = slot_raw < P;
      const int slot = in_sched ? slot_raw : 0;
      const int inst = (wave << (6 - log2P)) + iw;
      const int lane0 = iw << log2P;
      const Real a0[6] = {Real(0), Real(0), Real(0), -grav<Real>(dm, 0), -grav<Real>(dm, 1), -grav<Real>(dm, 2)};
      Real Rw[9], pw[3], v[6], a[6], phi[6];
      auto reset = [&]() {
#pragma unroll
        for (int k = 0; k < 9; ++k) Rw[k] = (k % 4 == 0) ? Real(1) : Real(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) pw[k] = Real(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          v[k] = Real(0);
          a[k] = a0[k];
          phi[k] = Real(0);
        }
      };
      reset();
      int lstart = 0;
      if (FREE) {
        // Level 0 holds only the free root, at the base origin; every slot
        // evaluates it (so every slot carries its state into level 1) and
        // slot 0 stores it.  Its six motion subspace columns are [0; R e_k]
        // for the linear and [R e_k; 0] for the angular velocity coordinates.
        Real qr[7], o[3];
#pragma unroll
        for (int k = 0; k < 7; ++k) qr[k] = q_l[k * T + inst];
        free_root_pose(tb.cst, qr, Rw, o);
        if (RNEA) {
          const Real* qdi = qd_l + inst;
          const Real* qddi = qdd_l + inst;
          const Real* tbi = tb_l + inst;
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            const Real* Ri = Rw + 3 * i;
            v[i] = Ri[0] * qdi[3 * T] + Ri[1] * qdi[4 * T] + Ri[2] * qdi[5 * T];
            v[3 + i] = Ri[0] * qdi[0] + Ri[1] * qdi[T] + Ri[2] * qdi[2 * T];
            a[i] = a0[i] + Ri[0] * qddi[3 * T] + Ri[1] * qddi[4 * T] + Ri[2] * qddi[5 * T];
            a[3 + i] = a0[3 + i] + Ri[0] * qddi[0] + Ri[1] * qddi[T] + Ri[2] * qddi[2 * T];
            phi[i] = Ri[0] * tbi[3 * T] + Ri[1] * tbi[4 * T] + Ri[2] * tbi[5 * T];
            phi[3 + i] = Ri[0] * tbi[0] + Ri[1] * tbi[T] + Ri[2] * tbi[2 * T];
          }
        }
        if (slot_raw == 0) {
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
          Real* br = body_l + tb.bm2[0].x * SB + inst;
#pragma unroll
          for (int k = 0; k < 9; ++k) br[k * T] = Rw[k];
#pragma unroll
          for (int k = 0; k < 3; ++k) br[(9 + k) * T] = pw[k];
          if (RNEA) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
              br[(12 + k) * T] = v[k];
              br[(18 + k) * T] = a[k];
              br[(24 + k) * T] = phi[k];
            }
          }
        }
        lstart = 1;
      }
      // one packed record per (level, slot), read a level ahead (as in the
      // forward kernels), and the branching levels as a scalar mask
      const I4* srec = tb.srec + slot;
      I4 rnext = I4{0, 0, 0, 0};
      if (lstart < dm.depth) rnext = srec[lstart * P];
      for (int l = lstart; l < dm.depth; ++l) {
        const I4 rec = rnext;
        if (l + 1 < dm.depth) rnext = srec[(l + 1) * P];
        const bool act = in_sched && ((rec.w >> 16) & 1);
        const int bb = rec.x;
        const int pos = rec.y, vi = rec.w & 255;
        const bool rev = (rec.w >> 17) & 1;
        const Real qv = q_l[rec.z * T + inst];
        if ((dm.xmask >> l) & 1) {
          const int src = lane0 + (in_sched ? ((rec.w >> 8) & 255) : slot_raw);
#pragma unroll
          for (int k = 0; k < 9; ++k) Rw[k] = xch(Rw[k], src);
#pragma unroll
          for (int k = 0; k < 3; ++k) pw[k] = xch(pw[k], src);
          if (RNEA) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
              v[k] = xch(v[k], src);
              a[k] = xch(a[k], src);
              phi[k] = xch(phi[k], src);
            }
          }
        }
        // Bodies on the world all sit at level 0, where every lane starts from
        // the base state set above; the carried state is never reset.
        Real s[6];
        joint_step(tb.cst + bb * CST, rev, qv, Rw, pw, s);
        if (RNEA) {
          const Real qdv = qd_l[vi * T + inst];
          const Real qddv = qdd_l[vi * T + inst];
          const Real tbv = tb_l[vi * T + inst];
          Real vJ[6], cJ[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) vJ[k] = s[k] * qdv;
          crm(v, vJ, cJ);  // v_parent x (s qd)
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            a[k] = a[k] + s[k] * qddv + cJ[k];
            v[k] = v[k] + vJ[k];
            phi[k] = phi[k] + tbv * s[k];
          }
        }
        if (act) {
          Real* sr = s_l + vi * SD + inst;
#pragma unroll
          for (int k = 0; k < 6; ++k) sr[k * T] = s[k];
          Real* br = body_l + pos * SB + inst;
#pragma unroll
          for (int k = 0; k < 9; ++k) br[k * T] = Rw[k];
#pragma unroll
          for (int k = 0; k < 3; ++k) br[(9 + k) * T] = pw[k];
          if (RNEA) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
              br[(12 + k) * T] = v[k];
              br[(18 + k) * T] = a[k];
              br[(24 + k) * T] = phi[k];
            }
          }
        }
      }
    }
    __syncthreads();

    Real pf[PF];
    if (can_pf && nxt < ar.ntiles)
#pragma unroll
      for (int j = 0; j < PF; ++j) {
        const int i = tid + j * nt;
        pf[j] = (i < KIN * T) ? input(i >> LOGT, nxt * T + (i & (T - 1))) : Real(0);
      }

    // ---------------- body phase: one (body, instance) item per thread ----------------
    // The T lanes of a row group share the body, so the batch sum of the
    // inertial-parameter gradient is a butterfly inside the group.
    for (int b0 = 0; b0 < n; b0 += rstep) {
      const int bb = b0 + r0;
      if (bb >= n) break;
      Real* br = body_l + tb.bm2[bb].x * SB + in;
      Real R[9], p[3];
#pragma unroll
      for (int k = 0; k < 9; ++k) R[k] = br[k * T];
#pragma unroll
      for (int k = 0; k < 3; ++k) p[k] = br[(9 + k) * T];
      if (!RNEA) {
        // w = [vee(Rbar R^T) + p x pbar; pbar]; poses_bar is 3x4 row-major [Rbar | pbar]
        const int64_t b = bok ? bo : ar.B - 1;
        const Real* pb = ar.poses_bar + b * ar.spb_b + (int64_t)(bb * 12) * ar.spb_k;
        Real Rb[9], pbar[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
          for (int c = 0; c < 3; ++c) Rb[3 * r + c] = pb[(4 * r + c) * ar.spb_k];
          pbar[r] = pb[(4 * r + 3) * ar.spb_k];
        }
        auto G = [&](int i, int j) { return Rb[3 * i] * R[3 * j] + Rb[3 * i + 1] * R[3 * j + 1] + Rb[3 * i + 2] * R[3 * j + 2]; };
        Real pxb[3];
        cross3(p, pbar, pxb);
        br[0] = G(2, 1) - G(1, 2) + pxb[0];
        br[T] = G(0, 2) - G(2, 0) + pxb[1];
        br[2 * T] = G(1, 0) - G(0, 1) + pxb[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) br[(3 + k) * T] = pbar[k];
      } else {
        Real v[6], a[6], phi[6], pic[10], I0[10];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          v[k] = br[(12 + k) * T];
          a[k] = br[(18 + k) * T];
          phi[k] = br[(24 + k) * T];
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) pic[k] = ar.pi_ovr ? ar.pi_ovr[bb * 10 + k] : tb.cst[bb * CST + C_PI + k];
        world_inertia(pic, R, p, I0);
        Real Ia[6], h[6], vxh[6], psi[6], abar[6], Ipsi[6], t0[6];
        inertia_mul(I0, a, Ia);
        inertia_mul(I0, v, h);
        crf(v, h, vxh);
        crm(v, phi, t0);
#pragma unroll
        for (int k = 0; k < 6; ++k) psi[k] = -t0[k];
        inertia_mul(I0, phi, abar);
        inertia_mul(I0, psi, Ipsi);
        // vbar_own = [h_w x phi_w + h_u x phi_u; h_u x phi_w] + I psi, then g = vbar_own + v x* abar
        Real c1[3], c2[3], c3[3], g[6];
        cross3(h, phi, c1);
        cross3(h + 3, phi + 3, c2);
        cross3(h + 3, phi, c3);
        crf(v, abar, t0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          g[k] = c1[k] + c2[k] + Ipsi[k] + t0[k];
          g[3 + k] = c3[k] + Ipsi[3 + k] + t0[3 + k];
        }
        // wI = -(phi x* I a + a x* abar + psi x* h + v x* I psi)
        Real wI[6], t1[6], t2[6], t3[6];
        crf(phi, Ia, t0);
        crf(a, abar, t1);
        crf(psi, h, t2);
        crf(v, Ipsi, t3);
#pragma unroll
        for (int k = 0; k < 6; ++k) wI[k] = -(t0[k] + t1[k] + t2[k] + t3[k]);
        if (want_pi) {
          Real gp[10];
          inertia_param_grad(R, p, a, phi, v, psi, gp);
          double sum[10];
#pragma unroll
          for (int k = 0; k < 10; ++k) sum[k] = bok ? (double)gp[k] : 0.0;
#pragma unroll
          for (int sh = 1; sh < T; sh <<= 1)
#pragma unroll
            for (int k = 0; k < 10; ++k) sum[k] += xch(sum[k], lane ^ sh);
          if (in == 0)
#pragma unroll
            for (int k = 0; k < 10; ++k) acc_l[bb * 10 + k] += sum[k];
        }
        // rows 0-5 f, 6-11 abar, 12-17 g, 18-23 v, 24-29 wI
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          br[k * T] = Ia[k] + vxh[k];
          br[(6 + k) * T] = abar[k];
          br[(12 + k) * T] = g[k];
          br[(18 + k) * T] = v[k];
          br[(24 + k) * T] = wI[k];
        }
      }
    }
    __syncthreads();

    if (RNEA) {
      // ---------------- subtree phase 1: F, Abar, G -> qd_bar, qdd_bar, w ----------------
      subtree_sums<Real, 18, 0, LOGT, SB>(tb, dm, body_l, tid, nt, [&](int bb, const I4& m2, int part, const Real* S) {
        if (part != 0) return;
        // m2.w dofs from v index m2.z (one for a revolute or prismatic
        // joint, six for the free root, whose parent velocity is zero)
        Real v[6], w[6], vpar[6];
        Real* br = body_l + m2.x * SB + in;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          v[k] = br[(18 + k) * T];
          w[k] = br[(24 + k) * T];
          vpar[k] = v[k];
        }
        const int nd = FREE ? m2.w : 1;
        for (int d = m2.z; d < m2.z + nd; ++d) {
          const Real* sr = s_l + d * SD + in;
          const Real qdv = qd_l[d * T + in];
#pragma unroll
          for (int k = 0; k < 6; ++k) vpar[k] -= sr[k * T] * qdv;
        }
        const Real* F = S;
        const Real* A = S + 6;
        const Real* G = S + 12;
        Real vxA[6], vpxA[6], vJb[6];
        crf(v, A, vxA);
        crf(vpar, A, vpxA);
#pragma unroll
        for (int k = 0; k < 6; ++k) vJb[k] = G[k] - vxA[k] - vpxA[k];
        for (int d = m2.z; d < m2.z + nd; ++d) {
          const Real* sr = s_l + d * SD + in;
          const Real qdv = qd_l[d * T + in], qddv = qdd_l[d * T + in], tbv = tb_l[d * T + in];
          Real s[6], sb[6], ws[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            s[k] = sr[k * T];
            sb[k] = tbv * F[k] + qdv * vJb[k] + qddv * A[k];
          }
          crf(s, sb, ws);
#pragma unroll
          for (int k = 0; k < 6; ++k) w[k] += ws[k];
          if (bok) {
            ar.qd_bar[bo * ar.sqdo_b + (int64_t)d * ar.sqdo_k] = dot6(s, vJb);
            if (ar.qdd_bar) ar.qdd_bar[bo * ar.sqddo_b + (int64_t)d * ar.sqddo_k] = dot6(s, A);
          }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) br[(24 + k) * T] = w[k];
      });
      __syncthreads();
    }

    // ---------------- subtree phase 2: q_bar = s . (sum of w) ----------------
    constexpr int WROW = RNEA ? 24 : 0;
    subtree_sums<Real, 6, WROW, LOGT, SB>(tb, dm, body_l, tid, nt, [&](int bb, const I4& m2, int part, const Real* S) {
      if (part != 0 || !bok) return;
      const I4 meta = tb.meta[bb];
      Real* qo = ar.q_bar + bo * ar.sqo_b;
      if (FREE && meta.y == J_FREE) {
        // The free root's subtree is the whole tree, so S sums every body's
        // sensitivity: its angular part is the gradient with respect to a
        // rotation of the tree about the base origin, its linear part that
        // with respect to a translation.  With R = R0 R(q^), q^ = q / |q|,
        // a change of q^ rotates the tree by R0 dth, dth = 2 (w dv - dw v +
        // v x dv) for q^ = (v, w) (quaternion product dq^ q^*), so
        // vbar = 2 (w th - v x th), wbar = -2 v . th with th = R0^T (angular
        // part); this is orthogonal to q^, so the normalisation only
        // divides by |q|.  The position moves the tree by R0 dp; RNEA does
        // not depend on it (the frame sits at the base).
        const Real* c = tb.cst + bb * CST + C_R0;
        Real th[3], pb[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          th[j] = c[j] * S[0] + c[3 + j] * S[1] + c[6 + j] * S[2];
          pb[j] = RNEA ? Real(0) : c[j] * S[3] + c[3 + j] * S[4] + c[6 + j] * S[5];
        }
        const int qz = meta.z;
        const Real x = q_l[(qz + 3) * T + in], y = q_l[(qz + 4) * T + in], z = q_l[(qz + 5) * T + in],
                   ww = q_l[(qz + 6) * T + in];
        const Real inv = Real(1) / sqrt(x * x + y * y + z * z + ww * ww);
        const Real u[3] = {x * inv, y * inv, z * inv}, uw = ww * inv;
        Real uxt[3];
        cross3(u, th, uxt);
        const Real g2 = Real(2) * inv;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          qo[(int64_t)(qz + j) * ar.sqo_k] = pb[j];
          qo[(int64_t)(qz + 3 + j) * ar.sqo_k] = g2 * (uw * th[j] - uxt[j]);
        }
        qo[(int64_t)(qz + 6) * ar.sqo_k] = -g2 * (u[0] * th[0] + u[1] * th[1] + u[2] * th[2]);
        return;
      }
      const Real* sr = s_l + m2.z * SD + in;
      Real s[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) s[k] = sr[k * T];
      qo[(int64_t)meta.z * ar.sqo_k] = dot6(s, S);
    });
    if (nxt < ar.ntiles) {
      Real* dst = inbuf[cur ^ 1];  // the previous tile's buffer, no longer read
      if (can_pf) {
#pragma unroll
        for (int j = 0; j < PF; ++j)
          if (tid + j * nt < KIN * T) dst[tid + j * nt] = pf[j];
      } else {
        for (int i = tid; i < KIN * T; i += nt) dst[i] = input(i >> LOGT, nxt * T + (i & (T - 1)));
      }
    }
    cur ^= 1;
  }
  __syncthreads();  // every thread's last inertial-parameter sums are in LDS

  if (want_pi) {
    double* out = ar.partial + (int64_t)blockIdx.x * n * 10;
    for (int i = tid; i < n * 10; i += nt) out[i] = acc_l[i];
  }
}

// ---------------------------------------------------------------------------
// Scratch of bard_rnea_vjp_noalloc: the per-workgroup inertial-parameter sums
// live in this file-scope array (one copy per GPU, held until the process
// ends) instead of a buffer the library allocates.  Host code reaches it only
// through the device address hipGetSymbolAddress returns for the current
// device; the array's name in host code is not a device address.
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

hipError_t noalloc_scratch(double** out) {
  static std::mutex mu;
  static double* addr[BARD_MAX_DEVICES] = {nullptr};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= BARD_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *out = addr[dev];
  return hipSuccess;
}

// Fixed-order batch reduction of the per-workgroup inertial-parameter sums.
template <class Real>
__global__ void __launch_bounds__(256) param_reduce_kernel(const double* partial, int groups, int count, Real* out) {
  __shared__ double red[256];
  const int idx = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int g = t; g < groups; g += 256) s += partial[(int64_t)g * count + idx];
  red[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[idx] = (Real)red[0];
}

template <class Real, bool RNEA, bool FREE, int LOGT>
static hipError_t launch_adjoint_t(const DevModel& dm, const AdjArgs<Real>& ar, int grid, int block, size_t lds,
                                   hipStream_t st) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)adjoint_kernel<Real, RNEA, FREE, LOGT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((adjoint_kernel<Real, RNEA, FREE, LOGT>), dim3(grid), dim3(block), lds, st, dm, ar);
  return hipGetLastError();
}

template <class Real, bool RNEA, bool FREE>
static hipError_t launch_adjoint_f(const DevModel& dm, const AdjArgs<Real>& ar, int grid, int block, size_t lds,
                                   hipStream_t st) {
  switch (ar.logT) {
    case 3: return launch_adjoint_t<Real, RNEA, FREE, 3>(dm, ar, grid, block, lds, st);
    case 4: return launch_adjoint_t<Real, RNEA, FREE, 4>(dm, ar, grid, block, lds, st);
    case 5: return launch_adjoint_t<Real, RNEA, FREE, 5>(dm, ar, grid, block, lds, st);
    case 6: return launch_adjoint_t<Real, RNEA, FREE, 6>(dm, ar, grid, block, lds, st);
    default: return hipErrorInvalidValue;
  }
}

template <class Real, bool RNEA>
hipError_t launch_adjoint(const DevModel& dm, const AdjArgs<Real>& ar, int grid, int block, size_t lds,
                          hipStream_t st) {
  return dm.free_root ? launch_adjoint_f<Real, RNEA, true>(dm, ar, grid, block, lds, st)
                      : launch_adjoint_f<Real, RNEA, false>(dm, ar, grid, block, lds, st);
}

template <class Real, bool RNEA, bool FREE, int LOGT>
static hipError_t adjoint_resident_t(int block, size_t lds, int* per_cu) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)adjoint_kernel<Real, RNEA, FREE, LOGT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, adjoint_kernel<Real, RNEA, FREE, LOGT>, block, lds);
}

template <class Real, bool RNEA, bool FREE>
static hipError_t adjoint_resident_f(int logT, int block, size_t lds, int* per_cu) {
  switch (logT) {
    case 3: return adjoint_resident_t<Real, RNEA, FREE, 3>(block, lds, per_cu);
    case 4: return adjoint_resident_t<Real, RNEA, FREE, 4>(block, lds, per_cu);
    case 5: return adjoint_resident_t<Real, RNEA, FREE, 5>(block, lds, per_cu);
    case 6: return adjoint_resident_t<Real, RNEA, FREE, 6>(block, lds, per_cu);
    default: return hipErrorInvalidValue;
  }
}

template <class Real, bool RNEA>
hipError_t adjoint_resident(int logT, int free_root, int block, size_t lds, int* per_cu) {
  return free_root ? adjoint_resident_f<Real, RNEA, true>(logT, block, lds, per_cu)
                   : adjoint_resident_f<Real, RNEA, false>(logT, block, lds, per_cu);
}

template <class Real>
hipError_t launch_param_reduce(const double* partial, int groups, int count, Real* out, hipStream_t st) {
  hipLaunchKernelGGL((param_reduce_kernel<Real>), dim3(count), dim3(256), 0, st, partial, groups, count, out);
  return hipGetLastError();
}

#define BARD_ADJ_INST(R)                                                                                      \
  template hipError_t launch_adjoint<R, true>(const DevModel&, const AdjArgs<R>&, int, int, size_t, hipStream_t); \
  template hipError_t launch_adjoint<R, false>(const DevModel&, const AdjArgs<R>&, int, int, size_t, hipStream_t); \
  template hipError_t launch_param_reduce<R>(const double*, int, int, R*, hipStream_t);                            \
  template hipError_t adjoint_resident<R, true>(int, int, int, size_t, int*);                                          \
  template hipError_t adjoint_resident<R, false>(int, int, int, size_t, int*);

BARD_ADJ_INST(float)
BARD_ADJ_INST(double)

}  // namespace bard
