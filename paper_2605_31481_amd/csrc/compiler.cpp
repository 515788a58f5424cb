// Host-side model compiler: validation, level schedule, joint constants, tables.
//
// The paper parses a robot once into an immutable model holding topology,
// inertias and precomputed constants (Fig. 1, Sec. 3).  This compile step
// produces, per body, the Rodrigues constants of eqs. (2)-(3) so that kernels
// evaluate each joint transform with one sincos and element-wise terms
// (eqs. (4)-(5)), and the level-order grouping of Sec. 3.3 laid out as a lane
// schedule: every level is one step, every body of a level gets a lane slot,
// and a child continues in its parent's slot when it can, so state moves
// between lanes only where the tree branches.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "model.h"
#include "status.h"

namespace bard {

namespace {

void skew(const double a[3], double K[9]) {
  K[0] = 0; K[1] = -a[2]; K[2] = a[1];
  K[3] = a[2]; K[4] = 0; K[5] = -a[0];
  K[6] = -a[1]; K[7] = a[0]; K[8] = 0;
}

void mul3(const double* a, const double* b, double* c) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

// Positive definiteness of a symmetric 3x3 by leading principal minors.
bool spd3(const double S[9]) {
  double d1 = S[0];
  double d2 = S[0] * S[4] - S[1] * S[3];
  double d3 = S[0] * (S[4] * S[8] - S[5] * S[7]) - S[1] * (S[3] * S[8] - S[5] * S[6]) +
              S[2] * (S[3] * S[7] - S[4] * S[6]);
  return d1 > 0 && d2 > 0 && d3 > 0;
}

bool is_ancestor(const bard_model* m, int a, int b) {  // a is b or an ancestor of b
  for (int k = b; k >= 0; k = m->parent[k])
    if (k == a) return true;
  return false;
}

}  // namespace

int compile_model(bard_model* m, std::string* err) {
  const int n = m->n;
  if (n < 1 || n > BARD_MAX_BODIES) {
    *err = "n_bodies must be in 1.." + std::to_string(BARD_MAX_BODIES);
    return BARD_E_ARG;
  }
  m->qi.assign(n, 0);
  m->vi.assign(n, 0);
  m->nvi.assign(n, 0);
  m->nq = m->nv = 0;
  for (int i = 0; i < n; ++i) {
    int p = m->parent[i];
    if (p < -1 || p >= i) {
      *err = "parent[" + std::to_string(i) + "] = " + std::to_string(p) + " must be in [-1, i-1]";
      return BARD_E_TOPOLOGY;
    }
    int t = m->jtype[i];
    if (t == J_FIXED) {
      *err = "fixed joints are not supported (merge the body into its parent)";
      return BARD_E_UNSUPPORTED;
    }
    if (t != J_REV && t != J_PRI && t != J_FREE) {
      *err = "joint_type[" + std::to_string(i) + "] is not a valid bard_joint";
      return BARD_E_TOPOLOGY;
    }
    if (t == J_FREE && (i != 0 || p != -1)) {
      *err = "a free joint is only allowed on body 0 attached to the world";
      return BARD_E_TOPOLOGY;
    }
    if (i > 0 && p == -1 && m->jtype[0] == J_FREE) {
      *err = "with a free root every other body must descend from it (body " + std::to_string(i) +
             " is attached to the world)";
      return BARD_E_TOPOLOGY;
    }
    if (t != J_FREE) {
      double* a = &m->axis[3 * i];
      double nrm = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
      if (!(nrm > 1e-12)) {
        *err = "axis of body " + std::to_string(i) + " is zero";
        return BARD_E_TOPOLOGY;
      }
      for (int k = 0; k < 3; ++k) a[k] /= nrm;
    }
    const double* X = &m->xtree[12 * i];
    double R[9], RtR[9], Rt[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        R[3 * r + c] = X[4 * r + c];
        Rt[3 * c + r] = X[4 * r + c];
      }
    mul3(Rt, R, RtR);
    double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                 R[2] * (R[3] * R[7] - R[4] * R[6]);
    double dev = std::fabs(det - 1.0);
    for (int k = 0; k < 9; ++k) dev = std::max(dev, std::fabs(RtR[k] - (k % 4 == 0 ? 1.0 : 0.0)));
    if (!(dev < 1e-6)) {
      *err = "X_tree rotation of body " + std::to_string(i) + " is not a rotation matrix";
      return BARD_E_ARG;
    }
    const double* pi = &m->inertia[10 * i];
    double mass = pi[0];
    if (!(mass > 0)) {
      *err = "mass of body " + std::to_string(i) + " must be positive";
      return BARD_E_INERTIA;
    }
    double c[3] = {pi[1] / mass, pi[2] / mass, pi[3] / mass};
    double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    double Io[9] = {pi[4], pi[5], pi[7], pi[5], pi[6], pi[8], pi[7], pi[8], pi[9]};
    double Ic[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) Ic[3 * r + k] = Io[3 * r + k] - mass * ((r == k ? cc : 0.0) - c[r] * c[k]);
    if (!spd3(Ic)) {
      *err = "COM inertia of body " + std::to_string(i) + " is not positive definite";
      return BARD_E_INERTIA;
    }
    m->qi[i] = m->nq;
    m->vi[i] = m->nv;
    m->nvi[i] = (t == J_FREE) ? 6 : 1;
    m->nq += (t == J_FREE) ? 7 : 1;
    m->nv += m->nvi[i];
  }
  if (m->nv > BARD_MAX_NV) {
    *err = "nv exceeds " + std::to_string(BARD_MAX_NV);
    return BARD_E_CAPACITY;
  }
  m->free_root = (m->jtype[0] == J_FREE);

  // ---- levels (Sec. 3.3): depth 1 for bodies on the world/base ----
  m->level_of.assign(n, 0);
  m->children.assign(n, {});
  int depth = 0;
  for (int i = 0; i < n; ++i) {
    int p = m->parent[i];
    m->level_of[i] = (p < 0) ? 0 : m->level_of[p] + 1;
    if (p >= 0) m->children[p].push_back(i);
    depth = std::max(depth, m->level_of[i] + 1);
  }
  m->depth = depth;
  std::vector<std::vector<int>> levels(depth);
  for (int i = 0; i < n; ++i) levels[m->level_of[i]].push_back(i);
  int width = 0;
  for (auto& l : levels) width = std::max<int>(width, (int)l.size());

  // ---- lane slots: a child continues in its parent's slot when that slot is unclaimed ----
  m->slot_of.assign(n, -1);
  for (int l = 0; l < depth; ++l) {
    std::vector<char> taken(width, 0);
    std::vector<int> rest;
    for (int b : levels[l]) {
      int p = m->parent[b];
      if (l > 0 && !taken[m->slot_of[p]]) {
        m->slot_of[b] = m->slot_of[p];
        taken[m->slot_of[b]] = 1;
      } else {
        rest.push_back(b);
      }
    }
    for (int b : rest) {
      int s = 0;
      while (taken[s]) ++s;
      m->slot_of[b] = s;
      taken[s] = 1;
    }
  }
  int P = 1, log2P = 0;
  while (P < width) {
    P <<= 1;
    ++log2P;
  }
  m->P = P;
  m->log2P = log2P;

  int kmax = 1;
  for (int i = 0; i < n; ++i) kmax = std::max<int>(kmax, (int)m->children[i].size());
  m->kmax = kmax;
  m->sched_body.assign(depth * P, -1);
  m->sched_src.assign(depth * P, 0);
  m->child_slot.assign(depth * P * kmax, -1);
  m->level_info.assign(depth * 2, 0);
  for (int l = 0; l < depth; ++l) {
    for (int s = 0; s < P; ++s) m->sched_src[l * P + s] = (int8_t)s;
    int K = 0, shuffle = 0;
    for (int b : levels[l]) {
      int s = m->slot_of[b];
      m->sched_body[l * P + s] = (int16_t)b;
      if (m->parent[b] >= 0) {
        int ps = m->slot_of[m->parent[b]];
        m->sched_src[l * P + s] = (int8_t)ps;
        if (ps != s) shuffle = 1;
      }
      const auto& ch = m->children[b];
      K = std::max<int>(K, (int)ch.size());
      for (size_t k = 0; k < ch.size(); ++k) m->child_slot[(l * P + s) * kmax + k] = (int8_t)m->slot_of[ch[k]];
    }
    m->level_info[2 * l] = K;
    m->level_info[2 * l + 1] = shuffle;
  }

  // ---- preorder positions: every subtree is a contiguous range of positions ----
  m->dfs.assign(n, 0);
  m->sub_size.assign(n, 1);
  for (int i = n - 1; i >= 0; --i)
    if (m->parent[i] >= 0) m->sub_size[m->parent[i]] += m->sub_size[i];
  {
    int pos = 0;
    std::vector<int> stack;
    for (int i = n - 1; i >= 0; --i)
      if (m->parent[i] < 0) stack.push_back(i);
    while (!stack.empty()) {
      int b = stack.back();
      stack.pop_back();
      m->dfs[b] = pos++;
      const auto& ch = m->children[b];
      for (int k = (int)ch.size() - 1; k >= 0; --k) stack.push_back(ch[k]);
    }
  }
  // ---- level-sweep records: everything one (level, slot) step needs, in one
  // 16-byte entry, so a lane reads it a level ahead and issues all of the
  // step's loads at once: {body, preorder position, q index,
  // v index | source slot << 8 | active << 16 | revolute << 17}.  Empty slots
  // step on body 0 and store nothing.
  m->srec.assign((size_t)depth * P, I4{0, 0, 0, 0});
  m->xmask = 0;
  for (int l = 0; l < depth; ++l) {
    if (m->level_info[2 * l + 1]) m->xmask |= 1ull << l;
    for (int s = 0; s < P; ++s) {
      const int b = m->sched_body[l * P + s];
      const int bb = b >= 0 ? b : 0;
      const int flags = m->vi[bb] | (int)(uint8_t)m->sched_src[l * P + s] << 8 | (b >= 0 ? 1 : 0) << 16 |
                        (m->jtype[bb] == J_REV ? 1 : 0) << 17;
      m->srec[(size_t)l * P + s] = I4{bb, m->dfs[bb], m->qi[bb], flags};
    }
  }
  // ---- pointer-jumping tables: ancestor of each body at distance 2^s ----
  m->jsteps = 0;
  while ((1 << m->jsteps) < m->depth) ++m->jsteps;
  m->jump.assign((size_t)m->jsteps * n, -1);
  for (int s = 0; s < m->jsteps; ++s)
    for (int i = 0; i < n; ++i) {
      int a = i;
      for (int k = 0; k < (1 << s) && a >= 0; ++k) a = m->parent[a];
      m->jump[(size_t)s * n + i] = (int8_t)a;
    }
  m->dlist.resize(n);
  for (int i = 0; i < n; ++i) m->dlist[i] = i;
  std::stable_sort(m->dlist.begin(), m->dlist.end(),
                   [&](int a, int b) { return m->sub_size[a] > m->sub_size[b]; });

  for (int k = 0; k < 4; ++k) m->ulist[k] = subtree_units(m, 1 << k);

  // ---- joint constants (eqs. (2)-(3)) and inertial parameters ----
  m->cst64.assign((size_t)n * CST, 0.0);
  for (int i = 0; i < n; ++i) {
    double* c = &m->cst64[(size_t)i * CST];
    const double* X = &m->xtree[12 * i];
    double Rp[9], tp[3];
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) Rp[3 * r + k] = X[4 * r + k];
      tp[r] = X[4 * r + 3];
    }
    const double* a = &m->axis[3 * i];
    double K[9], K2[9], A[9], B[9];
    skew(a, K);
    mul3(K, K, K2);
    mul3(Rp, K, A);
    mul3(Rp, K2, B);
    for (int k = 0; k < 9; ++k) {
      c[C_R0 + k] = Rp[k];
      c[C_A + k] = (m->jtype[i] == J_REV) ? A[k] : 0.0;
      c[C_B + k] = (m->jtype[i] == J_REV) ? B[k] : 0.0;
    }
    for (int k = 0; k < 3; ++k) {
      c[C_T0 + k] = tp[k];
      c[C_AX + k] = (m->jtype[i] == J_FREE) ? 0.0 : a[k];
      c[C_D + k] = (m->jtype[i] == J_PRI) ? (Rp[3 * k] * a[0] + Rp[3 * k + 1] * a[1] + Rp[3 * k + 2] * a[2]) : 0.0;
    }
    for (int k = 0; k < 10; ++k) c[C_PI + k] = m->inertia[10 * i + k];
  }
  m->cst32.resize(m->cst64.size());
  for (size_t k = 0; k < m->cst64.size(); ++k) m->cst32[k] = (float)m->cst64[k];

  // ---- mass-matrix output lists ----
  // Pairs: every dof pair (a, d) where body(a) is an ancestor of body(d), or
  // the same body with a <= d; M[a][d] = M[d][a] = s_a . (Ic_body(d) s_d).
  // Code a | d << 16.  Zeros: the row-major index of every other entry.
  // Both lists share one region of nv*nv ints (pairs first); their lengths
  // add up to nv*nv - n_pairs + nv <= nv*nv.
  std::vector<int> body_of(m->nv);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < m->nvi[i]; ++k) body_of[m->vi[i] + k] = i;
  std::vector<int> pairs, zeros;
  for (int r = 0; r < m->nv; ++r)
    for (int cc = 0; cc < m->nv; ++cc) {
      const int br = body_of[r], bc = body_of[cc];
      const bool related = br == bc || is_ancestor(m, br, bc) || is_ancestor(m, bc, br);
      if (!related) {
        zeros.push_back(r * m->nv + cc);
        continue;
      }
      // record each unordered pair once, from the upper triangle of its (a, d) order
      int a, d;
      if (br == bc) {
        a = std::min(r, cc);
        d = std::max(r, cc);
      } else if (is_ancestor(m, br, bc)) {
        a = r;
        d = cc;
      } else {
        a = cc;
        d = r;
      }
      if (r == a && cc == d) pairs.push_back(a | (d << 16));
    }
  m->n_mpair = (int)pairs.size();
  m->n_mzero = (int)zeros.size();
  m->mtab = pairs;
  m->mtab.insert(m->mtab.end(), zeros.begin(), zeros.end());
  return BARD_OK;
}

std::vector<int> subtree_units(const bard_model* m, int U) {
  std::vector<int> out;
  std::vector<int> small;
  for (int b : m->dlist) {
    if (U > 1 && m->sub_size[b] > 2 * U)
      for (int p = 0; p < U; ++p) out.push_back(b | (p << 8) | (U << 12));
    else
      small.push_back(b | (1 << 12));
  }
  out.insert(out.end(), small.begin(), small.end());
  while (out.size() % U) out.push_back(-1);
  return out;
}

std::vector<int> jacobian_table(const bard_model* m, const std::vector<int>& ee, int* n_cols, int* n_zeros) {
  // Columns: every (end effector e, dof c) with c on the root path of e; the
  // kernel writes its 6 rows from s_c.  Code c | e << 8.  Zeros: the index of
  // every row (e, r, c) of the [n_ee][6][nv] output whose dof is off the path.
  const int nv = m->nv;
  std::vector<char> on(nv);
  std::vector<int> cols, zeros;
  for (size_t e = 0; e < ee.size(); ++e) {
    std::fill(on.begin(), on.end(), 0);
    for (int k = ee[e]; k >= 0; k = m->parent[k])
      for (int j = 0; j < m->nvi[k]; ++j) on[m->vi[k] + j] = 1;
    for (int c = 0; c < nv; ++c)
      if (on[c]) cols.push_back(c | ((int)e << 8));
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < nv; ++c)
        if (!on[c]) zeros.push_back(((int)e * 6 + r) * nv + c);
  }
  *n_cols = (int)cols.size();
  *n_zeros = (int)zeros.size();
  cols.insert(cols.end(), zeros.begin(), zeros.end());
  return cols;
}

}  // namespace bard
