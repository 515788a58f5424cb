// FP64 CPU oracle for batched rigid-body kinematics and dynamics.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load this library.  It shares no code, header,
// table or constant with the GPU library and is built by g++ on its own.
//
// What it computes, and the passage each routine follows:
//   * FK         -- world pose of every body, T_0i = T_0parent * T_joint * J(q)
//                   (the parent-child composition of Sec. 3.2, eq. (1)), built from
//                   naive 4x4 products with the joint rotation taken from a unit
//                   quaternion, i.e. not from the precomputed Rodrigues constants.
//   * Jacobian   -- per joint on the root-to-end-effector path, the column
//                   Ad(T_0k) S_k formed with an explicit 6x6 adjoint: the
//                   "standard approach" that Sec. 3.4 replaces by eq. (7).
//   * RNEA, CRBA, ABA -- the textbook recursions the paper implements (Sec. 3,
//                   Featherstone's algorithms), in body coordinates with explicit
//                   6x6 Plucker transforms, run sequentially over body index.
//   * kinetic and potential energy, used by the invariant checks.
//   * the spatial force each joint transmits (the RNEA backward pass's f_i),
//     whose size sets the tests' per-entry torque tolerance; and the RNEA and
//     CRBA recursions instantiated in single precision, which the tests use
//     only to show that tolerance is attainable by a plain evaluation.
//   * vector-Jacobian products of RNEA and FK by reverse-mode automatic
//     differentiation on a private tape (Sec. 3.5 functional mode and Sec. 4.3
//     gradient-based identification use autograd for the same derivatives).
//
// Conventions:
//   spatial motion vectors are [w; v], force vectors [n; f];
//   free joint: q = [x y z qx qy qz qw] (quaternion normalised on read),
//   velocity = body-frame twist [v; w];
//   gravity enters as the base acceleration a_0 = -g;
//   Jacobian rows are [linear; angular]; frame 0 = world origin (spatial),
//   frame 1 = velocity of the end-effector origin expressed in world axes.
//
// Functions are templated on the scalar so the same text runs on double and on
// the tape type used for the adjoints.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace orc {

// ----------------------------------------------------------------------------
// Reverse-mode automatic differentiation on a per-thread tape.
// ----------------------------------------------------------------------------
struct Node {
  int p0, p1;        // parent node indices (-1 = none)
  double d0, d1;     // partial derivatives with respect to the parents
};

struct Tape {
  std::vector<Node> nodes;
  int push(int p0, double d0, int p1, double d1) {
    nodes.push_back(Node{p0, p1, d0, d1});
    return (int)nodes.size() - 1;
  }
};

thread_local Tape* g_tape = nullptr;

struct Var {
  double v;
  int id;  // -1 for a constant
  Var() : v(0.0), id(-1) {}
  Var(double x) : v(x), id(-1) {}
  Var(double x, int i) : v(x), id(i) {}
};

static inline Var mk(double v, int p0, double d0, int p1, double d1) {
  if (p0 < 0 && p1 < 0) return Var(v);
  return Var(v, g_tape->push(p0, d0, p1, d1));
}
static inline Var leaf(double v) { return Var(v, g_tape->push(-1, 0.0, -1, 0.0)); }

static inline Var operator+(const Var& a, const Var& b) { return mk(a.v + b.v, a.id, 1.0, b.id, 1.0); }
static inline Var operator-(const Var& a, const Var& b) { return mk(a.v - b.v, a.id, 1.0, b.id, -1.0); }
static inline Var operator*(const Var& a, const Var& b) { return mk(a.v * b.v, a.id, b.v, b.id, a.v); }
static inline Var operator/(const Var& a, const Var& b) {
  double r = a.v / b.v;
  return mk(r, a.id, 1.0 / b.v, b.id, -r / b.v);
}
static inline Var operator-(const Var& a) { return mk(-a.v, a.id, -1.0, -1, 0.0); }
static inline Var& operator+=(Var& a, const Var& b) { a = a + b; return a; }
static inline Var& operator-=(Var& a, const Var& b) { a = a - b; return a; }
static inline Var sin(const Var& a) { return mk(std::sin(a.v), a.id, std::cos(a.v), -1, 0.0); }
static inline Var cos(const Var& a) { return mk(std::cos(a.v), a.id, -std::sin(a.v), -1, 0.0); }
static inline Var sqrt(const Var& a) {
  double r = std::sqrt(a.v);
  return mk(r, a.id, 0.5 / r, -1, 0.0);
}
static inline double val(const Var& a) { return a.v; }
static inline double val(double a) { return a; }

using std::sin;
using std::cos;
using std::sqrt;

// ----------------------------------------------------------------------------
// Small dense algebra.
// ----------------------------------------------------------------------------
template <class S> struct M3 { S a[3][3]; };
template <class S> struct V3 { S a[3]; };
template <class S> struct M6 { S a[6][6]; };
template <class S> struct V6 { S a[6]; };
template <class S> struct M4 { S a[4][4]; };

template <class S> M3<S> m3_zero() { M3<S> r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.a[i][j] = S(0.0); return r; }
template <class S> M3<S> m3_eye() { M3<S> r = m3_zero<S>(); for (int i = 0; i < 3; ++i) r.a[i][i] = S(1.0); return r; }
template <class S> M3<S> m3_mul(const M3<S>& x, const M3<S>& y) {
  M3<S> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S s(0.0);
      for (int k = 0; k < 3; ++k) s += x.a[i][k] * y.a[k][j];
      r.a[i][j] = s;
    }
  return r;
}
template <class S> M3<S> m3_t(const M3<S>& x) { M3<S> r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.a[i][j] = x.a[j][i]; return r; }
template <class S> M3<S> skew(const V3<S>& v) {
  M3<S> r = m3_zero<S>();
  r.a[0][1] = -v.a[2]; r.a[0][2] = v.a[1];
  r.a[1][0] = v.a[2];  r.a[1][2] = -v.a[0];
  r.a[2][0] = -v.a[1]; r.a[2][1] = v.a[0];
  return r;
}
template <class S> V3<S> m3v(const M3<S>& m, const V3<S>& v) {
  V3<S> r;
  for (int i = 0; i < 3; ++i) r.a[i] = m.a[i][0] * v.a[0] + m.a[i][1] * v.a[1] + m.a[i][2] * v.a[2];
  return r;
}
template <class S> V3<S> cross3(const V3<S>& x, const V3<S>& y) {
  V3<S> r;
  r.a[0] = x.a[1] * y.a[2] - x.a[2] * y.a[1];
  r.a[1] = x.a[2] * y.a[0] - x.a[0] * y.a[2];
  r.a[2] = x.a[0] * y.a[1] - x.a[1] * y.a[0];
  return r;
}

template <class S> M6<S> m6_zero() { M6<S> r; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) r.a[i][j] = S(0.0); return r; }
template <class S> V6<S> v6_zero() { V6<S> r; for (int i = 0; i < 6; ++i) r.a[i] = S(0.0); return r; }
template <class S> M6<S> m6_mul(const M6<S>& x, const M6<S>& y) {
  M6<S> r;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      S s(0.0);
      for (int k = 0; k < 6; ++k) s += x.a[i][k] * y.a[k][j];
      r.a[i][j] = s;
    }
  return r;
}
template <class S> M6<S> m6_t(const M6<S>& x) { M6<S> r; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) r.a[i][j] = x.a[j][i]; return r; }
template <class S> M6<S> m6_add(const M6<S>& x, const M6<S>& y) { M6<S> r; for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) r.a[i][j] = x.a[i][j] + y.a[i][j]; return r; }
template <class S> V6<S> m6v(const M6<S>& m, const V6<S>& v) {
  V6<S> r;
  for (int i = 0; i < 6; ++i) {
    S s(0.0);
    for (int k = 0; k < 6; ++k) s += m.a[i][k] * v.a[k];
    r.a[i] = s;
  }
  return r;
}
template <class S> V6<S> m6tv(const M6<S>& m, const V6<S>& v) {
  V6<S> r;
  for (int i = 0; i < 6; ++i) {
    S s(0.0);
    for (int k = 0; k < 6; ++k) s += m.a[k][i] * v.a[k];
    r.a[i] = s;
  }
  return r;
}
template <class S> V6<S> v6_add(const V6<S>& x, const V6<S>& y) { V6<S> r; for (int i = 0; i < 6; ++i) r.a[i] = x.a[i] + y.a[i]; return r; }
template <class S> S v6_dot(const V6<S>& x, const V6<S>& y) { S s(0.0); for (int i = 0; i < 6; ++i) s += x.a[i] * y.a[i]; return s; }

// Plucker motion transform X = rot(E) xlt(r) = [E 0; -E r^ E].
template <class S> M6<S> plux(const M3<S>& E, const V3<S>& r) {
  M6<S> X = m6_zero<S>();
  M3<S> Er = m3_mul(E, skew(r));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      X.a[i][j] = E.a[i][j];
      X.a[i + 3][j + 3] = E.a[i][j];
      X.a[i + 3][j] = -Er.a[i][j];
    }
  return X;
}

// Spatial cross products: crm(v) acting on motion vectors, crf(v) = -crm(v)^T on forces.
template <class S> M6<S> crm(const V6<S>& v) {
  V3<S> w{{v.a[0], v.a[1], v.a[2]}}, u{{v.a[3], v.a[4], v.a[5]}};
  M3<S> W = skew(w), U = skew(u);
  M6<S> r = m6_zero<S>();
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      r.a[i][j] = W.a[i][j];
      r.a[i + 3][j + 3] = W.a[i][j];
      r.a[i + 3][j] = U.a[i][j];
    }
  return r;
}
template <class S> M6<S> crf(const V6<S>& v) {
  M6<S> c = crm(v);
  M6<S> r;
  for (int i = 0; i < 6; ++i) for (int j = 0; j < 6; ++j) r.a[i][j] = -c.a[j][i];
  return r;
}

// Rotation matrix of a unit quaternion (x, y, z, w): columns are the rotated axes.
template <class S> M3<S> quat_to_R(S x, S y, S z, S w) {
  M3<S> R;
  R.a[0][0] = S(1.0) - S(2.0) * (y * y + z * z);
  R.a[0][1] = S(2.0) * (x * y - z * w);
  R.a[0][2] = S(2.0) * (x * z + y * w);
  R.a[1][0] = S(2.0) * (x * y + z * w);
  R.a[1][1] = S(1.0) - S(2.0) * (x * x + z * z);
  R.a[1][2] = S(2.0) * (y * z - x * w);
  R.a[2][0] = S(2.0) * (x * z - y * w);
  R.a[2][1] = S(2.0) * (y * z + x * w);
  R.a[2][2] = S(1.0) - S(2.0) * (x * x + y * y);
  return R;
}

// Rotation by angle q about the unit axis a, through the half-angle quaternion.
template <class S> M3<S> axis_angle_R(const double* a, const S& q) {
  S h = q * S(0.5);
  S s = sin(h), c = cos(h);
  return quat_to_R<S>(s * S(a[0]), s * S(a[1]), s * S(a[2]), c);
}

// ----------------------------------------------------------------------------
// Model.
// ----------------------------------------------------------------------------
enum { REV = 0, PRI = 1, FREE = 2, FIXED = 3 };

struct Model {
  int n = 0, nq = 0, nv = 0;
  std::vector<int> parent, jtype, qo, vo, nqi, nvi;
  std::vector<double> axis, xtree, inertia;
  double g[3] = {0.0, 0.0, -9.81};
};

// Spatial inertia in body coordinates from [m, h(3), Ixx Ixy Iyy Ixz Iyz Izz] about the body origin:
// I = [I_O, h^; h^T, m 1].
template <class S> M6<S> spatial_inertia(const S* p) {
  M6<S> I = m6_zero<S>();
  S m = p[0];
  V3<S> h{{p[1], p[2], p[3]}};
  M3<S> Io;
  Io.a[0][0] = p[4]; Io.a[0][1] = p[5]; Io.a[1][1] = p[6];
  Io.a[0][2] = p[7]; Io.a[1][2] = p[8]; Io.a[2][2] = p[9];
  Io.a[1][0] = p[5]; Io.a[2][0] = p[7]; Io.a[2][1] = p[8];
  M3<S> H = skew(h);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      I.a[i][j] = Io.a[i][j];
      I.a[i][j + 3] = H.a[i][j];
      I.a[i + 3][j] = H.a[j][i];
    }
  for (int i = 0; i < 3; ++i) I.a[i + 3][i + 3] = m;
  return I;
}

// Pose of joint i's frame in the parent body frame.
template <class S> void tree_offset(const Model& M, int i, M3<S>& R, V3<S>& t) {
  const double* x = &M.xtree[12 * i];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) R.a[r][c] = S(x[4 * r + c]);
    t.a[r] = S(x[4 * r + 3]);
  }
}

// Rotation and translation of the body frame relative to its joint frame.
template <class S> void joint_motion(const Model& M, int i, const S* q, M3<S>& R, V3<S>& t) {
  const double* a = &M.axis[3 * i];
  const S* qi = q + M.qo[i];
  switch (M.jtype[i]) {
    case REV:
      R = axis_angle_R<S>(a, qi[0]);
      t = V3<S>{{S(0.0), S(0.0), S(0.0)}};
      break;
    case PRI:
      R = m3_eye<S>();
      t = V3<S>{{qi[0] * S(a[0]), qi[0] * S(a[1]), qi[0] * S(a[2])}};
      break;
    case FREE: {
      S nrm = sqrt(qi[3] * qi[3] + qi[4] * qi[4] + qi[5] * qi[5] + qi[6] * qi[6]);
      R = quat_to_R<S>(qi[3] / nrm, qi[4] / nrm, qi[5] / nrm, qi[6] / nrm);
      t = V3<S>{{qi[0], qi[1], qi[2]}};
      break;
    }
    default:
      R = m3_eye<S>();
      t = V3<S>{{S(0.0), S(0.0), S(0.0)}};
  }
}

// Motion subspace columns (body coordinates), 6 x nvi.
template <class S> void motion_subspace(const Model& M, int i, V6<S>* cols) {
  const double* a = &M.axis[3 * i];
  switch (M.jtype[i]) {
    case REV:
      cols[0] = V6<S>{{S(a[0]), S(a[1]), S(a[2]), S(0.0), S(0.0), S(0.0)}};
      break;
    case PRI:
      cols[0] = V6<S>{{S(0.0), S(0.0), S(0.0), S(a[0]), S(a[1]), S(a[2])}};
      break;
    case FREE:
      // velocity coordinates [v; w] -> spatial [w; v]
      for (int k = 0; k < 6; ++k) cols[k] = v6_zero<S>();
      for (int k = 0; k < 3; ++k) {
        cols[k].a[3 + k] = S(1.0);
        cols[3 + k].a[k] = S(1.0);
      }
      break;
    default:
      break;
  }
}

// X_up[i] = X_J(q_i) * X_tree[i]: parent-body coordinates -> body-i coordinates.
template <class S> M6<S> x_up(const Model& M, int i, const S* q) {
  M3<S> Rp, Rj;
  V3<S> tp, tj;
  tree_offset<S>(M, i, Rp, tp);
  joint_motion<S>(M, i, q, Rj, tj);
  M6<S> XT = plux<S>(m3_t(Rp), tp);
  M6<S> XJ = plux<S>(m3_t(Rj), tj);
  return m6_mul(XJ, XT);
}

template <class S> V6<S> base_accel(const Model& M) {
  return V6<S>{{S(0.0), S(0.0), S(0.0), S(-M.g[0]), S(-M.g[1]), S(-M.g[2])}};
}

template <class S> V6<S> subspace_times(const V6<S>* cols, int ni, const S* x) {
  V6<S> r = v6_zero<S>();
  for (int k = 0; k < ni; ++k)
    for (int c = 0; c < 6; ++c) r.a[c] += cols[k].a[c] * x[k];
  return r;
}

// ----------------------------------------------------------------------------
// Forward kinematics: 4x4 homogeneous products, T_0i = T_0p * T_tree * T_joint.
// ----------------------------------------------------------------------------
template <class S> M4<S> homog(const M3<S>& R, const V3<S>& t) {
  M4<S> T;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) T.a[r][c] = R.a[r][c];
    T.a[r][3] = t.a[r];
    T.a[3][r] = S(0.0);
  }
  T.a[3][3] = S(1.0);
  return T;
}
template <class S> M4<S> m4_mul(const M4<S>& x, const M4<S>& y) {
  M4<S> r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      S s(0.0);
      for (int k = 0; k < 4; ++k) s += x.a[i][k] * y.a[k][j];
      r.a[i][j] = s;
    }
  return r;
}

template <class S> void fk_one(const Model& M, const S* q, std::vector<M4<S>>& T) {
  T.resize(M.n);
  for (int i = 0; i < M.n; ++i) {
    M3<S> Rp, Rj;
    V3<S> tp, tj;
    tree_offset<S>(M, i, Rp, tp);
    joint_motion<S>(M, i, q, Rj, tj);
    M4<S> local = m4_mul(homog(Rp, tp), homog(Rj, tj));
    if (M.parent[i] < 0) T[i] = local;
    else T[i] = m4_mul(T[M.parent[i]], local);
  }
}

// ----------------------------------------------------------------------------
// Jacobian: columns Ad(T_0k) S_k for every joint k on the path to the end effector.
// ----------------------------------------------------------------------------
template <class S> void jacobian_one(const Model& M, const S* q, int n_ee, const int* ee, int frame, S* J) {
  std::vector<M4<S>> T;
  fk_one<S>(M, q, T);
  for (int e = 0; e < n_ee; ++e) {
    S* Je = J + (size_t)e * 6 * M.nv;
    for (int r = 0; r < 6 * M.nv; ++r) Je[r] = S(0.0);
    int body = ee[e];
    V3<S> pe{{T[body].a[0][3], T[body].a[1][3], T[body].a[2][3]}};
    for (int k = body; k >= 0; k = M.parent[k]) {
      M3<S> R;
      V3<S> p;
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R.a[r][c] = T[k].a[r][c];
        p.a[r] = T[k].a[r][3];
      }
      // Ad(T) = [R 0; p^ R  R] maps body-k motion coordinates to world coordinates.
      M6<S> Ad = m6_zero<S>();
      M3<S> pR = m3_mul(skew(p), R);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          Ad.a[r][c] = R.a[r][c];
          Ad.a[r + 3][c + 3] = R.a[r][c];
          Ad.a[r + 3][c] = pR.a[r][c];
        }
      V6<S> cols[6];
      motion_subspace<S>(M, k, cols);
      for (int j = 0; j < M.nvi[k]; ++j) {
        V6<S> s = m6v(Ad, cols[j]);
        V3<S> w{{s.a[0], s.a[1], s.a[2]}};
        V3<S> v{{s.a[3], s.a[4], s.a[5]}};
        if (frame == 1) {
          V3<S> wp = cross3(w, pe);
          for (int r = 0; r < 3; ++r) v.a[r] += wp.a[r];
        }
        int col = M.vo[k] + j;
        for (int r = 0; r < 3; ++r) {
          Je[r * M.nv + col] = v.a[r];
          Je[(r + 3) * M.nv + col] = w.a[r];
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// RNEA (body coordinates): tau = M(q) qdd + C(q, qd) qd + g(q).
// ----------------------------------------------------------------------------
// If f_joint is not null it receives, per body i, the spatial force the joint
// transmits from the parent to body i (the f_i of the backward pass once every
// descendant has been added), in body-i coordinates about the body origin,
// which lies on the joint axis.
template <class S>
void rnea_one(const Model& M, const S* q, const S* qd, const S* qdd, const S* pi /*[n][10]*/, S* tau,
              V6<S>* f_joint = nullptr) {
  int n = M.n;
  std::vector<M6<S>> X(n);
  std::vector<V6<S>> v(n), a(n), f(n);
  std::vector<V6<S>> S_(6 * n);
  V6<S> a0 = base_accel<S>(M);
  for (int i = 0; i < n; ++i) {
    X[i] = x_up<S>(M, i, q);
    motion_subspace<S>(M, i, &S_[6 * i]);
    V6<S> vJ = subspace_times(&S_[6 * i], M.nvi[i], qd + M.vo[i]);
    V6<S> aJ = subspace_times(&S_[6 * i], M.nvi[i], qdd + M.vo[i]);
    int p = M.parent[i];
    if (p < 0) {
      v[i] = vJ;
      a[i] = v6_add(m6v(X[i], a0), aJ);
    } else {
      v[i] = v6_add(m6v(X[i], v[p]), vJ);
      a[i] = v6_add(v6_add(m6v(X[i], a[p]), aJ), m6v(crm(v[i]), vJ));
    }
    M6<S> I = spatial_inertia<S>(pi + 10 * i);
    f[i] = v6_add(m6v(I, a[i]), m6v(crf(v[i]), m6v(I, v[i])));
  }
  for (int i = n - 1; i >= 0; --i) {
    for (int k = 0; k < M.nvi[i]; ++k) tau[M.vo[i] + k] = v6_dot(S_[6 * i + k], f[i]);
    int p = M.parent[i];
    if (p >= 0) f[p] = v6_add(f[p], m6tv(X[i], f[i]));
  }
  if (f_joint)
    for (int i = 0; i < n; ++i) f_joint[i] = f[i];
}

// ----------------------------------------------------------------------------
// CRBA: composite inertias Ic_parent += X^T Ic X, then the column walk.
// ----------------------------------------------------------------------------
template <class S> void crba_one(const Model& M, const S* q, const S* pi, S* Mout) {
  int n = M.n, nv = M.nv;
  std::vector<M6<S>> X(n), Ic(n);
  std::vector<V6<S>> S_(6 * n);
  for (int i = 0; i < n; ++i) {
    X[i] = x_up<S>(M, i, q);
    motion_subspace<S>(M, i, &S_[6 * i]);
    Ic[i] = spatial_inertia<S>(pi + 10 * i);
  }
  for (int i = n - 1; i >= 0; --i) {
    int p = M.parent[i];
    if (p >= 0) Ic[p] = m6_add(Ic[p], m6_mul(m6_t(X[i]), m6_mul(Ic[i], X[i])));
  }
  for (int r = 0; r < nv * nv; ++r) Mout[r] = S(0.0);
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < M.nvi[i]; ++k) {
      V6<S> F = m6v(Ic[i], S_[6 * i + k]);
      int col = M.vo[i] + k;
      for (int l = 0; l < M.nvi[i]; ++l) Mout[(M.vo[i] + l) * nv + col] = v6_dot(S_[6 * i + l], F);
      int j = i;
      while (M.parent[j] >= 0) {
        F = m6tv(X[j], F);
        j = M.parent[j];
        for (int l = 0; l < M.nvi[j]; ++l) {
          S val = v6_dot(S_[6 * j + l], F);
          Mout[(M.vo[j] + l) * nv + col] = val;
          Mout[col * nv + M.vo[j] + l] = val;
        }
      }
    }
  }
}

// Solve the small dense system A x = b (ni <= 6) by Gaussian elimination with partial pivoting.
template <class S> void small_solve(int ni, S A[6][6], S* b) {
  for (int c = 0; c < ni; ++c) {
    int piv = c;
    for (int r = c + 1; r < ni; ++r)
      if (std::fabs(val(A[r][c])) > std::fabs(val(A[piv][c]))) piv = r;
    if (piv != c) {
      for (int k = 0; k < ni; ++k) { S t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t; }
      S t = b[c]; b[c] = b[piv]; b[piv] = t;
    }
    for (int r = c + 1; r < ni; ++r) {
      S fct = A[r][c] / A[c][c];
      for (int k = c; k < ni; ++k) A[r][k] = A[r][k] - fct * A[c][k];
      b[r] = b[r] - fct * b[c];
    }
  }
  for (int r = ni - 1; r >= 0; --r) {
    S s = b[r];
    for (int k = r + 1; k < ni; ++k) s = s - A[r][k] * b[k];
    b[r] = s / A[r][r];
  }
}

// ----------------------------------------------------------------------------
// ABA: three passes (velocities; articulated inertias leaf to root; accelerations).
// ----------------------------------------------------------------------------
template <class S> void aba_one(const Model& M, const S* q, const S* qd, const S* tau, const S* pi, S* qdd) {
  int n = M.n;
  std::vector<M6<S>> X(n), IA(n);
  std::vector<V6<S>> v(n), c(n), pA(n), a(n), S_(6 * n), U(6 * n);
  std::vector<S> Dinv(36 * n), u(6 * n);
  for (int i = 0; i < n; ++i) {
    X[i] = x_up<S>(M, i, q);
    motion_subspace<S>(M, i, &S_[6 * i]);
    V6<S> vJ = subspace_times(&S_[6 * i], M.nvi[i], qd + M.vo[i]);
    int p = M.parent[i];
    v[i] = (p < 0) ? vJ : v6_add(m6v(X[i], v[p]), vJ);
    c[i] = m6v(crm(v[i]), vJ);
    IA[i] = spatial_inertia<S>(pi + 10 * i);
    pA[i] = m6v(crf(v[i]), m6v(IA[i], v[i]));
  }
  for (int i = n - 1; i >= 0; --i) {
    int ni = M.nvi[i];
    S D[6][6];
    for (int k = 0; k < ni; ++k) U[6 * i + k] = m6v(IA[i], S_[6 * i + k]);
    for (int r = 0; r < ni; ++r)
      for (int k = 0; k < ni; ++k) D[r][k] = v6_dot(S_[6 * i + r], U[6 * i + k]);
    for (int k = 0; k < ni; ++k) u[6 * i + k] = tau[M.vo[i] + k] - v6_dot(S_[6 * i + k], pA[i]);
    // Dinv by solving D X = I column by column.
    for (int col = 0; col < ni; ++col) {
      S A[6][6], b[6];
      for (int r = 0; r < ni; ++r) {
        for (int k = 0; k < ni; ++k) A[r][k] = D[r][k];
        b[r] = (r == col) ? S(1.0) : S(0.0);
      }
      small_solve<S>(ni, A, b);
      for (int r = 0; r < ni; ++r) Dinv[36 * i + r * 6 + col] = b[r];
    }
    int p = M.parent[i];
    if (p >= 0) {
      // Ia = IA - U Dinv U^T ; pa = pA + Ia c + U Dinv u
      M6<S> Ia = IA[i];
      S Du[6];
      for (int r = 0; r < ni; ++r) {
        S s(0.0);
        for (int k = 0; k < ni; ++k) s += Dinv[36 * i + r * 6 + k] * u[6 * i + k];
        Du[r] = s;
      }
      for (int r = 0; r < 6; ++r)
        for (int cc = 0; cc < 6; ++cc) {
          S s(0.0);
          for (int k = 0; k < ni; ++k)
            for (int l = 0; l < ni; ++l) s += U[6 * i + k].a[r] * Dinv[36 * i + k * 6 + l] * U[6 * i + l].a[cc];
          Ia.a[r][cc] = Ia.a[r][cc] - s;
        }
      V6<S> pa = v6_add(pA[i], m6v(Ia, c[i]));
      for (int k = 0; k < ni; ++k)
        for (int r = 0; r < 6; ++r) pa.a[r] += U[6 * i + k].a[r] * Du[k];
      IA[p] = m6_add(IA[p], m6_mul(m6_t(X[i]), m6_mul(Ia, X[i])));
      pA[p] = v6_add(pA[p], m6tv(X[i], pa));
    }
  }
  V6<S> a0 = base_accel<S>(M);
  for (int i = 0; i < n; ++i) {
    int p = M.parent[i], ni = M.nvi[i];
    V6<S> ap = v6_add(m6v(X[i], p < 0 ? a0 : a[p]), c[i]);
    S rhs[6];
    for (int k = 0; k < ni; ++k) rhs[k] = u[6 * i + k] - v6_dot(U[6 * i + k], ap);
    for (int r = 0; r < ni; ++r) {
      S s(0.0);
      for (int k = 0; k < ni; ++k) s += Dinv[36 * i + r * 6 + k] * rhs[k];
      qdd[M.vo[i] + r] = s;
    }
    a[i] = v6_add(ap, subspace_times(&S_[6 * i], ni, qdd + M.vo[i]));
  }
}

// ----------------------------------------------------------------------------
// Energies: kinetic sum 1/2 v^T I v (body velocities from the forward recursion),
// potential -sum m g . c_world (COM positions from FK).
// ----------------------------------------------------------------------------
template <class S> void energy_one(const Model& M, const S* q, const S* qd, const S* pi, S* ke, S* pe) {
  int n = M.n;
  std::vector<V6<S>> v(n);
  S kin(0.0);
  for (int i = 0; i < n; ++i) {
    M6<S> X = x_up<S>(M, i, q);
    V6<S> cols[6];
    motion_subspace<S>(M, i, cols);
    V6<S> vJ = subspace_times(cols, M.nvi[i], qd + M.vo[i]);
    int p = M.parent[i];
    v[i] = (p < 0) ? vJ : v6_add(m6v(X, v[p]), vJ);
    M6<S> I = spatial_inertia<S>(pi + 10 * i);
    kin += S(0.5) * v6_dot(v[i], m6v(I, v[i]));
  }
  std::vector<M4<S>> T;
  fk_one<S>(M, q, T);
  S pot(0.0);
  for (int i = 0; i < n; ++i) {
    const S* p = pi + 10 * i;
    for (int r = 0; r < 3; ++r) {
      // m * c_world[r] = R[r,:] . h + m p[r]
      S mc = T[i].a[r][0] * p[1] + T[i].a[r][1] * p[2] + T[i].a[r][2] * p[3] + p[0] * T[i].a[r][3];
      pot = pot - S(M.g[r]) * mc;
    }
  }
  *ke = kin;
  *pe = pot;
}

}  // namespace orc

// ============================================================================
// C ABI.  All arrays are float64, instance-major: q[B][nq], qd/qdd/tau[B][nv],
// poses[B][n][12] (row-major 3x4 [R|p]), J[B][n_ee][6][nv], M[B][nv][nv].
// ============================================================================
using namespace orc;

extern "C" {

void* orc_model_new(int n, const int* parent, const int* jtype, const double* axis, const double* xtree,
                    const double* inertia, const double* gravity) {
  Model* M = new Model();
  M->n = n;
  M->parent.assign(parent, parent + n);
  M->jtype.assign(jtype, jtype + n);
  M->axis.assign(axis, axis + 3 * n);
  M->xtree.assign(xtree, xtree + 12 * n);
  M->inertia.assign(inertia, inertia + 10 * n);
  if (gravity) for (int k = 0; k < 3; ++k) M->g[k] = gravity[k];
  for (int i = 0; i < n; ++i) {
    int a = 0, b = 0;
    switch (jtype[i]) {
      case REV: case PRI: a = 1; b = 1; break;
      case FREE: a = 7; b = 6; break;
      default: a = 0; b = 0;
    }
    M->qo.push_back(M->nq);
    M->vo.push_back(M->nv);
    M->nqi.push_back(a);
    M->nvi.push_back(b);
    M->nq += a;
    M->nv += b;
  }
  return M;
}

void orc_model_free(void* m) { delete (Model*)m; }

void orc_dims(void* m, int* nq, int* nv) {
  Model* M = (Model*)m;
  *nq = M->nq;
  *nv = M->nv;
}

static int threads_or_default(int nt) { return nt > 0 ? nt : omp_get_max_threads(); }

void orc_fk(void* m, int64_t B, const double* q, double* poses, int nthreads) {
  const Model& M = *(Model*)m;
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    std::vector<M4<double>> T;
    fk_one<double>(M, q + b * M.nq, T);
    double* out = poses + b * 12 * M.n;
    for (int i = 0; i < M.n; ++i)
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) out[12 * i + 4 * r + c] = T[i].a[r][c];
  }
}

void orc_jacobian(void* m, int64_t B, const double* q, int n_ee, const int* ee, int frame, double* J,
                  int nthreads) {
  const Model& M = *(Model*)m;
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b)
    jacobian_one<double>(M, q + b * M.nq, n_ee, ee, frame, J + b * (int64_t)n_ee * 6 * M.nv);
}

void orc_rnea(void* m, int64_t B, const double* q, const double* qd, const double* qdd,
              const double* inertia_override, double* tau, int nthreads) {
  const Model& M = *(Model*)m;
  const double* pi = inertia_override ? inertia_override : M.inertia.data();
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b)
    rnea_one<double>(M, q + b * M.nq, qd + b * M.nv, qdd + b * M.nv, pi, tau + b * M.nv);
}

void orc_crba(void* m, int64_t B, const double* q, double* Mout, int nthreads) {
  const Model& M = *(Model*)m;
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b)
    crba_one<double>(M, q + b * M.nq, M.inertia.data(), Mout + b * (int64_t)M.nv * M.nv);
}

// CRBA with the inertial parameters [n][10] given by the caller (M is linear
// in them, as RNEA is), e.g. one body's parameters alone.
void orc_crba_pi(void* m, int64_t B, const double* q, const double* inertia, double* Mout, int nthreads) {
  const Model& M = *(Model*)m;
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b)
    crba_one<double>(M, q + b * M.nq, inertia, Mout + b * (int64_t)M.nv * M.nv);
}

void orc_aba(void* m, int64_t B, const double* q, const double* qd, const double* tau, double* qdd,
             int nthreads) {
  const Model& M = *(Model*)m;
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b)
    aba_one<double>(M, q + b * M.nq, qd + b * M.nv, tau + b * M.nv, M.inertia.data(), qdd + b * M.nv);
}

// The fused reference chain a user of the metric would run: RNEA, CRBA and the Jacobian.
void orc_chain(void* m, int64_t B, const double* q, const double* qd, const double* qdd, int n_ee,
               const int* ee, int frame, double* tau, double* Mout, double* J, int nthreads) {
  const Model& M = *(Model*)m;
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    rnea_one<double>(M, q + b * M.nq, qd + b * M.nv, qdd + b * M.nv, M.inertia.data(), tau + b * M.nv);
    crba_one<double>(M, q + b * M.nq, M.inertia.data(), Mout + b * (int64_t)M.nv * M.nv);
    jacobian_one<double>(M, q + b * M.nq, n_ee, ee, frame, J + b * (int64_t)n_ee * 6 * M.nv);
  }
}

void orc_energy(void* m, int64_t B, const double* q, const double* qd, double* ke, double* pe, int nthreads) {
  const Model& M = *(Model*)m;
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b)
    energy_one<double>(M, q + b * M.nq, qd + b * M.nv, M.inertia.data(), ke + b, pe + b);
}

// The spatial force transmitted across every joint by the RNEA backward pass,
// f_out [B][n][6] = [moment; force] in body coordinates about the body origin
// (tau_i is its projection on the joint's motion subspace).  inertia_override
// may be null.
void orc_rnea_forces(void* m, int64_t B, const double* q, const double* qd, const double* qdd,
                     const double* inertia_override, double* f_out, int nthreads) {
  const Model& M = *(Model*)m;
  const double* pi = inertia_override ? inertia_override : M.inertia.data();
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    std::vector<double> tau(M.nv);
    std::vector<V6<double>> f(M.n);
    rnea_one<double>(M, q + b * M.nq, qd + b * M.nv, qdd + b * M.nv, pi, tau.data(), f.data());
    for (int i = 0; i < M.n; ++i)
      for (int k = 0; k < 6; ++k) f_out[(b * M.n + i) * 6 + k] = f[i].a[k];
  }
}

// The same RNEA and CRBA recursions evaluated in single precision, inputs and
// parameters rounded to float.  Not a reference: the tests use them to show
// that the single-precision tolerance is attainable by a plain evaluation of
// the textbook recursion.
void orc_rnea_f32(void* m, int64_t B, const float* q, const float* qd, const float* qdd, const float* inertia,
                  float* tau, int nthreads) {
  const Model& M = *(Model*)m;
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b)
    rnea_one<float>(M, q + b * M.nq, qd + b * M.nv, qdd + b * M.nv, inertia, tau + b * M.nv);
}

void orc_crba_f32(void* m, int64_t B, const float* q, const float* inertia, float* Mout, int nthreads) {
  const Model& M = *(Model*)m;
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b) crba_one<float>(M, q + b * M.nq, inertia, Mout + b * (int64_t)M.nv * M.nv);
}

// Reverse-mode gradient of <tau_bar, RNEA(q, qd, qdd; pi)>.  inertia_bar is per instance
// ([B][n][10], not reduced).  Any of the output pointers may be null.
void orc_rnea_vjp(void* m, int64_t B, const double* q, const double* qd, const double* qdd,
                  const double* inertia_override, const double* tau_bar, double* q_bar, double* qd_bar,
                  double* qdd_bar, double* inertia_bar, int nthreads) {
  const Model& M = *(Model*)m;
  const double* pi0 = inertia_override ? inertia_override : M.inertia.data();
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    Tape tape;
    g_tape = &tape;
    int nq = M.nq, nv = M.nv, np = 10 * M.n;
    std::vector<Var> vq(nq), vqd(nv), vqdd(nv), vpi(np), vtau(nv);
    for (int k = 0; k < nq; ++k) vq[k] = leaf(q[b * nq + k]);
    for (int k = 0; k < nv; ++k) vqd[k] = leaf(qd[b * nv + k]);
    for (int k = 0; k < nv; ++k) vqdd[k] = leaf(qdd[b * nv + k]);
    for (int k = 0; k < np; ++k) vpi[k] = leaf(pi0[k]);
    rnea_one<Var>(M, vq.data(), vqd.data(), vqdd.data(), vpi.data(), vtau.data());
    std::vector<double> adj(tape.nodes.size(), 0.0);
    for (int k = 0; k < nv; ++k)
      if (vtau[k].id >= 0) adj[vtau[k].id] += tau_bar[b * nv + k];
    for (int i = (int)tape.nodes.size() - 1; i >= 0; --i) {
      const Node& nd = tape.nodes[i];
      if (adj[i] == 0.0) continue;
      if (nd.p0 >= 0) adj[nd.p0] += nd.d0 * adj[i];
      if (nd.p1 >= 0) adj[nd.p1] += nd.d1 * adj[i];
    }
    if (q_bar) for (int k = 0; k < nq; ++k) q_bar[b * nq + k] = adj[vq[k].id];
    if (qd_bar) for (int k = 0; k < nv; ++k) qd_bar[b * nv + k] = adj[vqd[k].id];
    if (qdd_bar) for (int k = 0; k < nv; ++k) qdd_bar[b * nv + k] = adj[vqdd[k].id];
    if (inertia_bar) for (int k = 0; k < np; ++k) inertia_bar[b * np + k] = adj[vpi[k].id];
    g_tape = nullptr;
  }
}

// Reverse-mode gradient of <M_bar, CRBA(q; pi)> (M_bar [nv][nv] row-major per
// instance): q_bar [nq] and, if inertia_bar is not null, the per-instance
// parameter gradient [n][10].  The derivatives of the mass matrix that
// analytical forward-dynamics derivatives need (the paper's outlook on
// trajectory optimisation, Sec. 5).
void orc_crba_vjp(void* m, int64_t B, const double* q, const double* inertia_override, const double* M_bar,
                  double* q_bar, double* inertia_bar, int nthreads) {
  const Model& M = *(Model*)m;
  const double* pi0 = inertia_override ? inertia_override : M.inertia.data();
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    Tape tape;
    g_tape = &tape;
    int nq = M.nq, nv = M.nv, np = 10 * M.n;
    std::vector<Var> vq(nq), vpi(np), vM(nv * nv);
    for (int k = 0; k < nq; ++k) vq[k] = leaf(q[b * nq + k]);
    for (int k = 0; k < np; ++k) vpi[k] = leaf(pi0[k]);
    crba_one<Var>(M, vq.data(), vpi.data(), vM.data());
    std::vector<double> adj(tape.nodes.size(), 0.0);
    const double* mb = M_bar + b * (int64_t)nv * nv;
    for (int k = 0; k < nv * nv; ++k)
      if (vM[k].id >= 0) adj[vM[k].id] += mb[k];
    for (int i = (int)tape.nodes.size() - 1; i >= 0; --i) {
      const Node& nd = tape.nodes[i];
      if (adj[i] == 0.0) continue;
      if (nd.p0 >= 0) adj[nd.p0] += nd.d0 * adj[i];
      if (nd.p1 >= 0) adj[nd.p1] += nd.d1 * adj[i];
    }
    for (int k = 0; k < nq; ++k) q_bar[b * nq + k] = adj[vq[k].id];
    if (inertia_bar) for (int k = 0; k < np; ++k) inertia_bar[b * np + k] = adj[vpi[k].id];
    g_tape = nullptr;
  }
}

// Reverse-mode gradient of <poses_bar, FK(q)> with poses laid out [n][12] (3x4 [R|p]).
void orc_fk_vjp(void* m, int64_t B, const double* q, const double* poses_bar, double* q_bar, int nthreads) {
  const Model& M = *(Model*)m;
#pragma omp parallel for num_threads(threads_or_default(nthreads)) schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    Tape tape;
    g_tape = &tape;
    int nq = M.nq;
    std::vector<Var> vq(nq);
    for (int k = 0; k < nq; ++k) vq[k] = leaf(q[b * nq + k]);
    std::vector<M4<Var>> T;
    fk_one<Var>(M, vq.data(), T);
    std::vector<double> adj(tape.nodes.size(), 0.0);
    const double* pb = poses_bar + b * 12 * M.n;
    for (int i = 0; i < M.n; ++i)
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) {
          const Var& x = T[i].a[r][c];
          if (x.id >= 0) adj[x.id] += pb[12 * i + 4 * r + c];
        }
    for (int i = (int)tape.nodes.size() - 1; i >= 0; --i) {
      const Node& nd = tape.nodes[i];
      if (adj[i] == 0.0) continue;
      if (nd.p0 >= 0) adj[nd.p0] += nd.d0 * adj[i];
      if (nd.p1 >= 0) adj[nd.p1] += nd.d1 * adj[i];
    }
    for (int k = 0; k < nq; ++k) q_bar[b * nq + k] = adj[vq[k].id];
    g_tape = nullptr;
  }
}

}  // extern "C"
