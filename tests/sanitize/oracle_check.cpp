// The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Reads valid trees in the format of compiler_check.cpp, calls every export of
// the oracle library on a few random states (two OpenMP threads), and checks
// that the results are finite and consistent: ABA inverts RNEA, the mass
// matrix is symmetric, the fused chain returns the separate operators'
// results, and the reverse-mode products and energies run.  Exit status 0
// when every check holds.

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
void* orc_model_new(int n, const int* parent, const int* jtype, const double* axis, const double* xtree,
                    const double* inertia, const double* gravity);
void orc_model_free(void* m);
void orc_dims(void* m, int* nq, int* nv);
void orc_fk(void* m, int64_t B, const double* q, double* poses, int nthreads);
void orc_jacobian(void* m, int64_t B, const double* q, int n_ee, const int* ee, int frame, double* J, int nthreads);
void orc_rnea(void* m, int64_t B, const double* q, const double* qd, const double* qdd, const double* pi, double* tau,
              int nthreads);
void orc_crba(void* m, int64_t B, const double* q, double* M, int nthreads);
void orc_crba_pi(void* m, int64_t B, const double* q, const double* pi, double* M, int nthreads);
void orc_aba(void* m, int64_t B, const double* q, const double* qd, const double* tau, double* qdd, int nthreads);
void orc_chain(void* m, int64_t B, const double* q, const double* qd, const double* qdd, int n_ee, const int* ee,
               int frame, double* tau, double* M, double* J, int nthreads);
void orc_energy(void* m, int64_t B, const double* q, const double* qd, double* ke, double* pe, int nthreads);
void orc_rnea_forces(void* m, int64_t B, const double* q, const double* qd, const double* qdd, const double* pi,
                     double* f, int nthreads);
void orc_rnea_f32(void* m, int64_t B, const float* q, const float* qd, const float* qdd, const float* pi, float* tau,
                  int nthreads);
void orc_crba_f32(void* m, int64_t B, const float* q, const float* pi, float* M, int nthreads);
void orc_rnea_vjp(void* m, int64_t B, const double* q, const double* qd, const double* qdd, const double* pi,
                  const double* tau_bar, double* q_bar, double* qd_bar, double* qdd_bar, double* pi_bar, int nthreads);
void orc_crba_vjp(void* m, int64_t B, const double* q, const double* pi, const double* M_bar, double* q_bar,
                  double* pi_bar, int nthreads);
void orc_fk_vjp(void* m, int64_t B, const double* q, const double* poses_bar, double* q_bar, int nthreads);
}

static int failures = 0;
static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double uniform() {  // xorshift64*, in [-1, 1)
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (double)((rng_state * 0x2545f4914f6cdd1dull) >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static bool finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

template <class T>
static bool read_n(FILE* f, std::vector<T>& v, int n) {
  v.resize(n);
  for (int i = 0; i < n; ++i) {
    double x;
    if (std::fscanf(f, "%lf", &x) != 1) return false;
    v[i] = (T)x;
  }
  return true;
}

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* f = std::fopen(argv[1], "r");
  if (!f) return 2;
  int count = 0;
  if (std::fscanf(f, "%d", &count) != 1) return 2;
  const int B = 3, T = 2;
  int checked = 0;
  for (int t = 0; t < count; ++t) {
    int expect = 0, n = 0;
    if (std::fscanf(f, "%d %d", &expect, &n) != 2) return 2;
    std::vector<int> parent, jtype;
    std::vector<double> axis, xtree, inertia;
    if (!read_n(f, parent, n) || !read_n(f, jtype, n) || !read_n(f, axis, 3 * n) || !read_n(f, xtree, 12 * n) ||
        !read_n(f, inertia, 10 * n))
      return 2;
    if (expect != 0) continue;  // the oracle takes valid trees only
    const double g[3] = {0.0, 0.0, -9.81};
    void* m = orc_model_new(n, parent.data(), jtype.data(), axis.data(), xtree.data(), inertia.data(), g);
    int nq = 0, nv = 0;
    orc_dims(m, &nq, &nv);
    std::vector<double> q(B * nq), qd(B * nv), qdd(B * nv);
    for (int b = 0; b < B; ++b) {
      int k = 0;
      for (int i = 0; i < n; ++i) {
        if (jtype[i] == 2) {  // free root: position, then a unit quaternion
          for (int c = 0; c < 3; ++c) q[b * nq + k + c] = uniform();
          double s = 0.0;
          for (int c = 3; c < 7; ++c) s += (q[b * nq + k + c] = uniform()) * q[b * nq + k + c];
          for (int c = 3; c < 7; ++c) q[b * nq + k + c] /= std::sqrt(s);
          k += 7;
        } else if (jtype[i] == 0 || jtype[i] == 1) {
          q[b * nq + k++] = 3.0 * uniform();
        }
      }
    }
    for (double& x : qd) x = uniform();
    for (double& x : qdd) x = uniform();
    std::vector<int> ee;
    for (int i = 0; i < n && ee.size() < 4; ++i) {
      bool leaf = true;
      for (int j = i + 1; j < n; ++j)
        if (parent[j] == i) leaf = false;
      if (leaf) ee.push_back(i);
    }
    const int ne = (int)ee.size();
    std::vector<double> poses(B * 12 * n), J(B * ne * 6 * nv), tau(B * nv), M(B * nv * nv), qdd2(B * nv);
    std::vector<double> tau_c(B * nv), M_c(B * nv * nv), J_c(B * ne * 6 * nv), ke(B), pe(B), fj(B * n * 6);
    orc_fk(m, B, q.data(), poses.data(), T);
    for (int frame = 0; frame < 2; ++frame) orc_jacobian(m, B, q.data(), ne, ee.data(), frame, J.data(), T);
    orc_rnea(m, B, q.data(), qd.data(), qdd.data(), nullptr, tau.data(), T);
    orc_crba(m, B, q.data(), M.data(), T);
    std::vector<double> M_pi(B * nv * nv);
    orc_crba_pi(m, B, q.data(), inertia.data(), M_pi.data(), T);
    orc_aba(m, B, q.data(), qd.data(), tau.data(), qdd2.data(), T);
    orc_chain(m, B, q.data(), qd.data(), qdd.data(), ne, ee.data(), 1, tau_c.data(), M_c.data(), J_c.data(), T);
    orc_energy(m, B, q.data(), qd.data(), ke.data(), pe.data(), T);
    orc_rnea_forces(m, B, q.data(), qd.data(), qdd.data(), nullptr, fj.data(), T);
    std::vector<float> q32(q.begin(), q.end()), qd32(qd.begin(), qd.end()), qdd32(qdd.begin(), qdd.end());
    std::vector<float> pi32(inertia.begin(), inertia.end()), tau32(B * nv), M32(B * nv * nv);
    orc_rnea_f32(m, B, q32.data(), qd32.data(), qdd32.data(), pi32.data(), tau32.data(), T);
    orc_crba_f32(m, B, q32.data(), pi32.data(), M32.data(), T);
    std::vector<double> tb(B * nv), qb(B * nq), qdb(B * nv), qddb(B * nv), pib(B * n * 10), mb(B * nv * nv),
        pb(B * 12 * n), fq(B * nq), cq(B * nq), cpi(B * n * 10);
    for (double& x : tb) x = uniform();
    for (double& x : mb) x = uniform();
    for (double& x : pb) x = uniform();
    orc_rnea_vjp(m, B, q.data(), qd.data(), qdd.data(), nullptr, tb.data(), qb.data(), qdb.data(), qddb.data(),
                 pib.data(), T);
    orc_crba_vjp(m, B, q.data(), nullptr, mb.data(), cq.data(), cpi.data(), T);
    orc_fk_vjp(m, B, q.data(), pb.data(), fq.data(), T);
    for (const auto* v : {&poses, &J, &tau, &M, &qdd2, &ke, &pe, &fj, &qb, &qdb, &qddb, &pib, &cq, &cpi, &fq})
      if (!finite(*v)) {
        std::fprintf(stderr, "tree %d: non-finite output\n", t);
        ++failures;
      }
    double err = 0.0, scale = 1.0;
    for (int k = 0; k < B * nv; ++k) {
      err = std::fmax(err, std::fabs(qdd2[k] - qdd[k]));
      scale = std::fmax(scale, std::fabs(qdd[k]));
    }
    if (err > 1e-7 * scale) {
      std::fprintf(stderr, "tree %d: ABA does not invert RNEA (%g)\n", t, err);
      ++failures;
    }
    // symmetric to rounding (a free root's block forms M_lk and M_kl
    // separately); the three CRBA entry points give the same bits
    double mmax = 0.0;
    for (double x : M) mmax = std::fmax(mmax, std::fabs(x));
    bool ok = true;
    for (int b = 0; b < B; ++b)
      for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
          const double x = M[(b * nv + i) * nv + j];
          if (std::fabs(x - M[(b * nv + j) * nv + i]) > 1e-13 * mmax || x != M_c[(b * nv + i) * nv + j] ||
              x != M_pi[(b * nv + i) * nv + j])
            ok = false;
        }
    if (!ok) {
      std::fprintf(stderr, "tree %d: mass matrix not symmetric or not reproduced\n", t);
      ++failures;
    }
    for (int k = 0; k < B * nv; ++k)
      if (tau[k] != tau_c[k]) {
        std::fprintf(stderr, "tree %d: chain torque differs from RNEA\n", t);
        ++failures;
        break;
      }
    orc_model_free(m);
    ++checked;
  }
  std::fclose(f);
  std::printf("oracle check: %d trees, %d failures\n", checked, failures);
  return failures ? 1 : 0;
}
