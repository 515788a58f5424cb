// Host-side model compiler under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Reads trees from a text file (written by tests/test_sanitizers.py from the
// seeded generators: count, then per tree the expected status (0 = valid), n,
// parent[n], joint_type[n], axis[3n], X_tree[12n], inertia[10n]), compiles
// each one the way bard_model_create does, and checks the compiled tables'
// invariants: preorder positions form a permutation, the level schedule
// places every body exactly once, every subtree work list covers every body,
// the mass-matrix lists index inside [nv][nv] and the Jacobian lists of the
// leaf end effectors account for every row of the [n_ee][6][nv] output.
// Malformed trees must be rejected.  Exit status 0 when every check holds.

#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_2605_31481_amd/csrc/model.h"
#include "../../paper_2605_31481_amd/csrc/status.h"

static int failures = 0;
#define CHECK(c, ...)                                   \
  do {                                                  \
    if (!(c)) {                                         \
      std::fprintf(stderr, "tree %d: ", tree_index);    \
      std::fprintf(stderr, __VA_ARGS__);                \
      std::fprintf(stderr, "\n");                       \
      ++failures;                                       \
    }                                                   \
  } while (0)

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
  for (int tree_index = 0; tree_index < count; ++tree_index) {
    int expect = 0, n = 0;
    if (std::fscanf(f, "%d %d", &expect, &n) != 2) return 2;
    bard_model* m = new bard_model();
    m->n = n;
    if (!read_n(f, m->parent, n) || !read_n(f, m->jtype, n) || !read_n(f, m->axis, 3 * n) ||
        !read_n(f, m->xtree, 12 * n) || !read_n(f, m->inertia, 10 * n))
      return 2;
    std::string err;
    const int rc = bard::compile_model(m, &err);
    if (expect != 0) {
      CHECK(rc != BARD_OK, "malformed tree accepted");
      delete m;
      continue;
    }
    CHECK(rc == BARD_OK, "valid tree rejected: %s", err.c_str());
    if (rc != BARD_OK) {
      delete m;
      continue;
    }
    std::vector<int> seen(n, 0);
    for (int i = 0; i < n; ++i) {
      CHECK(m->dfs[i] >= 0 && m->dfs[i] < n, "preorder position out of range");
      if (m->dfs[i] >= 0 && m->dfs[i] < n) ++seen[m->dfs[i]];
      CHECK(m->sub_size[i] >= 1 && m->dfs[i] + m->sub_size[i] <= n, "subtree range out of bounds");
    }
    for (int i = 0; i < n; ++i) CHECK(seen[i] == 1, "preorder positions are not a permutation");
    std::vector<int> placed(n, 0);
    for (int16_t b : m->sched_body)
      if (b >= 0) {
        CHECK(b < n, "schedule body out of range");
        if (b < n) ++placed[b];
      }
    for (int i = 0; i < n; ++i) CHECK(placed[i] == 1, "body %d placed %d times by the level schedule", i, placed[i]);
    for (int U : {1, 2, 4, 8}) {
      std::vector<int> units = bard::subtree_units(m, U);
      std::vector<int> cov(n, 0);
      CHECK(units.size() % U == 0, "work list not a multiple of %d", U);
      for (int code : units)
        if (code >= 0) {
          const int b = code & 0xff;
          CHECK(b < n, "work-list body out of range");
          if (b < n && ((code >> 8) & 0xf) == 0) ++cov[b];
        }
      for (int i = 0; i < n; ++i) CHECK(cov[i] == 1, "work list (U=%d) covers body %d %d times", U, i, cov[i]);
    }
    const int nv = m->nv;
    CHECK((int)m->mtab.size() == m->n_mpair + m->n_mzero, "mass-matrix list size");
    for (int k = 0; k < m->n_mpair; ++k) {
      const int a = m->mtab[k] & 0xffff, d = m->mtab[k] >> 16;
      CHECK(a < nv && d < nv, "mass-matrix pair out of range");
    }
    for (int k = m->n_mpair; k < (int)m->mtab.size(); ++k)
      CHECK(m->mtab[k] >= 0 && m->mtab[k] < nv * nv, "mass-matrix zero entry out of range");
    std::vector<int> ee;
    for (int i = 0; i < n; ++i) {
      bool leaf = true;
      for (int j = i + 1; j < n; ++j)
        if (m->parent[j] == i) leaf = false;
      if (leaf && (int)ee.size() < BARD_MAX_EE) ee.push_back(i);
    }
    int n_cols = 0, n_zeros = 0;
    std::vector<int> jt = bard::jacobian_table(m, ee, &n_cols, &n_zeros);
    CHECK(6 * n_cols + n_zeros == 6 * nv * (int)ee.size(), "Jacobian lists do not cover the output");
    for (int k = 0; k < n_cols; ++k) CHECK((jt[k] & 0xff) < nv && (jt[k] >> 8) < (int)ee.size(), "column code");
    delete m;
  }
  std::fclose(f);
  std::printf("compiler check: %d trees, %d failures\n", count, failures);
  return failures ? 1 : 0;
}
