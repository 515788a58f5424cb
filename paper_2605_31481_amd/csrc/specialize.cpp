// Model-specialised chain kernels: the model compiler writes HIP source for one
// tree -- RNEA, CRBA and the end-effector Jacobians fused, every model
// constant a literal, the traversal unrolled body by body -- and compiles it
// at run time with hipRTC.
//
// Mapping.  One lane per instance, 64 instances per workgroup, all lanes of a
// wave at the same body at the same time, so every constant is wave-uniform
// and folds into the instructions; no tables are staged.  Entering a body the
// code composes the joint transform (eqs. (4)-(5)), the world pose, the axis
// and the velocity and acceleration; leaving it (after its children) it forms
// the subtree force and composite inertia, the torque, the mass-matrix column
// and, walking up the ancestors, the entries that couple it to them.  Every
// index is known when the code is written, so ancestors' state stays in
// registers.  Two forms: the whole tree in one wave, or split over the waves
// of the workgroup by limbs (SplitPlan below), which shortens the serial
// chain of instructions each wave issues -- the bound when a batch leaves most
// of the device idle.  Products with the zero half of a motion-subspace
// column and with zero inertial parameters are not emitted; every input is
// loaded ahead of the code that uses it; every output is addressed by a
// wave-uniform row base plus a 32-bit per-lane offset.
//
// Frames.  Motion and force vectors are kept about each body's own origin
// with world axes: a child's state is its parent's moved by the link offset
// r = R_parent t_pc (a translation-only transform), forces and composite
// inertias move back up by the same offsets.  Only relative positions enter
// the dynamics, so no quantity grows with the distance from the base.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace bard {

namespace {

const char kSpatialHeader[] =
#include "spatial_h.inc"
    ;

// How one instance's work is spread over the waves of a workgroup.  The
// trunk is every body with two or more children and all their ancestors; what
// hangs off it (or off the world, outside the trunk) are limbs, each a chain.
// Every wave computes the trunk's kinematics, then one or more whole limbs:
// their poses, torques, Jacobians, mass-matrix columns and the entries coupling
// them to the trunk (the walks go up through the trunk's state, which each wave
// holds).  A limb's subtree force and composite inertia, moved to its trunk
// parent's origin, go to LDS; after one barrier the last wave (the least
// loaded one, which also forms the trunk's body forces beforehand) sums the
// trunk.  Limbs are dealt to at most kMaxWaves waves, longest first, onto the
// least loaded wave.  A tree that is one chain keeps a single wave.
struct SplitPlan {
  static constexpr int kMaxWaves = 8;
  bool split = false;
  int waves = 1;
  std::vector<char> trunk;
  std::vector<std::vector<int>> limbs;  // bodies root first
  std::vector<std::vector<int>> bins;   // limbs per wave; the last wave merges
  std::vector<int> limb_slot;           // LDS slot of each limb's sum, -1 for a root limb
  std::vector<char> limb_first;         // first limb writing its slot
  std::vector<int> slot_body;           // trunk body each slot adds into
};

SplitPlan make_plan(const bard_model* m, bool whole, bool fp64, int max_waves = SplitPlan::kMaxWaves) {
  SplitPlan pl;
  const int n = m->n;
  pl.trunk.assign(n, 0);
  if (whole) return pl;
  for (int i = 0; i < n; ++i)
    if (m->children[i].size() >= 2)
      for (int k = i; k >= 0 && !pl.trunk[k]; k = m->parent[k]) pl.trunk[k] = 1;
  std::vector<double> cost;
  for (int i = 0; i < n; ++i) {
    if (pl.trunk[i] || (m->parent[i] >= 0 && !pl.trunk[m->parent[i]])) continue;
    std::vector<int> chain;
    double c = 0;
    for (int k = i;; k = m->children[k][0]) {
      chain.push_back(k);
      int depth = 0;
      for (int a = m->parent[k]; a >= 0; a = m->parent[a]) ++depth;
      c += 12.0 + (double)m->nvi[k] * depth;  // a body's forward pass ~ 12 steps of its mass-matrix walks
      if (m->children[k].empty()) break;
    }
    pl.limbs.push_back(chain);
    cost.push_back(c);
  }
  const int nl = (int)pl.limbs.size();
  pl.waves = std::min(nl, max_waves);
  std::vector<int> order(nl);
  for (int l = 0; l < nl; ++l) order[l] = l;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<std::vector<int>> bins(pl.waves);
  std::vector<double> load(pl.waves, 0.0);
  for (int l : order) {
    const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    bins[w].push_back(l);
    load[w] += cost[l];
  }
  std::vector<int> wo(pl.waves);
  for (int w = 0; w < pl.waves; ++w) wo[w] = w;
  std::stable_sort(wo.begin(), wo.end(), [&](int a, int b) { return load[a] > load[b]; });
  for (int w : wo) pl.bins.push_back(bins[w]);
  pl.limb_slot.assign(nl, -1);
  pl.limb_first.assign(nl, 0);
  for (const auto& bin : pl.bins) {
    std::vector<std::pair<int, int>> seen;  // (trunk body, slot) within this wave
    for (int l : bin) {
      const int at = m->parent[pl.limbs[l][0]];
      if (at < 0) continue;
      int sl = -1;
      for (const auto& [body, slot] : seen)
        if (body == at) sl = slot;
      if (sl < 0) {
        sl = (int)pl.slot_body.size();
        pl.slot_body.push_back(at);
        seen.push_back({at, sl});
        pl.limb_first[l] = 1;
      }
      pl.limb_slot[l] = sl;
    }
  }
  // LDS: 16 values per slot and lane; keep within 64 KB (with one wave, a
  // slot per trunk body that has limbs; past that no split plan)
  if (pl.slot_body.size() * 16 * 64 * (fp64 ? 8 : 4) > 65536)
    return max_waves > 1 ? make_plan(m, false, fp64, 1) : make_plan(m, true, fp64);
  pl.split = true;
  return pl;
}

// Emits the source text of one specialised chain kernel.
class Emitter {
 public:
  // ops: the outputs the kernel computes (1 torques, 2 mass matrix, 4
  // Jacobians, 8 world poses; the split and whole forms only)
  Emitter(const bard_model* m, const std::vector<int>& ee, int frame, bool fp64, int form,
          int max_waves = SplitPlan::kMaxWaves, int ops = 7)
      : m_(m), ee_(ee), frame_(frame), fp64_(fp64), ops_(ops), parts_(form == 2 ? 2 : form == 3 ? 3 : 1),
        dual_(parts_ > 1), pl_(make_plan(m, form == 1, fp64, max_waves)), split_(pl_.split || dual_) {
    trunk_ = pl_.trunk;
    slot_body_ = pl_.slot_body;
  }

  // Helpers and accessor macros every generated chain source starts with.
  static std::string prologue(bool fp64) {
    std::ostringstream o;
    o << "#include \"spatial.h\"\n";
    o << "typedef " << (fp64 ? "double" : "float") << " Real;\n";
    o << "template <class T>\n"
         "__device__ __forceinline__ T* bard_at(T* base, long long k, long long sk, unsigned ob) {\n"
         "  return (T*)((const char*)(base + k * sk) + ob);\n"
         "}\n"
         "#define Q(k) (*bard_at(q, (k), sq_k, oq_))\n"
         "#define QD(k) (*bard_at(qd, (k), sqd_k, oqd_))\n"
         "#define QDD(k) (*bard_at(qdd, (k), sqdd_k, oqdd_))\n"
         "__device__ __forceinline__ void bard_st(__amdgpu_buffer_rsrc_t r, unsigned row, unsigned ob, float v) {\n"
         "  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)ob, (int)row, 2);\n"
         "}\n"
         "__device__ __forceinline__ void bard_st(__amdgpu_buffer_rsrc_t r, unsigned row, unsigned ob, double v) {\n"
         "  typedef unsigned U2 __attribute__((ext_vector_type(2)));\n"
         "  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, (int)ob, (int)row, 2);\n"
         "}\n"
         "#define TAU(k, v) bard_st(rt_, (unsigned)(k) * ut_, ot_, (v))\n"
         "#define MA(k, v) bard_st(rM_, (unsigned)(k) * uM_, oM_, (v))\n"
         "#define JA(k, v) bard_st(rJ_, (unsigned)(k) * uJ_, oJ_, (v))\n"
         "#define PA(k, v) bard_st(rP_, (unsigned)(k) * uP_, oP_, (v))\n"
         "#define Qv(k) Qv_##k\n"
         "#define QDv(k) QDv_##k\n"
         "#define QDDv(k) QDDv_##k\n";
    return o.str();
  }

  std::string source() {
    o_ << "// generated: fused RNEA + CRBA + Jacobian for one tree (" << m_->n << " bodies, nv " << m_->nv
       << ", " << ee_.size() << " end effectors, frame " << frame_ << ", " << (fp64_ ? "FP64" : "FP32") << ")\n";
    o_ << prologue(fp64_);
    emit_zero_tables();
    const int nw = pl_.waves;
    o_ << "static constexpr int NW = " << nw << ";  // waves per workgroup, 64 instances\n";
    o_ << "static constexpr int WG_PER_GROUP = " << parts_ << ";  // workgroups per 64 instances\n";
    o_ << "extern \"C\" __global__ void __launch_bounds__(" << 64 * nw << ") bard_spec_chain(\n"
          "    const Real* __restrict__ q, const Real* __restrict__ qd, const Real* __restrict__ qdd,\n"
          "    Real* __restrict__ tau, Real* __restrict__ M, Real* __restrict__ J,\n"
          "    long long sq_b, long long sq_k, long long sqd_b, long long sqd_k, long long sqdd_b, long long sqdd_k,\n"
          "    long long st_b, long long st_k, long long sM_b, long long sM_k, long long sJ_b, long long sJ_k,\n"
          "    long long B, Real g0, Real g1, Real g2, int main_blocks, int zero_blocks,\n"
          "    Real* __restrict__ P, long long sp_b, long long sp_k) {\n"
          "  if ((int)blockIdx.x >= main_blocks) {\n"
          "    // structural zeros, instance-minor layout: the zero rows cut into\n"
          "    // chunks of 1024 16-byte vectors, one chunk per workgroup in turn\n"
          "    constexpr int V = 16 / (int)sizeof(Real);\n"
          "    typedef Real Zv __attribute__((vector_size(16)));\n"
          "    const Zv zero = {};\n"
          "    const long long per = B / V;\n"
          "    const long long nch = (per + 1023) / 1024;\n"
          "    for (long long u = blockIdx.x - main_blocks; u < (NZM + NZJ) * nch; u += zero_blocks) {\n"
          "      const long long r = u / nch, c = u - r * nch;\n"
          "      Real* row = r < NZM ? M + (long long)ZM[r] * sM_k : J + (long long)ZJ[r - NZM] * sJ_k;\n"
          "      const long long end = per < (c + 1) * 1024 ? per : (c + 1) * 1024;\n"
          "      for (long long j = c * 1024 + threadIdx.x; j < end; j += 64 * NW)\n"
          "        *reinterpret_cast<Zv*>(row + j * V) = zero;\n"
          "    }\n"
          "    return;\n"
          "  }\n";
    body();
    o_ << "}\n";
    return o_.str();
  }

  // The tree's code as a member of a multi-tree kernel: namespace bard_t<k>
  // with its tables and run(io, blk, xch_), which evaluates the 64-instance
  // group (or dual half) `blk` of a batch of B instances held instance-minor
  // ([K][B], the layout of plans); xch_ is the kernel's LDS hand-over area.
  // The kernel's workgroups may have more waves than this tree uses: those
  // skip the tree's work and still reach its barrier.
  std::string member(int k, int64_t B) {
    member_ = true;
    blk_ = "blk";
    o_ << "namespace bard_t" << k << " {  // " << m_->n << " bodies, nv " << m_->nv << ", batch " << B << "\n";
    emit_zero_tables();
    o_ << "static constexpr int NW = " << pl_.waves << ";\n";
    o_ << "__device__ __forceinline__ void run(const PlanIO& io, long long blk, Real* xch_) {\n";
    const long long ld = std::max<int64_t>(B, 1);
    o_ << "  const Real* __restrict__ q = io.q;\n  const Real* __restrict__ qd = io.qd;\n"
          "  const Real* __restrict__ qdd = io.qdd;\n  Real* __restrict__ tau = io.tau;\n"
          "  Real* __restrict__ M = io.M;\n  Real* __restrict__ J = io.J;\n"
       << "  const long long B = " << B << "LL;\n"
       << "  const long long sq_b = 1, sqd_b = 1, sqdd_b = 1, st_b = 1, sM_b = 1, sJ_b = 1;\n"
       << "  const long long sq_k = " << ld << "LL, sqd_k = " << ld << "LL, sqdd_k = " << ld << "LL, st_k = " << ld
       << "LL, sM_k = " << ld << "LL, sJ_k = " << ld << "LL;\n"
       << "  const Real g0 = io.g[0], g1 = io.g[1], g2 = io.g[2];\n"
          "  const int zero_blocks = 0;\n"
          "  Real* const P = nullptr;\n  const long long sp_b = 0, sp_k = 0;\n";
    body();
    o_ << "}\n}  // namespace bard_t" << k << "\n";
    return o_.str();
  }

  int waves() const { return pl_.waves; }
  int wg_per_group() const { return parts_; }
  // LDS values of the hand-over area (trunk slots x 16 x 64 lanes)
  int xch_values() const { return split_ ? (int)slot_body_.size() * 16 * 64 : 0; }

  // The code of one workgroup after the structural-zero workgroups.
  void body() {
    if (!split_) {
      set_parts(ops_ & 1, ops_ & 2, ops_ & 4);
      if (member_) o_ << "  if (threadIdx.x >= 64) return;\n";
      o_ << "  const long long b = (long long)" << blk_ << " * 64 + threadIdx.x;\n"
            "  if (b >= B) return;\n";
      pointers();
      std::vector<int> all(m_->n);
      for (int i = 0; i < m_->n; ++i) all[i] = i;
      loads(all);
      emit_zero_stores();
      for (int i = 0; i < m_->n; ++i)
        if (m_->parent[i] < 0) visit(i);
      set_parts(true, true, true);
      return;
    }
    // Every lane of every wave reaches the barrier: lanes past the batch
    // repeat the last instance (the same values to the same addresses).
    o_ << "  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);\n"
          "  const int lane = (int)threadIdx.x & 63;\n";
    if (parts_ == 2)
      o_ << "  const int part = (int)" << blk_ << " & 1;  // 0: torques, 1: mass matrix and Jacobians\n"
         << "  long long b = ((long long)" << blk_ << " >> 1) * 64 + lane;\n";
    else if (parts_ == 3)
      o_ << "  const int part = (int)((long long)" << blk_ << " % 3);  // 0: torques, 1: mass matrix, 2: Jacobians\n"
         << "  long long b = ((long long)" << blk_ << " / 3) * 64 + lane;\n";
    else
      o_ << "  long long b = (long long)" << blk_ << " * 64 + lane;\n";
    o_ << "  if (b > B - 1) b = B - 1;\n";
    pointers();
    if (!slot_body_.empty() && !member_) o_ << "  __shared__ Real xch_[" << slot_body_.size() * 16 * 64 << "];\n";
    if (parts_ == 2) {
      o_ << "  if (part == 0) {\n";
      set_parts(true, false, false);
      split_body();
      o_ << "  } else {\n";
      set_parts(false, true, true);
      split_body();
      o_ << "  }\n";
      set_parts(true, true, true);
    } else if (parts_ == 3) {
      o_ << "  if (part == 0) {\n";
      set_parts(true, false, false);
      split_body();
      o_ << "  } else if (part == 1) {\n";
      set_parts(false, true, false);
      split_body();
      o_ << "  } else {\n";
      set_parts(false, false, true);
      split_body();
      o_ << "  }\n";
      set_parts(true, true, true);
    } else {
      set_parts(ops_ & 1, ops_ & 2, ops_ & 4);
      split_body();
      set_parts(true, true, true);
    }
  }

  void set_parts(bool rnea, bool crba, bool jac) {
    do_rnea_ = rnea;
    do_crba_ = crba;
    do_jac_ = jac;
  }

  // The workgroup's code for the parts selected by do_rnea_ / do_crba_ /
  // do_jac_: the
  // waves' branches (loads, trunk kinematics, limbs), one barrier, the
  // trunk's sums in the merging wave.  The trunk's state lives at the scope
  // of this code (the merging wave reads it after the barrier); each wave's
  // branch issues all its loads -- its limbs' and the trunk's -- before
  // computing anything (one memory round trip).
  void split_body() {
    const int nw = pl_.waves;
    o_ << "  {\n";
    // the lanes' structural-zero stores (when no extra workgroups write
    // them) go with the part that stores little else: the torques' in the
    // dual form, the Jacobians' in the triple form
    if (parts_ == 1 || (parts_ == 2 && do_rnea_) || (parts_ == 3 && !do_rnea_ && !do_crba_)) emit_zero_stores();
    std::vector<int> tb;
    bool any_trunk = false;
    for (int i = 0; i < m_->n; ++i)
      if (trunk_[i]) {
        tb.push_back(i);
        o_ << "  Real " << v("R", i) << "[9], " << v("p", i) << "[3], " << v("r", i) << "[3], " << v("a", i)
           << "[3], " << v("v", i) << "[6], " << v("c", i) << "[6], " << v("I", i) << "[10], " << v("f", i)
           << "[6];\n";
        any_trunk = true;
      }
    const int merge = nw - 1;
    for (int w = 0; w < nw; ++w) {
      o_ << (w ? "  else if" : "  if") << " (wave == " << w << ") {\n";
      std::vector<int> lb;
      for (int l : pl_.bins[w]) lb.insert(lb.end(), pl_.limbs[l].begin(), pl_.limbs[l].end());
      loads(lb);
      loads(tb);
      for (int i : tb) forward_kin(i, false);
      for (int l : pl_.bins[w]) limb(l);
      if (w == merge) {
        if (ops_ & 8)
          for (int i : tb) store_pose(i);
        for (int i = 0; i < m_->n; ++i)
          if (trunk_[i]) body_force(i, false);
        if (do_jac_)
          for (size_t e = 0; e < ee_.size(); ++e)
            if (trunk_[ee_[e]]) jacobian((int)e);
      }
      o_ << "  }\n";
    }
    if (any_trunk && (do_rnea_ || do_crba_)) {
      o_ << "  __syncthreads();\n  if (wave == " << merge << ") {\n";
      for (int i = m_->n - 1; i >= 0; --i)
        if (trunk_[i]) backward(i);
      o_ << "  }\n";
    }
    o_ << "  }\n";
  }

  // The inputs of the given bodies, loaded at once ahead of the code that
  // uses them (one memory round trip instead of one per body); velocities
  // and accelerations only where the torques are computed.
  void loads(const std::vector<int>& bodies) {
    for (int i : bodies) {
      const int nq = m_->jtype[i] == J_FREE ? 7 : 1;
      for (int k = 0; k < nq; ++k) o_ << "  const Real Qv_" << m_->qi[i] + k << " = Q(" << m_->qi[i] + k << ");\n";
      if (do_rnea_)
        for (int k = 0; k < m_->nvi[i]; ++k)
          o_ << "  const Real QDv_" << m_->vi[i] + k << " = QD(" << m_->vi[i] + k << ");\n  const Real QDDv_"
             << m_->vi[i] + k << " = QDD(" << m_->vi[i] + k << ");\n";
    }
  }

  void pointers() {
    o_ << "  const unsigned oq_ = (unsigned)(b * sq_b) * (unsigned)sizeof(Real);\n"
          "  const unsigned oqd_ = (unsigned)(b * sqd_b) * (unsigned)sizeof(Real);\n"
          "  const unsigned oqdd_ = (unsigned)(b * sqdd_b) * (unsigned)sizeof(Real);\n"
          "  const unsigned ot_ = (unsigned)(b * st_b) * (unsigned)sizeof(Real);\n"
          "  const unsigned oM_ = (unsigned)(b * sM_b) * (unsigned)sizeof(Real);\n"
          "  const unsigned oJ_ = (unsigned)(b * sJ_b) * (unsigned)sizeof(Real);\n"
          // outputs: buffer stores from a resource per array, the row's byte
          // offset in a scalar register and the lane's in a vector register
          "  const __amdgpu_buffer_rsrc_t rt_ = __builtin_amdgcn_make_buffer_rsrc(tau, (short)0, -1, 0x00020000);\n"
          "  const __amdgpu_buffer_rsrc_t rM_ = __builtin_amdgcn_make_buffer_rsrc(M, (short)0, -1, 0x00020000);\n"
          "  const __amdgpu_buffer_rsrc_t rJ_ = __builtin_amdgcn_make_buffer_rsrc(J, (short)0, -1, 0x00020000);\n"
          "  const unsigned ut_ = (unsigned)st_k * (unsigned)sizeof(Real);\n"
          "  const unsigned uM_ = (unsigned)sM_k * (unsigned)sizeof(Real);\n"
          "  const unsigned uJ_ = (unsigned)sJ_k * (unsigned)sizeof(Real);\n";
    if (ops_ & 8)
      o_ << "  const unsigned oP_ = (unsigned)(b * sp_b) * (unsigned)sizeof(Real);\n"
            "  const __amdgpu_buffer_rsrc_t rP_ = __builtin_amdgcn_make_buffer_rsrc(P, (short)0, -1, 0x00020000);\n"
            "  const unsigned uP_ = (unsigned)sp_k * (unsigned)sizeof(Real);\n";
  }

  // FK output: body i's world pose [R | p], 3x4 row-major (p about the world
  // origin: the kinematics keep world positions)
  void store_pose(int i) {
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k)
        o_ << "  PA(" << 12 * i + 4 * r + k << ", " << v("R", i) << "[" << 3 * r + k << "]);\n";
      o_ << "  PA(" << 12 * i + 4 * r + 3 << ", " << v("p", i) << "[" << r << "]);\n";
    }
  }

  // One limb (a chain): forward, its end effectors' Jacobians, backward with
  // the mass-matrix walks up to the root, then its sum moved to the trunk
  // parent's origin into its LDS slot.
  void limb(int l) {
    const std::vector<int>& ch = pl_.limbs[l];
    o_ << "  {\n";
    for (int i : ch) {
      forward(i);
      if (do_jac_)
        for (size_t e = 0; e < ee_.size(); ++e)
          if (ee_[e] == i) jacobian((int)e);
    }
    if (do_rnea_ || do_crba_)
      for (auto it = ch.rbegin(); it != ch.rend(); ++it) backward(*it);
    const int sl = pl_.limb_slot[l], r = ch[0];
    if (sl >= 0) {
      const char* op = pl_.limb_first[l] ? " = " : " += ";
      o_ << "  {\n    Real t_[3], S_[10];\n";
      if (do_rnea_)
        o_ << "    bard::cross3(" << v("r", r) << ", " << v("F", r) << " + 3, t_);\n"
           << "    for (int k = 0; k < 3; ++k) {\n      xch_[(" << sl * 16 << " + k) * 64 + lane]" << op << v("F", r)
           << "[k] + t_[k];\n      xch_[(" << sl * 16 + 3 << " + k) * 64 + lane]" << op << v("F", r)
           << "[3 + k];\n    }\n";
      if (do_crba_)
        o_ << "    bard::shift_inertia(" << v("K", r) << ", " << v("r", r) << ", S_);\n"
           << "    for (int k = 0; k < 10; ++k) xch_[(" << sl * 16 + 6 << " + k) * 64 + lane]" << op << "S_[k];\n";
      o_ << "  }\n";
    }
    o_ << "  }\n";
  }

 protected:
  const bard_model* m_;
  std::vector<int> ee_;
  int frame_;
  bool fp64_;
  int ops_;          // outputs computed (1 torques, 2 mass matrix, 4 Jacobians)
  int parts_;        // workgroups per 64 instances: 1; 2 (RNEA | CRBA + Jacobians); 3 (RNEA | CRBA | Jacobians)
  bool dual_;        // parts_ > 1
  bool do_rnea_ = true, do_crba_ = true, do_jac_ = true;  // parts of the output the code being emitted computes
  SplitPlan pl_;
  bool split_;
  std::vector<char> trunk_;
  std::vector<int> slot_body_;
  std::ostringstream o_;
  bool member_ = false;             // emitting a member of a multi-tree kernel
  std::string blk_ = "blockIdx.x";  // the workgroup's group index in the emitted code

  double c(int body, int k) const { return fp64_ ? m_->cst64[body * CST + k] : (double)m_->cst32[body * CST + k]; }
  std::string lit(double x) const {
    char buf[64];
    if (fp64_) std::snprintf(buf, sizeof buf, "%.17g", x);
    else std::snprintf(buf, sizeof buf, "%.9g", x);
    std::string s(buf);
    if (s.find_first_of(".eEn") == std::string::npos) s += ".0";
    if (!fp64_) s += "f";
    return "Real(" + s + ")";
  }
  static std::string v(const char* name, int body) { return std::string(name) + std::to_string(body); }

  // sum of terms coef * factor, omitting exact zeros (x + 0 y = x exactly)
  std::string lin(const std::vector<std::pair<double, std::string>>& t) const {
    std::string s;
    for (const auto& [coef, f] : t) {
      if (coef == 0.0) continue;
      std::string term = f.empty() ? lit(coef) : (coef == 1.0 ? f : lit(coef) + " * " + f);
      s += s.empty() ? term : " + " + term;
    }
    return s.empty() ? "Real(0)" : s;
  }

  // The zero rows of M and J as tables (NZM, ZM, NZJ, ZJ); the kernel writes
  // them either from its computing lanes (zero_blocks == 0) or from extra
  // workgroups when the layout is instance-minor.
  void emit_zero_tables() {
    zero_lists();
    auto table = [&](const char* name, const char* count, const std::vector<int>& z) {
      o_ << "static constexpr int " << count << " = " << z.size() << ";\n";
      o_ << "static __device__ constexpr int " << name << "[" << (z.empty() ? 1 : z.size()) << "] = {";
      if (z.empty()) o_ << "0";
      for (size_t i = 0; i < z.size(); ++i) o_ << (i ? "," : "") << z[i];
      o_ << "};\n";
    };
    table("ZM", "NZM", zm_);
    table("ZJ", "NZJ", zj_);
  }

  void emit_zero_stores() {
    const char* first = split_ ? "wave" : "0";
    o_ << (split_ ? "  if (zero_blocks == 0 && wave < NW) {\n" : "  if (zero_blocks == 0) {\n")
       << "    for (int i = " << first << "; i < NZM; i += NW) MA(ZM[i], Real(0));\n"
          "    for (int i = " << first << "; i < NZJ; i += NW) JA(ZJ[i], Real(0));\n"
          "  }\n";
  }

  std::vector<int> zm_, zj_;

  void zero_lists() {
    // mass-matrix entries of unrelated dofs and Jacobian rows of dofs off an
    // end effector's root path are zero for every configuration
    const int nv = m_->nv;
    std::vector<int> zm, zj;
    std::vector<int> body_of(nv);
    for (int i = 0; i < m_->n; ++i)
      for (int d = 0; d < m_->nvi[i]; ++d) body_of[m_->vi[i] + d] = i;
    auto related = [&](int a, int bb) {
      for (int k = a; k >= 0; k = m_->parent[k])
        if (k == bb) return true;
      for (int k = bb; k >= 0; k = m_->parent[k])
        if (k == a) return true;
      return false;
    };
    for (int r = 0; r < nv; ++r)
      for (int col = 0; col < nv; ++col)
        if (!related(body_of[r], body_of[col])) zm.push_back(r * nv + col);
    for (size_t e = 0; e < ee_.size(); ++e) {
      std::vector<char> on(nv, 0);
      for (int k = ee_[e]; k >= 0; k = m_->parent[k])
        for (int d = 0; d < m_->nvi[k]; ++d) on[m_->vi[k] + d] = 1;
      for (int r = 0; r < 6; ++r)
        for (int col = 0; col < nv; ++col)
          if (!on[col]) zj.push_back(((int)e * 6 + r) * nv + col);
    }
    zm_ = (ops_ & 2) ? zm : std::vector<int>();
    zj_ = (ops_ & 4) ? zj : std::vector<int>();
  }

  // ---- entering body i: pose, axis, velocity, acceleration, body force ----
  void forward(int i) {
    forward_kin(i);
    if (ops_ & 8) store_pose(i);
    body_force(i, true);
  }

  // declare: define the body's state here; otherwise assign variables
  // declared beforehand in an outer scope
  void forward_kin(int i, bool declare = true) {
    const int p = m_->parent[i], t = m_->jtype[i], qi = m_->qi[i], vi = m_->vi[i];
    o_ << "  // body " << i << " (" << (t == J_REV ? "revolute" : t == J_PRI ? "prismatic" : "free") << ", parent "
       << p << ")\n";
    if (declare)
      o_ << "  Real " << v("R", i) << "[9], " << v("p", i) << "[3], " << v("r", i) << "[3], " << v("a", i)
         << "[3], " << v("v", i) << "[6], " << v("c", i) << "[6];\n";
    o_ << "  {\n";
    if (t == J_FREE) {
      o_ << "    Real x_ = Qv(" << qi + 3 << "), y_ = Qv(" << qi + 4 << "), z_ = Qv(" << qi + 5
         << "), w_ = Qv(" << qi + 6 << ");\n"
            "    const Real n_ = Real(1) / sqrt(x_ * x_ + y_ * y_ + z_ * z_ + w_ * w_);\n"
            "    x_ *= n_; y_ *= n_; z_ *= n_; w_ *= n_;\n"
            "    const Real Rq[9] = {Real(1) - Real(2) * (y_ * y_ + z_ * z_), Real(2) * (x_ * y_ - z_ * w_),"
            " Real(2) * (x_ * z_ + y_ * w_), Real(2) * (x_ * y_ + z_ * w_), Real(1) - Real(2) * (x_ * x_ + z_ * z_),"
            " Real(2) * (y_ * z_ - x_ * w_), Real(2) * (x_ * z_ - y_ * w_), Real(2) * (y_ * z_ + x_ * w_),"
            " Real(1) - Real(2) * (x_ * x_ + y_ * y_)};\n";
      o_ << "    const Real P_[3] = {Qv(" << qi << "), Qv(" << qi + 1 << "), Qv(" << qi + 2
         << ")};\n";
      for (int r = 0; r < 3; ++r)
        for (int col = 0; col < 3; ++col)
          o_ << "    " << v("R", i) << "[" << 3 * r + col << "] = "
             << lin({{c(i, C_R0 + 3 * r), "Rq[" + std::to_string(col) + "]"},
                     {c(i, C_R0 + 3 * r + 1), "Rq[" + std::to_string(3 + col) + "]"},
                     {c(i, C_R0 + 3 * r + 2), "Rq[" + std::to_string(6 + col) + "]"}})
             << ";\n";
      for (int r = 0; r < 3; ++r)
        o_ << "    " << v("p", i) << "[" << r << "] = "
           << lin({{c(i, C_R0 + 3 * r), "P_[0]"}, {c(i, C_R0 + 3 * r + 1), "P_[1]"}, {c(i, C_R0 + 3 * r + 2), "P_[2]"},
                   {c(i, C_T0 + r), ""}})
           << ";\n";
      o_ << "    for (int k = 0; k < 3; ++k) " << v("r", i) << "[k] = " << v("p", i) << "[k];\n";
    }
    if (t == J_FREE && do_rnea_) {
      // velocity coordinates [v; w] in the body frame -> world axes at the body origin
      o_ << "    Real vb_[3], wb_[3], ab_[3], wd_[3];\n";
      for (int k = 0; k < 3; ++k)
        o_ << "    vb_[" << k << "] = QDv(" << vi + k << "); wb_[" << k << "] = QDv(" << vi + 3 + k
           << "); ab_[" << k << "] = QDDv(" << vi + k << "); wd_[" << k << "] = QDDv("
           << vi + 3 + k << ");\n";
      const std::string R = v("R", i);
      for (int r = 0; r < 3; ++r) {
        auto row = [&](const char* x) {
          return R + "[" + std::to_string(3 * r) + "] * " + x + "[0] + " + R + "[" + std::to_string(3 * r + 1) +
                 "] * " + x + "[1] + " + R + "[" + std::to_string(3 * r + 2) + "] * " + x + "[2]";
        };
        o_ << "    " << v("v", i) << "[" << r << "] = " << row("wb_") << ";\n";
        o_ << "    " << v("v", i) << "[" << 3 + r << "] = " << row("vb_") << ";\n";
        o_ << "    " << v("c", i) << "[" << r << "] = " << row("wd_") << ";\n";
        o_ << "    " << v("c", i) << "[" << 3 + r << "] = " << row("ab_") << " - g" << r << ";\n";
      }
    }
    if (t != J_FREE) {
      // joint transform (eqs. (4)-(5))
      if (t == J_REV)
        o_ << "    Real s_, c_;\n    bard::sincos_r(Qv(" << qi << "), &s_, &c_);\n"
           << "    const Real o_ = Real(1) - c_;\n";
      else
        o_ << "    const Real x_ = Qv(" << qi << ");\n";
      o_ << "    Real Rpc[9], tpc[3];\n";
      for (int k = 0; k < 9; ++k)
        o_ << "    Rpc[" << k << "] = "
           << (t == J_REV ? lin({{c(i, C_R0 + k), ""}, {c(i, C_A + k), "s_"}, {c(i, C_B + k), "o_"}})
                          : lin({{c(i, C_R0 + k), ""}}))
           << ";\n";
      for (int k = 0; k < 3; ++k)
        o_ << "    tpc[" << k << "] = "
           << (t == J_PRI ? lin({{c(i, C_T0 + k), ""}, {c(i, C_D + k), "x_"}}) : lin({{c(i, C_T0 + k), ""}}))
           << ";\n";
      // the joint axis in the parent frame: R0 axis (R0 = R_pre, the joint frame
      // in the parent), taken in FP64 and rounded once by the literal
      double d[3];
      for (int k = 0; k < 3; ++k)
        d[k] = m_->cst64[i * CST + C_R0 + 3 * k] * m_->cst64[i * CST + C_AX] +
               m_->cst64[i * CST + C_R0 + 3 * k + 1] * m_->cst64[i * CST + C_AX + 1] +
               m_->cst64[i * CST + C_R0 + 3 * k + 2] * m_->cst64[i * CST + C_AX + 2];
      if (p < 0) {
        o_ << "    for (int k = 0; k < 9; ++k) " << v("R", i) << "[k] = Rpc[k];\n";
        o_ << "    for (int k = 0; k < 3; ++k) { " << v("r", i) << "[k] = tpc[k]; " << v("p", i)
           << "[k] = tpc[k]; }\n";
        for (int k = 0; k < 3; ++k) o_ << "    " << v("a", i) << "[" << k << "] = " << lit(d[k]) << ";\n";
      } else {
        const std::string Rp = v("R", p);
        o_ << "    bard::mul33(" << Rp << ", Rpc, " << v("R", i) << ");\n";
        for (int r = 0; r < 3; ++r) {
          o_ << "    " << v("r", i) << "[" << r << "] = " << Rp << "[" << 3 * r << "] * tpc[0] + " << Rp << "["
             << 3 * r + 1 << "] * tpc[1] + " << Rp << "[" << 3 * r + 2 << "] * tpc[2];\n";
          o_ << "    " << v("p", i) << "[" << r << "] = " << v("p", p) << "[" << r << "] + " << v("r", i) << "[" << r
             << "];\n";
          o_ << "    " << v("a", i) << "[" << r << "] = "
             << lin({{d[0], Rp + "[" + std::to_string(3 * r) + "]"}, {d[1], Rp + "[" + std::to_string(3 * r + 1) + "]"},
                     {d[2], Rp + "[" + std::to_string(3 * r + 2) + "]"}})
             << ";\n";
        }
      }
    }
    if (t != J_FREE && do_rnea_) {
      // parent state moved to this body's origin: u += w x r (velocity and spatial acceleration)
      o_ << "    Real vs_[6], as_[6];\n";
      if (p < 0) {
        o_ << "    for (int k = 0; k < 6; ++k) vs_[k] = Real(0);\n"
              "    as_[0] = Real(0); as_[1] = Real(0); as_[2] = Real(0); as_[3] = -g0; as_[4] = -g1; as_[5] = -g2;\n";
      } else {
        o_ << "    {\n      Real t_[3];\n      bard::cross3(" << v("v", p) << ", " << v("r", i) << ", t_);\n"
           << "      for (int k = 0; k < 3; ++k) { vs_[k] = " << v("v", p) << "[k]; vs_[3 + k] = " << v("v", p)
           << "[3 + k] + t_[k]; }\n      bard::cross3(" << v("c", p) << ", " << v("r", i) << ", t_);\n"
           << "      for (int k = 0; k < 3; ++k) { as_[k] = " << v("c", p) << "[k]; as_[3 + k] = " << v("c", p)
           << "[3 + k] + t_[k]; }\n    }\n";
      }
      o_ << "    const Real qd_ = QDv(" << vi << "), qdd_ = QDDv(" << vi << ");\n"
         << "    Real sq_[3], t_[3];\n    for (int k = 0; k < 3; ++k) sq_[k] = " << v("a", i) << "[k] * qd_;\n";
      const int off = (t == J_REV) ? 0 : 3;  // s = [a; 0] revolute, [0; a] prismatic
      o_ << "    for (int k = 0; k < 6; ++k) " << v("v", i) << "[k] = vs_[k];\n"
         << "    for (int k = 0; k < 3; ++k) " << v("v", i) << "[" << off << " + k] += sq_[k];\n"
         << "    for (int k = 0; k < 6; ++k) " << v("c", i) << "[k] = as_[k];\n"
         << "    for (int k = 0; k < 3; ++k) " << v("c", i) << "[" << off << " + k] += " << v("a", i)
         << "[k] * qdd_;\n";
      // v x (s qd): revolute [w x sq; u x sq], prismatic [0; w x sq]
      if (t == J_REV)
        o_ << "    bard::cross3(" << v("v", i) << ", sq_, t_);\n    for (int k = 0; k < 3; ++k) " << v("c", i)
           << "[k] += t_[k];\n    bard::cross3(" << v("v", i) << " + 3, sq_, t_);\n    for (int k = 0; k < 3; ++k) "
           << v("c", i) << "[3 + k] += t_[k];\n";
      else
        o_ << "    bard::cross3(" << v("v", i) << ", sq_, t_);\n    for (int k = 0; k < 3; ++k) " << v("c", i)
           << "[3 + k] += t_[k];\n";
    }
    o_ << "  }\n";
  }

  // body force about the body origin, f = I a + v x* I v, into I_i and f_i
  // (declared here, or beforehand in an outer scope)
  void body_force(int i, bool declare) {
    if (declare) o_ << "  Real " << v("I", i) << "[10], " << v("f", i) << "[6];\n";
    if (!do_rnea_ && !do_crba_) return;  // the Jacobians' part needs only poses

    // [m, R h, R Ibar R^T] about the body origin, world axes; the constant
    // parameters as literals, zero ones left out
    const std::string R = v("R", i), I = v("I", i);
    auto Rk = [&](int k) { return R + "[" + std::to_string(k) + "]"; };
    const double pi[10] = {c(i, C_PI), c(i, C_PI + 1), c(i, C_PI + 2), c(i, C_PI + 3), c(i, C_PI + 4),
                           c(i, C_PI + 5), c(i, C_PI + 6), c(i, C_PI + 7), c(i, C_PI + 8), c(i, C_PI + 9)};
    const double Ib[9] = {pi[4], pi[5], pi[7], pi[5], pi[6], pi[8], pi[7], pi[8], pi[9]};
    o_ << "  {\n    " << I << "[0] = " << lit(pi[0]) << ";\n";
    for (int r = 0; r < 3; ++r)
      o_ << "    " << I << "[" << 1 + r << "] = "
         << lin({{pi[1], Rk(3 * r)}, {pi[2], Rk(3 * r + 1)}, {pi[3], Rk(3 * r + 2)}}) << ";\n";
    o_ << "    Real X_[9];\n";
    for (int r = 0; r < 3; ++r)
      for (int col = 0; col < 3; ++col)
        o_ << "    X_[" << 3 * r + col << "] = "
           << lin({{Ib[col], Rk(3 * r)}, {Ib[3 + col], Rk(3 * r + 1)}, {Ib[6 + col], Rk(3 * r + 2)}}) << ";\n";
    const int ij[6][2] = {{0, 0}, {0, 1}, {1, 1}, {0, 2}, {1, 2}, {2, 2}};
    for (int k = 0; k < 6; ++k) {
      const int a = ij[k][0], b = ij[k][1];
      o_ << "    " << I << "[" << 4 + k << "] = X_[" << 3 * a << "] * " << Rk(3 * b) << " + X_[" << 3 * a + 1 << "] * "
         << Rk(3 * b + 1) << " + X_[" << 3 * a + 2 << "] * " << Rk(3 * b + 2) << ";\n";
    }
    if (do_rnea_)
      o_ << "    Real Iv_[6], vIv_[6];\n    bard::inertia_mul(" << v("I", i) << ", " << v("v", i) << ", Iv_);\n"
         << "    bard::crf(" << v("v", i) << ", Iv_, vIv_);\n    bard::inertia_mul(" << v("I", i) << ", " << v("c", i)
         << ", " << v("f", i) << ");\n    for (int k = 0; k < 6; ++k) " << v("f", i) << "[k] += vIv_[k];\n";
    o_ << "  }\n";
  }

  // motion-subspace column d of body j about the body origin (world axes)
  std::string s_col(int j, int d) const {
    const int t = m_->jtype[j];
    const std::string a = v("a", j), R = v("R", j);
    auto z = [](int n) { std::string s; for (int k = 0; k < n; ++k) s += "Real(0), "; return s; };
    if (t == J_REV) return "{" + a + "[0], " + a + "[1], " + a + "[2], Real(0), Real(0), Real(0)}";
    if (t == J_PRI) return "{Real(0), Real(0), Real(0), " + a + "[0], " + a + "[1], " + a + "[2]}";
    const int e = d % 3;
    const std::string col = R + "[" + std::to_string(e) + "], " + R + "[" + std::to_string(3 + e) + "], " + R + "[" +
                            std::to_string(6 + e) + "]";
    return d < 3 ? "{" + z(3) + col + "}" : "{" + col + ", Real(0), Real(0), Real(0)}";
  }

  // The non-zero halves of motion-subspace column d of body j: angular
  // (w) and linear (u) parts as three expressions each, empty when zero.
  void s_parts(int j, int d, std::vector<std::string>* w, std::vector<std::string>* u) const {
    const int t = m_->jtype[j];
    const std::string a = v("a", j), R = v("R", j);
    w->clear();
    u->clear();
    auto col = [&](int e) {
      return std::vector<std::string>{R + "[" + std::to_string(e) + "]", R + "[" + std::to_string(3 + e) + "]",
                                      R + "[" + std::to_string(6 + e) + "]"};
    };
    if (t == J_REV) *w = {a + "[0]", a + "[1]", a + "[2]"};
    else if (t == J_PRI) *u = {a + "[0]", a + "[1]", a + "[2]"};
    else if (d < 3) *u = col(d);
    else *w = col(d - 3);
  }

  // s_j,d . f for a force f (name[0..5]), structural zeros left out
  std::string dot_s(int j, int d, const std::string& f) const {
    std::vector<std::string> w, u;
    s_parts(j, d, &w, &u);
    std::string e;
    for (int k = 0; k < 3 && !w.empty(); ++k) e += (e.empty() ? "" : " + ") + w[k] + " * " + f + "[" + std::to_string(k) + "]";
    for (int k = 0; k < 3 && !u.empty(); ++k)
      e += (e.empty() ? "" : " + ") + u[k] + " * " + f + "[" + std::to_string(3 + k) + "]";
    return e;
  }

  // out = K s_j,d for a rigid-body inertia K = [m, h, Ibar]:
  // [Ibar w + h x u; m u - h x w], with the zero half of s left out
  void emit_Ks(const std::string& K, int j, int d, const std::string& out) {
    std::vector<std::string> w, u;
    s_parts(j, d, &w, &u);
    auto k = [&](int i) { return K + "[" + std::to_string(i) + "]"; };
    if (!w.empty()) {
      o_ << "      " << out << "[0] = " << k(4) << " * " << w[0] << " + " << k(5) << " * " << w[1] << " + " << k(7)
         << " * " << w[2] << ";\n";
      o_ << "      " << out << "[1] = " << k(5) << " * " << w[0] << " + " << k(6) << " * " << w[1] << " + " << k(8)
         << " * " << w[2] << ";\n";
      o_ << "      " << out << "[2] = " << k(7) << " * " << w[0] << " + " << k(8) << " * " << w[1] << " + " << k(9)
         << " * " << w[2] << ";\n";
      o_ << "      " << out << "[3] = " << w[1] << " * " << k(3) << " - " << w[2] << " * " << k(2) << ";\n";
      o_ << "      " << out << "[4] = " << w[2] << " * " << k(1) << " - " << w[0] << " * " << k(3) << ";\n";
      o_ << "      " << out << "[5] = " << w[0] << " * " << k(2) << " - " << w[1] << " * " << k(1) << ";\n";
    } else {
      o_ << "      " << out << "[0] = " << k(2) << " * " << u[2] << " - " << k(3) << " * " << u[1] << ";\n";
      o_ << "      " << out << "[1] = " << k(3) << " * " << u[0] << " - " << k(1) << " * " << u[2] << ";\n";
      o_ << "      " << out << "[2] = " << k(1) << " * " << u[1] << " - " << k(2) << " * " << u[0] << ";\n";
      for (int i = 0; i < 3; ++i) o_ << "      " << out << "[" << 3 + i << "] = " << k(0) << " * " << u[i] << ";\n";
    }
  }

  void store_M(int r, int col, const std::string& val) {
    const int nv = m_->nv;
    o_ << "    MA(" << r * nv + col << ", " << val << ");\n";
    if (r != col) o_ << "    MA(" << col * nv + r << ", " << val << ");\n";
  }

  // ---- leaving body i: subtree force, torque, composite inertia, M ----
  void backward(int i) {
    const int t = m_->jtype[i], vi = m_->vi[i], nd = m_->nvi[i];
    o_ << "  // body " << i << ": subtree sums\n  Real " << v("F", i) << "[6], " << v("K", i) << "[10];\n  {\n";
    if (do_rnea_) o_ << "    for (int k = 0; k < 6; ++k) " << v("F", i) << "[k] = " << v("f", i) << "[k];\n";
    if (do_crba_) o_ << "    for (int k = 0; k < 10; ++k) " << v("K", i) << "[k] = " << v("I", i) << "[k];\n";
    for (int ch : m_->children[i]) {
      if (split_ && trunk_[i] && !trunk_[ch]) continue;  // a limb: its wave's sum arrives through LDS
      o_ << "    {\n      Real t_[3], S_[10];\n";
      if (do_rnea_)
        o_ << "      bard::cross3(" << v("r", ch) << ", " << v("F", ch) << " + 3, t_);\n"
           << "      for (int k = 0; k < 3; ++k) { " << v("F", i) << "[k] += " << v("F", ch) << "[k] + t_[k]; "
           << v("F", i) << "[3 + k] += " << v("F", ch) << "[3 + k]; }\n";
      if (do_crba_)
        o_ << "      bard::shift_inertia(" << v("K", ch) << ", " << v("r", ch) << ", S_);\n"
           << "      for (int k = 0; k < 10; ++k) " << v("K", i) << "[k] += S_[k];\n";
      o_ << "    }\n";
    }
    for (size_t sl = 0; sl < slot_body_.size(); ++sl)
      if (split_ && slot_body_[sl] == i) {
        if (do_rnea_)
          o_ << "    for (int k = 0; k < 6; ++k) " << v("F", i) << "[k] += xch_[(" << sl * 16 << " + k) * 64 + lane];\n";
        if (do_crba_)
          o_ << "    for (int k = 0; k < 10; ++k) " << v("K", i) << "[k] += xch_[(" << sl * 16 + 6
             << " + k) * 64 + lane];\n";
      }
    if (do_rnea_) torque(i);
    if (do_crba_) mass_columns(i);
    o_ << "  }\n";
  }

  void torque(int i) {
    const int t = m_->jtype[i], vi = m_->vi[i];
    const std::string F = v("F", i), a = v("a", i), R = v("R", i);
    if (t == J_REV)
      o_ << "    TAU(" << vi << ", " << a << "[0] * " << F << "[0] + " << a << "[1] * " << F << "[1] + "
         << a << "[2] * " << F << "[2]);\n";
    else if (t == J_PRI)
      o_ << "    TAU(" << vi << ", " << a << "[0] * " << F << "[3] + " << a << "[1] * " << F << "[4] + "
         << a << "[2] * " << F << "[5]);\n";
    else
      for (int d = 0; d < 6; ++d) {
        const int e = d % 3, base = d < 3 ? 3 : 0;  // [f; n] in the body frame: R^T f, R^T n
        o_ << "    TAU(" << vi + d << ", " << R << "[" << e << "] * " << F << "[" << base << "] + " << R
           << "[" << 3 + e << "] * " << F << "[" << base + 1 << "] + " << R << "[" << 6 + e << "] * " << F << "["
           << base + 2 << "]);\n";
      }
  }

  // mass-matrix columns of this body's dofs, and up the ancestors
  void mass_columns(int i) {
    const int vi = m_->vi[i], nd = m_->nvi[i];
    for (int d = 0; d < nd; ++d) {
      o_ << "    {\n      Real fc_[6];\n";
      emit_Ks(v("K", i), i, d, "fc_");
      for (int d2 = 0; d2 <= d; ++d2) {
        o_ << "      {\n        const Real m_ = " << dot_s(i, d2, "fc_") << ";\n";
        store_M(vi + d2, vi + d, "m_");
        o_ << "      }\n";
      }
      // up the ancestors: the force moves to the parent's origin, n += r x f
      int ch = i;
      for (int j = m_->parent[i]; j >= 0; ch = j, j = m_->parent[j]) {
        o_ << "      {\n        Real t_[3];\n        bard::cross3(" << v("r", ch) << ", fc_ + 3, t_);\n"
           << "        for (int k = 0; k < 3; ++k) fc_[k] += t_[k];\n";
        for (int e = 0; e < m_->nvi[j]; ++e) {
          o_ << "        {\n          const Real m_ = " << dot_s(j, e, "fc_") << ";\n";
          store_M(m_->vi[j] + e, vi + d, "m_");
          o_ << "        }\n";
        }
        o_ << "      }\n";
      }
      o_ << "    }\n";
    }
  }

  // Jacobian columns of end effector e (rows [linear; angular]).
  void jacobian(int ei) {
    const int e = ee_[ei], nv = m_->nv;
    o_ << "  // Jacobian of end effector " << ei << " (body " << e << ")\n  {\n";
    for (int j = e; j >= 0; j = m_->parent[j]) {
      const int t = m_->jtype[j];
      for (int d = 0; d < m_->nvi[j]; ++d) {
        const int col = m_->vi[j] + d;
        o_ << "    {\n      const Real s_[6] = " << s_col(j, d) << ";\n      Real l_[3];\n";
        // angular part w = s[0..2]; linear part: velocity of the chosen point
        if (t == J_PRI || (t == J_FREE && d < 3)) {
          o_ << "      for (int k = 0; k < 3; ++k) l_[k] = s_[3 + k];\n";
        } else if (frame_ == 0) {  // the body-fixed point at the world origin: p_j x w
          o_ << "      bard::cross3(" << v("p", j) << ", s_, l_);\n";
        } else {  // the end effector's origin: w x (p_e - p_j)
          o_ << "      Real d_[3];\n      for (int k = 0; k < 3; ++k) d_[k] = " << v("p", e) << "[k] - " << v("p", j)
             << "[k];\n      bard::cross3(s_, d_, l_);\n";
        }
        for (int r = 0; r < 6; ++r)
          o_ << "      JA(" << (ei * 6 + r) * nv + col << ", " << (r < 3 ? "l_[" : "s_[")
             << (r % 3) << "]);\n";
        o_ << "    }\n";
      }
    }
    o_ << "  }\n";
  }

  void visit(int i) {
    forward(i);
    if (do_jac_)
      for (size_t e = 0; e < ee_.size(); ++e)
        if (ee_[e] == i) jacobian((int)e);
    for (int ch : m_->children[i]) visit(ch);
    if (do_rnea_ || do_crba_) backward(i);
  }
};


// Emits the source of one specialised forward-dynamics (ABA) kernel: one
// wave per 64 instances over the whole tree, in base-frame coordinates (world
// axes, vectors about the root's origin -- a fixed base's world origin, a
// free root's own origin), so a child's articulated inertia and bias force
// add to its parent's without a transform, as in the generic kernel.
// Passes 1 and 2 run in one depth-first walk: entering a body its pose,
// motion subspace, velocity, velocity-product acceleration, rigid inertia
// and bias force; leaving it (after its children) its articulated inertia,
// U = IA s, D = s^T U, u = tau - s^T pA, and what it hands to its parent, so
// only the state of the bodies on the current path is held.  Pass 3 needs
// per body only W = U / D and e = (u - U.c) / D (qdd = e - W.a_parent) and
// recomputes the kinematics and velocities on a second walk.  A free root
// factors its 6x6 D by Cholesky.
class AbaEmitter : public Emitter {
 public:
  // split: limbs in waves of their own (the chain kernel's plan) when the
  // tree has one and its LDS hand-over fits; otherwise the whole tree in one
  // wave
  AbaEmitter(const bard_model* m, bool fp64, bool split) : Emitter(m, {}, 0, fp64, split ? 0 : 1) {
    do_rnea_ = false;
    aba_split_ = split && split_ && split_fits();
  }

  bool is_split() const { return aba_split_; }
  int waves() const { return aba_split_ ? pl_.waves : 1; }

  // every loop of the generated code has constant bounds; unrolled, the
  // arrays it indexes stay in registers
  std::string source() {
    std::string src = aba_split_ ? source_split() : source_whole();
    std::string out;
    const std::string pat = "for (int ";
    size_t at = 0;
    for (size_t k; (k = src.find(pat, at)) != std::string::npos; at = k + pat.size()) {
      out.append(src, at, k - at);
      out += "_Pragma(\"unroll\") " + pat;
    }
    out.append(src, at, std::string::npos);
    return out;
  }

  void header() {
    const int n = m_->n;
    o_ << "// generated: forward dynamics (ABA) for one tree (" << n << " bodies, nv " << m_->nv << ", "
       << (fp64_ ? "FP64" : "FP32") << (aba_split_ ? ", split over waves by limbs" : ", one wave per instance group")
       << ")\n#include \"spatial.h\"\n";
    o_ << "typedef " << (fp64_ ? "double" : "float") << " Real;\n";
    o_ << "template <class T>\n"
          "__device__ __forceinline__ T* bard_at(T* base, long long k, long long sk, unsigned ob) {\n"
          "  return (T*)((const char*)(base + k * sk) + ob);\n"
          "}\n"
          "#define Q(k) (*bard_at(q, (k), sq_k, oq_))\n"
          "#define QD(k) (*bard_at(qd, (k), sqd_k, oqd_))\n"
          "#define TIN(k) (*bard_at(tau, (k), st_k, ot_))\n"
          "#define QDDO(k, v) (*bard_at(qdd, (k), so_k, oo_) = (v))\n"
          "#define WL(slot, k) wl_[((slot) * 7 + (k)) * 64 + lane]\n"
          "#define Qv(k) Qv_##k\n"
          "#define QDv(k) QDv_##k\n"
          "#define TAUv(k) TAUv_##k\n"
          // upper-triangle index of a symmetric 6x6 matrix
          "__device__ constexpr int SI(int r, int c) { return r <= c ? r * 6 - r * (r - 1) / 2 + (c - r)"
          " : c * 6 - c * (c - 1) / 2 + (r - c); }\n";
  }

  void params() {
    o_ << "    const Real* __restrict__ q, const Real* __restrict__ qd, const Real* __restrict__ tau,\n"
          "    Real* __restrict__ qdd, long long sq_b, long long sq_k, long long sqd_b, long long sqd_k,\n"
          "    long long st_b, long long st_k, long long so_b, long long so_k, long long B, Real g0, Real g1,\n"
          "    Real g2) {\n";
  }

  void offsets() {
    o_ << "  const unsigned oq_ = (unsigned)(b * sq_b) * (unsigned)sizeof(Real);\n"
          "  const unsigned oqd_ = (unsigned)(b * sqd_b) * (unsigned)sizeof(Real);\n"
          "  const unsigned ot_ = (unsigned)(b * st_b) * (unsigned)sizeof(Real);\n"
          "  const unsigned oo_ = (unsigned)(b * so_b) * (unsigned)sizeof(Real);\n"
          "  const Real a0_[6] = {Real(0), Real(0), Real(0), -g0, -g1, -g2};\n";
  }

  std::string source_whole() {
    const int n = m_->n;
    header();
    o_ << "static constexpr int NW = 1;  // waves per workgroup, 64 instances\n";
    o_ << "extern \"C\" __global__ void __launch_bounds__(64) bard_spec_aba(\n";
    params();
    o_ << "  const long long b = (long long)blockIdx.x * 64 + threadIdx.x;\n"
          "  if (b >= B) return;\n"
          "  const int lane = (int)threadIdx.x;\n";
    offsets();
    // what pass 3 needs of each body: W = U / D and e in LDS (7 values per
    // lane; each lane reads only its own), a free root's factors in registers
    // (formed last in pass 2, used first in pass 3)
    slot_.assign(n, -1);
    int ns = 0;
    for (int i = 0; i < n; ++i)
      if (m_->jtype[i] == J_FREE) o_ << "  Real Ur" << i << "[36], Lr" << i << "[21], ur" << i << "[6];\n";
      else slot_[i] = ns++;
    // W and e in LDS while it fits, else in registers (they then spill)
    we_lds_ = (size_t)ns * 7 * 64 * (fp64_ ? 8 : 4) <= 150 * 1024;
    if (ns && we_lds_) o_ << "  __shared__ Real wl_[" << ns * 7 * 64 << "];\n";
    if (!we_lds_)
      for (int i = 0; i < n; ++i)
        if (slot_[i] >= 0) o_ << "  Real W" << i << "[6], e" << i << ";\n";
    o_ << "  // passes 1 and 2\n";
    for (int i = 0; i < n; ++i)
      if (m_->parent[i] < 0) walk12(i);
    o_ << "  // pass 3\n";
    for (int i = 0; i < n; ++i)
      if (m_->parent[i] < 0) walk3(i);
    o_ << "}\n";
    return o_.str();
  }

 private:
  // upper-triangle index of a symmetric 6x6 matrix, at generation time
  static int si(int r, int c) {
    if (r > c) std::swap(r, c);
    return r * 6 - r * (r - 1) / 2 + (c - r);
  }
  static std::string ix(const std::string& a, int k) { return a + "[" + std::to_string(k) + "]"; }

  std::vector<int> slot_;  // LDS slot of each body's W and e
  bool we_lds_ = true;     // W and e in LDS (else in registers, whole form only)
  bool aba_split_ = false;
  enum Mode { WHOLE, LIMB, TRUNK };
  Mode mode_ = WHOLE;
  std::vector<int> at_slot_;  // LDS slot of the acceleration of each trunk body with limbs attached

  // LDS of the split form: W and e of every non-free body, a limb sum (21 +
  // 6) per (wave, trunk body) slot, a trunk body's acceleration per attach
  // body; a free root inside a limb would need its factors across barriers
  bool split_fits() {
    const int n = m_->n;
    int nwl = 0, nat = 0;
    std::vector<char> has_limb(n, 0);
    for (size_t l = 0; l < pl_.limbs.size(); ++l) {
      const int r = pl_.limbs[l][0], at = m_->parent[r];
      if (at >= 0) has_limb[at] = 1;
      else if (m_->jtype[r] == J_FREE && !pl_.slot_body.empty()) return false;
    }
    bool any_trunk = false;
    for (int i = 0; i < n; ++i) {
      if (m_->jtype[i] != J_FREE) ++nwl;
      nat += has_limb[i];
      any_trunk = any_trunk || trunk_[i];
    }
    if (!any_trunk) nat = 0;
    const size_t bytes = (size_t)(nwl * 7 + pl_.slot_body.size() * 27 + nat * 6) * 64 * (fp64_ ? 8 : 4);
    return bytes <= 150 * 1024;
  }

  // pose, motion subspace s (or the free root's S), velocity v, velocity-
  // product acceleration cJ, all about the reference point; the body's joint
  // inputs loaded here
  void kin_vel(int i) {
    const int p = m_->parent[i], t = m_->jtype[i], vi = m_->vi[i];
    const int nq = t == J_FREE ? 7 : 1;
    for (int k = 0; k < nq; ++k) o_ << "  const Real Qv_" << m_->qi[i] + k << " = Q(" << m_->qi[i] + k << ");\n";
    for (int k = 0; k < m_->nvi[i]; ++k) o_ << "  const Real QDv_" << vi + k << " = QD(" << vi + k << ");\n";
    forward_kin(i);
    if (t == J_FREE && p < 0)
      o_ << "  for (int k = 0; k < 3; ++k) { " << v("p", i) << "[k] = Real(0); " << v("r", i) << "[k] = Real(0); }\n";
    const std::string R = v("R", i);
    if (t == J_FREE) {
      // columns [0; R e_d] for the linear dofs, [R e_d; 0] for the angular ones
      o_ << "  Real " << v("S", i) << "[36], " << v("V", i) << "[6], " << v("cJ", i) << "[6];\n  {\n";
      for (int d = 0; d < 6; ++d)
        for (int k = 0; k < 6; ++k) {
          const bool lin_dof = d < 3;
          const bool nz = lin_dof ? k >= 3 : k < 3;
          const int e = d % 3, row = k % 3;
          o_ << "    " << v("S", i) << "[" << d * 6 + k << "] = "
             << (nz ? R + "[" + std::to_string(3 * row + e) + "]" : std::string("Real(0)")) << ";\n";
        }
      o_ << "    for (int k = 0; k < 6; ++k) { " << v("V", i) << "[k] = Real(0);";
      for (int d = 0; d < 6; ++d) o_ << " " << v("V", i) << "[k] += " << v("S", i) << "[" << d * 6 << " + k] * QDv(" << vi + d << ");";
      o_ << " }\n";
      if (p >= 0) o_ << "    // (a free joint below the root is refused by the model compiler)\n";
      o_ << "    for (int k = 0; k < 6; ++k) " << v("cJ", i) << "[k] = Real(0);\n  }\n";
      return;
    }
    o_ << "  Real " << v("s", i) << "[6], " << v("V", i) << "[6], " << v("cJ", i) << "[6];\n  {\n";
    const std::string a = v("a", i), pp = v("p", i), s = v("s", i);
    if (t == J_REV)
      o_ << "    for (int k = 0; k < 3; ++k) " << s << "[k] = " << a << "[k];\n    bard::cross3(" << pp << ", " << a
         << ", " << s << " + 3);\n";
    else
      o_ << "    for (int k = 0; k < 3; ++k) { " << s << "[k] = Real(0); " << s << "[3 + k] = " << a << "[k]; }\n";
    o_ << "    Real vJ_[6];\n    for (int k = 0; k < 6; ++k) vJ_[k] = " << s << "[k] * QDv(" << vi << ");\n";
    if (p >= 0)
      o_ << "    bard::crm(" << v("V", p) << ", vJ_, " << v("cJ", i) << ");\n    for (int k = 0; k < 6; ++k) "
         << v("V", i) << "[k] = " << v("V", p) << "[k] + vJ_[k];\n";
    else
      o_ << "    for (int k = 0; k < 6; ++k) { " << v("cJ", i) << "[k] = Real(0); " << v("V", i) << "[k] = vJ_[k]; }\n";
    o_ << "  }\n";
  }

  // whether body i hands its articulated inertia to its parent through LDS
  bool to_slot(int i) const { return mode_ == LIMB && m_->parent[i] >= 0 && trunk_[m_->parent[i]]; }

  void walk12(int i) {
    const int t = m_->jtype[i], vi = m_->vi[i];
    if (m_->parent[i] >= 0 && !to_slot(i)) o_ << "  Real " << v("Ia", i) << "[21], " << v("pa", i) << "[6];\n";
    o_ << "  {\n";
    kin_vel(i);
    for (int ch : m_->children[i])
      if (!(mode_ == TRUNK && !trunk_[ch])) walk12(ch);
    // leaving the body: its rigid inertia about the body origin (world axes),
    // about the reference point, and its bias force pA = v x* (I v)
    body_force(i, true);
    o_ << "  Real " << v("I0", i) << "[10], " << v("pA", i) << "[6];\n  {\n    bard::shift_inertia(" << v("I", i)
       << ", " << v("p", i) << ", " << v("I0", i) << ");\n    Real Iv_[6];\n    bard::inertia_mul(" << v("I0", i)
       << ", " << v("V", i) << ", Iv_);\n    bard::crf(" << v("V", i) << ", Iv_, " << v("pA", i) << ");\n  }\n";
    // leaving the body: articulated inertia and bias force with the children's
    const std::string I0 = v("I0", i);
    // the rigid inertia [Ibar, h x; -h x, m 1] as a symmetric 6x6
    const std::string ent[6][6] = {
        {ix(I0, 4), ix(I0, 5), ix(I0, 7), "Real(0)", "-" + ix(I0, 3), ix(I0, 2)},
        {"", ix(I0, 6), ix(I0, 8), ix(I0, 3), "Real(0)", "-" + ix(I0, 1)},
        {"", "", ix(I0, 9), "-" + ix(I0, 2), ix(I0, 1), "Real(0)"},
        {"", "", "", ix(I0, 0), "Real(0)", "Real(0)"},
        {"", "", "", "", ix(I0, 0), "Real(0)"},
        {"", "", "", "", "", ix(I0, 0)}};
    o_ << "  {\n    Real IA_[21], pA_[6];\n";
    for (int r = 0; r < 6; ++r)
      for (int c = r; c < 6; ++c) o_ << "    IA_[" << si(r, c) << "] = " << ent[r][c] << ";\n";
    o_ << "    for (int k = 0; k < 6; ++k) pA_[k] = " << v("pA", i) << "[k];\n";
    for (int ch : m_->children[i])
      if (!(mode_ == TRUNK && !trunk_[ch]))
        o_ << "    for (int k = 0; k < 21; ++k) IA_[k] += " << v("Ia", ch) << "[k];\n    for (int k = 0; k < 6; ++k) pA_[k] += "
           << v("pa", ch) << "[k];\n";
    if (mode_ == TRUNK)
      for (size_t sl = 0; sl < pl_.slot_body.size(); ++sl)
        if (pl_.slot_body[sl] == i)
          o_ << "    for (int k = 0; k < 21; ++k) IA_[k] += xa_[(" << sl * 27 << " + k) * 64 + lane];\n"
             << "    for (int k = 0; k < 6; ++k) pA_[k] += xa_[(" << sl * 27 + 21 << " + k) * 64 + lane];\n";
    for (int k = 0; k < m_->nvi[i]; ++k) o_ << "    const Real TAUv_" << vi + k << " = TIN(" << vi + k << ");\n";
    if (t == J_FREE) {
      const std::string S = v("S", i), U = "Ur" + std::to_string(i), L = "Lr" + std::to_string(i),
                        u = "ur" + std::to_string(i);
      o_ << "    Real D_[21];\n";
      for (int d = 0; d < 6; ++d)
        for (int r = 0; r < 6; ++r) {
          o_ << "    " << ix(U, d * 6 + r) << " = ";
          for (int c = 0; c < 6; ++c) o_ << (c ? " + " : "") << "IA_[" << si(r, c) << "] * " << ix(S, d * 6 + c);
          o_ << ";\n";
        }
      for (int d = 0; d < 6; ++d) {
        o_ << "    " << ix(u, d) << " = TAUv(" << vi + d << ") - (";
        for (int k = 0; k < 6; ++k) o_ << (k ? " + " : "") << ix(S, d * 6 + k) << " * pA_[" << k << "]";
        o_ << ");\n";
      }
      for (int r = 0; r < 6; ++r)
        for (int c = r; c < 6; ++c) {
          o_ << "    D_[" << si(r, c) << "] = ";
          for (int k = 0; k < 6; ++k) o_ << (k ? " + " : "") << ix(S, r * 6 + k) << " * " << ix(U, c * 6 + k);
          o_ << ";\n";
        }
      // D = L L^T
      for (int jj = 0; jj < 6; ++jj) {
        o_ << "    {\n      Real d_ = D_[" << si(jj, jj) << "];\n";
        for (int k = 0; k < jj; ++k) o_ << "      d_ -= " << ix(L, si(jj, k)) << " * " << ix(L, si(jj, k)) << ";\n";
        o_ << "      " << ix(L, si(jj, jj)) << " = sqrt(d_);\n      const Real il_ = Real(1) / " << ix(L, si(jj, jj))
           << ";\n";
        for (int r = jj + 1; r < 6; ++r) {
          o_ << "      " << ix(L, si(r, jj)) << " = (D_[" << si(r, jj) << "]";
          for (int k = 0; k < jj; ++k) o_ << " - " << ix(L, si(r, k)) << " * " << ix(L, si(jj, k));
          o_ << ") * il_;\n";
        }
        o_ << "    }\n";
      }
      if (m_->parent[i] >= 0) o_ << "    // (not reached: a free joint is always a root)\n";
      o_ << "  }\n  }\n";
      return;
    }
    const std::string s = v("s", i), cJ = v("cJ", i), sl = std::to_string(slot_[i]);
    o_ << "    Real U_[6];\n";
    for (int r = 0; r < 6; ++r) {
      o_ << "    U_[" << r << "] = ";
      for (int c = 0; c < 6; ++c) o_ << (c ? " + " : "") << "IA_[" << si(r, c) << "] * " << ix(s, c);
      o_ << ";\n";
    }
    o_
       << "    const Real D_ = " << s << "[0] * U_[0] + " << s << "[1] * U_[1] + " << s << "[2] * U_[2] + " << s
       << "[3] * U_[3] + " << s << "[4] * U_[4] + " << s << "[5] * U_[5];\n"
       << "    const Real Di_ = Real(1) / D_;\n"
       << "    const Real u_ = TAUv(" << vi << ") - (" << s << "[0] * pA_[0] + " << s << "[1] * pA_[1] + " << s
       << "[2] * pA_[2] + " << s << "[3] * pA_[3] + " << s << "[4] * pA_[4] + " << s << "[5] * pA_[5]);\n"
       ;
    const std::string Wk = we_lds_ ? "WL(" + sl + ", " : "W" + std::to_string(i) + "[";
    const std::string Wc = we_lds_ ? ")" : "]";
    for (int k = 0; k < 6; ++k) o_ << "    " << Wk << k << Wc << " = U_[" << k << "] * Di_;\n";
    o_ << "    " << (we_lds_ ? "WL(" + sl + ", 6)" : "e" + std::to_string(i)) << " = (u_ - (U_[0] * " << cJ
       << "[0] + U_[1] * " << cJ << "[1] + U_[2] * " << cJ << "[2] + U_[3] * " << cJ << "[3] + U_[4] * " << cJ
       << "[4] + U_[5] * " << cJ << "[5])) * Di_;\n";
    if (m_->parent[i] >= 0) {
      const bool lds = to_slot(i);
      const std::string Ia = lds ? std::string("Ia_") : v("Ia", i), pa = lds ? std::string("pa_") : v("pa", i);
      if (lds) o_ << "    Real Ia_[21], pa_[6];\n";
      for (int r = 0; r < 6; ++r)
        for (int c = r; c < 6; ++c)
          o_ << "    " << ix(Ia, si(r, c)) << " = IA_[" << si(r, c) << "] - U_[" << r << "] * U_[" << c << "] * Di_;\n";
      o_ << "    const Real uD_ = u_ * Di_;\n";
      for (int r = 0; r < 6; ++r) {
        o_ << "    " << ix(pa, r) << " = pA_[" << r << "] + U_[" << r << "] * uD_";
        for (int c = 0; c < 6; ++c) o_ << " + " << ix(Ia, si(r, c)) << " * " << ix(cJ, c);
        o_ << ";\n";
      }
      if (lds) {
        int l = -1;
        for (size_t k = 0; k < pl_.limbs.size(); ++k)
          if (pl_.limbs[k][0] == i) l = (int)k;
        const int sl = pl_.limb_slot[l];
        const char* op = pl_.limb_first[l] ? " = " : " += ";
        o_ << "    for (int k = 0; k < 21; ++k) xa_[(" << sl * 27 << " + k) * 64 + lane]" << op << "Ia_[k];\n"
           << "    for (int k = 0; k < 6; ++k) xa_[(" << sl * 27 + 21 << " + k) * 64 + lane]" << op << "pa_[k];\n";
      }
    }
    o_ << "  }\n  }\n";
  }

  void walk3(int i) {
    const int p = m_->parent[i], t = m_->jtype[i], vi = m_->vi[i];
    o_ << "  {\n";
    kin_vel(i);
    o_ << "  Real " << v("A", i) << "[6];\n  {\n";
    const std::string ap = p >= 0 ? v("A", p) : std::string("a0_");
    if (t == J_FREE) {
      const std::string S = v("S", i), U = "Ur" + std::to_string(i), L = "Lr" + std::to_string(i),
                        u = "ur" + std::to_string(i);
      o_ << "    Real x_[6];\n";
      for (int d = 0; d < 6; ++d) {
        o_ << "    x_[" << d << "] = " << ix(u, d);
        for (int k = 0; k < 6; ++k) o_ << " - " << ix(U, d * 6 + k) << " * " << ap << "[" << k << "]";
        o_ << ";\n";
      }
      for (int r = 0; r < 6; ++r) {  // L y = x
        o_ << "    x_[" << r << "] = (x_[" << r << "]";
        for (int k = 0; k < r; ++k) o_ << " - " << ix(L, si(r, k)) << " * x_[" << k << "]";
        o_ << ") / " << ix(L, si(r, r)) << ";\n";
      }
      for (int r = 5; r >= 0; --r) {  // L^T z = y
        o_ << "    x_[" << r << "] = (x_[" << r << "]";
        for (int k = r + 1; k < 6; ++k) o_ << " - " << ix(L, si(k, r)) << " * x_[" << k << "]";
        o_ << ") / " << ix(L, si(r, r)) << ";\n";
      }
      for (int k = 0; k < 6; ++k) {
        o_ << "    " << v("A", i) << "[" << k << "] = " << ap << "[" << k << "] + " << v("cJ", i) << "[" << k << "]";
        for (int d = 0; d < 6; ++d) o_ << " + " << ix(S, d * 6 + k) << " * x_[" << d << "]";
        o_ << ";\n";
      }
      for (int d = 0; d < 6; ++d) o_ << "    QDDO(" << vi + d << ", x_[" << d << "]);\n";
    } else {
      const std::string s = v("s", i), sl = std::to_string(slot_[i]);
      const std::string Wk = we_lds_ ? "WL(" + sl + ", " : "W" + std::to_string(i) + "[";
      const std::string Wc = we_lds_ ? ")" : "]";
      o_ << "    Real qdd_ = " << (we_lds_ ? "WL(" + sl + ", 6)" : "e" + std::to_string(i)) << ";\n";
      for (int k = 0; k < 6; ++k) o_ << "    qdd_ -= " << Wk << k << Wc << " * " << ap << "[" << k << "];\n";
      o_
         << "    for (int k = 0; k < 6; ++k) " << v("A", i) << "[k] = " << ap << "[k] + " << v("cJ", i) << "[k] + " << s
         << "[k] * qdd_;\n    QDDO(" << vi << ", qdd_);\n";
    }
    if (mode_ == TRUNK && at_slot_[i] >= 0)
      o_ << "  for (int k = 0; k < 6; ++k) at_[(" << at_slot_[i] * 6 << " + k) * 64 + lane] = " << v("A", i) << "[k];\n";
    o_ << "  }\n";
    for (int ch : m_->children[i])
      if (!(mode_ == TRUNK && !trunk_[ch])) walk3(ch);
    o_ << "  }\n";
  }

  // The split form: phase A (every wave: the trunk's kinematics, its limbs'
  // passes 1 and 2, each limb's articulated inertia and bias force moved into
  // LDS), phase B (the merging wave: the trunk's passes 2 and 3, the
  // accelerations of the trunk bodies with limbs attached into LDS), phase C
  // (every wave: the kinematics again and its limbs' pass 3).  A tree without
  // a trunk runs A and C back to back in each wave, with no barrier.
  std::string source_split() {
    const int n = m_->n, nw = pl_.waves;
    header();
    o_ << "static constexpr int NW = " << nw << ";  // waves per workgroup, 64 instances\n";
    o_ << "extern \"C\" __global__ void __launch_bounds__(" << 64 * nw << ") bard_spec_aba(\n";
    params();
    o_ << "  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);\n"
          "  const int lane = (int)threadIdx.x & 63;\n"
          "  long long b = (long long)blockIdx.x * 64 + lane;\n"
          "  if (b > B - 1) b = B - 1;  // every lane reaches the barriers\n";
    offsets();
    slot_.assign(n, -1);
    at_slot_.assign(n, -1);
    int ns = 0, nat = 0;
    bool any_trunk = false;
    for (int i = 0; i < n; ++i) {
      if (m_->jtype[i] != J_FREE) slot_[i] = ns++;
      any_trunk = any_trunk || trunk_[i];
    }
    for (const auto& limb : pl_.limbs) {
      const int at = m_->parent[limb[0]];
      if (at >= 0 && at_slot_[at] < 0) at_slot_[at] = nat++;
    }
    if (ns) o_ << "  __shared__ Real wl_[" << ns * 7 * 64 << "];\n";
    if (!pl_.slot_body.empty()) o_ << "  __shared__ Real xa_[" << pl_.slot_body.size() * 27 * 64 << "];\n";
    if (nat) o_ << "  __shared__ Real at_[" << nat * 6 * 64 << "];\n";
    std::vector<int> tb;
    for (int i = 0; i < n; ++i)
      if (trunk_[i]) tb.push_back(i);
    auto free_roots = [&](const std::vector<int>& bodies) {
      for (int i : bodies)
        if (m_->jtype[i] == J_FREE) o_ << "  Real Ur" << i << "[36], Lr" << i << "[21], ur" << i << "[6];\n";
    };
    const int merge = nw - 1;
    for (int w = 0; w < nw; ++w) {
      o_ << (w ? "  else if" : "  if") << " (wave == " << w << ") {\n";
      mode_ = LIMB;
      for (int i : tb) kin_vel(i);
      std::vector<int> roots;
      for (int l : pl_.bins[w]) roots.push_back(pl_.limbs[l][0]);
      if (!any_trunk) free_roots(roots);
      for (int r : roots) walk12(r);
      if (!any_trunk)
        for (int r : roots) walk3(r);
      o_ << "  }\n";
    }
    if (any_trunk) {
      o_ << "  __syncthreads();\n  if (wave == " << merge << ") {\n";
      mode_ = TRUNK;
      free_roots(tb);
      for (int i : tb)
        if (m_->parent[i] < 0) walk12(i);
      for (int i : tb)
        if (m_->parent[i] < 0) walk3(i);
      o_ << "  }\n  __syncthreads();\n";
      for (int w = 0; w < nw; ++w) {
        o_ << (w ? "  else if" : "  if") << " (wave == " << w << ") {\n";
        mode_ = LIMB;
        for (int i : tb) kin_vel(i);
        std::vector<int> ats;
        for (int l : pl_.bins[w]) {
          const int at = m_->parent[pl_.limbs[l][0]];
          if (at >= 0 && std::find(ats.begin(), ats.end(), at) == ats.end()) ats.push_back(at);
        }
        for (int at : ats)
          o_ << "  Real " << v("A", at) << "[6];\n  for (int k = 0; k < 6; ++k) " << v("A", at) << "[k] = at_[("
             << at_slot_[at] * 6 << " + k) * 64 + lane];\n";
        for (int l : pl_.bins[w]) walk3(pl_.limbs[l][0]);
        o_ << "  }\n";
      }
    }
    o_ << "}\n";
    mode_ = WHOLE;
    return o_.str();
  }
};
}  // namespace

int spec_tier(int64_t B) {
  int t = 0;
  while (t + 1 < kSpecTiers && B >= kSpecTierBatch[t + 1]) ++t;
  return t;
}

std::string spec_key(int dtype, int frame, const std::vector<int>& ee, int form) {
  std::string k = std::to_string(form) + ":" + std::to_string(dtype) + ":" + std::to_string(frame) + ":";
  for (int e : ee) k += std::to_string(e) + ",";
  return k;
}

std::string spec_chain_source(const bard_model* m, const std::vector<int>& ee, int frame, bool fp64, int form) {
  return Emitter(m, ee, frame, fp64, form).source();
}

std::string spec_op_source(const bard_model* m, bool fp64, int form, int ops, const std::vector<int>& ee, int frame) {
  return Emitter(m, ee, frame, fp64, form, SplitPlan::kMaxWaves, ops).source();
}

std::string spec_op_key(int ops, int dtype, int form, const std::vector<int>& ee, int frame) {
  std::string k = "op" + std::to_string(ops) + ":" + std::to_string(form) + ":" + std::to_string(dtype) + ":" +
                  std::to_string(frame) + ":";
  for (int e : ee) k += std::to_string(e) + ",";
  return k;
}

std::string spec_plan_source(const std::vector<bard_model*>& ms, const std::vector<std::vector<int>>& ee,
                             const std::vector<int64_t>& batch, bool fp64, int max_waves, int* waves,
                             int64_t* blocks) {
  std::ostringstream o;
  const int n = (int)ms.size();
  o << "// generated: fused RNEA + CRBA + Jacobian of " << n << " trees in one launch ("
    << (fp64 ? "FP64" : "FP32") << ")\n"
    << Emitter::prologue(fp64)
    << "struct PlanIO {\n  const Real* q;\n  const Real* qd;\n  const Real* qdd;\n  Real* tau;\n  Real* M;\n"
       "  Real* J;\n  Real g[4];\n};\n";
  // trees of larger nv first: their workgroups run longest, and the
  // dispatcher hands workgroups out in order
  std::vector<int> order(n);
  for (int k = 0; k < n; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ms[a]->nv > ms[b]->nv; });
  int nwb = 1, xmax = 0;
  std::vector<int64_t> first(n, 0), count(n, 0);
  int64_t at = 0;
  for (int k : order) {
    if (batch[k] <= 0) continue;
    const int form = spec_form_ok(ms[k], fp64, 2) ? 2 : 0;
    Emitter e(ms[k], ee[k], 0, fp64, form, max_waves);
    o << e.member(k, batch[k]);
    nwb = std::max(nwb, e.waves());
    xmax = std::max(xmax, e.xch_values());
    first[k] = at;
    count[k] = (batch[k] + 63) / 64 * e.wg_per_group();
    at += count[k];
  }
  o << "extern \"C\" __global__ void __launch_bounds__(" << 64 * nwb
    << ") bard_spec_plan(const PlanIO* __restrict__ io) {\n";
  if (xmax) o << "  __shared__ Real xch_[" << xmax << "];\n";
  else o << "  Real* xch_ = nullptr;\n";
  o << "  const long long blk = blockIdx.x;\n";
  for (int k : order)
    if (count[k])
      o << "  if (blk < " << first[k] + count[k] << "LL) {\n    bard_t" << k << "::run(io[" << k << "], blk - "
        << first[k] << "LL, xch_);\n    return;\n  }\n";
  o << "}\n";
  *waves = nwb;
  *blocks = at;
  return o.str();
}

std::string spec_aba_source(const bard_model* m, bool fp64, bool split) {
  return AbaEmitter(m, fp64, split).source();
}

int spec_aba_waves(const bard_model* m, bool fp64, bool split) { return AbaEmitter(m, fp64, split).waves(); }

int spec_waves(const bard_model* m, bool fp64, int form) { return make_plan(m, form == 1, fp64).waves; }

bool spec_form_ok(const bard_model* m, bool fp64, int form) {
  return (form != 2 && form != 3) || make_plan(m, false, fp64).split;
}



int spec_zero_rows(const bard_model* m, const std::vector<int>& ee) {
  // unrelated dof pairs of M plus the off-path rows of J
  const int nv = m->nv;
  std::vector<int> body_of(nv);
  for (int i = 0; i < m->n; ++i)
    for (int d = 0; d < m->nvi[i]; ++d) body_of[m->vi[i] + d] = i;
  auto anc = [&](int a, int b) {
    for (int k = a; k >= 0; k = m->parent[k])
      if (k == b) return true;
    return false;
  };
  int z = 0;
  for (int r = 0; r < nv; ++r)
    for (int c = 0; c < nv; ++c)
      if (!anc(body_of[r], body_of[c]) && !anc(body_of[c], body_of[r])) ++z;
  for (int e : ee) {
    int on = 0;
    for (int k = e; k >= 0; k = m->parent[k]) on += m->nvi[k];
    z += 6 * (nv - on);
  }
  return z;
}

int spec_compile(const std::string& src, std::vector<char>* code, std::string* log) {
  hiprtcProgram prog;
  const char* hdr[] = {kSpatialHeader};
  const char* hdr_name[] = {"spatial.h"};
  if (hiprtcCreateProgram(&prog, src.c_str(), "bard_spec_chain.hip", 1, hdr, hdr_name) != HIPRTC_SUCCESS) {
    *log = "hiprtcCreateProgram failed";
    return BARD_E_DEVICE;
  }
  // the library's own flags: multiply-adds fused within an expression only,
  // packed FP32 instructions off
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-ffp-contract=on", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops"};
  const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(prog, &ls);
  if (ls > 1) {
    log->resize(ls);
    hiprtcGetProgramLog(prog, &(*log)[0]);
  }
  if (rc != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    return BARD_E_DEVICE;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  code->resize(cs);
  hiprtcGetCode(prog, code->data());
  hiprtcDestroyProgram(&prog);
  return BARD_OK;
}

// Compiles (once per key) and loads on the current device.
namespace {

// Compiles (once per key) and, if `load`, loads on the current device the
// kernel `fname` of the source `gen` writes; `init` fills the kernel's launch
// facts at compile time.
template <class Gen, class Init>
int prepare_kernel(bard_model* m, DeviceCopy* dc, const std::string& key, Gen gen, const char* fname, Init init,
                   bool load, SpecKernel** out) {
  std::lock_guard<std::mutex> lk(m->mu);
  auto it = dc->spec.find(key);
  if (it != dc->spec.end() && (it->second.fn || !load)) {
    *out = &it->second;
    return BARD_OK;
  }
  SpecKernel sk;
  if (it != dc->spec.end()) sk = it->second;
  if (sk.code.empty()) {
    const auto t0 = std::chrono::steady_clock::now();
    std::string log;
    init(&sk);
    const int rc = spec_compile(gen(), &sk.code, &log);
    sk.compile_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc) return fail(rc, "hipRTC compile of the specialised kernel failed: " + log.substr(0, 2000));
  }
  if (load) {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    if (hipModuleLoadData(&mod, sk.code.data()) != hipSuccess) {
      (void)hipGetLastError();
      return fail(BARD_E_DEVICE, "hipModuleLoadData of the specialised kernel failed");
    }
    if (hipModuleGetFunction(&fn, mod, fname) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipModuleUnload(mod);
      return fail(BARD_E_DEVICE, "specialised kernel not found in its module");
    }
    sk.mod = mod;
    sk.fn = fn;
    int regs = 0, local = 0;
    if (hipFuncGetAttribute(&regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, fn) != hipSuccess ||
        hipFuncGetAttribute(&local, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, fn) != hipSuccess)
      (void)hipGetLastError();
    sk.vgprs = regs;
    sk.scratch = local;
    // workgroups of 64 lanes resident at once: four SIMDs per compute unit,
    // each holding as many waves as its 512 registers per lane allow
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      (void)hipGetLastError();
      cus = 0;
    }
    const int per_simd = regs > 0 ? std::max(1, std::min(8, 512 / ((regs + 7) / 8 * 8))) : 1;
    sk.slots = std::max<int64_t>(1, (int64_t)cus * 4 * per_simd / sk.waves);
  }
  dc->spec[key] = sk;
  *out = &dc->spec[key];
  return BARD_OK;
}

}  // namespace

int spec_prepare(bard_model* m, DeviceCopy* dc, int dtype, int frame, const std::vector<int>& ee, int form,
                 bool load, SpecKernel** out) {
  return prepare_kernel(
      m, dc, spec_key(dtype, frame, ee, form), [&] { return spec_chain_source(m, ee, frame, dtype == BARD_F64, form); },
      "bard_spec_chain",
      [&](SpecKernel* sk) {
        sk->form = form;
        sk->zero_rows = spec_zero_rows(m, ee);
        sk->waves = spec_waves(m, dtype == BARD_F64, form);
      },
      load, out);
}

std::string spec_aba_key(int dtype) { return "aba:" + std::to_string(dtype); }

int spec_prepare_aba(bard_model* m, DeviceCopy* dc, int dtype, bool load, SpecKernel** out) {
  return prepare_kernel(
      m, dc, spec_aba_key(dtype), [&] { return spec_aba_source(m, dtype == BARD_F64, true); }, "bard_spec_aba",
      [&](SpecKernel* sk) {
        sk->waves = spec_aba_waves(m, dtype == BARD_F64, true);
        sk->form = sk->waves > 1 ? 0 : 1;
      },
      load, out);
}

int spec_plan_build(const std::vector<bard_model*>& ms, const std::vector<std::vector<int>>& ee,
                    const std::vector<int64_t>& batch, bool fp64, int max_waves, SpecKernel* sk, int64_t* blocks) {
  const auto t0 = std::chrono::steady_clock::now();
  int waves = 1;
  const std::string src = spec_plan_source(ms, ee, batch, fp64, max_waves, &waves, blocks);
  SpecKernel out;
  out.waves = waves;
  {
    // code objects by source: plans over the same trees and batches share one
    // compilation per process
    static std::mutex mu;
    static std::map<std::string, std::vector<char>> done;
    std::lock_guard<std::mutex> lk(mu);
    auto it = done.find(src);
    if (it != done.end()) {
      out.code = it->second;
      out.compile_s = -1.0;  // reused
    } else {
      std::string log;
      const int rc = spec_compile(src, &out.code, &log);
      if (rc) return fail(rc, "hipRTC compile of the multi-tree kernel failed: " + log.substr(0, 2000));
      if (done.size() >= 16) done.clear();
      done[src] = out.code;
    }
  }
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  if (hipModuleLoadData(&mod, out.code.data()) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BARD_E_DEVICE, "hipModuleLoadData of the multi-tree kernel failed");
  }
  if (hipModuleGetFunction(&fn, mod, "bard_spec_plan") != hipSuccess) {
    (void)hipGetLastError();
    (void)hipModuleUnload(mod);
    return fail(BARD_E_DEVICE, "multi-tree kernel not found in its module");
  }
  out.mod = mod;
  out.fn = fn;
  int regs = 0, local = 0;
  if (hipFuncGetAttribute(&regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, fn) != hipSuccess ||
      hipFuncGetAttribute(&local, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, fn) != hipSuccess)
    (void)hipGetLastError();
  out.vgprs = regs;
  out.scratch = local;
  out.compile_s = out.compile_s < 0 ? 0.0 : std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *sk = std::move(out);
  return BARD_OK;
}

int spec_prepare_op(bard_model* m, DeviceCopy* dc, int dtype, int form, int ops, const std::vector<int>& ee,
                    int frame, bool load, SpecKernel** out) {
  return prepare_kernel(
      m, dc, spec_op_key(ops, dtype, form, ee, frame),
      [&] { return spec_op_source(m, dtype == BARD_F64, form, ops, ee, frame); }, "bard_spec_chain",
      [&](SpecKernel* sk) {
        sk->form = form;
        // the zero rows of the outputs written: M's, the Jacobians'
        const int zm = spec_zero_rows(m, {});
        sk->zero_rows = ((ops & 2) ? zm : 0) + ((ops & 4) ? spec_zero_rows(m, ee) - zm : 0);
        sk->waves = spec_waves(m, dtype == BARD_F64, form);
      },
      load, out);
}

SpecKernel* spec_lookup_op(bard_model* m, DeviceCopy* dc, int dtype, int ops, const std::vector<int>& ee, int frame,
                           int64_t B) {
  if (!m->spec_route.load()) return nullptr;
  const int bit = 1 << spec_tier(B);
  std::lock_guard<std::mutex> lk(m->mu);
  for (int form = 0; form < 2; ++form) {
    auto it = dc->spec.find(spec_op_key(ops, dtype, form, ee, frame));
    if (it != dc->spec.end() && it->second.fn && (it->second.route_tiers & bit)) return &it->second;
  }
  return nullptr;
}

SpecKernel* spec_lookup_aba(bard_model* m, DeviceCopy* dc, int dtype, int64_t B) {
  if (!m->spec_route.load()) return nullptr;
  std::lock_guard<std::mutex> lk(m->mu);
  auto it = dc->spec.find(spec_aba_key(dtype));
  if (it == dc->spec.end() || !it->second.fn || !(it->second.route_tiers & (1 << spec_tier(B)))) return nullptr;
  return &it->second;
}

SpecKernel* spec_lookup(bard_model* m, DeviceCopy* dc, int dtype, int frame, int n_ee, const int32_t* ee,
                        int64_t B) {
  if (!m->spec_route.load()) return nullptr;
  std::vector<int> v(ee, ee + n_ee);
  const int bit = 1 << spec_tier(B);
  std::lock_guard<std::mutex> lk(m->mu);
  for (int form = 0; form < kSpecForms; ++form) {
    auto it = dc->spec.find(spec_key(dtype, frame, v, form));
    if (it != dc->spec.end() && it->second.fn && (it->second.route_tiers & bit)) return &it->second;
  }
  return nullptr;
}

template <class Real>
int spec_launch(const SpecKernel* sk, const Args<Real>& a, const double g[3], hipStream_t st) {
  long long sq_b = a.sq_b, sq_k = a.sq_k, sqd_b = a.sqd_b, sqd_k = a.sqd_k, sqdd_b = a.sqdd_b, sqdd_k = a.sqdd_k;
  long long st_b = a.st_b, st_k = a.st_k, sM_b = a.sM_b, sM_k = a.sM_k, sJ_b = a.sJ_b, sJ_k = a.sJ_k, B = a.B;
  Real g0 = (Real)g[0], g1 = (Real)g[1], g2 = (Real)g[2];
  const Real *q = a.q, *qd = a.qd, *qdd = a.qdd;
  Real *tau = a.tau, *M = a.M, *J = a.J;
  const int64_t main = (a.B + 63) / 64 * (sk->form == 2 ? 2 : sk->form == 3 ? 3 : 1);
  // Structural zeros: when every zero row is a run of B contiguous, 16-byte
  // aligned values (instance-minor M and J) and the computing workgroups fill
  // at most a third of the device's wave slots, extra workgroups of the same
  // launch write them beside the computing waves (a few waves storing one
  // value per lane per zero entry are bound by instruction issue, not by
  // HBM); with more computing waves than that each lane writes its own,
  // coalesced across the wavefront, and the launch is bound by HBM writes.
  const int64_t V = 16 / (int64_t)sizeof(Real);
  // (an array the kernel does not write, NULL, imposes nothing)
  const bool rows = a.B % V == 0 &&
                    (!a.M || (a.sM_b == 1 && a.sM_k % V == 0 && ((uintptr_t)a.M % 16) == 0)) &&
                    (!a.J || (a.sJ_b == 1 && a.sJ_k % V == 0 && ((uintptr_t)a.J % 16) == 0));
  int64_t zb = 0;
  if (rows && sk->zero_rows > 0 && main * 3 <= sk->slots) {
    const int64_t chunks = (int64_t)sk->zero_rows * ((a.B / V + 1023) / 1024);
    zb = std::min<int64_t>(chunks, sk->slots - main);
  }
  int main_blocks = (int)main, zero_blocks = (int)zb;
  Real* P = a.poses;
  long long sp_b = a.sp_b, sp_k = a.sp_k;
  void* args[] = {&q,     &qd,    &qdd,  &tau,   &M,    &J,    &sq_b, &sq_k,        &sqd_b,       &sqd_k,
                  &sqdd_b, &sqdd_k, &st_b, &st_k,  &sM_b, &sM_k, &sJ_b, &sJ_k,        &B,           &g0,
                  &g1,    &g2,    &main_blocks, &zero_blocks, &P, &sp_b, &sp_k};
  const int64_t grid = main + zb;
  if (grid > 0x7fffffff) return fail(BARD_E_CAPACITY, "batch too large for one launch");
  if (hipModuleLaunchKernel((hipFunction_t)sk->fn, (unsigned)grid, 1, 1, 64 * sk->waves, 1, 1, 0, st, args,
                            nullptr) !=
      hipSuccess) {
    (void)hipGetLastError();
    return fail(BARD_E_DEVICE, "launch of the specialised kernel failed");
  }
  return BARD_OK;
}

template <class Real>
bool spec_aba_fits(const Args<Real>& a) {
  const int64_t last = a.B > 0 ? a.B - 1 : 0;
  const int64_t lim = (int64_t)(0xffffffffu / sizeof(Real));
  const int64_t s[4] = {a.sq_b, a.sqd_b, a.sti_b, a.sqo_b};
  for (int64_t x : s)
    if (x < 0 || last * x > lim) return false;
  return true;
}

template <class Real>
int spec_aba_launch(const SpecKernel* sk, const Args<Real>& a, const double g[3], hipStream_t st) {
  long long sq_b = a.sq_b, sq_k = a.sq_k, sqd_b = a.sqd_b, sqd_k = a.sqd_k, st_b = a.sti_b, st_k = a.sti_k;
  long long so_b = a.sqo_b, so_k = a.sqo_k, B = a.B;
  Real g0 = (Real)g[0], g1 = (Real)g[1], g2 = (Real)g[2];
  const Real *q = a.q, *qd = a.qd, *tau = a.tau_in;
  Real* qdd = a.qdd_out;
  void* args[] = {&q, &qd, &tau, &qdd, &sq_b, &sq_k, &sqd_b, &sqd_k, &st_b, &st_k, &so_b, &so_k, &B, &g0, &g1, &g2};
  const int64_t grid = (a.B + 63) / 64;
  if (grid > 0x7fffffff) return fail(BARD_E_CAPACITY, "batch too large for one launch");
  if (hipModuleLaunchKernel((hipFunction_t)sk->fn, (unsigned)grid, 1, 1, 64 * sk->waves, 1, 1, 0, st, args,
                            nullptr) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BARD_E_DEVICE, "launch of the specialised kernel failed");
  }
  return BARD_OK;
}

template bool spec_aba_fits<float>(const Args<float>&);
template bool spec_aba_fits<double>(const Args<double>&);
template int spec_aba_launch<float>(const SpecKernel*, const Args<float>&, const double*, hipStream_t);
template int spec_aba_launch<double>(const SpecKernel*, const Args<double>&, const double*, hipStream_t);

template <class Real>
bool spec_fits(const Args<Real>& a, int nv, int n_ee, int n_pose) {
  const int64_t last = a.B > 0 ? a.B - 1 : 0;
  const int64_t lim = (int64_t)(0xffffffffu / sizeof(Real));
  if (n_pose > 0 && (a.sp_b < 0 || a.sp_k < 0 || (12LL * n_pose - 1) * a.sp_k + last * a.sp_b > lim)) return false;
  const int64_t s[6] = {a.sq_b, a.sqd_b, a.sqdd_b, a.st_b, a.sM_b, a.sJ_b};
  for (int64_t x : s)
    if (x < 0 || last * x > lim) return false;
  // outputs: last row's offset plus the last lane's
  const int64_t rows[3] = {nv, (int64_t)nv * nv, 6LL * nv * n_ee};
  const int64_t sk[3] = {a.st_k, a.sM_k, a.sJ_k}, sb[3] = {a.st_b, a.sM_b, a.sJ_b};
  for (int k = 0; k < 3; ++k)
    if (sk[k] < 0 || (rows[k] - 1) * sk[k] + last * sb[k] > lim) return false;
  return true;
}

template bool spec_fits<float>(const Args<float>&, int, int, int);
template bool spec_fits<double>(const Args<double>&, int, int, int);
template int spec_launch<float>(const SpecKernel*, const Args<float>&, const double*, hipStream_t);
template int spec_launch<double>(const SpecKernel*, const Args<double>&, const double*, hipStream_t);

}  // namespace bard
