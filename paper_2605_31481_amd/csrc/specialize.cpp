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
  Emitter(const bard_model* m, const std::vector<int>& ee, int frame, bool fp64, int form)
      : m_(m), ee_(ee), frame_(frame), fp64_(fp64), dual_(form == 2), pl_(make_plan(m, form == 1, fp64)),
        split_(pl_.split || dual_) {
    trunk_ = pl_.trunk;
    slot_body_ = pl_.slot_body;
  }

  std::string source() {
    o_ << "// generated: fused RNEA + CRBA + Jacobian for one tree (" << m_->n << " bodies, nv " << m_->nv
       << ", " << ee_.size() << " end effectors, frame " << frame_ << ", " << (fp64_ ? "FP64" : "FP32")
       << ")\n#include \"spatial.h\"\n";
    o_ << "typedef " << (fp64_ ? "double" : "float") << " Real;\n";
    o_ << "template <class T>\n"
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
          "#define Qv(k) Qv_##k\n"
          "#define QDv(k) QDv_##k\n"
          "#define QDDv(k) QDDv_##k\n";
    emit_zero_tables();
    const int nw = pl_.waves;
    o_ << "static constexpr int NW = " << nw << ";  // waves per workgroup, 64 instances\n";
    o_ << "static constexpr int WG_PER_GROUP = " << (dual_ ? 2 : 1) << ";  // workgroups per 64 instances\n";
    o_ << "extern \"C\" __global__ void __launch_bounds__(" << 64 * nw << ") bard_spec_chain(\n"
          "    const Real* __restrict__ q, const Real* __restrict__ qd, const Real* __restrict__ qdd,\n"
          "    Real* __restrict__ tau, Real* __restrict__ M, Real* __restrict__ J,\n"
          "    long long sq_b, long long sq_k, long long sqd_b, long long sqd_k, long long sqdd_b, long long sqdd_k,\n"
          "    long long st_b, long long st_k, long long sM_b, long long sM_k, long long sJ_b, long long sJ_k,\n"
          "    long long B, Real g0, Real g1, Real g2, int main_blocks, int zero_blocks) {\n"
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
          "  }\n"
          ;
    if (!split_) {
      o_ << "  const long long b = (long long)blockIdx.x * 64 + threadIdx.x;\n"
            "  if (b >= B) return;\n";
      pointers();
      std::vector<int> all(m_->n);
      for (int i = 0; i < m_->n; ++i) all[i] = i;
      loads(all);
      emit_zero_stores();
      for (int i = 0; i < m_->n; ++i)
        if (m_->parent[i] < 0) visit(i);
      o_ << "}\n";
      return o_.str();
    }
    // Every lane of every wave reaches the barrier: lanes past the batch
    // repeat the last instance (the same values to the same addresses).
    o_ << "  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);\n"
          "  const int lane = (int)threadIdx.x & 63;\n";
    if (dual_)
      o_ << "  const int part = (int)blockIdx.x & 1;  // 0: torques, 1: mass matrix and Jacobians\n"
            "  long long b = ((long long)blockIdx.x >> 1) * 64 + lane;\n";
    else
      o_ << "  long long b = (long long)blockIdx.x * 64 + lane;\n";
    o_ << "  if (b > B - 1) b = B - 1;\n";
    pointers();
    if (!slot_body_.empty()) o_ << "  __shared__ Real xch_[" << slot_body_.size() * 16 * 64 << "];\n";
    if (dual_) {
      o_ << "  if (part == 0) {\n";
      do_rnea_ = true;
      do_crba_ = false;
      split_body();
      o_ << "  } else {\n";
      do_rnea_ = false;
      do_crba_ = true;
      split_body();
      o_ << "  }\n";
      do_rnea_ = do_crba_ = true;
    } else {
      split_body();
    }
    o_ << "}\n";
    return o_.str();
  }

  // The workgroup's code for the parts selected by do_rnea_ / do_crba_: the
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
    // dual form
    if (dual_ ? do_rnea_ : do_crba_) emit_zero_stores();
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
        for (int i = 0; i < m_->n; ++i)
          if (trunk_[i]) body_force(i, false);
        if (do_crba_)
          for (size_t e = 0; e < ee_.size(); ++e)
            if (trunk_[ee_[e]]) jacobian((int)e);
      }
      o_ << "  }\n";
    }
    if (any_trunk) {
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
  }

  // One limb (a chain): forward, its end effectors' Jacobians, backward with
  // the mass-matrix walks up to the root, then its sum moved to the trunk
  // parent's origin into its LDS slot.
  void limb(int l) {
    const std::vector<int>& ch = pl_.limbs[l];
    o_ << "  {\n";
    for (int i : ch) {
      forward(i);
      if (do_crba_)
        for (size_t e = 0; e < ee_.size(); ++e)
          if (ee_[e] == i) jacobian((int)e);
    }
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

 private:
  const bard_model* m_;
  std::vector<int> ee_;
  int frame_;
  bool fp64_;
  bool dual_;        // two workgroups per 64 instances: RNEA in one, CRBA and Jacobians in the other
  bool do_rnea_ = true, do_crba_ = true;  // parts of the output the code being emitted computes
  SplitPlan pl_;
  bool split_;
  std::vector<char> trunk_;
  std::vector<int> slot_body_;
  std::ostringstream o_;

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
    o_ << "  if (zero_blocks == 0) {\n"
          "    for (int i = " << first << "; i < NZM; i += NW) MA(ZM[i], Real(0));\n"
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
    zm_ = zm;
    zj_ = zj;
  }

  // ---- entering body i: pose, axis, velocity, acceleration, body force ----
  void forward(int i) {
    forward_kin(i);
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
    for (size_t e = 0; e < ee_.size(); ++e)
      if (ee_[e] == i) jacobian((int)e);
    for (int ch : m_->children[i]) visit(ch);
    backward(i);
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

int spec_waves(const bard_model* m, bool fp64, int form) { return make_plan(m, form == 1, fp64).waves; }

bool spec_form_ok(const bard_model* m, bool fp64, int form) {
  return form != 2 || make_plan(m, false, fp64).split;
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
int spec_prepare(bard_model* m, DeviceCopy* dc, int dtype, int frame, const std::vector<int>& ee, int form,
                 bool load, SpecKernel** out) {
  const std::string key = spec_key(dtype, frame, ee, form);
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
    sk.form = form;
    const int rc = spec_compile(spec_chain_source(m, ee, frame, dtype == BARD_F64, form), &sk.code, &log);
    sk.zero_rows = spec_zero_rows(m, ee);
    sk.waves = spec_waves(m, dtype == BARD_F64, form);
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
    if (hipModuleGetFunction(&fn, mod, "bard_spec_chain") != hipSuccess) {
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
  const int64_t main = (a.B + 63) / 64 * (sk->form == 2 ? 2 : 1);
  // Structural zeros: when every zero row is a run of B contiguous, 16-byte
  // aligned values (instance-minor M and J) and the computing workgroups fill
  // at most a third of the device's wave slots, extra workgroups of the same
  // launch write them beside the computing waves (a few waves storing one
  // value per lane per zero entry are bound by instruction issue, not by
  // HBM); with more computing waves than that each lane writes its own,
  // coalesced across the wavefront, and the launch is bound by HBM writes.
  const int64_t V = 16 / (int64_t)sizeof(Real);
  const bool rows = a.sM_b == 1 && a.sJ_b == 1 && a.B % V == 0 && a.sM_k % V == 0 && a.sJ_k % V == 0 &&
                    ((uintptr_t)a.M % 16) == 0 && ((uintptr_t)a.J % 16) == 0;
  int64_t zb = 0;
  if (rows && sk->zero_rows > 0 && main * 3 <= sk->slots) {
    const int64_t chunks = (int64_t)sk->zero_rows * ((a.B / V + 1023) / 1024);
    zb = std::min<int64_t>(chunks, sk->slots - main);
  }
  int main_blocks = (int)main, zero_blocks = (int)zb;
  void* args[] = {&q, &qd, &qdd, &tau, &M, &J, &sq_b, &sq_k, &sqd_b, &sqd_k, &sqdd_b, &sqdd_k,
                  &st_b, &st_k, &sM_b, &sM_k, &sJ_b, &sJ_k, &B, &g0, &g1, &g2, &main_blocks, &zero_blocks};
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
bool spec_fits(const Args<Real>& a, int nv, int n_ee) {
  const int64_t last = a.B > 0 ? a.B - 1 : 0;
  const int64_t lim = (int64_t)(0xffffffffu / sizeof(Real));
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

template bool spec_fits<float>(const Args<float>&, int, int);
template bool spec_fits<double>(const Args<double>&, int, int);
template int spec_launch<float>(const SpecKernel*, const Args<float>&, const double*, hipStream_t);
template int spec_launch<double>(const SpecKernel*, const Args<double>&, const double*, hipStream_t);

}  // namespace bard
