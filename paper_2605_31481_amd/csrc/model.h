// Internal model representation shared by the host-side compiler, the launch
// code and the kernels.  Not part of the public ABI (see include/bard.h).
#pragma once

#include <atomic>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#define BARD_MAX_BODIES 64
#define BARD_MAX_NV 128
#define BARD_MAX_DEVICES 16
#define BARD_MAX_EE 16

namespace bard {

enum JointType { J_REV = 0, J_PRI = 1, J_FREE = 2, J_FIXED = 3 };

// Per-body constant record (CST scalars, FP32 and FP64 copies).
//   [0..8]   R0 = R_pre R_post                     (eq. (2); R_post = I through the ABI)
//   [9..17]  A  = R_pre K R_post, K = [axis]x      (eq. (2))
//   [18..26] Bq = R_pre K^2 R_post                 (eq. (2))
//   [27..29] t0 = R_pre t_post + t_pre             (eq. (3); t_post = 0 so a = b = 0)
//   [30..32] axis in the body frame
//   [33..35] d = R_pre axis (prismatic translation direction in the parent frame)
//   [36..45] inertial parameters m, h(3), I_O(6) about the body origin
// Revolute:  R_pc = R0 + sin(q) A + (1 - cos q) Bq,  t_pc = t0           (eqs. (4)-(5))
// Prismatic: R_pc = R0,  t_pc = t0 + q d
// Free:      R_pc = R0 R(quat),  t_pc = R0 p + t0
constexpr int CST = 48;
constexpr int C_R0 = 0, C_A = 9, C_B = 18, C_T0 = 27, C_AX = 30, C_D = 33, C_PI = 36;

struct I4 {
  int x, y, z, w;
};

// Device view of a compiled model; a POD passed to kernels by value.  The
// tables live in two images (FP32 and FP64 constants) whose layout is
// tab_layout() in launch.h; kernels copy them into LDS.
struct DevModel {
  const unsigned char* img32;
  const unsigned char* img64;
  int n, nq, nv, depth, P, log2P, kmax, free_root;
  int ulen[4];  // entries of the subtree work lists for 1, 2, 4, 8 row groups per wave
  int n_mpair, n_mzero;  // mass-matrix output lists (pairs, then zero entries)
  int jsteps;            // pointer-jumping steps: ceil(log2(depth))
  int use_scan;          // 1: kinematics by pointer jumping instead of the level sweep
  unsigned long long xmask;  // bit l: level l pulls link state across lanes (a branching level)
  float g32[3];
  double g64[3];
};

// Per end-effector-set image: the Jacobian column list (dof | ee << 8) and
// then the zero-row list, in a region of n_ee*6*nv ints, then ee_body.
struct DevEE {
  const unsigned char* img;
  int n_ee;
  int n_col, n_zero;
};

// A model-specialised chain kernel (hipRTC): code object, module and function
// handles on one device (void* so this header stays free of HIP types), its
// resources, and whether matching chain calls go to it.
struct SpecKernel {
  std::vector<char> code;
  void* mod = nullptr;  // hipModule_t
  void* fn = nullptr;   // hipFunction_t
  int vgprs = 0, scratch = 0;
  int zero_rows = 0;  // structural-zero rows of M and J
  int waves = 1;      // waves per workgroup (64 instances)
  int64_t slots = 0;  // 64-lane workgroups the device holds at once at this register count
  double compile_s = 0.0;
  int form = 0;         // 0: split over waves by limbs, 1: one wave per instance over the whole tree
  int route_tiers = 0;  // bit k: chain calls whose batch falls in tier k (spec_tier) launch this kernel
};

struct DeviceCopy {
  bool ready = false;
  void* blob = nullptr;
  DevModel dm{};
  std::map<std::vector<int>, std::pair<void*, DevEE>> ee_sets;
  double* adj_partial = nullptr;  // per-workgroup inertial-parameter sums of the RNEA adjoint
  std::map<std::string, SpecKernel> spec;  // by (dtype, frame, end-effector set)
};

}  // namespace bard

struct bard_model {
  int n = 0, nq = 0, nv = 0, depth = 0, P = 1, log2P = 0, kmax = 0;
  bool free_root = false;
  std::vector<int> parent, jtype, qi, vi, nvi, level_of, slot_of;
  std::vector<int> dfs, sub_size, dlist;  // preorder position, subtree size, bodies by subtree size
  int jsteps = 0;
  std::vector<int8_t> jump;               // [jsteps][n]: ancestor at distance 2^step, or -1
  std::vector<int> ulist[4];              // subtree work lists (see subtree_units)
  std::vector<double> axis, xtree, inertia;
  double g[3] = {0.0, 0.0, -9.81};
  std::atomic<uint64_t> g_gen{0};  // bumped by every gravity change (keys the bias tier and plans)
  std::vector<double> cst64;
  std::vector<float> cst32;
  std::vector<int16_t> sched_body;
  std::vector<int8_t> sched_src, child_slot;
  std::vector<int> level_info, mtab;  // mtab: mass-matrix pair list, then zero list
  std::vector<bard::I4> srec;         // [depth][P] level-sweep records (see compile_model)
  unsigned long long xmask = 0;       // bit l: level l exchanges state across lanes
  int n_mpair = 0, n_mzero = 0;
  std::vector<std::vector<int>> children;
  bard::DeviceCopy dev[BARD_MAX_DEVICES];
  std::atomic<bool> spec_route{false};  // some specialised kernel takes chain calls
  std::mutex mu;
};

namespace bard {
// Host-side compile of a model (compiler.cpp).  Returns a bard_status.
int compile_model(bard_model* m, std::string* err);
// Subtree-phase work list for U row groups per wave: entries body | part << 8 |
// parts << 12 (-1 = idle).  Bodies whose subtree exceeds 2U bodies come first
// as U-entry groups, each aligned to a wave, so one wave splits the sum.
std::vector<int> subtree_units(const bard_model* m, int U);
// Output lists of the dense Jacobian for a set of end effectors: the column
// list (n_cols entries) followed by the zero-row list (n_zeros entries).
std::vector<int> jacobian_table(const bard_model* m, const std::vector<int>& ee, int* n_cols, int* n_zeros);
}  // namespace bard
