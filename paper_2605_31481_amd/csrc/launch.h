// Kernel argument block and launcher declarations shared by the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "model.h"

namespace bard {

// OP_CVJP (with OP_CRBA): the reverse-mode product of CRBA, q_bar = d<M_bar, M(q)>/dq,
// instead of the mass-matrix output.  OP_KIN: per-body blocks for the
// kinematics alone, so that a Jacobian launch on a deep tree takes the
// kinematics by pointer jumping, as every other operator does there (a
// kinematics-tier entry one operator stores is then what another computes).
enum { OP_FK = 1, OP_JAC = 2, OP_RNEA = 4, OP_CRBA = 8, OP_BIAS = 16, OP_CVJP = 32, OP_KIN = 64 };

// Rows of a per-body LDS block: R, p, v, a (24); an RNEA launch that also
// returns the bias forces RNEA(q, qd, 0) carries the acceleration without the
// qdd terms in 6 more.
__host__ __device__ constexpr int body_rows(int ops) { return (ops & OP_BIAS) ? 30 : 24; }

template <class Real>
struct Args {
  const Real* q;
  const Real* qd;
  const Real* qdd;
  const Real* tau_in;
  const Real* pi_ovr;
  Real* poses;
  Real* J;
  Real* tau;
  Real* M;
  Real* qdd_out;
  Real* bias;  // OP_BIAS: RNEA(q, qd, 0) [nv]
  int64_t sq_b, sq_k, sqd_b, sqd_k, sqdd_b, sqdd_k, sti_b, sti_k, sb_b, sb_k;
  int64_t sp_b, sp_k, sJ_b, sJ_k, st_b, st_k, sM_b, sM_k, sqo_b, sqo_k;
  int64_t B;
  int logT;
  int log2P;  // lanes per instance of this launch, log2 (>= the model's minimum)
  int frame;
  int xcd_remap;
  int stream_out;  // 1: dense outputs use non-temporal (streaming) stores
  int aba_solve;   // ABA only: 1 = qdd = M^-1 tau (no velocity, no gravity; qd not read)
  // Kinematics tier of a workspace (see kin_rows): instance-minor rows with
  // stride kin_ld.  kin_mode 0: unused; 1: store the poses, motion subspaces
  // and base origin this launch computes; 2: load them instead of computing.
  Real* kin;
  int64_t kin_ld;
  int kin_mode;
  // OP_CVJP: the cotangent M_bar [nv*nv] in, q_bar [nq] out
  const Real* Mbar;
  Real* q_bar;
  int64_t sMb_b, sMb_k, sqb_b, sqb_k;
};

// Rows of the kinematics tier per instance: 12 per body by preorder position
// (world R row-major, then p relative to the base origin), 6 per dof (s),
// then the base origin o (3).
__host__ __device__ inline int kin_rows(int n, int nv) { return 12 * n + 6 * nv + 3; }

template <class Real, int OPS>
hipError_t launch_tree(const DevModel& dm, const DevEE& ee, const Args<Real>& ar, int grid, int block, size_t lds,
                       hipStream_t st);

// Workspace result tiers (tiers.hip): dst[k][b] = src[k][b] for `rows` rows,
// and tau = M qdd + b from an M tier and a bias tier of row stride ld.
template <class Real>
hipError_t launch_tier_copy(const Real* src, int64_t s_b, int64_t s_k, Real* dst, int64_t d_b, int64_t d_k, int rows,
                            int64_t B, hipStream_t st);
template <class Real>
hipError_t launch_tier_matvec(const Real* Mt, const Real* bt, int64_t ld, const Real* qdd, int64_t sq_b, int64_t sq_k,
                              Real* tau, int64_t st_b, int64_t st_k, int nv, int64_t B, hipStream_t st);

// Device arrays of a multi-tree launch: per model its tables, end effectors
// and I/O arguments, and the work items {model, tile} of the launch starting
// at item0 (one workgroup each).
template <class Real>
struct PlanPtrs {
  const DevModel* dm;
  const DevEE* ee;
  const Args<Real>* args;
  const int2* items;
  int item0;
};
template <class Real, int OPS>
hipError_t launch_plan(const PlanPtrs<Real>& pp, int logT, int grid, int block, size_t lds, hipStream_t st);
template <class Real>
hipError_t launch_aba(const DevModel& dm, const Args<Real>& ar, int grid, int block, size_t lds, hipStream_t st);

// Standalone kinematics of one chain (path.hip): the bodies on the path from
// the root to one end effector, root first, and the Jacobian columns that
// path leaves zero.  Passed by value (kernel arguments, no device tables of
// its own).
template <class Real>
struct PathArgs {
  const Real* q;
  Real* pose;  // [12] or NULL
  Real* J;     // [6*nv] or NULL
  int64_t sq_b, sq_k, sp_b, sp_k, sJ_b, sJ_k;
  int64_t B;
  int len;           // bodies on the path
  int seg;           // lane-parallel form: path bodies per lane (16 lanes per instance)
  int nqp;           // position coordinates of the path's joints
  int n_zero;        // columns off the path
  int zero_groups;   // workgroup rows (gridDim.y - 1) that store those columns
  int8_t body[64];   // the path, root first
  uint8_t vcol[64];  // first velocity column of each path body
  uint8_t qsrc[72];  // q index of each of the path's nqp coordinates, in path order
  uint8_t zcol[128];  // the columns off the path
};
// par: the lane-parallel form (16 lanes per instance, the path's poses by a
// scan across the lanes) instead of one lane per instance.
template <class Real>
hipError_t launch_path(const DevModel& dm, const PathArgs<Real>& pa, bool lwa, bool par, hipStream_t st);

__host__ __device__ inline int lds_align(int x) { return (x + 15) & ~15; }

// Threads per workgroup the tree kernels are compiled for: 16 waves in FP32
// (4 per SIMD; the kernels fit 128 VGPRs without spills), 8 in FP64 (whose
// kernels need more registers).  The phases after the level sweep use every
// wave, and more waves per SIMD hide more of their LDS latency.
__host__ __device__ constexpr int tree_max_threads(int rs) { return rs == 4 ? 1024 : 512; }
// Threads per workgroup of the articulated-body kernel (its sweep waves only);
// FP64 keeps 4 waves, whose register budget its 6x6 free-root solve needs.
__host__ __device__ constexpr int aba_max_threads(int rs) { return rs == 4 ? 512 : 256; }
// Threads per workgroup of the adjoint kernels.
constexpr int kAdjMaxThreads = 512;

// Layout of the model's table image.  The device keeps one image per scalar
// type laid out exactly as the workgroup wants it in LDS, so staging is a
// single copy of 16-byte chunks.  mtab comes last so kernels that do not need
// it copy only the prefix.
struct TabLayout {
  int cst, meta, sbody, ssrc, cslot, linfo, srec, bm2, dlist, ulist, jump, pre, mtab, end_nomtab, end;
};

__host__ __device__ inline TabLayout tab_layout(int n, int P, int depth, int kmax, int nv, int rs) {
  TabLayout t{};
  int off = 0;
  auto take = [&](int bytes) {
    int at = off;
    off = lds_align(off + bytes);
    return at;
  };
  t.cst = take(n * CST * rs);
  t.meta = take(n * 16);
  t.sbody = take(depth * P * 2);
  t.ssrc = take(depth * P);
  t.cslot = take(depth * P * kmax);
  t.linfo = take(depth * 2 * 4);
  t.srec = take(depth * P * 16);  // per (level, slot) {body, position, q index, packed flags}
  t.bm2 = take(n * 16);    // per body {preorder position, subtree size, v index, dofs}
  t.dlist = take(n * 4);   // bodies by decreasing subtree size
  t.ulist = take(4 * 8 * n * 4);  // subtree-phase work lists for 1, 2, 4, 8 row groups per wave
  t.jump = take(6 * n);           // pointer-jumping ancestors for up to 6 steps (depth <= 64)
  t.pre = take(n);                // body at each preorder position
  t.end_nomtab = off;
  t.mtab = take(nv * nv * 4);
  t.end = off;
  return t;
}

// Byte size of an end-effector image: jrow [n_ee*6*nv] then ee_body [n_ee].
__host__ __device__ inline int ee_image_bytes(int n_ee, int nv) {
  return lds_align(n_ee * 6 * nv * 4) + lds_align(n_ee * 4);
}

// Padding (in elements) added to the stride of every per-dof and per-body
// block of rows.  A row holds one scalar of the T instances of a tile, so a
// 64-lane FP32 access touches 64 / T blocks at once; unpadded strides (6T or
// 24T words) are multiples of the 64 LDS banks for T = 8, 16, 32, and a pad
// of T words puts those blocks on disjoint banks.
__host__ __device__ constexpr int block_pad(int T, int rs) { return (rs == 4 && T < 64) ? T : 0; }

// Byte offsets of the regions a workgroup stages in LDS.  Computed by the same
// function on the host (to size the launch) and in the kernels.  Per-dof
// blocks (s, fc) hold 6 rows and get one extra all-zero block (index nv) that
// structural zeros of the dense outputs read, so the output loops need no
// branches.  Per-body blocks hold body_rows(ops) rows (R, p, v, a and, with
// OP_BIAS, the acceleration without qdd terms after the sweep; f, the world
// inertia and the bias force after the body phase) and are indexed by
// preorder position so every subtree is a contiguous range.
struct LdsPlan {
  int q, qd, qdd, tin;        // input tiles [K][T]
  int s, fc, body, o, pe;     // tree-kernel state
  int cvd, cvb;               // OP_CVJP state: per dof (cvjp_dof_rows), per body by preorder position
  int c, ia, pa, u;           // ABA state
  int tab;                    // table image
  int tab_bytes;              // bytes of the image this kernel stages
  int ee;                     // end-effector image
  int total;
};

// Rows of the CRBA adjoint's blocks: per dof y (6), z (6), w_a (6); per body,
// by preorder position, the composite inertia Ic (10), the packed symmetric
// Pc (21), e (6) and t (6).
__host__ __device__ constexpr int cvjp_dof_rows() { return 18; }
__host__ __device__ constexpr int cvjp_body_rows() { return 43; }

// kind: 0 = tree kernel with op mask `ops`, 1 = ABA kernel.
__host__ __device__ inline LdsPlan lds_plan(int kind, int ops, int n, int nq, int nv, int n_ee, int frame, int T,
                                            int rs, int P, int depth, int kmax) {
  LdsPlan L{};
  int off = 0;
  auto take = [&](int bytes) {
    int at = off;
    off = lds_align(off + bytes);
    return at;
  };
  const int pad = block_pad(T, rs);
  const bool vel = kind == 1 || (ops & OP_RNEA);
  L.q = take(nq * T * rs);
  L.qd = vel ? take(nv * T * rs) : off;
  L.qdd = (kind == 0 && (ops & OP_RNEA)) ? take(nv * T * rs) : off;
  L.tin = (kind == 1) ? take(nv * T * rs) : off;
  if (kind == 0) {
    const bool need_s = ops & (OP_JAC | OP_RNEA | OP_CRBA);
    const bool need_body = ops & (OP_FK | OP_RNEA | OP_CRBA | OP_KIN);
    L.s = need_s ? take((nv + 1) * (6 * T + pad) * rs) : off;
    L.body = need_body ? take(n * (body_rows(ops) * T + pad) * rs) : off;
    // fc: CRBA's Ic_i s blocks; RNEA kernels use them first as the scratch of
    // the velocity and acceleration scans
    L.fc = (ops & (OP_CRBA | OP_RNEA)) ? take((nv + 1) * (6 * T + pad) * rs) : off;
    L.o = take(3 * T * rs);
    L.pe = ((ops & OP_JAC) && frame == 1) ? take(n_ee * 3 * T * rs) : off;
    L.cvd = (ops & OP_CVJP) ? take(nv * (cvjp_dof_rows() * T + pad) * rs) : off;
    L.cvb = (ops & OP_CVJP) ? take(n * (cvjp_body_rows() * T + pad) * rs) : off;
  } else {
    L.s = take(nv * 6 * T * rs);
    L.c = take(n * 6 * T * rs);
    L.ia = take(n * 21 * T * rs);
    L.pa = take(n * 6 * T * rs);
    L.u = take(n * 8 * T * rs);
  }
  const TabLayout tl = tab_layout(n, P, depth, kmax, nv, rs);
  L.tab_bytes = (kind == 0 && (ops & OP_CRBA) && !(ops & OP_CVJP)) ? tl.end : tl.end_nomtab;
  L.tab = take(L.tab_bytes);
  L.ee = (kind == 0 && (ops & OP_JAC)) ? take(ee_image_bytes(n_ee, nv)) : off;
  L.total = off;
  return L;
}

// ----------------------------------------------------------------------------
// Reverse-mode kernels (adjoint.hip): FK and RNEA vector-Jacobian products.
// ----------------------------------------------------------------------------
template <class Real>
struct AdjArgs {
  const Real* q;
  const Real* qd;
  const Real* qdd;
  const Real* tau_bar;
  const Real* pi_ovr;
  const Real* poses_bar;
  Real* q_bar;
  Real* qd_bar;
  Real* qdd_bar;
  double* partial;  // [gridDim.x][n][10] per-workgroup inertial-parameter gradients, or NULL
  Real tb_scale;    // tau_bar is read as tb_scale * tau_bar (1 for the plain product)
  int64_t sq_b, sq_k, sqd_b, sqd_k, sqdd_b, sqdd_k, stb_b, stb_k, spb_b, spb_k;
  int64_t sqo_b, sqo_k, sqdo_b, sqdo_k, sqddo_b, sqddo_k;
  int64_t B, ntiles;
  int logT;
  int log2P;
};

// Rows of a per-body LDS block: RNEA adjoint 30 (R, p, v, a, phi after the
// sweep), FK adjoint 12 (R, p).
__host__ __device__ constexpr int adj_rows(bool rnea) { return rnea ? 30 : 12; }

struct AdjPlan {
  int in0, in1;  // two input tiles [K][T] (q, then for RNEA qd, qdd, tau_bar rows): one in use, one filling
  int s, body;   // per-dof and per-body blocks
  int acc;       // [n][10] FP64 inertial-parameter sums of the workgroup
  int tab, tab_bytes, total;
};

// Input rows of an adjoint tile.
__host__ __device__ inline int adj_in_rows(bool rnea, int nq, int nv) { return rnea ? nq + 3 * nv : nq; }

__host__ __device__ inline AdjPlan adj_plan(bool rnea, int n, int nq, int nv, int T, int rs, int P, int depth,
                                            int kmax) {
  AdjPlan L{};
  int off = 0;
  auto take = [&](int bytes) {
    int at = off;
    off = lds_align(off + bytes);
    return at;
  };
  const int pad = block_pad(T, rs);
  L.in0 = take(adj_in_rows(rnea, nq, nv) * T * rs);
  L.in1 = take(adj_in_rows(rnea, nq, nv) * T * rs);
  L.s = take(nv * (6 * T + pad) * rs);
  L.body = take(n * (adj_rows(rnea) * T + pad) * rs);
  L.acc = rnea ? take(n * 10 * 8) : off;
  L.tab_bytes = tab_layout(n, P, depth, kmax, nv, rs).end_nomtab;
  L.tab = take(L.tab_bytes);
  L.total = off;
  return L;
}

template <class Real, bool RNEA>
hipError_t launch_adjoint(const DevModel& dm, const AdjArgs<Real>& ar, int grid, int block, size_t lds,
                          hipStream_t st);
// Workgroups of the adjoint kernel that fit one CU at once (also grants the LDS).
template <class Real, bool RNEA>
hipError_t adjoint_resident(int logT, int free_root, int block, size_t lds, int* per_cu);
// out[i] = sum over g < groups of partial[g * count + i], in a fixed order.
template <class Real>
hipError_t launch_param_reduce(const double* partial, int groups, int count, Real* out, hipStream_t st);

// Most workgroups of an RNEA adjoint launch that returns the inertial-parameter
// gradient: each loops over tiles and keeps its own FP64 sums, so the batch
// reduction is two fixed-order stages and its buffer is bounded by the model.
constexpr int kAdjGroups = 2048;
// Values of the file-scope scratch array that holds those sums for the
// entry point that allocates nothing: enough for kAdjGroups workgroups of a
// model of BARD_MAX_BODIES bodies (10 MiB per GPU).
constexpr int64_t kNoAllocScratchDoubles = (int64_t)kAdjGroups * BARD_MAX_BODIES * 10;
// Device address of that array on the current device, looked up once per
// device (with the device current) and kept; never the array's own name.
hipError_t noalloc_scratch(double** out);

}  // namespace bard
