// C ABI of the library: argument checks, per-device model upload, launch
// configuration.  Every operator validates on the host before launching and
// never allocates per call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "launch.h"
#include "status.h"

namespace bard {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// Launch shape chosen per model: T instances per workgroup.
struct Shape {
  int waves, logT, T, log2P;
};

}  // namespace bard

// A workspace: the kinematics tier of one stream (Sec. 3.1's cached
// kinematic state).  Each component (poses, motion subspaces, base origin)
// records the q tag it was computed for; the tier is allocated on the first
// call that uses it.
struct bard_ws {
  bard_model* model;
  bard_dtype dtype;
  int64_t max_batch;
  int policy = BARD_TIER_KINEMATICS;  // tiers in use (bard_ws_set_policy)
  void* kin = nullptr;                // kinematics tier [kin_rows][max_batch]
  void* mt = nullptr;                 // mass-matrix tier [nv*nv][max_batch]
  void* bt = nullptr;                 // bias-force tier [nv][max_batch]
  int dev = -1;
  int64_t tier_B = -1;
  uint64_t pose_tag = 0, s_tag = 0, o_tag = 0;
  int64_t m_B = -1, b_B = -1;
  uint64_t m_tag = 0, bq_tag = 0, bqd_tag = 0, b_gen = 0;
  uint64_t hits[3] = {0, 0, 0}, misses[3] = {0, 0, 0};  // per tier: kinematics, mass, bias
};

using namespace bard;

namespace bard {

int check_device_state() {
  hipError_t e = hipPeekAtLastError();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(BARD_E_DEVICE, std::string("earlier device error: ") + hipGetErrorString(e));
  }
  return BARD_OK;
}

size_t lds_limit(int dev) {
  static size_t cache[BARD_MAX_DEVICES] = {0};
  if (dev < 0 || dev >= BARD_MAX_DEVICES) return 65536;
  if (!cache[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    cache[dev] = (size_t)v;
  }
  return cache[dev];
}

int default_target_T() {
  const char* e = getenv("BARD_TILE");
  if (e) {
    int t = atoi(e);
    if (t >= 1 && t <= 256) return t;
  }
  return 16;
}

// Host image of the model tables with constants of scalar size rs (layout tab_layout()).
std::vector<unsigned char> table_image(const bard_model* m, int rs) {
  const TabLayout t = tab_layout(m->n, m->P, m->depth, m->kmax, m->nv, rs);
  std::vector<unsigned char> img(t.end, 0);
  if (rs == 4) std::memcpy(&img[t.cst], m->cst32.data(), m->cst32.size() * sizeof(float));
  else std::memcpy(&img[t.cst], m->cst64.data(), m->cst64.size() * sizeof(double));
  std::vector<I4> meta(m->n);
  for (int i = 0; i < m->n; ++i) meta[i] = I4{m->parent[i], m->jtype[i], m->qi[i], m->vi[i]};
  std::memcpy(&img[t.meta], meta.data(), meta.size() * sizeof(I4));
  std::memcpy(&img[t.sbody], m->sched_body.data(), m->sched_body.size() * sizeof(int16_t));
  std::memcpy(&img[t.ssrc], m->sched_src.data(), m->sched_src.size());
  std::memcpy(&img[t.cslot], m->child_slot.data(), m->child_slot.size());
  std::memcpy(&img[t.linfo], m->level_info.data(), m->level_info.size() * sizeof(int));
  std::memcpy(&img[t.srec], m->srec.data(), m->srec.size() * sizeof(I4));
  std::vector<I4> bm2(m->n);
  for (int i = 0; i < m->n; ++i) bm2[i] = I4{m->dfs[i], m->sub_size[i], m->vi[i], m->nvi[i]};
  std::memcpy(&img[t.bm2], bm2.data(), bm2.size() * sizeof(I4));
  std::memcpy(&img[t.dlist], m->dlist.data(), m->dlist.size() * sizeof(int));
  for (int k = 0; k < 4; ++k)
    std::memcpy(&img[t.ulist + k * 8 * m->n * 4], m->ulist[k].data(), m->ulist[k].size() * sizeof(int));
  if (!m->jump.empty()) std::memcpy(&img[t.jump], m->jump.data(), m->jump.size());
  for (int i = 0; i < m->n; ++i) img[t.pre + m->dfs[i]] = (unsigned char)i;
  std::memcpy(&img[t.mtab], m->mtab.data(), m->mtab.size() * sizeof(int));
  return img;
}

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // the query's own failure is not a device fault
    // the legacy default stream may not be used while another stream captures
    return e == hipErrorStreamCaptureImplicit;
  }
  return cs != hipStreamCaptureStatusNone;
}

static int capture_refusal(const char* what) {
  return fail(BARD_E_CAPTURE, std::string(what) +
                                  " would be allocated while the stream is being captured into a HIP graph; "
                                  "run the call once before capturing (or call bard_model_upload)");
}

// Upload the compiled model to the current device (once per device).
int ensure_device(bard_model* m, DeviceCopy** out, hipStream_t st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BARD_E_DEVICE, "hipGetDevice failed (no GPU?)");
  if (dev < 0 || dev >= BARD_MAX_DEVICES) return fail(BARD_E_DEVICE, "device index out of range");
  DeviceCopy& dc = m->dev[dev];
  if (dc.ready) {
    *out = &dc;
    return BARD_OK;
  }
  if (capturing(st)) return capture_refusal("the model's device tables");
  std::lock_guard<std::mutex> lk(m->mu);
  if (dc.ready) {
    *out = &dc;
    return BARD_OK;
  }
  std::vector<unsigned char> i32 = table_image(m, 4), i64 = table_image(m, 8);
  std::vector<unsigned char> host(i32.size() + i64.size());
  std::memcpy(host.data(), i32.data(), i32.size());
  std::memcpy(host.data() + i32.size(), i64.data(), i64.size());
  void* blob = nullptr;
  if (hipMalloc(&blob, host.size()) != hipSuccess) return fail(BARD_E_NOMEM, "hipMalloc of the model tables failed");
  if (hipMemcpy(blob, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(blob);
    return fail(BARD_E_DEVICE, "upload of the model tables failed");
  }
  DevModel& dm = dc.dm;
  dm.img32 = (const unsigned char*)blob;
  dm.img64 = (const unsigned char*)blob + i32.size();
  dm.n = m->n;
  dm.nq = m->nq;
  dm.nv = m->nv;
  dm.depth = m->depth;
  dm.P = m->P;
  dm.log2P = m->log2P;
  dm.kmax = m->kmax;
  dm.free_root = m->free_root ? 1 : 0;
  for (int k = 0; k < 4; ++k) dm.ulen[k] = (int)m->ulist[k].size();
  dm.n_mpair = m->n_mpair;
  dm.n_mzero = m->n_mzero;
  dm.jsteps = m->jsteps;
  dm.xmask = m->xmask;
  // Pointer jumping takes three scans of jsteps barrier steps plus three
  // setup phases, each moving all state through LDS; the sweep keeps it in
  // registers.  Measured per chain launch at B = 4096 (FP32): depth 64 chain
  // 102 us scan vs 131 us sweep; depth 16 tree 62 vs 50; depth 9 humanoid
  // 23 vs 20; depth 7-8 chains even.
  dm.use_scan = m->depth >= 32 ? 1 : 0;
  if (const char* k = getenv("BARD_KINEMATICS")) {  // "scan" or "sweep" forces one path
    if (!strcmp(k, "scan")) dm.use_scan = 1;
    if (!strcmp(k, "sweep")) dm.use_scan = 0;
  }
  for (int k = 0; k < 3; ++k) {
    dm.g32[k] = (float)m->g[k];
    dm.g64[k] = m->g[k];
  }
  dc.blob = blob;
  dc.ready = true;
  *out = &dc;
  return BARD_OK;
}

int ensure_ee(bard_model* m, DeviceCopy* dc, int n_ee, const int32_t* ee_body, DevEE* out, hipStream_t st) {
  if (n_ee < 1 || n_ee > BARD_MAX_EE) return fail(BARD_E_ARG, "n_ee must be in 1..16");
  if (!ee_body) return fail(BARD_E_ARG, "ee_body is NULL");
  std::vector<int> key(ee_body, ee_body + n_ee);
  for (int b : key)
    if (b < 0 || b >= m->n) return fail(BARD_E_ARG, "end-effector body index out of range");
  std::lock_guard<std::mutex> lk(m->mu);
  auto it = dc->ee_sets.find(key);
  if (it != dc->ee_sets.end()) {
    *out = it->second.second;
    return BARD_OK;
  }
  if (capturing(st)) return capture_refusal("the end-effector table");
  int n_col = 0, n_zero = 0;
  std::vector<int> jt = jacobian_table(m, key, &n_col, &n_zero);
  const int bytes = ee_image_bytes(n_ee, m->nv);
  std::vector<unsigned char> host(bytes, 0);
  std::memcpy(host.data(), jt.data(), jt.size() * sizeof(int));
  std::memcpy(host.data() + lds_align(n_ee * 6 * m->nv * 4), key.data(), key.size() * sizeof(int));  // offset as in ee_image_bytes
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(BARD_E_NOMEM, "hipMalloc failed");
  if (hipMemcpy(p, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p);
    return fail(BARD_E_DEVICE, "upload of the end-effector table failed");
  }
  DevEE e;
  e.img = (const unsigned char*)p;
  e.n_ee = n_ee;
  e.n_col = n_col;
  e.n_zero = n_zero;
  dc->ee_sets[key] = {p, e};
  *out = e;
  return BARD_OK;
}

// Waves per workgroup for the phases after the level sweep (no serial
// dependency; more waves hide more LDS latency).  FP32 default 12 (measured
// on the 36-DOF humanoid: 12 waves 19.9 us, 16 waves 20.1 us, 8 waves
// 22.0 us per launch at B = 4096); BARD_OUT_WAVES overrides up to the most
// the kernels are compiled for.
int out_waves(int rs) {
  const int cap = tree_max_threads(rs) / 64;
  const char* e = getenv("BARD_OUT_WAVES");
  if (e) {
    int w = atoi(e);
    if (w >= 1 && w <= cap) return w;
  }
  return rs == 4 ? 12 : cap;
}

}  // namespace bard

namespace {

bool layout_of(const bard_layout* L, int idx, int64_t B, int64_t K, int64_t* sb, int64_t* sk) {
  if (!L) {
    *sb = 1;
    *sk = B;
    return true;
  }
  *sb = L[idx].stride_b;
  *sk = L[idx].stride_k;
  if (*sb < 1 || *sk < 1) return false;
  (void)K;
  return true;
}

// Instances per workgroup T = wavesA * (64 >> log2P).  Start from the model's
// lanes per instance and the target tile; shrink the tile (fewer sweep waves,
// then more lanes per instance) until the LDS plan fits.
template <class PlanBytes>
Shape pick_shape(const bard_model* m, int dev, PlanBytes bytes_for) {
  // T = waves * (64 >> log2P) instances per workgroup, a power of two in
  // [8, 64] (the kernels are instantiated for those tiles).  Start from the
  // model's lanes per instance and the target tile; shrink the tile (fewer
  // sweep waves, then more lanes per instance) until the LDS plan fits.
  int log2P = m->log2P;
  int target = default_target_T();
  // Narrow trees (a chain has one lane per instance) would put 64 instances
  // in one wave; more lanes per instance keep the tile at the target, so a
  // batch spreads over more workgroups (idle lanes cost nothing extra).
  while ((64 >> log2P) > target && log2P < 6) ++log2P;
  int waves = std::max(1, std::min(4, target / (64 >> log2P)));
  while (waves * (64 >> log2P) < 8) ++waves;  // wide trees: at least 8 instances
  size_t lim = lds_limit(dev);
  for (;;) {
    int T = waves * (64 >> log2P);
    if ((size_t)bytes_for(T, log2P) <= lim || T <= 8) break;
    if (waves > 1) waves >>= 1;
    else ++log2P;
  }
  int T = waves * (64 >> log2P);
  int logT = 0;
  while ((1 << logT) < T) ++logT;
  return Shape{waves, logT, T, log2P};
}

int common_checks(bard_model* m, bard_ws_t ws, int dtype, int64_t B) {
  if (!m) return fail(BARD_E_ARG, "model is NULL");
  if (dtype != BARD_F32 && dtype != BARD_F64) return fail(BARD_E_ARG, "dtype must be BARD_F32 or BARD_F64");
  if (B < 0) return fail(BARD_E_ARG, "batch must be >= 0");
  if (B > ((int64_t)1 << 40)) return fail(BARD_E_CAPACITY, "batch too large");
  if (ws) {
    if (ws->model != m) return fail(BARD_E_ARG, "workspace belongs to another model");
    if (ws->dtype != dtype) return fail(BARD_E_ARG, "workspace dtype differs from the call's dtype");
    if (B > ws->max_batch) return fail(BARD_E_CAPACITY, "batch exceeds the workspace capacity");
  }
  return BARD_OK;
}

template <class Real>
Args<Real> blank_args(int64_t B) {
  Args<Real> a;
  std::memset(&a, 0, sizeof(a));
  a.B = B;
  a.xcd_remap = 1;
  const char* e = getenv("BARD_STREAM_OUT");
  a.stream_out = e ? atoi(e) : 1;
  return a;
}

// Decide how a launch uses the workspace's kinematics tier: load it when
// every component the kernel needs was computed for q_tag on this batch,
// else store what the kernel computes.  Returns the tag bookkeeping to apply
// after a successful launch.
struct TierUse {
  int mode = 0;
  bool pose = false, s = false;
};

// Allocate one tier of `rows` instance-minor rows on the workspace's device
// (the device of its first use).
template <class Real>
int ensure_tier(bard_ws* ws, void** tier, int rows, hipStream_t st) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (ws->dev >= 0 && ws->dev != dev) return fail(BARD_E_ARG, "workspace used on another device");
  if (*tier) return BARD_OK;
  if (capturing(st)) return capture_refusal("a workspace tier");
  const size_t bytes = (size_t)rows * ws->max_batch * sizeof(Real);
  if (hipMalloc(tier, bytes) != hipSuccess) {
    *tier = nullptr;
    return fail(BARD_E_NOMEM, "hipMalloc of a workspace tier failed");
  }
  ws->dev = dev;
  return BARD_OK;
}

template <class Real, int OPS>
int plan_tier(bard_model* m, bard_ws* ws, uint64_t q_tag, int64_t B, int frame, Args<Real>* ar, TierUse* tu,
              hipStream_t st) {
  if (!ws || !(ws->policy & BARD_TIER_KINEMATICS) || q_tag == 0) return BARD_OK;
  int rc = ensure_tier<Real>(ws, &ws->kin, kin_rows(m->n, m->nv), st);
  if (rc) return rc;
  const bool need_body = OPS & (OP_FK | OP_RNEA | OP_CRBA | OP_KIN);
  const bool need_s = OPS & (OP_JAC | OP_RNEA | OP_CRBA);
  const bool need_pose = need_body || ((OPS & OP_JAC) && frame == 1);
  const bool same = ws->tier_B == B;
  const bool hit = same && ws->o_tag == q_tag && (!need_pose || ws->pose_tag == q_tag) &&
                   (!need_s || ws->s_tag == q_tag);
  ar->kin = (Real*)ws->kin;
  ar->kin_ld = ws->max_batch;
  tu->mode = hit ? 2 : 1;
  ++(hit ? ws->hits : ws->misses)[0];
  tu->pose = need_body;
  tu->s = need_s;
  ar->kin_mode = tu->mode;
  return BARD_OK;
}

void commit_tier(bard_ws* ws, uint64_t q_tag, int64_t B, const TierUse& tu) {
  if (tu.mode != 1) return;
  if (ws->tier_B != B) {
    ws->pose_tag = ws->s_tag = ws->o_tag = 0;
    ws->tier_B = B;
  }
  if (tu.pose) ws->pose_tag = q_tag;
  if (tu.s) ws->s_tag = q_tag;
  ws->o_tag = q_tag;
}

template <class Real, int OPS>
int run_tree(bard_model* m, Args<Real> ar, int n_ee, const int32_t* ee_body, int frame, hipStream_t st,
             bard_ws* ws = nullptr, uint64_t q_tag = 0) {
  DeviceCopy* dc = nullptr;
  int rc = ensure_device(m, &dc, st);
  if (rc) return rc;
  TierUse tu;
  if ((rc = plan_tier<Real, OPS>(m, ws, q_tag, ar.B, frame, &ar, &tu, st))) return rc;
  DevEE ee{nullptr, 0};
  if (OPS & OP_JAC) {
    rc = ensure_ee(m, dc, n_ee, ee_body, &ee, st);
    if (rc) return rc;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int ne = (OPS & OP_JAC) ? n_ee : 0;
  auto bytes_for = [&](int T, int) {
    return lds_plan(0, OPS, m->n, m->nq, m->nv, ne, frame, T, (int)sizeof(Real), m->P, m->depth, m->kmax).total;
  };
  Shape sh = pick_shape(m, dev, bytes_for);
  size_t lds = (size_t)bytes_for(sh.T, sh.log2P);
  if (lds > lds_limit(dev)) return fail(BARD_E_CAPACITY, "model too large for on-chip staging");
  ar.logT = sh.logT;
  ar.log2P = sh.log2P;
  ar.frame = frame;
  int waves = (sh.T << sh.log2P) >> 6;
  if (OPS & (OP_CRBA | OP_JAC | OP_RNEA | OP_FK)) waves = std::max(waves, out_waves((int)sizeof(Real)));
  if (waves * 64 > tree_max_threads((int)sizeof(Real)))
    return fail(BARD_E_CAPACITY, "tree too wide for one workgroup's level sweep");
  int64_t grid = (ar.B + sh.T - 1) / sh.T;
  if (grid > 0x7fffffff) return fail(BARD_E_CAPACITY, "batch too large for one launch");
  hipError_t e = launch_tree<Real, OPS>(dc->dm, ee, ar, (int)grid, waves * 64, lds, st);
  if (e != hipSuccess) return fail(BARD_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  if (ws) commit_tier(ws, q_tag, ar.B, tu);
  return BARD_OK;
}

template <class Real>
int run_aba(bard_model* m, Args<Real> ar, hipStream_t st) {
  DeviceCopy* dc = nullptr;
  int rc = ensure_device(m, &dc, st);
  if (rc) return rc;
  int dev = 0;
  (void)hipGetDevice(&dev);
  auto bytes_for = [&](int T, int) {
    return lds_plan(1, 0, m->n, m->nq, m->nv, 0, 0, T, (int)sizeof(Real), m->P, m->depth, m->kmax).total;
  };
  Shape sh = pick_shape(m, dev, bytes_for);
  size_t lds = (size_t)bytes_for(sh.T, sh.log2P);
  if (lds > lds_limit(dev)) return fail(BARD_E_CAPACITY, "model too large for on-chip staging");
  ar.logT = sh.logT;
  ar.log2P = sh.log2P;
  int waves = (sh.T << sh.log2P) >> 6;
  if (waves * 64 > aba_max_threads((int)sizeof(Real)))
    return fail(BARD_E_CAPACITY, "tree too wide for the articulated-body kernel in this precision");
  int64_t grid = (ar.B + sh.T - 1) / sh.T;
  if (grid > 0x7fffffff) return fail(BARD_E_CAPACITY, "batch too large for one launch");
  hipError_t e = launch_aba<Real>(dc->dm, ar, (int)grid, waves * 64, lds, st);
  if (e != hipSuccess) return fail(BARD_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return BARD_OK;
}

// The adjoint grid (at most kAdjGroups workgroups when the inertial-parameter
// gradient is returned) depends only on the batch, the tile and the device,
// so results are identical run to run on one GPU model.

int ensure_adj_partial(bard_model* m, DeviceCopy* dc, hipStream_t st) {
  std::lock_guard<std::mutex> lk(m->mu);
  if (dc->adj_partial) return BARD_OK;
  if (capturing(st)) return capture_refusal("the adjoint reduction buffer");
  void* p = nullptr;
  if (hipMalloc(&p, (size_t)kAdjGroups * m->n * 10 * sizeof(double)) != hipSuccess)
    return fail(BARD_E_NOMEM, "hipMalloc of the adjoint reduction buffer failed");
  dc->adj_partial = (double*)p;
  return BARD_OK;
}

// The model's device copy on the current device if it has been uploaded
// (by an earlier call or bard_model_upload); BARD_E_STATE otherwise.
int uploaded_copy(bard_model* m, DeviceCopy** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BARD_E_DEVICE, "hipGetDevice failed (no GPU?)");
  if (dev < 0 || dev >= BARD_MAX_DEVICES) return fail(BARD_E_DEVICE, "device index out of range");
  DeviceCopy& dc = m->dev[dev];
  if (!dc.ready)
    return fail(BARD_E_STATE, "the model's tables are not on the current device: call bard_model_upload (or any "
                              "operator) with this device current first");
  *out = &dc;
  return BARD_OK;
}

// noalloc: the model must already be on the device and the per-workgroup
// inertial-parameter sums go to the file-scope scratch array; nothing is
// allocated.
template <class Real, bool RNEA>
int run_adjoint(bard_model* m, AdjArgs<Real> ar, Real* inertia_bar, hipStream_t st, bool noalloc = false) {
  DeviceCopy* dc = nullptr;
  int rc = noalloc ? uploaded_copy(m, &dc) : ensure_device(m, &dc, st);
  if (rc) return rc;
  int dev = 0;
  (void)hipGetDevice(&dev);
  auto bytes_for = [&](int T, int) {
    return adj_plan(RNEA, m->n, m->nq, m->nv, T, (int)sizeof(Real), m->P, m->depth, m->kmax).total;
  };
  Shape sh = pick_shape(m, dev, bytes_for);
  size_t lds = (size_t)bytes_for(sh.T, sh.log2P);
  if (lds > lds_limit(dev)) return fail(BARD_E_CAPACITY, "model too large for on-chip staging");
  ar.logT = sh.logT;
  ar.log2P = sh.log2P;
  ar.ntiles = (ar.B + sh.T - 1) / sh.T;
  const int waves = std::max((sh.T << sh.log2P) >> 6, 4);
  if (waves * 64 > kAdjMaxThreads) return fail(BARD_E_CAPACITY, "tree too wide for the adjoint kernel");
  // One workgroup per resident slot, each looping over tiles (it prefetches
  // the next tile's inputs while it works on the current one).
  int per_cu = 0, cus = 0;
  hipError_t eo = adjoint_resident<Real, RNEA>(sh.logT, dc->dm.free_root, waves * 64, lds, &per_cu);
  if (eo != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(BARD_E_DEVICE, "occupancy query failed");
  int64_t grid = std::min<int64_t>(ar.ntiles, (int64_t)std::max(per_cu, 1) * std::max(cus, 1));
  if (RNEA && inertia_bar) {
    grid = std::min<int64_t>(grid, kAdjGroups);
    if (noalloc) {
      if (grid * m->n * 10 > kNoAllocScratchDoubles)
        return fail(BARD_E_CAPACITY, "inertial-parameter sums exceed the scratch array");
      double* p = nullptr;
      if (noalloc_scratch(&p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(BARD_E_DEVICE, "device address of the scratch array not available");
      }
      ar.partial = p;
    } else {
      if ((rc = ensure_adj_partial(m, dc, st))) return rc;
      ar.partial = dc->adj_partial;
    }
  }
  if (grid > 0x7fffffff) return fail(BARD_E_CAPACITY, "batch too large for one launch");
  hipError_t e = launch_adjoint<Real, RNEA>(dc->dm, ar, (int)grid, waves * 64, lds, st);
  if (e == hipSuccess && ar.partial) e = launch_param_reduce<Real>(ar.partial, (int)grid, m->n * 10, inertia_bar, st);
  if (e != hipSuccess) return fail(BARD_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return BARD_OK;
}

// Mean time of `reps` launches after 2 warm-ups, from an event pair on `st`.
template <class F>
int time_launches(F launch, hipStream_t st, int reps, double* us) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return fail(BARD_E_DEVICE, "event");
  int rc = BARD_OK;
  for (int k = 0; k < 2 && !rc; ++k) rc = launch();
  if (!rc && hipEventRecord(a, st) != hipSuccess) rc = fail(BARD_E_DEVICE, "event record");
  for (int k = 0; k < reps && !rc; ++k) rc = launch();
  if (!rc && hipEventRecord(b, st) != hipSuccess) rc = fail(BARD_E_DEVICE, "event record");
  float ms = 0.0f;
  if (!rc && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
    rc = fail(BARD_E_DEVICE, "event timing");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *us = 1e3 * ms / reps;
  return rc;
}

}  // namespace

extern "C" {

const char* bard_status_str(int s) {
  switch (s) {
    case BARD_OK: return "BARD_OK";
    case BARD_E_ARG: return "BARD_E_ARG";
    case BARD_E_TOPOLOGY: return "BARD_E_TOPOLOGY";
    case BARD_E_INERTIA: return "BARD_E_INERTIA";
    case BARD_E_NOMEM: return "BARD_E_NOMEM";
    case BARD_E_DEVICE: return "BARD_E_DEVICE";
    case BARD_E_CAPACITY: return "BARD_E_CAPACITY";
    case BARD_E_UNSUPPORTED: return "BARD_E_UNSUPPORTED";
    case BARD_E_CAPTURE: return "BARD_E_CAPTURE";
    case BARD_E_STATE: return "BARD_E_STATE";
    default: return "BARD_E_UNKNOWN";
  }
}

const char* bard_last_error(void) { return g_err.c_str(); }

const char* bard_version(void) { return "bard 0.1 gfx950"; }

int bard_model_create(int32_t n, const int32_t* parent, const int32_t* joint_type, const double* axis,
                      const double* X_tree, const double* inertia, bard_model_t* out) {
  g_err.clear();
  if (!out) return fail(BARD_E_ARG, "out is NULL");
  if (!parent || !joint_type || !axis || !X_tree || !inertia) return fail(BARD_E_ARG, "NULL model array");
  if (n < 1 || n > BARD_MAX_BODIES) return fail(BARD_E_ARG, "n_bodies must be in 1..64");
  bard_model* m = new (std::nothrow) bard_model();
  if (!m) return fail(BARD_E_NOMEM, "host allocation failed");
  m->n = n;
  m->parent.assign(parent, parent + n);
  m->jtype.assign(joint_type, joint_type + n);
  m->axis.assign(axis, axis + 3 * n);
  m->xtree.assign(X_tree, X_tree + 12 * n);
  m->inertia.assign(inertia, inertia + 10 * n);
  for (double x : m->axis)
    if (!std::isfinite(x)) { delete m; return fail(BARD_E_ARG, "non-finite axis"); }
  for (double x : m->xtree)
    if (!std::isfinite(x)) { delete m; return fail(BARD_E_ARG, "non-finite X_tree"); }
  for (double x : m->inertia)
    if (!std::isfinite(x)) { delete m; return fail(BARD_E_INERTIA, "non-finite inertia"); }
  std::string err;
  int rc = compile_model(m, &err);
  if (rc != BARD_OK) {
    delete m;
    return fail(rc, err);
  }
  *out = m;
  return BARD_OK;
}

int bard_model_set_gravity(bard_model_t m, const double* g) {
  if (!m || !g) return fail(BARD_E_ARG, "NULL argument");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(g[k])) return fail(BARD_E_ARG, "non-finite gravity");
  std::lock_guard<std::mutex> lk(m->mu);
  for (int k = 0; k < 3; ++k) m->g[k] = g[k];
  ++m->g_gen;
  for (auto& dc : m->dev)
    if (dc.ready)
      for (int k = 0; k < 3; ++k) {
        dc.dm.g32[k] = (float)g[k];
        dc.dm.g64[k] = g[k];
      }
  return BARD_OK;
}

int bard_model_info(bard_model_t m, int32_t* nq, int32_t* nv, int32_t* n_bodies, int32_t* depth) {
  if (!m) return fail(BARD_E_ARG, "model is NULL");
  if (nq) *nq = m->nq;
  if (nv) *nv = m->nv;
  if (n_bodies) *n_bodies = m->n;
  if (depth) *depth = m->depth;
  return BARD_OK;
}

int bard_model_schedule(bard_model_t m, int32_t* lanes, int32_t* levels) {
  if (!m) return fail(BARD_E_ARG, "model is NULL");
  if (lanes) *lanes = m->P;
  if (levels) *levels = m->depth;
  return BARD_OK;
}

int bard_model_joint_transform(bard_model_t m, int32_t body, const double* q, double* R, double* t) {
  if (!m || !q || !R || !t) return fail(BARD_E_ARG, "NULL argument");
  if (body < 0 || body >= m->n) return fail(BARD_E_ARG, "body out of range");
  const double* c = &m->cst64[(size_t)body * CST];
  if (m->jtype[body] == J_FREE) {
    double x = q[3], y = q[4], z = q[5], w = q[6];
    double inv = 1.0 / std::sqrt(x * x + y * y + z * z + w * w);
    x *= inv; y *= inv; z *= inv; w *= inv;
    double Rq[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                    2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                    2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)};
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j)
        R[3 * i + j] = c[C_R0 + 3 * i] * Rq[j] + c[C_R0 + 3 * i + 1] * Rq[3 + j] + c[C_R0 + 3 * i + 2] * Rq[6 + j];
      t[i] = c[C_R0 + 3 * i] * q[0] + c[C_R0 + 3 * i + 1] * q[1] + c[C_R0 + 3 * i + 2] * q[2] + c[C_T0 + i];
    }
    return BARD_OK;
  }
  double s = std::sin(q[0]), co = std::cos(q[0]);
  for (int k = 0; k < 9; ++k) R[k] = c[C_R0 + k] + s * c[C_A + k] + (1.0 - co) * c[C_B + k];
  for (int k = 0; k < 3; ++k) t[k] = c[C_T0 + k] + q[0] * c[C_D + k];
  return BARD_OK;
}

int bard_model_upload(bard_model_t m, int32_t n_ee, const int32_t* ee_body, int32_t flags) {
  if (!m) return fail(BARD_E_ARG, "model is NULL");
  if (flags & ~BARD_UPLOAD_ADJOINT) return fail(BARD_E_ARG, "flags must be 0 or BARD_UPLOAD_ADJOINT");
  if (n_ee < 0 || n_ee > BARD_MAX_EE || (n_ee > 0 && !ee_body)) return fail(BARD_E_ARG, "n_ee must be in 0..16");
  int rc = check_device_state();
  if (rc) return rc;
  DeviceCopy* dc = nullptr;
  if ((rc = ensure_device(m, &dc, nullptr))) return rc;
  if (n_ee > 0) {
    DevEE ee;
    if ((rc = ensure_ee(m, dc, n_ee, ee_body, &ee, nullptr))) return rc;
  }
  if ((flags & BARD_UPLOAD_ADJOINT) && (rc = ensure_adj_partial(m, dc, nullptr))) return rc;
  return BARD_OK;
}

int bard_model_destroy(bard_model_t m) {
  if (!m) return fail(BARD_E_ARG, "model is NULL");
  int cur = -1;
  (void)hipGetDevice(&cur);
  for (int d = 0; d < BARD_MAX_DEVICES; ++d) {
    DeviceCopy& dc = m->dev[d];
    if (!dc.ready) continue;
    (void)hipSetDevice(d);
    (void)hipFree(dc.blob);
    for (auto& kv : dc.ee_sets) (void)hipFree(kv.second.first);
    if (dc.adj_partial) (void)hipFree(dc.adj_partial);
    for (auto& kv : dc.spec)
      if (kv.second.mod) (void)hipModuleUnload((hipModule_t)kv.second.mod);
  }
  if (cur >= 0) (void)hipSetDevice(cur);
  delete m;
  return BARD_OK;
}

static int spec_args(bard_model_t m, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body, bard_frame frame,
                     std::vector<int>* ee) {
  if (!m) return fail(BARD_E_ARG, "model is NULL");
  if (dtype != BARD_F32 && dtype != BARD_F64) return fail(BARD_E_ARG, "bad dtype");
  if (frame != BARD_WORLD && frame != BARD_LOCAL_WORLD_ALIGNED) return fail(BARD_E_ARG, "bad frame");
  if (n_ee < 1 || n_ee > BARD_MAX_EE || !ee_body) return fail(BARD_E_ARG, "n_ee must be in 1..16 with ee_body");
  ee->assign(ee_body, ee_body + n_ee);
  for (int e : *ee)
    if (e < 0 || e >= m->n) return fail(BARD_E_ARG, "end-effector body out of range");
  return BARD_OK;
}

// Whether any loaded specialised kernel takes chain calls (m->mu held).
static void spec_refresh_route(bard_model* m) {
  bool any = false;
  for (const auto& d : m->dev)
    for (const auto& kv : d.spec) any = any || kv.second.route_tiers != 0;
  m->spec_route.store(any);
}

static int spec_form(int32_t flags) {
  return (flags & BARD_SPEC_WHOLE) ? 1 : (flags & BARD_SPEC_DUAL) ? 2 : (flags & BARD_SPEC_TRIPLE) ? 3 : 0;
}

// flags: only the form bits (and `extra`), at most one form
static bool spec_flags_ok(int32_t flags, int32_t extra) {
  const int32_t forms = BARD_SPEC_WHOLE | BARD_SPEC_DUAL | BARD_SPEC_TRIPLE;
  if (flags & ~(forms | extra)) return false;
  const int32_t f = flags & forms;
  return (f & (f - 1)) == 0;
}

int bard_model_specialize(bard_model_t m, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body, bard_frame frame,
                          int32_t flags) {
  std::vector<int> ee;
  int rc = spec_args(m, dtype, n_ee, ee_body, frame, &ee);
  if (rc) return rc;
  if (!spec_flags_ok(flags, BARD_SPEC_ROUTE | BARD_SPEC_COMPILE_ONLY))
    return fail(BARD_E_ARG, "unknown flags, or more than one form");
  // The generated code grows with the ancestor walks of the mass-matrix
  // columns (one step per dof and ancestor body); past this size the compile
  // time and register pressure outgrow what specialisation gains.
  int steps = 0;
  for (int i = 0; i < m->n; ++i)
    for (int k = m->parent[i]; k >= 0; k = m->parent[k]) steps += m->nvi[i];
  if (m->depth > kSpecMaxDepth || steps > kSpecMaxWalkSteps)
    return fail(BARD_E_UNSUPPORTED, "tree too deep for a specialised kernel (depth " + std::to_string(m->depth) +
                                        ", " + std::to_string(steps) + " ancestor-walk steps); the generic kernel "
                                        "serves it");
  const int form = spec_form(flags);
  if (!spec_form_ok(m, dtype == BARD_F64, form))
    return fail(BARD_E_UNSUPPORTED, "the dual and triple forms need a split plan whose limb sums fit in LDS");
  if (flags & BARD_SPEC_COMPILE_ONLY) {
    std::vector<char> code;
    std::string log;
    rc = spec_compile(spec_chain_source(m, ee, (int)frame, dtype == BARD_F64, form), &code, &log);
    return rc ? fail(rc, "hipRTC compile of the specialised kernel failed: " + log.substr(0, 2000)) : BARD_OK;
  }
  if ((rc = check_device_state())) return rc;
  DeviceCopy* dc = nullptr;
  if ((rc = ensure_device(m, &dc, nullptr))) return rc;
  SpecKernel* sk = nullptr;
  if ((rc = spec_prepare(m, dc, (int)dtype, (int)frame, ee, form, true, &sk))) return rc;
  std::lock_guard<std::mutex> lk(m->mu);
  if (flags & BARD_SPEC_ROUTE) {
    // every batch to this form; the other forms of the same arguments keep none
    for (int f = 0; f < kSpecForms; ++f) {
      auto other = dc->spec.find(spec_key((int)dtype, (int)frame, ee, f));
      if (f != form && other != dc->spec.end()) other->second.route_tiers = 0;
    }
    sk->route_tiers = (1 << kSpecTiers) - 1;
  } else {
    sk->route_tiers = 0;
  }
  spec_refresh_route(m);
  return BARD_OK;
}

int bard_model_specialized_info(bard_model_t m, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                                bard_frame frame, int32_t flags, int32_t* vgprs, int32_t* scratch_bytes,
                                double* compile_seconds, int32_t* routed_tiers, int32_t* waves) {
  std::vector<int> ee;
  int rc = spec_args(m, dtype, n_ee, ee_body, frame, &ee);
  if (rc) return rc;
  if (!spec_flags_ok(flags, 0)) return fail(BARD_E_ARG, "unknown flags, or more than one form");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= BARD_MAX_DEVICES) return fail(BARD_E_DEVICE, "no device");
  const std::string key = spec_key((int)dtype, (int)frame, ee, spec_form(flags));
  std::lock_guard<std::mutex> lk(m->mu);
  auto it = m->dev[dev].spec.find(key);
  if (it == m->dev[dev].spec.end() || !it->second.fn)
    return fail(BARD_E_STATE, "no specialised kernel for these arguments on the current device");
  if (vgprs) *vgprs = it->second.vgprs;
  if (scratch_bytes) *scratch_bytes = it->second.scratch;
  if (compile_seconds) *compile_seconds = it->second.compile_s;
  if (routed_tiers) *routed_tiers = it->second.route_tiers;
  if (waves) *waves = it->second.waves;
  return BARD_OK;
}

int bard_chain_autotune(bard_model_t m, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body, bard_frame frame,
                        void* stream, int64_t* min_batch) {
  std::vector<int> ee;
  int rc = spec_args(m, dtype, n_ee, ee_body, frame, &ee);
  if (rc) return rc;
  if ((rc = check_device_state())) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (capturing(st)) return fail(BARD_E_CAPTURE, "autotuning allocates and synchronises; not under capture");
  DeviceCopy* dc = nullptr;
  if ((rc = ensure_device(m, &dc, st))) return rc;
  // the candidates: the split form, the whole form when the tree splits
  // over several waves (else it is the same code), the dual and triple
  // forms when the tree has a plan for them
  bool use[kSpecForms] = {true, spec_waves(m, dtype == BARD_F64, 0) > 1, spec_form_ok(m, dtype == BARD_F64, 2),
                          spec_form_ok(m, dtype == BARD_F64, 3)};
  SpecKernel* sk[kSpecForms] = {};
  for (int f = 0; f < kSpecForms; ++f)
    if (use[f] && (rc = spec_prepare(m, dc, (int)dtype, (int)frame, ee, f, true, &sk[f]))) return rc;
  // Scratch arrays for the largest batch tried, inputs filled with 0.1 (the
  // kernels have no data-dependent branches at these values).
  const int64_t Bmax = kSpecTierBatch[kSpecTiers - 1];
  const size_t rs = dtype == BARD_F64 ? 8 : 4;
  const int64_t nin = (int64_t)m->nq + 2 * m->nv, nout = (int64_t)m->nv + (int64_t)m->nv * m->nv + 6LL * m->nv * n_ee;
  void* buf = nullptr;
  if (hipMalloc(&buf, (size_t)(nin + nout) * Bmax * rs) != hipSuccess)
    return fail(BARD_E_NOMEM, "hipMalloc of the autotuning arrays failed");
  {
    std::vector<unsigned char> host((size_t)nin * Bmax * rs);
    for (int64_t k = 0; k < nin * Bmax; ++k) {
      if (dtype == BARD_F64) reinterpret_cast<double*>(host.data())[k] = 0.1;
      else reinterpret_cast<float*>(host.data())[k] = 0.1f;
    }
    if (hipMemcpy(buf, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(buf);
      return fail(BARD_E_DEVICE, "upload of the autotuning inputs failed");
    }
  }
  double t[kSpecTiers][1 + kSpecForms] = {};  // generic, then each form
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    for (int k = 0; k < kSpecTiers; ++k) {
      const int64_t B = kSpecTierBatch[k];
      R* base = (R*)buf;
      Args<R> a = blank_args<R>(B);
      a.q = base;
      a.qd = base + m->nq * B;
      a.qdd = base + (int64_t)(m->nq + m->nv) * B;
      a.tau = base + nin * Bmax;
      a.M = a.tau + (int64_t)m->nv * B;
      a.J = a.M + (int64_t)m->nv * m->nv * B;
      a.sq_b = a.sqd_b = a.sqdd_b = a.st_b = a.sM_b = a.sJ_b = 1;
      a.sq_k = a.sqd_k = a.sqdd_k = a.st_k = a.sM_k = a.sJ_k = B;
      const int reps = B >= 16384 ? 5 : 20;
      int r = time_launches([&] { return run_tree<R, OP_RNEA | OP_CRBA | OP_JAC>(m, a, n_ee, ee_body, (int)frame, st); },
                            st, reps, &t[k][0]);
      for (int f = 0; f < kSpecForms && !r; ++f)
        if (use[f]) r = time_launches([&] { return spec_launch<R>(sk[f], a, m->g, st); }, st, reps, &t[k][1 + f]);
      if (r) return r;
    }
    return BARD_OK;
  };
  rc = dtype == BARD_F32 ? go(0.0f) : go(0.0);
  (void)hipDeviceSynchronize();
  (void)hipFree(buf);
  if (rc) return rc;
  // each tier to the fastest of the generic kernel and the forms
  int tiers[kSpecForms] = {};
  int64_t first = -1;
  for (int k = 0; k < kSpecTiers; ++k) {
    int best = 0;
    for (int f = 0; f < kSpecForms; ++f)
      if (use[f] && t[k][1 + f] < t[k][best]) best = 1 + f;
    if (best > 0) {
      tiers[best - 1] |= 1 << k;
      if (first < 0) first = k == 0 ? 0 : kSpecTierBatch[k];
    }
  }
  {
    std::lock_guard<std::mutex> lk(m->mu);
    for (int f = 0; f < kSpecForms; ++f) {
      if (use[f]) {
        sk[f]->route_tiers = tiers[f];
      } else {  // a form not timed takes no calls
        auto it = dc->spec.find(spec_key((int)dtype, (int)frame, ee, f));
        if (it != dc->spec.end()) it->second.route_tiers = 0;
      }
    }
    spec_refresh_route(m);
  }
  if (min_batch) *min_batch = first;
  return BARD_OK;
}

int bard_model_specialized_source(bard_model_t m, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                                  bard_frame frame, int32_t flags, char* buf, int64_t cap, int64_t* len) {
  std::vector<int> ee;
  int rc = spec_args(m, dtype, n_ee, ee_body, frame, &ee);
  if (rc) return rc;
  if (!spec_flags_ok(flags, 0)) return fail(BARD_E_ARG, "unknown flags, or more than one form");
  if (!spec_form_ok(m, dtype == BARD_F64, spec_form(flags)))
    return fail(BARD_E_UNSUPPORTED, "the dual and triple forms need a split plan whose limb sums fit in LDS");
  const std::string src = spec_chain_source(m, ee, (int)frame, dtype == BARD_F64, spec_form(flags));
  if (len) *len = (int64_t)src.size();
  if (buf && cap > 0) {
    const size_t k = std::min<size_t>((size_t)cap - 1, src.size());
    std::memcpy(buf, src.data(), k);
    buf[k] = 0;
  }
  return BARD_OK;
}

// ---- single-operator specialised kernels (inverse dynamics, mass matrix) ----

static int spec_op_args(bard_model_t m, bard_dtype dtype, int32_t flags, int32_t extra) {
  if (!m) return fail(BARD_E_ARG, "NULL model");
  if (dtype != BARD_F32 && dtype != BARD_F64) return fail(BARD_E_ARG, "bad dtype");
  if (flags & ~(BARD_SPEC_WHOLE | extra)) return fail(BARD_E_ARG, "unknown flags");
  if (m->depth > kSpecMaxDepth)
    return fail(BARD_E_UNSUPPORTED, "tree too deep for a specialised kernel (depth " + std::to_string(m->depth) +
                                        "); the generic kernel serves it");
  return BARD_OK;
}

static int spec_op_specialize(bard_model_t m, bard_dtype dtype, int32_t flags, int ops,
                              const std::vector<int>& ee = {}, int frame = 0) {
  int rc = spec_op_args(m, dtype, flags, BARD_SPEC_ROUTE | BARD_SPEC_COMPILE_ONLY);
  if (rc) return rc;
  const int form = (flags & BARD_SPEC_WHOLE) ? 1 : 0;
  if (flags & BARD_SPEC_COMPILE_ONLY) {
    std::vector<char> code;
    std::string log;
    rc = spec_compile(spec_op_source(m, dtype == BARD_F64, form, ops, ee, frame), &code, &log);
    return rc ? fail(rc, "hipRTC compile of the specialised kernel failed: " + log.substr(0, 2000)) : BARD_OK;
  }
  if ((rc = check_device_state())) return rc;
  DeviceCopy* dc = nullptr;
  if ((rc = ensure_device(m, &dc, nullptr))) return rc;
  SpecKernel* sk = nullptr;
  if ((rc = spec_prepare_op(m, dc, (int)dtype, form, ops, ee, frame, true, &sk))) return rc;
  std::lock_guard<std::mutex> lk(m->mu);
  auto other = dc->spec.find(spec_op_key(ops, (int)dtype, 1 - form, ee, frame));
  if ((flags & BARD_SPEC_ROUTE) && other != dc->spec.end()) other->second.route_tiers = 0;
  sk->route_tiers = (flags & BARD_SPEC_ROUTE) ? (1 << kSpecTiers) - 1 : 0;
  spec_refresh_route(m);
  return BARD_OK;
}

static int spec_op_info(bard_model_t m, bard_dtype dtype, int32_t flags, int ops, int32_t* vgprs,
                        int32_t* scratch_bytes, double* compile_seconds, int32_t* routed_tiers, int32_t* waves,
                        const std::vector<int>& ee = {}, int frame = 0) {
  int rc = spec_op_args(m, dtype, flags, 0);
  if (rc) return rc;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= BARD_MAX_DEVICES) return fail(BARD_E_DEVICE, "no device");
  std::lock_guard<std::mutex> lk(m->mu);
  auto it = m->dev[dev].spec.find(spec_op_key(ops, (int)dtype, (flags & BARD_SPEC_WHOLE) ? 1 : 0, ee, frame));
  if (it == m->dev[dev].spec.end() || !it->second.fn)
    return fail(BARD_E_STATE, "no specialised kernel of this operator and form on the current device");
  if (vgprs) *vgprs = it->second.vgprs;
  if (scratch_bytes) *scratch_bytes = it->second.scratch;
  if (compile_seconds) *compile_seconds = it->second.compile_s;
  if (routed_tiers) *routed_tiers = it->second.route_tiers;
  if (waves) *waves = it->second.waves;
  return BARD_OK;
}

static int spec_op_source_copy(bard_model_t m, bard_dtype dtype, int32_t flags, int ops, char* buf, int64_t cap,
                               int64_t* len, const std::vector<int>& ee = {}, int frame = 0) {
  int rc = spec_op_args(m, dtype, flags, 0);
  if (rc) return rc;
  if (!len) return fail(BARD_E_ARG, "len is NULL");
  const std::string src = spec_op_source(m, dtype == BARD_F64, (flags & BARD_SPEC_WHOLE) ? 1 : 0, ops, ee, frame);
  *len = (int64_t)src.size();
  if (buf && cap > 0) {
    const size_t n = std::min<size_t>(src.size(), (size_t)cap - 1);
    std::memcpy(buf, src.data(), n);
    buf[n] = 0;
  }
  return BARD_OK;
}

int bard_model_specialize_rnea(bard_model_t m, bard_dtype dtype, int32_t flags) {
  return spec_op_specialize(m, dtype, flags, 1);
}

int bard_model_specialized_rnea_info(bard_model_t m, bard_dtype dtype, int32_t flags, int32_t* vgprs,
                                     int32_t* scratch_bytes, double* compile_seconds, int32_t* routed_tiers,
                                     int32_t* waves) {
  return spec_op_info(m, dtype, flags, 1, vgprs, scratch_bytes, compile_seconds, routed_tiers, waves);
}

int bard_model_specialized_rnea_source(bard_model_t m, bard_dtype dtype, int32_t flags, char* buf, int64_t cap,
                                       int64_t* len) {
  return spec_op_source_copy(m, dtype, flags, 1, buf, cap, len);
}

int bard_model_specialize_crba(bard_model_t m, bard_dtype dtype, int32_t flags) {
  return spec_op_specialize(m, dtype, flags, 2);
}

int bard_model_specialized_crba_info(bard_model_t m, bard_dtype dtype, int32_t flags, int32_t* vgprs,
                                     int32_t* scratch_bytes, double* compile_seconds, int32_t* routed_tiers,
                                     int32_t* waves) {
  return spec_op_info(m, dtype, flags, 2, vgprs, scratch_bytes, compile_seconds, routed_tiers, waves);
}

int bard_model_specialized_crba_source(bard_model_t m, bard_dtype dtype, int32_t flags, char* buf, int64_t cap,
                                       int64_t* len) {
  return spec_op_source_copy(m, dtype, flags, 2, buf, cap, len);
}

int bard_model_specialize_fk(bard_model_t m, bard_dtype dtype, int32_t flags) {
  return spec_op_specialize(m, dtype, flags, 8);
}

int bard_model_specialized_fk_info(bard_model_t m, bard_dtype dtype, int32_t flags, int32_t* vgprs,
                                   int32_t* scratch_bytes, double* compile_seconds, int32_t* routed_tiers,
                                   int32_t* waves) {
  return spec_op_info(m, dtype, flags, 8, vgprs, scratch_bytes, compile_seconds, routed_tiers, waves);
}

int bard_model_specialized_fk_source(bard_model_t m, bard_dtype dtype, int32_t flags, char* buf, int64_t cap,
                                     int64_t* len) {
  return spec_op_source_copy(m, dtype, flags, 8, buf, cap, len);
}

int bard_model_specialize_jacobian(bard_model_t m, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                                   bard_frame frame, int32_t flags) {
  std::vector<int> ee;
  int rc = spec_args(m, dtype, n_ee, ee_body, frame, &ee);
  return rc ? rc : spec_op_specialize(m, dtype, flags, 4, ee, (int)frame);
}

int bard_model_specialized_jacobian_info(bard_model_t m, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                                         bard_frame frame, int32_t flags, int32_t* vgprs, int32_t* scratch_bytes,
                                         double* compile_seconds, int32_t* routed_tiers, int32_t* waves) {
  std::vector<int> ee;
  int rc = spec_args(m, dtype, n_ee, ee_body, frame, &ee);
  return rc ? rc
            : spec_op_info(m, dtype, flags, 4, vgprs, scratch_bytes, compile_seconds, routed_tiers, waves, ee,
                           (int)frame);
}

int bard_model_specialized_jacobian_source(bard_model_t m, bard_dtype dtype, int32_t n_ee, const int32_t* ee_body,
                                           bard_frame frame, int32_t flags, char* buf, int64_t cap, int64_t* len) {
  std::vector<int> ee;
  int rc = spec_args(m, dtype, n_ee, ee_body, frame, &ee);
  return rc ? rc : spec_op_source_copy(m, dtype, flags, 4, buf, cap, len, ee, (int)frame);
}

static int spec_aba_args(bard_model_t m, bard_dtype dtype) {
  if (!m) return fail(BARD_E_ARG, "NULL model");
  if (dtype != BARD_F32 && dtype != BARD_F64) return fail(BARD_E_ARG, "bad dtype");
  if (m->depth > kSpecAbaMaxDepth)
    return fail(BARD_E_UNSUPPORTED, "tree too deep for a specialised forward-dynamics kernel (depth " +
                                        std::to_string(m->depth) + "); the generic kernel serves it");
  return BARD_OK;
}

int bard_model_specialize_aba(bard_model_t m, bard_dtype dtype, int32_t flags) {
  int rc = spec_aba_args(m, dtype);
  if (rc) return rc;
  if (flags & ~(BARD_SPEC_ROUTE | BARD_SPEC_COMPILE_ONLY)) return fail(BARD_E_ARG, "unknown flags");
  if (flags & BARD_SPEC_COMPILE_ONLY) {
    std::vector<char> code;
    std::string log;
    rc = spec_compile(spec_aba_source(m, dtype == BARD_F64, true), &code, &log);
    return rc ? fail(rc, "hipRTC compile of the specialised kernel failed: " + log.substr(0, 2000)) : BARD_OK;
  }
  if ((rc = check_device_state())) return rc;
  DeviceCopy* dc = nullptr;
  if ((rc = ensure_device(m, &dc, nullptr))) return rc;
  SpecKernel* sk = nullptr;
  if ((rc = spec_prepare_aba(m, dc, (int)dtype, true, &sk))) return rc;
  std::lock_guard<std::mutex> lk(m->mu);
  sk->route_tiers = (flags & BARD_SPEC_ROUTE) ? (1 << kSpecTiers) - 1 : 0;
  spec_refresh_route(m);
  return BARD_OK;
}

int bard_model_specialized_aba_info(bard_model_t m, bard_dtype dtype, int32_t* vgprs, int32_t* scratch_bytes,
                                    double* compile_seconds, int32_t* routed_tiers) {
  if (!m) return fail(BARD_E_ARG, "NULL model");
  if (dtype != BARD_F32 && dtype != BARD_F64) return fail(BARD_E_ARG, "bad dtype");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= BARD_MAX_DEVICES) return fail(BARD_E_DEVICE, "no device");
  std::lock_guard<std::mutex> lk(m->mu);
  auto it = m->dev[dev].spec.find(spec_aba_key((int)dtype));
  if (it == m->dev[dev].spec.end() || !it->second.fn)
    return fail(BARD_E_STATE, "no specialised forward-dynamics kernel on the current device");
  if (vgprs) *vgprs = it->second.vgprs;
  if (scratch_bytes) *scratch_bytes = it->second.scratch;
  if (compile_seconds) *compile_seconds = it->second.compile_s;
  if (routed_tiers) *routed_tiers = it->second.route_tiers;
  return BARD_OK;
}

int bard_aba_autotune(bard_model_t m, bard_dtype dtype, void* stream, int64_t* min_batch) {
  int rc = spec_aba_args(m, dtype);
  if (rc) return rc;
  if ((rc = check_device_state())) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (capturing(st)) return fail(BARD_E_CAPTURE, "autotuning allocates and synchronises; not under capture");
  DeviceCopy* dc = nullptr;
  if ((rc = ensure_device(m, &dc, st))) return rc;
  SpecKernel* sk = nullptr;
  if ((rc = spec_prepare_aba(m, dc, (int)dtype, true, &sk))) return rc;
  const int64_t Bmax = kSpecTierBatch[kSpecTiers - 1];
  const size_t rs = dtype == BARD_F64 ? 8 : 4;
  const int64_t nin = (int64_t)m->nq + 2 * m->nv, nout = m->nv;
  void* buf = nullptr;
  if (hipMalloc(&buf, (size_t)(nin + nout) * Bmax * rs) != hipSuccess)
    return fail(BARD_E_NOMEM, "hipMalloc of the autotuning arrays failed");
  {
    // q = 0.1 everywhere (a unit quaternion is not needed: the kernels
    // normalise), qd = 0.1, tau = 0.1
    std::vector<unsigned char> host((size_t)nin * Bmax * rs);
    for (int64_t k = 0; k < nin * Bmax; ++k) {
      if (dtype == BARD_F64) reinterpret_cast<double*>(host.data())[k] = 0.1;
      else reinterpret_cast<float*>(host.data())[k] = 0.1f;
    }
    if (hipMemcpy(buf, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(buf);
      return fail(BARD_E_DEVICE, "upload of the autotuning inputs failed");
    }
  }
  double t[kSpecTiers][2] = {};
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    for (int k = 0; k < kSpecTiers; ++k) {
      const int64_t B = kSpecTierBatch[k];
      R* base = (R*)buf;
      Args<R> a = blank_args<R>(B);
      a.q = base;
      a.qd = base + m->nq * B;
      a.tau_in = base + (int64_t)(m->nq + m->nv) * B;
      a.qdd_out = base + nin * Bmax;
      a.sq_b = a.sqd_b = a.sti_b = a.sqo_b = 1;
      a.sq_k = a.sqd_k = a.sti_k = a.sqo_k = B;
      const int reps = B >= 16384 ? 5 : 20;
      int r = time_launches([&] { return run_aba<R>(m, a, st); }, st, reps, &t[k][0]);
      if (!r) r = time_launches([&] { return spec_aba_launch<R>(sk, a, m->g, st); }, st, reps, &t[k][1]);
      if (r) return r;
    }
    return BARD_OK;
  };
  rc = dtype == BARD_F32 ? go(0.0f) : go(0.0);
  (void)hipDeviceSynchronize();
  (void)hipFree(buf);
  if (rc) return rc;
  int tiers = 0;
  int64_t first = -1;
  for (int k = 0; k < kSpecTiers; ++k)
    if (t[k][1] < t[k][0]) {
      tiers |= 1 << k;
      if (first < 0) first = k == 0 ? 0 : kSpecTierBatch[k];
    }
  {
    std::lock_guard<std::mutex> lk(m->mu);
    sk->route_tiers = tiers;
    spec_refresh_route(m);
  }
  if (min_batch) *min_batch = first;
  return BARD_OK;
}

int bard_model_specialized_aba_source(bard_model_t m, bard_dtype dtype, char* buf, int64_t cap, int64_t* len) {
  int rc = spec_aba_args(m, dtype);
  if (rc) return rc;
  const std::string src = spec_aba_source(m, dtype == BARD_F64, true);
  if (len) *len = (int64_t)src.size();
  if (buf && cap > 0) {
    const size_t k = std::min<size_t>((size_t)cap - 1, src.size());
    std::memcpy(buf, src.data(), k);
    buf[k] = 0;
  }
  return BARD_OK;
}

int bard_ws_create(bard_model_t m, bard_dtype dtype, int64_t max_batch, bard_ws_t* out) {
  if (!m || !out) return fail(BARD_E_ARG, "NULL argument");
  if (dtype != BARD_F32 && dtype != BARD_F64) return fail(BARD_E_ARG, "bad dtype");
  if (max_batch < 1) return fail(BARD_E_ARG, "max_batch must be >= 1");
  bard_ws* w = new (std::nothrow) bard_ws();
  if (!w) return fail(BARD_E_NOMEM, "host allocation failed");
  w->model = m;
  w->dtype = dtype;
  w->max_batch = max_batch;
  *out = w;
  return BARD_OK;
}

int bard_ws_destroy(bard_ws_t w) {
  if (!w) return fail(BARD_E_ARG, "NULL workspace");
  if (w->dev >= 0) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(w->dev);
    (void)hipDeviceSynchronize();
    for (void* t : {w->kin, w->mt, w->bt})
      if (t) (void)hipFree(t);
    if (cur >= 0) (void)hipSetDevice(cur);
  }
  delete w;
  return BARD_OK;
}

int bard_ws_stats(bard_ws_t w, uint64_t* hits, uint64_t* misses) {
  if (!w) return fail(BARD_E_ARG, "NULL workspace");
  for (int k = 0; k < 3; ++k) {
    if (hits) hits[k] = w->hits[k];
    if (misses) misses[k] = w->misses[k];
  }
  return BARD_OK;
}

int bard_ws_set_policy(bard_ws_t w, int32_t policy) {
  if (!w) return fail(BARD_E_ARG, "NULL workspace");
  if (policy & ~(BARD_TIER_KINEMATICS | BARD_TIER_MASS | BARD_TIER_BIAS))
    return fail(BARD_E_ARG, "policy must be an OR of BARD_TIER_* bits");
  w->policy = policy;
  return BARD_OK;
}

#define BARD_DISPATCH_DTYPE(dtype, CALL_F, CALL_D) ((dtype) == BARD_F32 ? (CALL_F) : (CALL_D))

int bard_fk(bard_model_t m, bard_ws_t ws, bard_dtype dtype, const void* q, void* poses, const bard_layout* L,
            uint64_t q_tag, int64_t B, void* stream) {
    int rc = common_checks(m, ws, dtype, B);
  if (rc) return rc;
  if (B == 0) return BARD_OK;
  if (!q || !poses) return fail(BARD_E_ARG, "NULL array");
  if ((rc = check_device_state())) return rc;
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    Args<R> a = blank_args<R>(B);
    a.q = (const R*)q;
    a.poses = (R*)poses;
    if (!layout_of(L, 0, B, m->nq, &a.sq_b, &a.sq_k) || !layout_of(L, 1, B, 12 * m->n, &a.sp_b, &a.sp_k))
      return fail(BARD_E_ARG, "bad layout stride");
    if (!ws && m->spec_route.load()) {
      // a routed pose-only specialised kernel (calls without a workspace)
      DeviceCopy* dc = nullptr;
      int rc2 = ensure_device(m, &dc, (hipStream_t)stream);
      if (rc2) return rc2;
      SpecKernel* sk = spec_lookup_op(m, dc, (int)dtype, 8, {}, 0, B);
      if (sk && spec_fits(a, m->nv, 0, m->n)) return spec_launch<R>(sk, a, m->g, (hipStream_t)stream);
    }
    return run_tree<R, OP_FK>(m, a, 0, nullptr, 0, (hipStream_t)stream, ws, q_tag);
  };
  return dtype == BARD_F32 ? go(0.0f) : go(0.0);
}

int bard_jacobian(bard_model_t m, bard_ws_t ws, bard_dtype dtype, const void* q, int32_t n_ee,
                  const int32_t* ee_body, bard_frame frame, void* J, const bard_layout* L, uint64_t q_tag, int64_t B,
                  void* stream) {
    int rc = common_checks(m, ws, dtype, B);
  if (rc) return rc;
  if (frame != BARD_WORLD && frame != BARD_LOCAL_WORLD_ALIGNED) return fail(BARD_E_ARG, "bad frame");
  if (n_ee < 1 || n_ee > BARD_MAX_EE || !ee_body) return fail(BARD_E_ARG, "n_ee must be in 1..16 with ee_body");
  if (B == 0) return BARD_OK;
  if (!q || !J) return fail(BARD_E_ARG, "NULL array");
  if ((rc = check_device_state())) return rc;
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    Args<R> a = blank_args<R>(B);
    a.q = (const R*)q;
    a.J = (R*)J;
    if (!layout_of(L, 0, B, m->nq, &a.sq_b, &a.sq_k) || !layout_of(L, 1, B, 6 * m->nv * n_ee, &a.sJ_b, &a.sJ_k))
      return fail(BARD_E_ARG, "bad layout stride");
    DeviceCopy* dc = nullptr;
    int rc2 = ensure_device(m, &dc, (hipStream_t)stream);
    if (rc2) return rc2;
    if (!ws && m->spec_route.load()) {
      // a routed Jacobian-only specialised kernel for these end effectors and frame
      SpecKernel* sk = spec_lookup_op(m, dc, (int)dtype, 4, std::vector<int>(ee_body, ee_body + n_ee), (int)frame, B);
      if (sk && spec_fits(a, m->nv, n_ee)) return spec_launch<R>(sk, a, m->g, (hipStream_t)stream);
    }
    if (dc->dm.use_scan)
      return run_tree<R, OP_JAC | OP_KIN>(m, a, n_ee, ee_body, (int)frame, (hipStream_t)stream, ws, q_tag);
    return run_tree<R, OP_JAC>(m, a, n_ee, ee_body, (int)frame, (hipStream_t)stream, ws, q_tag);
  };
  return dtype == BARD_F32 ? go(0.0f) : go(0.0);
}

// Batch from which the path kinematics runs one lane per instance.
constexpr int64_t kPathParBatch = 65536;

int bard_path_kinematics(bard_model_t m, bard_dtype dtype, const void* q, int32_t ee_body, bard_frame frame,
                          void* pose, void* J, const bard_layout* L, int64_t B, void* stream) {
  int rc = common_checks(m, nullptr, dtype, B);
  if (rc) return rc;
  if (frame != BARD_WORLD && frame != BARD_LOCAL_WORLD_ALIGNED) return fail(BARD_E_ARG, "bad frame");
  if (ee_body < 0 || ee_body >= m->n) return fail(BARD_E_ARG, "ee_body out of range");
  if (B == 0) return BARD_OK;
  if (!q || (!pose && !J)) return fail(BARD_E_ARG, "NULL q, or neither pose nor J given");
  if ((rc = check_device_state())) return rc;
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    PathArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.B = B;
    a.q = (const R*)q;
    a.pose = (R*)pose;
    a.J = (R*)J;
    if (!layout_of(L, 0, B, m->nq, &a.sq_b, &a.sq_k) || !layout_of(L, 1, B, 12, &a.sp_b, &a.sp_k) ||
        !layout_of(L, 2, B, 6 * m->nv, &a.sJ_b, &a.sJ_k))
      return fail(BARD_E_ARG, "bad layout stride");
    std::vector<int> path;
    for (int j = ee_body; j >= 0; j = m->parent[j]) path.push_back(j);
    std::reverse(path.begin(), path.end());
    a.len = (int)path.size();
    for (int s = 0; s < a.len; ++s) {
      const int j = path[s];
      a.body[s] = (int8_t)j;
      a.vcol[s] = (uint8_t)m->vi[j];
      for (int k = 0; k < (m->jtype[j] == J_FREE ? 7 : 1); ++k) a.qsrc[a.nqp++] = (uint8_t)(m->qi[j] + k);
    }
    if (J) {
      std::vector<char> on(m->nv, 0);
      for (int j : path)
        for (int d = 0; d < m->nvi[j]; ++d) on[m->vi[j] + d] = 1;
      for (int c = 0; c < m->nv; ++c)
        if (!on[c]) a.zcol[a.n_zero++] = (uint8_t)c;
      a.zero_groups = (a.n_zero + 3) / 4;
    }
    DeviceCopy* dc = nullptr;
    int rc2 = ensure_device(m, &dc, (hipStream_t)stream);
    if (rc2) return rc2;
    // several lanes per instance below kPathParBatch instances (the walk's
    // latency sets the time there): 4 with segments of up to 4 bodies when
    // the path has at most 16, else 16; one lane per instance above (the
    // stores do).  BARD_PATH_LANES=1 or 16 pins the form (16: the
    // lane-parallel one)
    a.seg = a.len <= 16 ? (a.len + 3) / 4 : (a.len + 15) / 16;
    bool par = B < kPathParBatch;
    if (const char* env = getenv("BARD_PATH_LANES")) par = atoi(env) == 16;
    hipError_t e = launch_path<R>(dc->dm, a, frame == BARD_LOCAL_WORLD_ALIGNED, par, (hipStream_t)stream);
    if (e != hipSuccess) return fail(BARD_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return BARD_OK;
  };
  return dtype == BARD_F32 ? go(0.0f) : go(0.0);
}

int bard_rnea(bard_model_t m, bard_ws_t ws, bard_dtype dtype, const void* q, const void* qd, const void* qdd,
              const void* inertia_override, void* tau, const bard_layout* L, uint64_t q_tag, uint64_t qd_tag,
              int64_t B, void* stream) {
  int rc = common_checks(m, ws, dtype, B);
  if (rc) return rc;
  if (B == 0) return BARD_OK;
  if (!q || !qd || !qdd || !tau) return fail(BARD_E_ARG, "NULL array");
  if ((rc = check_device_state())) return rc;
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    Args<R> a = blank_args<R>(B);
    a.q = (const R*)q;
    a.qd = (const R*)qd;
    a.qdd = (const R*)qdd;
    a.pi_ovr = (const R*)inertia_override;
    a.tau = (R*)tau;
    if (!layout_of(L, 0, B, m->nq, &a.sq_b, &a.sq_k) || !layout_of(L, 1, B, m->nv, &a.sqd_b, &a.sqd_k) ||
        !layout_of(L, 2, B, m->nv, &a.sqdd_b, &a.sqdd_k) || !layout_of(L, 3, B, m->nv, &a.st_b, &a.st_k))
      return fail(BARD_E_ARG, "bad layout stride");
    const hipStream_t st = (hipStream_t)stream;
    if (!ws && !inertia_override && m->spec_route.load()) {
      // a routed inverse-dynamics-only specialised kernel (calls without a
      // workspace and with the model's own inertial parameters)
      DeviceCopy* dc = nullptr;
      int rc2 = ensure_device(m, &dc, st);
      if (rc2) return rc2;
      SpecKernel* sk = spec_lookup_op(m, dc, (int)dtype, 1, {}, 0, B);
      if (sk && spec_fits(a, m->nv, 0)) return spec_launch<R>(sk, a, m->g, st);
    }
    if (!ws || !(ws->policy & BARD_TIER_BIAS) || q_tag == 0 || qd_tag == 0 || inertia_override)
      return run_tree<R, OP_RNEA>(m, a, 0, nullptr, 0, st, ws, q_tag);
    DeviceCopy* dc = nullptr;
    int rc2 = ensure_device(m, &dc, st);
    if (rc2) return rc2;
    if ((rc2 = ensure_tier<R>(ws, &ws->bt, m->nv, st))) return rc2;
    const int64_t ld = ws->max_batch;
    const bool b_hit = ws->b_B == B && ws->bq_tag == q_tag && ws->bqd_tag == qd_tag && ws->b_gen == m->g_gen;
    const bool m_hit = ws->mt && ws->m_B == B && ws->m_tag == q_tag;
    ++((b_hit && m_hit) ? ws->hits : ws->misses)[2];
    if (b_hit && m_hit) {
      // tau = M qdd + b from the two tiers: no traversal
      if (launch_tier_matvec<R>((const R*)ws->mt, (const R*)ws->bt, ld, a.qdd, a.sqdd_b, a.sqdd_k, a.tau, a.st_b,
                                a.st_k, m->nv, B, st) != hipSuccess)
        return fail(BARD_E_DEVICE, "tier launch failed");
      return BARD_OK;
    }
    if (b_hit || dc->dm.use_scan) return run_tree<R, OP_RNEA>(m, a, 0, nullptr, 0, st, ws, q_tag);
    // one traversal for tau and b = RNEA(q, qd, 0), b into the tier
    a.bias = (R*)ws->bt;
    a.sb_b = 1;
    a.sb_k = ld;
    ws->bq_tag = 0;
    if ((rc2 = run_tree<R, OP_RNEA | OP_BIAS>(m, a, 0, nullptr, 0, st, ws, q_tag))) return rc2;
    ws->b_B = B;
    ws->bq_tag = q_tag;
    ws->bqd_tag = qd_tag;
    ws->b_gen = m->g_gen;
    return BARD_OK;
  };
  return dtype == BARD_F32 ? go(0.0f) : go(0.0);
}

int bard_crba(bard_model_t m, bard_ws_t ws, bard_dtype dtype, const void* q, void* M, const bard_layout* L,
              uint64_t q_tag, int64_t B, void* stream) {
    int rc = common_checks(m, ws, dtype, B);
  if (rc) return rc;
  if (B == 0) return BARD_OK;
  if (!q || !M) return fail(BARD_E_ARG, "NULL array");
  if ((rc = check_device_state())) return rc;
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    Args<R> a = blank_args<R>(B);
    a.q = (const R*)q;
    a.M = (R*)M;
    if (!layout_of(L, 0, B, m->nq, &a.sq_b, &a.sq_k) || !layout_of(L, 1, B, m->nv * m->nv, &a.sM_b, &a.sM_k))
      return fail(BARD_E_ARG, "bad layout stride");
    const hipStream_t st = (hipStream_t)stream;
    const int nn = m->nv * m->nv;
    if (!ws && m->spec_route.load()) {
      // a routed mass-matrix-only specialised kernel (calls without a workspace)
      DeviceCopy* dc = nullptr;
      int rc2 = ensure_device(m, &dc, st);
      if (rc2) return rc2;
      SpecKernel* sk = spec_lookup_op(m, dc, (int)dtype, 2, {}, 0, B);
      if (sk && spec_fits(a, m->nv, 0)) return spec_launch<R>(sk, a, m->g, st);
    }
    if (!ws || !(ws->policy & BARD_TIER_MASS) || q_tag == 0)
      return run_tree<R, OP_CRBA>(m, a, 0, nullptr, 0, st, ws, q_tag);
    int rc2 = ensure_tier<R>(ws, &ws->mt, nn, st);
    if (rc2) return rc2;
    R* mt = (R*)ws->mt;
    const int64_t ld = ws->max_batch;
    const bool mhit = ws->m_B == B && ws->m_tag == q_tag;
    ++(mhit ? ws->hits : ws->misses)[1];
    if (mhit) {
      // mass-matrix tier hit: no traversal, one copy into the caller's layout
      if (launch_tier_copy<R>(mt, 1, ld, a.M, a.sM_b, a.sM_k, nn, B, st) != hipSuccess)
        return fail(BARD_E_DEVICE, "tier copy launch failed");
      return BARD_OK;
    }
    if ((rc2 = run_tree<R, OP_CRBA>(m, a, 0, nullptr, 0, st, ws, q_tag))) return rc2;
    if (launch_tier_copy<R>(a.M, a.sM_b, a.sM_k, mt, 1, ld, nn, B, st) != hipSuccess) {
      ws->m_tag = 0;
      return fail(BARD_E_DEVICE, "tier copy launch failed");
    }
    ws->m_B = B;
    ws->m_tag = q_tag;
    return BARD_OK;
  };
  return dtype == BARD_F32 ? go(0.0f) : go(0.0);
}

int bard_aba(bard_model_t m, bard_ws_t ws, bard_dtype dtype, const void* q, const void* qd, const void* tau,
             void* qdd, const bard_layout* L, uint64_t q_tag, uint64_t qd_tag, int64_t B, void* stream) {
  (void)q_tag;
  (void)qd_tag;
  int rc = common_checks(m, ws, dtype, B);
  if (rc) return rc;
  if (B == 0) return BARD_OK;
  if (!q || !qd || !tau || !qdd) return fail(BARD_E_ARG, "NULL array");
  if ((rc = check_device_state())) return rc;
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    Args<R> a = blank_args<R>(B);
    a.q = (const R*)q;
    a.qd = (const R*)qd;
    a.tau_in = (const R*)tau;
    a.qdd_out = (R*)qdd;
    if (!layout_of(L, 0, B, m->nq, &a.sq_b, &a.sq_k) || !layout_of(L, 1, B, m->nv, &a.sqd_b, &a.sqd_k) ||
        !layout_of(L, 2, B, m->nv, &a.sti_b, &a.sti_k) || !layout_of(L, 3, B, m->nv, &a.sqo_b, &a.sqo_k))
      return fail(BARD_E_ARG, "bad layout stride");
    if (m->spec_route.load()) {
      DeviceCopy* dc = nullptr;
      if ((rc = ensure_device(m, &dc, (hipStream_t)stream))) return rc;
      SpecKernel* sk = spec_lookup_aba(m, dc, (int)dtype, B);
      if (sk && spec_aba_fits(a)) return spec_aba_launch<R>(sk, a, m->g, (hipStream_t)stream);
    }
    return run_aba<R>(m, a, (hipStream_t)stream);
  };
  return dtype == BARD_F32 ? go(0.0f) : go(0.0);
}

int bard_chain(bard_model_t m, bard_ws_t ws, bard_dtype dtype, const void* q, const void* qd, const void* qdd,
               int32_t n_ee, const int32_t* ee_body, bard_frame frame, void* tau, void* M, void* J,
               const bard_layout* L, int64_t B, void* stream) {
  int rc = common_checks(m, ws, dtype, B);
  if (rc) return rc;
  if (frame != BARD_WORLD && frame != BARD_LOCAL_WORLD_ALIGNED) return fail(BARD_E_ARG, "bad frame");
  if (n_ee < 1 || n_ee > BARD_MAX_EE || !ee_body) return fail(BARD_E_ARG, "n_ee must be in 1..16 with ee_body");
  if (B == 0) return BARD_OK;
  if (!q || !qd || !qdd || !tau || !M || !J) return fail(BARD_E_ARG, "NULL array");
  if ((rc = check_device_state())) return rc;
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    Args<R> a = blank_args<R>(B);
    a.q = (const R*)q;
    a.qd = (const R*)qd;
    a.qdd = (const R*)qdd;
    a.tau = (R*)tau;
    a.M = (R*)M;
    a.J = (R*)J;
    if (!layout_of(L, 0, B, m->nq, &a.sq_b, &a.sq_k) || !layout_of(L, 1, B, m->nv, &a.sqd_b, &a.sqd_k) ||
        !layout_of(L, 2, B, m->nv, &a.sqdd_b, &a.sqdd_k) || !layout_of(L, 3, B, m->nv, &a.st_b, &a.st_k) ||
        !layout_of(L, 4, B, m->nv * m->nv, &a.sM_b, &a.sM_k) ||
        !layout_of(L, 5, B, 6 * m->nv * n_ee, &a.sJ_b, &a.sJ_k))
      return fail(BARD_E_ARG, "bad layout stride");
    if (m->spec_route.load()) {
      DeviceCopy* dc = nullptr;
      if ((rc = ensure_device(m, &dc, (hipStream_t)stream))) return rc;
      SpecKernel* sk = spec_lookup(m, dc, (int)dtype, (int)frame, n_ee, ee_body, B);
      if (sk && spec_fits(a, m->nv, n_ee)) return spec_launch<R>(sk, a, m->g, (hipStream_t)stream);
    }
    return run_tree<R, OP_RNEA | OP_CRBA | OP_JAC>(m, a, n_ee, ee_body, (int)frame, (hipStream_t)stream);
  };
  return dtype == BARD_F32 ? go(0.0f) : go(0.0);
}

static int rnea_vjp_impl(bard_model_t m, bard_dtype dtype, const void* q, const void* qd, const void* qdd,
                         const void* inertia_override, const void* tau_bar, void* q_bar, void* qd_bar,
                         void* qdd_bar, void* inertia_bar, const bard_layout* L, int64_t B, void* stream,
                         bool noalloc) {
  int rc = common_checks(m, nullptr, dtype, B);
  if (rc) return rc;
  if (B == 0) return BARD_OK;
  if (!q || !qd || !qdd || !tau_bar || !q_bar || !qd_bar || !qdd_bar) return fail(BARD_E_ARG, "NULL array");
  if ((rc = check_device_state())) return rc;
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    AdjArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.B = B;
    a.q = (const R*)q;
    a.qd = (const R*)qd;
    a.qdd = (const R*)qdd;
    a.tau_bar = (const R*)tau_bar;
    a.tb_scale = R(1);
    a.pi_ovr = (const R*)inertia_override;
    a.q_bar = (R*)q_bar;
    a.qd_bar = (R*)qd_bar;
    a.qdd_bar = (R*)qdd_bar;
    if (!layout_of(L, 0, B, m->nq, &a.sq_b, &a.sq_k) || !layout_of(L, 1, B, m->nv, &a.sqd_b, &a.sqd_k) ||
        !layout_of(L, 2, B, m->nv, &a.sqdd_b, &a.sqdd_k) || !layout_of(L, 3, B, m->nv, &a.stb_b, &a.stb_k) ||
        !layout_of(L, 4, B, m->nq, &a.sqo_b, &a.sqo_k) || !layout_of(L, 5, B, m->nv, &a.sqdo_b, &a.sqdo_k) ||
        !layout_of(L, 6, B, m->nv, &a.sqddo_b, &a.sqddo_k))
      return fail(BARD_E_ARG, "bad layout stride");
    return run_adjoint<R, true>(m, a, (R*)inertia_bar, (hipStream_t)stream, noalloc);
  };
  return dtype == BARD_F32 ? go(0.0f) : go(0.0);
}

int bard_rnea_vjp(bard_model_t m, bard_dtype dtype, const void* q, const void* qd, const void* qdd,
                  const void* inertia_override, const void* tau_bar, void* q_bar, void* qd_bar, void* qdd_bar,
                  void* inertia_bar, const bard_layout* L, int64_t B, void* stream) {
  return rnea_vjp_impl(m, dtype, q, qd, qdd, inertia_override, tau_bar, q_bar, qd_bar, qdd_bar, inertia_bar, L, B,
                       stream, false);
}

int bard_rnea_vjp_noalloc(bard_model_t m, bard_dtype dtype, const void* q, const void* qd, const void* qdd,
                          const void* inertia_override, const void* tau_bar, void* q_bar, void* qd_bar,
                          void* qdd_bar, void* inertia_bar, const bard_layout* L, int64_t B, void* stream) {
  return rnea_vjp_impl(m, dtype, q, qd, qdd, inertia_override, tau_bar, q_bar, qd_bar, qdd_bar, inertia_bar, L, B,
                       stream, true);
}

int bard_fk_vjp(bard_model_t m, bard_dtype dtype, const void* q, const void* poses_bar, void* q_bar,
                const bard_layout* L, int64_t B, void* stream) {
  int rc = common_checks(m, nullptr, dtype, B);
  if (rc) return rc;
  if (B == 0) return BARD_OK;
  if (!q || !poses_bar || !q_bar) return fail(BARD_E_ARG, "NULL array");
  if ((rc = check_device_state())) return rc;
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    AdjArgs<R> a;
    std::memset(&a, 0, sizeof(a));
    a.B = B;
    a.q = (const R*)q;
    a.poses_bar = (const R*)poses_bar;
    a.q_bar = (R*)q_bar;
    if (!layout_of(L, 0, B, m->nq, &a.sq_b, &a.sq_k) || !layout_of(L, 1, B, 12 * m->n, &a.spb_b, &a.spb_k) ||
        !layout_of(L, 2, B, m->nq, &a.sqo_b, &a.sqo_k))
      return fail(BARD_E_ARG, "bad layout stride");
    return run_adjoint<R, false>(m, a, nullptr, (hipStream_t)stream);
  };
  return dtype == BARD_F32 ? go(0.0f) : go(0.0);
}

int bard_crba_vjp(bard_model_t m, bard_dtype dtype, const void* q, const void* M_bar, void* q_bar,
                  const bard_layout* L, int64_t B, void* stream) {
  int rc = common_checks(m, nullptr, dtype, B);
  if (rc) return rc;
  if (B == 0) return BARD_OK;
  if (!q || !M_bar || !q_bar) return fail(BARD_E_ARG, "NULL array");
  if ((rc = check_device_state())) return rc;
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    Args<R> a = blank_args<R>(B);
    a.q = (const R*)q;
    a.Mbar = (const R*)M_bar;
    a.q_bar = (R*)q_bar;
    if (!layout_of(L, 0, B, m->nq, &a.sq_b, &a.sq_k) || !layout_of(L, 1, B, m->nv * m->nv, &a.sMb_b, &a.sMb_k) ||
        !layout_of(L, 2, B, m->nq, &a.sqb_b, &a.sqb_k))
      return fail(BARD_E_ARG, "bad layout stride");
    return run_tree<R, OP_CRBA | OP_CVJP>(m, a, 0, nullptr, 0, (hipStream_t)stream);
  };
  return dtype == BARD_F32 ? go(0.0f) : go(0.0);
}

int bard_aba_vjp(bard_model_t m, bard_dtype dtype, const void* q, const void* qd, const void* qdd,
                 const void* qdd_bar, void* q_bar, void* qd_bar, void* tau_bar, const bard_layout* L, int64_t B,
                 void* stream) {
  int rc = common_checks(m, nullptr, dtype, B);
  if (rc) return rc;
  if (B == 0) return BARD_OK;
  if (!q || !qd || !qdd || !qdd_bar || !q_bar || !qd_bar || !tau_bar) return fail(BARD_E_ARG, "NULL array");
  if ((rc = check_device_state())) return rc;
  auto go = [&](auto zero) -> int {
    using R = decltype(zero);
    const hipStream_t st = (hipStream_t)stream;
    // 1. tau_bar = M^-1 qdd_bar: the articulated-body sweeps with no velocity
    //    and no gravity (M is symmetric, so M^-T = M^-1)
    Args<R> a = blank_args<R>(B);
    a.q = (const R*)q;
    a.qd = (const R*)qd;
    a.tau_in = (const R*)qdd_bar;
    a.qdd_out = (R*)tau_bar;
    a.aba_solve = 1;
    if (!layout_of(L, 0, B, m->nq, &a.sq_b, &a.sq_k) || !layout_of(L, 1, B, m->nv, &a.sqd_b, &a.sqd_k) ||
        !layout_of(L, 3, B, m->nv, &a.sti_b, &a.sti_k) || !layout_of(L, 6, B, m->nv, &a.sqo_b, &a.sqo_k))
      return fail(BARD_E_ARG, "bad layout stride");
    AdjArgs<R> j;
    std::memset(&j, 0, sizeof(j));
    j.B = B;
    j.q = (const R*)q;
    j.qd = (const R*)qd;
    j.qdd = (const R*)qdd;
    j.tau_bar = (const R*)tau_bar;
    j.tb_scale = R(-1);
    j.q_bar = (R*)q_bar;
    j.qd_bar = (R*)qd_bar;
    if (!layout_of(L, 0, B, m->nq, &j.sq_b, &j.sq_k) || !layout_of(L, 1, B, m->nv, &j.sqd_b, &j.sqd_k) ||
        !layout_of(L, 2, B, m->nv, &j.sqdd_b, &j.sqdd_k) || !layout_of(L, 6, B, m->nv, &j.stb_b, &j.stb_k) ||
        !layout_of(L, 4, B, m->nq, &j.sqo_b, &j.sqo_k) || !layout_of(L, 5, B, m->nv, &j.sqdo_b, &j.sqdo_k))
      return fail(BARD_E_ARG, "bad layout stride");
    int rc2 = run_aba<R>(m, a, st);
    if (rc2) return rc2;
    // 2. (q_bar, qd_bar) = -(dRNEA/d(q, qd))^T tau_bar at (q, qd, qdd): the
    //    RNEA adjoint with the cotangent read negated
    return run_adjoint<R, true>(m, j, nullptr, st);
  };
  return dtype == BARD_F32 ? go(0.0f) : go(0.0);
}

}  // extern "C"
