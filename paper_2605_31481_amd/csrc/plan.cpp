// Multi-tree plans: several models with their own batch sizes evaluated by
// one launch (or a few) over a list of work items {model, instance tile},
// captured once in a HIP graph and replayed.  An autotuner times the launch
// configurations (tile size, fusion, item order) and persists its choice.
//
// Each model's tables, end-effector lists and I/O arguments live in one
// device descriptor that the kernels read with uniform loads, so replacing
// the I/O pointers between runs is a small stream-ordered copy and the graph
// never has to be captured again.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

using namespace bard;

namespace {

constexpr int kMaxPlanModels = 64;
constexpr int kPlanMaxEE = 4;

// FUSE_SPEC: one launch of a kernel generated for the plan's trees (every
// model constant a literal, each tree's code specialised; hipRTC).
enum { FUSE_ALL = 0, FUSE_PER_MODEL = 1, FUSE_PER_OP = 2, FUSE_SPEC = 3 };
enum { ORDER_LONGEST_FIRST = 0, ORDER_MODEL = 1 };

struct PlanConfig {
  int logT = 4;
  int fusion = FUSE_ALL;
  int order = ORDER_LONGEST_FIRST;
  int lanes = 0;  // extra lanes per instance in the level sweep, log2 (0 or 1)
};

struct Group {
  int ops, item0, count, block;
  size_t lds;
};

// Tip end effectors of a model: its leaves of greatest depth, at most four,
// ties to the lowest body index.
std::vector<int> tip_ees(const bard_model* m) {
  std::vector<int> depth(m->n, 1), leaf(m->n, 1);
  for (int i = 0; i < m->n; ++i) {
    if (m->parent[i] >= 0) {
      depth[i] = depth[m->parent[i]] + 1;
      leaf[m->parent[i]] = 0;
    }
  }
  std::vector<int> leaves;
  for (int i = 0; i < m->n; ++i)
    if (leaf[i]) leaves.push_back(i);
  std::stable_sort(leaves.begin(), leaves.end(), [&](int a, int b) { return depth[a] > depth[b]; });
  if ((int)leaves.size() > kPlanMaxEE) leaves.resize(kPlanMaxEE);
  return leaves;
}

int mask_to_ops(uint32_t mask) {
  return ((mask & 1) ? OP_RNEA : 0) | ((mask & 2) ? OP_CRBA : 0) | ((mask & 4) ? OP_JAC : 0);
}

// Fused kernels exist for single operators and the full chain.
bool fusable(int ops) { return ops == OP_RNEA || ops == OP_CRBA || ops == OP_JAC || ops == (OP_RNEA | OP_CRBA | OP_JAC); }

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

}  // namespace

struct bard_plan {
  std::vector<bard_model*> models;
  std::vector<int64_t> batch;
  uint32_t op_mask = 0;
  bard_dtype dtype = BARD_F32;
  std::vector<std::vector<int>> ee;
  PlanConfig cfg;
  bool from_cache = false;
  // device state for cfg on `device`
  int device = -1;
  bool ready = false;
  int runs = 0;  // runs since the configuration was prepared (the first is eager)
  std::vector<Group> groups;
  std::vector<int> log2P;
  std::vector<uint64_t> g_gen;  // each model's gravity generation when the descriptor was uploaded
  int n_items = 0;
  unsigned char* d_buf = nullptr;
  size_t d_bytes = 0, off_ee = 0, off_args = 0, off_items = 0, args_bytes = 0;
  unsigned char* h_stage = nullptr;
  std::vector<unsigned char> h_last;
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // FUSE_SPEC: the generated kernel (loaded on `device`) and its launch size
  SpecKernel spk;
  int64_t spk_blocks = 0;
  int spk_max_waves = 0;  // the wave cap spk was generated for
};

namespace {

void drop_graph(bard_plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

std::string cache_path() {
  const char* e = getenv("BARD_TUNE_CACHE");
  if (e && *e) return e;
  const char* home = getenv("HOME");
  if (!home || !*home) return "";
  std::string dir = std::string(home) + "/.cache";
  ::mkdir(dir.c_str(), 0755);
  return dir + "/bard_plan_tune.json";
}

std::string plan_key(const bard_plan* p) {
  uint64_t h = 1469598103934665603ull;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) h = fnv1a(h, prop.gcnArchName, strlen(prop.gcnArchName));
  const int head[3] = {(int)p->dtype, (int)p->op_mask, (int)p->models.size()};
  h = fnv1a(h, head, sizeof(head));
  for (size_t i = 0; i < p->models.size(); ++i) {
    const bard_model* m = p->models[i];
    h = fnv1a(h, m->parent.data(), m->parent.size() * sizeof(int));
    h = fnv1a(h, m->jtype.data(), m->jtype.size() * sizeof(int));
    h = fnv1a(h, &p->batch[i], sizeof(int64_t));
  }
  char buf[17];
  snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  return buf;
}

// The cache is a JSON object with one entry per line:
//   "<key>": {"tile": 16, "fusion": 0, "order": 0, "lanes": 0, "us": 123.4}
std::map<std::string, std::pair<PlanConfig, double>> read_cache(const std::string& path) {
  std::map<std::string, std::pair<PlanConfig, double>> out;
  FILE* f = path.empty() ? nullptr : fopen(path.c_str(), "r");
  if (!f) return out;
  char line[512];
  while (fgets(line, sizeof(line), f)) {
    char key[65];
    int tile = 0, fusion = 0, order = 0, lanes = 0;
    double us = 0;
    if (sscanf(line, " \"%64[^\"]\": {\"tile\": %d, \"fusion\": %d, \"order\": %d, \"lanes\": %d, \"us\": %lf}", key,
               &tile, &fusion, &order, &lanes, &us) == 6) {
      PlanConfig c;
      int lt = 0;
      while ((1 << lt) < tile) ++lt;
      c.logT = lt;
      c.fusion = fusion;
      c.order = order;
      c.lanes = lanes;
      out[key] = {c, us};
    }
  }
  fclose(f);
  return out;
}

void write_cache(const std::string& path, const std::map<std::string, std::pair<PlanConfig, double>>& entries) {
  if (path.empty()) return;
  std::string tmp = path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& kv : entries) {
    fprintf(f, "\"%s\": {\"tile\": %d, \"fusion\": %d, \"order\": %d, \"lanes\": %d, \"us\": %.3f}%s\n",
            kv.first.c_str(), 1 << kv.second.first.logT, kv.second.first.fusion, kv.second.first.order,
            kv.second.first.lanes, kv.second.second, ++k < entries.size() ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
  (void)rename(tmp.c_str(), path.c_str());
}

bool valid_config(const bard_plan* p, const PlanConfig& c) {
  if (c.logT < 3 || c.logT > 5) return false;
  if (c.fusion < FUSE_ALL || c.fusion > FUSE_SPEC) return false;
  if (c.fusion == FUSE_SPEC && mask_to_ops(p->op_mask) != (OP_RNEA | OP_CRBA | OP_JAC)) return false;
  if (c.order != ORDER_LONGEST_FIRST && c.order != ORDER_MODEL) return false;
  if (c.lanes < 0 || c.lanes > 1) return false;
  if (c.fusion != FUSE_PER_OP && !fusable(mask_to_ops(p->op_mask))) return false;
  return true;
}

// Host-side buffers every configuration uses: the pinned staging copy of
// the arguments, its event and the capture stream.
int plan_host_state(bard_plan* p) {
  if (!p->h_stage) {
    const size_t hb = kMaxPlanModels * sizeof(Args<double>);
    if (hipHostMalloc((void**)&p->h_stage, hb, hipHostMallocDefault) != hipSuccess)
      return fail(BARD_E_NOMEM, "hipHostMalloc of the plan staging buffer failed");
  }
  if (!p->staged && hipEventCreateWithFlags(&p->staged, hipEventDisableTiming) != hipSuccess)
    return fail(BARD_E_DEVICE, "hipEventCreate failed");
  if (!p->cap && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
    return fail(BARD_E_DEVICE, "hipStreamCreate failed");
  return BARD_OK;
}

// FUSE_SPEC: waves per tree at most 8, or 4 with cfg.lanes = 1 (two
// workgroups of a wide tree then fit a CU where one of 8 waves did).
int spec_plan_waves(const PlanConfig& c) { return c.lanes ? 4 : 8; }

// FUSE_SPEC: generate and compile the plan's kernel once per plan and wave
// cap (on its device); its descriptor holds one SpecPlanIO per model.
template <class Real>
int prepare_spec(bard_plan* p) {
  const int mw = spec_plan_waves(p->cfg);
  if (p->spk.fn && p->spk_max_waves != mw) {
    if (hipDeviceSynchronize() != hipSuccess) return fail(BARD_E_DEVICE, "device error before a kernel change");
    (void)hipModuleUnload((hipModule_t)p->spk.mod);
    p->spk = SpecKernel();
  }
  if (!p->spk.fn) {
    std::vector<bard_model*> ms(p->models.begin(), p->models.end());
    int rc = spec_plan_build(ms, p->ee, p->batch, sizeof(Real) == 8, mw, &p->spk, &p->spk_blocks);
    if (rc) return rc;
    p->spk_max_waves = mw;
  }
  const int nm = (int)p->models.size();
  p->args_bytes = nm * sizeof(SpecPlanIO<Real>);
  p->off_args = 0;
  p->n_items = 0;
  p->groups.clear();
  if (p->spk_blocks > 0) p->groups.push_back(Group{-1, 0, 0, 64 * p->spk.waves, 0});
  if (p->spk_blocks > 0x7fffffff) return fail(BARD_E_CAPACITY, "too many workgroups for one launch");
  if (p->args_bytes > p->d_bytes) {
    if (hipDeviceSynchronize() != hipSuccess) return fail(BARD_E_DEVICE, "device error before plan upload");
    if (p->d_buf) (void)hipFree(p->d_buf);
    p->d_buf = nullptr;
    p->d_bytes = 0;
    if (hipMalloc((void**)&p->d_buf, p->args_bytes) != hipSuccess)
      return fail(BARD_E_NOMEM, "hipMalloc of the plan failed");
    p->d_bytes = p->args_bytes;
  }
  int rc = plan_host_state(p);
  if (rc) return rc;
  p->g_gen.assign(nm, 0);
  for (int i = 0; i < nm; ++i) p->g_gen[i] = p->models[i]->g_gen;
  p->h_last.clear();
  p->runs = 0;
  p->ready = true;
  return BARD_OK;
}

template <class Real>
int prepare_t(bard_plan* p) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BARD_E_DEVICE, "hipGetDevice failed (no GPU?)");
  if (p->device >= 0 && p->device != dev) return fail(BARD_E_ARG, "a plan runs on the device of its first use");
  p->device = dev;
  if (p->ready) return BARD_OK;
  drop_graph(p);
  if (p->cfg.fusion == FUSE_SPEC) return prepare_spec<Real>(p);
  const int nm = (int)p->models.size();
  const int T = 1 << p->cfg.logT;
  const int all_ops = mask_to_ops(p->op_mask);
  const int rs = (int)sizeof(Real);
  std::vector<DevModel> dms(nm);
  std::vector<DevEE> ees(nm);
  p->log2P.assign(nm, 0);
  p->g_gen.assign(nm, 0);
  std::vector<double> cost(nm);
  for (int i = 0; i < nm; ++i) {
    bard_model* m = p->models[i];
    DeviceCopy* dc = nullptr;
    int rc = ensure_device(m, &dc, nullptr);
    if (rc) return rc;
    {
      // the device copy carries the model's current gravity; remember which
      std::lock_guard<std::mutex> lk(m->mu);
      dms[i] = dc->dm;
      p->g_gen[i] = m->g_gen;
    }
    ees[i] = DevEE{nullptr, 0, 0, 0};
    if (all_ops & OP_JAC) {
      rc = ensure_ee(m, dc, (int)p->ee[i].size(), p->ee[i].data(), &ees[i], nullptr);
      if (rc) return rc;
    }
    int lp = std::max(m->log2P, 6 - p->cfg.logT) + p->cfg.lanes;
    if (((T << lp) >> 6) > 8 || lp > 6) return fail(BARD_E_CAPACITY, "tree too wide for this tile size");
    p->log2P[i] = lp;
    // serial sweep plus output rows per instance of the tile
    const int ne = (int)p->ee[i].size();
    cost[i] = 8.0 * m->depth + (double)(m->nv * m->nv + 6 * m->nv * ne + m->nv) / 16.0;
  }
  // work items
  std::vector<int2> items;
  for (int i = 0; i < nm; ++i) {
    const int64_t tiles = (p->batch[i] + T - 1) / T;
    for (int64_t t = 0; t < tiles; ++t) items.push_back(make_int2(i, (int)t));
  }
  if (items.size() > 0x7fffffff) return fail(BARD_E_CAPACITY, "too many work items");
  auto by_cost = [&](const int2& a, const int2& b) {
    if (cost[a.x] != cost[b.x]) return cost[a.x] > cost[b.x];
    if (a.x != b.x) return a.x < b.x;
    return a.y < b.y;
  };
  if (p->cfg.fusion == FUSE_PER_MODEL) {
    std::stable_sort(items.begin(), items.end(), [](const int2& a, const int2& b) { return a.x < b.x; });
  } else if (p->cfg.order == ORDER_LONGEST_FIRST) {
    std::stable_sort(items.begin(), items.end(), by_cost);
  }
  p->n_items = (int)items.size();
  // launch groups
  const size_t lim = lds_limit(dev);
  auto make_group = [&](int ops, int item0, int count, const std::vector<int>& which) -> int {
    Group g{ops, item0, count, 0, 0};
    int waves = out_waves(rs);
    for (int i : which) {
      const bard_model* m = p->models[i];
      const int ne = (int)p->ee[i].size();
      const size_t l =
          (size_t)lds_plan(0, ops, m->n, m->nq, m->nv, ne, 0, T, rs, m->P, m->depth, m->kmax).total;
      g.lds = std::max(g.lds, l);
      waves = std::max(waves, (T << p->log2P[i]) >> 6);
    }
    if (g.lds > lim) return fail(BARD_E_CAPACITY, "a tree is too large for on-chip staging at this tile size");
    if (waves * 64 > tree_max_threads(rs)) return fail(BARD_E_CAPACITY, "a tree is too wide for this tile size");
    g.block = waves * 64;
    if (count > 0) p->groups.push_back(g);
    return BARD_OK;
  };
  p->groups.clear();
  std::vector<int> all(nm);
  for (int i = 0; i < nm; ++i) all[i] = i;
  int rc = BARD_OK;
  if (p->cfg.fusion == FUSE_ALL) {
    rc = make_group(all_ops, 0, p->n_items, all);
  } else if (p->cfg.fusion == FUSE_PER_MODEL) {
    int at = 0;
    for (int i = 0; i < nm && !rc; ++i) {
      int cnt = 0;
      while (at + cnt < p->n_items && items[at + cnt].x == i) ++cnt;
      rc = make_group(all_ops, at, cnt, std::vector<int>{i});
      at += cnt;
    }
  } else {
    for (int op : {OP_RNEA, OP_CRBA, OP_JAC})
      if ((all_ops & op) && !rc) rc = make_group(op, 0, p->n_items, all);
  }
  if (rc) return rc;
  // device descriptor: [DevModel n][DevEE n][Args n][items]
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  p->off_ee = al(nm * sizeof(DevModel));
  p->off_args = p->off_ee + al(nm * sizeof(DevEE));
  p->args_bytes = nm * sizeof(Args<Real>);
  p->off_items = p->off_args + al(p->args_bytes);
  const size_t need = p->off_items + std::max<size_t>(1, items.size()) * sizeof(int2);
  if (need > p->d_bytes) {
    if (p->d_buf) (void)hipFree(p->d_buf);
    p->d_buf = nullptr;
    p->d_bytes = 0;
    if (hipMalloc((void**)&p->d_buf, need) != hipSuccess) return fail(BARD_E_NOMEM, "hipMalloc of the plan failed");
    p->d_bytes = need;
  }
  rc = plan_host_state(p);
  if (rc) return rc;
  // the descriptor may still be read by earlier work of this plan
  if (hipDeviceSynchronize() != hipSuccess) return fail(BARD_E_DEVICE, "device error before plan upload");
  bool ok = hipMemcpy(p->d_buf, dms.data(), nm * sizeof(DevModel), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(p->d_buf + p->off_ee, ees.data(), nm * sizeof(DevEE), hipMemcpyHostToDevice) == hipSuccess &&
            (items.empty() || hipMemcpy(p->d_buf + p->off_items, items.data(), items.size() * sizeof(int2),
                                        hipMemcpyHostToDevice) == hipSuccess);
  if (!ok) return fail(BARD_E_DEVICE, "upload of the plan descriptor failed");
  p->h_last.clear();
  p->runs = 0;
  p->ready = true;
  return BARD_OK;
}

int prepare(bard_plan* p) { return p->dtype == BARD_F32 ? prepare_t<float>(p) : prepare_t<double>(p); }

// Per-model kernel arguments from io (per model: q, qd, qdd, tau, M, J).
template <class Real>
int build_spec_args(const bard_plan* p, const void* const* io, std::vector<unsigned char>* out) {
  const int nm = (int)p->models.size();
  out->assign(nm * sizeof(SpecPlanIO<Real>), 0);
  SpecPlanIO<Real>* a = reinterpret_cast<SpecPlanIO<Real>*>(out->data());
  for (int i = 0; i < nm; ++i) {
    bard_model* m = p->models[i];
    const void* const* v = io + 6 * i;
    if (p->batch[i] > 0)
      for (int k = 0; k < 6; ++k)
        if (!v[k]) return fail(BARD_E_ARG, "NULL array in plan io");
    a[i].q = (const Real*)v[0];
    a[i].qd = (const Real*)v[1];
    a[i].qdd = (const Real*)v[2];
    a[i].tau = (Real*)v[3];
    a[i].M = (Real*)v[4];
    a[i].J = (Real*)v[5];
    std::lock_guard<std::mutex> lk(m->mu);
    for (int k = 0; k < 3; ++k) a[i].g[k] = (Real)m->g[k];
  }
  return BARD_OK;
}

template <class Real>
int build_args(const bard_plan* p, const void* const* io, std::vector<unsigned char>* out) {
  if (p->cfg.fusion == FUSE_SPEC) return build_spec_args<Real>(p, io, out);
  const int nm = (int)p->models.size();
  const int ops = mask_to_ops(p->op_mask);
  out->assign(p->args_bytes, 0);
  Args<Real>* a = reinterpret_cast<Args<Real>*>(out->data());
  for (int i = 0; i < nm; ++i) {
    const bard_model* m = p->models[i];
    const void* const* v = io + 6 * i;
    if (p->batch[i] > 0) {
      if (!v[0]) return fail(BARD_E_ARG, "NULL q in plan io");
      if ((ops & OP_RNEA) && (!v[1] || !v[2] || !v[3])) return fail(BARD_E_ARG, "NULL qd, qdd or tau in plan io");
      if ((ops & OP_CRBA) && !v[4]) return fail(BARD_E_ARG, "NULL M in plan io");
      if ((ops & OP_JAC) && !v[5]) return fail(BARD_E_ARG, "NULL J in plan io");
    }
    Args<Real>& x = a[i];
    const int64_t B = p->batch[i];
    x.q = (const Real*)v[0];
    x.qd = (const Real*)v[1];
    x.qdd = (const Real*)v[2];
    x.tau = (Real*)v[3];
    x.M = (Real*)v[4];
    x.J = (Real*)v[5];
    x.sq_b = x.sqd_b = x.sqdd_b = x.st_b = x.sM_b = x.sJ_b = 1;
    x.sq_k = x.sqd_k = x.sqdd_k = x.st_k = x.sM_k = x.sJ_k = std::max<int64_t>(B, 1);
    x.B = B;
    x.logT = p->cfg.logT;
    x.log2P = p->log2P[i];
    x.frame = 0;
    x.xcd_remap = 0;
    x.stream_out = 1;
    (void)m;
  }
  return BARD_OK;
}

// Stream-ordered update of the device copy of the arguments when they change.
int stage_args(bard_plan* p, const std::vector<unsigned char>& args, hipStream_t st) {
  if (args == p->h_last) return BARD_OK;
  if (p->staged_pending && hipEventSynchronize(p->staged) != hipSuccess)
    return fail(BARD_E_DEVICE, "waiting for the previous argument upload failed");
  std::memcpy(p->h_stage, args.data(), args.size());
  if (hipMemcpyAsync(p->d_buf + p->off_args, p->h_stage, args.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipEventRecord(p->staged, st) != hipSuccess)
    return fail(BARD_E_DEVICE, "upload of the plan arguments failed");
  p->staged_pending = true;
  p->h_last = args;
  return BARD_OK;
}

template <class Real>
hipError_t launch_groups_t(const bard_plan* p, hipStream_t st) {
  if (p->cfg.fusion == FUSE_SPEC) {
    if (p->groups.empty()) return hipSuccess;
    void* io = p->d_buf + p->off_args;
    void* args[] = {&io};
    return hipModuleLaunchKernel((hipFunction_t)p->spk.fn, (unsigned)p->spk_blocks, 1, 1, 64 * p->spk.waves, 1, 1, 0,
                                 st, args, nullptr);
  }
  for (const Group& g : p->groups) {
    PlanPtrs<Real> pp;
    pp.dm = reinterpret_cast<const DevModel*>(p->d_buf);
    pp.ee = reinterpret_cast<const DevEE*>(p->d_buf + p->off_ee);
    pp.args = reinterpret_cast<const Args<Real>*>(p->d_buf + p->off_args);
    pp.items = reinterpret_cast<const int2*>(p->d_buf + p->off_items);
    pp.item0 = g.item0;
    hipError_t e;
    switch (g.ops) {
      case OP_RNEA: e = launch_plan<Real, OP_RNEA>(pp, p->cfg.logT, g.count, g.block, g.lds, st); break;
      case OP_CRBA: e = launch_plan<Real, OP_CRBA>(pp, p->cfg.logT, g.count, g.block, g.lds, st); break;
      case OP_JAC: e = launch_plan<Real, OP_JAC>(pp, p->cfg.logT, g.count, g.block, g.lds, st); break;
      default: e = launch_plan<Real, OP_RNEA | OP_CRBA | OP_JAC>(pp, p->cfg.logT, g.count, g.block, g.lds, st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_groups(const bard_plan* p, hipStream_t st) {
  return p->dtype == BARD_F32 ? launch_groups_t<float>(p, st) : launch_groups_t<double>(p, st);
}

// A model's gravity lives in the plan's device descriptor (and so in its
// captured graph): a change since the upload prepares the plan again.
bool gravity_changed(const bard_plan* p) {
  if (p->g_gen.size() != p->models.size()) return false;
  for (size_t i = 0; i < p->models.size(); ++i)
    if (p->models[i]->g_gen != p->g_gen[i]) return true;
  return false;
}

int run_plan(bard_plan* p, const void* const* io, hipStream_t st, bool allow_graph) {
  if (p->ready && gravity_changed(p)) p->ready = false;
  if (capturing(st)) {
    // The caller is capturing `st`: nothing may synchronize or allocate, and
    // the plan's own graph is not launched inside another capture.  A plan
    // that ran eagerly with the same io records its kernel launches.
    if (!p->ready || p->runs == 0) return fail(BARD_E_CAPTURE, "a plan must run once before it is captured");
    std::vector<unsigned char> args;
    int rc = p->dtype == BARD_F32 ? build_args<float>(p, io, &args) : build_args<double>(p, io, &args);
    if (rc) return rc;
    if (args != p->h_last)
      return fail(BARD_E_CAPTURE, "a captured plan run must use the io of the plan's previous run");
    hipError_t e = launch_groups(p, st);
    if (e != hipSuccess) return fail(BARD_E_DEVICE, std::string("plan launch failed: ") + hipGetErrorString(e));
    return BARD_OK;
  }
  int rc = prepare(p);
  if (rc) return rc;
  std::vector<unsigned char> args;
  rc = p->dtype == BARD_F32 ? build_args<float>(p, io, &args) : build_args<double>(p, io, &args);
  if (rc) return rc;
  if ((rc = stage_args(p, args, st))) return rc;
  if (p->groups.empty()) return BARD_OK;
  // The first run of a configuration launches eagerly (it also sets the
  // kernels' LDS attributes); later runs replay one captured graph.
  if (!allow_graph || p->runs++ == 0) {
    hipError_t e = launch_groups(p, st);
    if (e != hipSuccess) return fail(BARD_E_DEVICE, std::string("plan launch failed: ") + hipGetErrorString(e));
    return BARD_OK;
  }
  if (!p->exec) {
    if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(BARD_E_DEVICE, "hipStreamBeginCapture failed");
    hipError_t e = launch_groups(p, p->cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(p->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return fail(BARD_E_DEVICE, "capture of the plan launch failed");
    }
    p->graph = g;
    if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      drop_graph(p);
      return fail(BARD_E_DEVICE, "hipGraphInstantiate failed");
    }
  }
  if (hipGraphLaunch(p->exec, st) != hipSuccess) return fail(BARD_E_DEVICE, "hipGraphLaunch failed");
  return BARD_OK;
}

}  // namespace

extern "C" {

int bard_plan_create(const bard_model_t* models, int32_t n_models, const int64_t* batch, uint32_t op_mask,
                     bard_dtype dtype, bard_plan_t* out) {
  if (!out || !models || !batch) return fail(BARD_E_ARG, "NULL argument");
  if (n_models < 1 || n_models > kMaxPlanModels) return fail(BARD_E_ARG, "n_models must be in 1..64");
  if (op_mask == 0 || op_mask > 7) return fail(BARD_E_ARG, "op_mask must be a non-empty subset of bits 0..2");
  if (dtype != BARD_F32 && dtype != BARD_F64) return fail(BARD_E_ARG, "dtype must be BARD_F32 or BARD_F64");
  for (int i = 0; i < n_models; ++i) {
    if (!models[i]) return fail(BARD_E_ARG, "NULL model");
    if (batch[i] < 0 || batch[i] > ((int64_t)1 << 31)) return fail(BARD_E_ARG, "batch out of range");
  }
  bard_plan* p = new (std::nothrow) bard_plan();
  if (!p) return fail(BARD_E_NOMEM, "host allocation failed");
  p->models.assign(models, models + n_models);
  p->batch.assign(batch, batch + n_models);
  p->op_mask = op_mask;
  p->dtype = dtype;
  for (int i = 0; i < n_models; ++i) p->ee.push_back(tip_ees(models[i]));
  if (!fusable(mask_to_ops(op_mask))) p->cfg.fusion = FUSE_PER_OP;
  // a configuration chosen earlier for the same trees, batches and device
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    p->device = dev;
    const auto cache = read_cache(cache_path());
    auto it = cache.find(plan_key(p));
    if (it != cache.end() && valid_config(p, it->second.first)) {
      p->cfg = it->second.first;
      p->from_cache = true;
    }
    p->device = -1;
  }
  *out = p;
  return BARD_OK;
}

int bard_plan_configure(bard_plan_t p, int32_t tile, int32_t fusion, int32_t order, int32_t lanes) {
  if (!p) return fail(BARD_E_ARG, "plan is NULL");
  PlanConfig c;
  c.logT = 0;
  while ((1 << c.logT) < tile && c.logT < 8) ++c.logT;
  if ((1 << c.logT) != tile) return fail(BARD_E_ARG, "tile must be 8, 16 or 32");
  c.fusion = fusion;
  c.order = order;
  c.lanes = lanes;
  if (!valid_config(p, c)) return fail(BARD_E_ARG, "invalid plan configuration");
  p->cfg = c;
  p->ready = false;
  return BARD_OK;
}

int bard_plan_get_config(bard_plan_t p, int32_t* tile, int32_t* fusion, int32_t* order, int32_t* lanes,
                         int32_t* from_cache) {
  if (!p) return fail(BARD_E_ARG, "plan is NULL");
  if (lanes) *lanes = p->cfg.lanes;
  if (tile) *tile = 1 << p->cfg.logT;
  if (fusion) *fusion = p->cfg.fusion;
  if (order) *order = p->cfg.order;
  if (from_cache) *from_cache = p->from_cache ? 1 : 0;
  return BARD_OK;
}

int bard_plan_ee(bard_plan_t p, int32_t model_index, int32_t* n_ee, int32_t* ee_body) {
  if (!p || !n_ee) return fail(BARD_E_ARG, "NULL argument");
  if (model_index < 0 || model_index >= (int)p->models.size()) return fail(BARD_E_ARG, "model index out of range");
  const std::vector<int>& e = p->ee[model_index];
  *n_ee = (int32_t)e.size();
  if (ee_body)
    for (size_t k = 0; k < e.size(); ++k) ee_body[k] = e[k];
  return BARD_OK;
}

int bard_plan_run(bard_plan_t p, const void* const* io, void* stream) {
  if (!p || !io) return fail(BARD_E_ARG, "NULL argument");
  int rc = check_device_state();
  if (rc) return rc;
  return run_plan(p, io, (hipStream_t)stream, true);
}

int bard_plan_autotune(bard_plan_t p, void* stream, int32_t budget_ms) {
  if (!p) return fail(BARD_E_ARG, "plan is NULL");
  if (budget_ms < 1) return fail(BARD_E_ARG, "budget_ms must be >= 1");
  int rc = check_device_state();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const size_t rs = p->dtype == BARD_F32 ? 4 : 8;
  // scratch I/O of the plan's shape, zero-filled
  std::vector<void*> bufs;
  std::vector<const void*> io;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    for (void* b : bufs) (void)hipFree(b);
  };
  for (size_t i = 0; i < p->models.size(); ++i) {
    const bard_model* m = p->models[i];
    const size_t B = (size_t)std::max<int64_t>(p->batch[i], 1);
    const size_t ks[6] = {(size_t)m->nq, (size_t)m->nv, (size_t)m->nv, (size_t)m->nv, (size_t)m->nv * m->nv,
                          (size_t)6 * m->nv * p->ee[i].size()};
    for (size_t k : ks) {
      void* b = nullptr;
      if (hipMalloc(&b, k * B * rs) != hipSuccess) {
        cleanup();
        return fail(BARD_E_NOMEM, "hipMalloc of autotune buffers failed");
      }
      bufs.push_back(b);
      io.push_back(b);
      if (hipMemsetAsync(b, 0, k * B * rs, st) != hipSuccess) {
        cleanup();
        return fail(BARD_E_DEVICE, "hipMemsetAsync failed");
      }
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const PlanConfig start = p->cfg;
  PlanConfig best = start;
  double best_us = 1e300;
  auto t_start = std::chrono::steady_clock::now();
  // the generated multi-tree kernel first (it is tried whatever the budget;
  // its compilation is not timed), then the generic configurations
  std::vector<PlanConfig> cands;
  cands.push_back(PlanConfig{4, FUSE_SPEC, ORDER_LONGEST_FIRST, 0});
  cands.push_back(PlanConfig{4, FUSE_SPEC, ORDER_LONGEST_FIRST, 1});
  for (int ln = 0; ln <= 1; ++ln)
    for (int lt = 3; lt <= 5; ++lt)
      for (int fu = FUSE_ALL; fu <= FUSE_PER_OP; ++fu)
        for (int od = ORDER_LONGEST_FIRST; od <= ORDER_MODEL; ++od) cands.push_back(PlanConfig{lt, fu, od, ln});
  for (const PlanConfig& c : cands) {
    const int fu = c.fusion, od = c.order;
    const double spent =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (spent > budget_ms && best_us < 1e300 && fu != FUSE_SPEC) continue;
    if (!valid_config(p, c) || (fu == FUSE_PER_MODEL && od == ORDER_MODEL)) continue;
    p->cfg = c;
    p->ready = false;
    if (run_plan(p, io.data(), st, false) != BARD_OK) continue;  // infeasible (LDS) or failed: skip
    const int reps = 10;
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) (void)launch_groups(p, st);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) continue;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double us = 1e3 * ms / reps;
    if (us < best_us) {
      best_us = us;
      best = c;
    }
    if (fu == FUSE_SPEC) t_start = std::chrono::steady_clock::now();
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cleanup();
  p->cfg = best;
  p->ready = false;
  p->h_last.clear();
  (void)check_device_state();
  if (best_us >= 1e300) return fail(BARD_E_CAPACITY, "no plan configuration could run");
  int dev = 0;
  (void)hipGetDevice(&dev);
  p->device = dev;
  const std::string path = cache_path();
  auto cache = read_cache(path);
  cache[plan_key(p)] = {best, best_us};
  write_cache(path, cache);
  p->from_cache = false;
  return BARD_OK;
}

int bard_plan_specialized_source(bard_plan_t p, int32_t compile_only, char* buf, int64_t cap, int64_t* len) {
  if (!p || !len) return fail(BARD_E_ARG, "NULL argument");
  if (mask_to_ops(p->op_mask) != (OP_RNEA | OP_CRBA | OP_JAC))
    return fail(BARD_E_UNSUPPORTED, "the generated multi-tree kernel covers plans of all three operators");
  std::vector<bard_model*> ms(p->models.begin(), p->models.end());
  int waves = 1;
  int64_t blocks = 0;
  const std::string src =
      spec_plan_source(ms, p->ee, p->batch, p->dtype == BARD_F64, spec_plan_waves(p->cfg), &waves, &blocks);
  *len = (int64_t)src.size();
  if (buf && cap > 0) {
    const size_t n = std::min<size_t>(src.size(), (size_t)cap - 1);
    std::memcpy(buf, src.data(), n);
    buf[n] = 0;
  }
  if (compile_only) {
    std::vector<char> code;
    std::string log;
    const int rc = spec_compile(src, &code, &log);
    if (rc) return fail(rc, "hipRTC compile of the multi-tree kernel failed: " + log.substr(0, 2000));
  }
  return BARD_OK;
}

int bard_plan_specialized_info(bard_plan_t p, int32_t* vgprs, int32_t* scratch_bytes, int32_t* waves,
                               int64_t* workgroups, double* compile_s) {
  if (!p) return fail(BARD_E_ARG, "plan is NULL");
  if (!p->spk.fn) return fail(BARD_E_STATE, "the plan's generated kernel is not built (run it in fusion 3 first)");
  if (vgprs) *vgprs = p->spk.vgprs;
  if (scratch_bytes) *scratch_bytes = p->spk.scratch;
  if (waves) *waves = p->spk.waves;
  if (workgroups) *workgroups = p->spk_blocks;
  if (compile_s) *compile_s = p->spk.compile_s;
  return BARD_OK;
}

int bard_plan_destroy(bard_plan_t p) {
  if (!p) return fail(BARD_E_ARG, "plan is NULL");
  if (p->device >= 0) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    drop_graph(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->staged) (void)hipEventDestroy(p->staged);
    if (p->d_buf) (void)hipFree(p->d_buf);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    if (p->spk.mod) (void)hipModuleUnload((hipModule_t)p->spk.mod);
    if (cur >= 0) (void)hipSetDevice(cur);
  }
  delete p;
  return BARD_OK;
}

}  // extern "C"
