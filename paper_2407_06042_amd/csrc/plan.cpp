// Uneven batches: shape classes, longest-processing-time ordering, one HIP graph
// per plan, and the per-class layout autotuner.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "host.hpp"

using namespace dmala;
using namespace dmala::host;

namespace {

struct ClassInfo {
  dmala_shape shape;
  int count = 0;
  int first = 0;          // first entry of the class in the descriptor table
  Plan pl;                // layout of this class (tile config applied)
  size_t ws_off = 0;      // offset of the class's workspace region
  double cost = 0.0;      // relative work estimate (LPT ordering)
  int tile_config = 0;    // 1 + sampler layout
  int cbw = 4;            // chain blocks per workgroup
  double tuned_ms = 0.0;
  int branch = 0;         // graph branch
};

constexpr int kMaxBranches = 8;

double class_cost(const dmala_shape& s, int count, const dmala_params& p) {
  // dominant per chain-iteration VALU work: proposal weights and draws over the
  // levels of 2 Nt dimensions, plus the contraction (on MFMA, lower weight)
  const double N = 2.0 * s.nt, Q = std::sqrt((double)s.qam_order);
  return (double)count * p.n_chains * std::max(1, p.n_iters) * (N * (Q + 20.0) + N * N / 64.0);
}

std::string class_key(const dmala_shape& s, const dmala_params& p) {
  char buf[160];
  snprintf(buf, sizeof buf, "nt=%d,nr=%d,M=%d,C=%d,T=%d,prec=%d,prop=%d", s.nt, s.nr, s.qam_order, p.n_chains,
           p.n_iters, (int)p.precision, (int)p.proposal);
  return buf;
}

}  // namespace

// One persistent launch: a kernel (setup, sampler or estimator instantiation) and the classes
// whose items it runs.
struct Family {
  int stage = 0;            // 0 setup, 1 sampler, 2 estimator
  const void* k = nullptr;
  int threads = 0;
  size_t lds = 0;           // largest body LDS of the member classes
  std::vector<int> cls;     // member classes, largest items first
  double cost = 0.0;
  int item_off = 0, n_items = 0, grid = 0;
};

struct dmala_plan_s {
  dmala_params params{};
  int n_inst = 0;
  std::vector<ClassInfo> classes;
  bool persistent = false;  // the graph is the persistent form
  std::vector<Family> fams;
  WorkItem* items_dev = nullptr;
  size_t items_cap = 0;
  unsigned char* args_dev = nullptr;  // per-class SetupArgs, SamplerArgs, EstArgs arrays
  size_t args_cap = 0;
  int32_t* counters = nullptr;        // two per family
  int counters_cap = 0;
  int n_cu = 0;
  std::vector<hipEvent_t> stage_ev;   // per stage: fork and branch joins of the persistent graph
  InstDesc* desc_dev = nullptr;
  size_t ws_total = 0;
  int n_branches = 1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> branches;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key.clear();
  }
  ~dmala_plan_s() {
    drop_graph();
    if (desc_dev) (void)hipFree(desc_dev);
    if (items_dev) (void)hipFree(items_dev);
    if (args_dev) (void)hipFree(args_dev);
    if (counters) (void)hipFree(counters);
    for (auto s : branches) (void)hipStreamDestroy(s);
    if (cap) (void)hipStreamDestroy(cap);
    for (auto e : joins) (void)hipEventDestroy(e);
    for (auto e : stage_ev) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
  }
};

namespace {

dmala_status class_plan(dmala_plan_s* P, ClassInfo& c) {
  dmala_params p = P->params;
  p.tile_config = c.tile_config;
  p.wg_chain_blocks = c.cbw;
  const dmala_status st = make_plan(c.count, c.shape.nt, c.shape.nr, c.shape.qam_order, &p, c.pl);
  c.pl.sh.share = 1;
  return st;
}

// Assign classes (already in decreasing cost order) to graph branches, each to the
// currently least loaded branch (longest processing time first).
void assign_branches(dmala_plan_s* P) {
  P->n_branches = std::min<int>(kMaxBranches, (int)P->classes.size());
  std::vector<double> load(P->n_branches, 0.0);
  for (auto& c : P->classes) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    c.branch = b;
    load[b] += c.cost;
  }
}

// Grow a device buffer (contents not kept).
template <typename T>
hipError_t ensure(T*& ptr, size_t& cap, size_t n) {
  if (n <= cap && ptr) return hipSuccess;
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  cap = 0;
  const hipError_t e = hipMalloc((void**)&ptr, n * sizeof(T) + 256);
  if (e == hipSuccess) cap = n;
  return e;
}

// The persistent form: the classes' setup, sampler and estimator work split into items
// (instance, or instance x chain group), grouped by the kernel instantiation that runs them; one
// persistent launch per group, groups in stage order on one stream, items of the classes with
// the largest items first.  DMALA_ERR_UNSUPPORTED when a class has no persistent kernel
// (float64, learned and MHGD chains), which then take the branch graph.
dmala_status build_graph_persistent(dmala_plan_s* P, const void* H, const void* y, const void* sigma2,
                                    const dmala_outputs* out, unsigned char* ws) {
  const int nc = (int)P->classes.size();
  hipError_t e;
  // an earlier launch of this plan may still read the tables rewritten below
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "synchronise");
  dmala_outputs o = *out;
  for (int i = 0; i < 4; ++i) o.stage_events[i] = nullptr;
  const bool est = wants_estimates(&o);
  std::vector<SetupArgs> sa(nc);
  std::vector<SamplerArgs> ka(nc);
  std::vector<EstArgs> ea(nc);
  std::vector<KernelCfg> cfg(3 * nc);
  for (int ci = 0; ci < nc; ++ci) {
    const ClassInfo& c = P->classes[ci];
    make_args(H, y, sigma2, c.count, c.pl, &P->params, &o, P->desc_dev + c.first, ws + c.ws_off, nullptr, nullptr,
              nullptr, nullptr, 0.0, sa[ci], ka[ci], ea[ci]);
    if (launch_setup(sa[ci], nullptr, nullptr, 0, &cfg[3 * ci]) != hipSuccess ||
        launch_sampler(c.pl.sh, ka[ci], false, nullptr, nullptr, 0, &cfg[3 * ci + 1]) != hipSuccess ||
        (est && launch_estimate(ea[ci], nullptr, nullptr, 0, &cfg[3 * ci + 2]) != hipSuccess))
      return DMALA_ERR_UNSUPPORTED;
  }
  if (!P->n_cu) {
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "get device");
    if ((e = hipDeviceGetAttribute(&P->n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
      return hip_fail(e, "device attribute");
  }
  // families: (stage, kernel, threads)
  P->fams.clear();
  std::map<std::tuple<int, const void*, int>, int> fidx;
  auto item_cost = [&](int stage, int ci) {
    const ClassInfo& c = P->classes[ci];
    const double nt = c.shape.nt, nr = c.shape.nr, M = c.shape.qam_order;
    if (stage == 0) return nt * nt * (nt + nr);
    if (stage == 1) return c.cost / ((double)c.count * std::max(1, cfg[3 * ci + 1].gy));
    return (double)P->params.n_chains * nt * (nr + M);
  };
  for (int stage = 0; stage < (est ? 3 : 2); ++stage)
    for (int ci = 0; ci < nc; ++ci) {
      const KernelCfg& k = cfg[3 * ci + stage];
      const auto key = std::make_tuple(stage, k.k, k.threads);
      auto it = fidx.find(key);
      if (it == fidx.end()) {
        it = fidx.emplace(key, (int)P->fams.size()).first;
        Family f;
        f.stage = stage;
        f.k = k.k;
        f.threads = k.threads;
        P->fams.push_back(f);
      }
      Family& f = P->fams[it->second];
      f.lds = std::max(f.lds, k.lds);
      f.cls.push_back(ci);
      f.cost += item_cost(stage, ci) * P->classes[ci].count * (stage == 1 ? k.gy : 1);
    }
  std::vector<WorkItem> items;
  for (auto& f : P->fams) {
    std::stable_sort(f.cls.begin(), f.cls.end(),
                     [&](int a, int b) { return item_cost(f.stage, a) > item_cost(f.stage, b); });
    f.item_off = (int)items.size();
    for (int ci : f.cls) {
      const int gy = f.stage == 1 ? cfg[3 * ci + 1].gy : 1;
      for (int i = 0; i < P->classes[ci].count; ++i)
        for (int g = 0; g < gy; ++g) items.push_back(WorkItem{ci, i, g, 0});
    }
    f.n_items = (int)items.size() - f.item_off;
    const size_t lds_run = ((f.lds + 15) & ~(size_t)15) + 16;
    if (lds_run > 65536 &&
        (e = hipFuncSetAttribute(f.k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_run)) != hipSuccess)
      return hip_fail(e, "kernel attribute");
    int nb = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f.k, f.threads, lds_run)) != hipSuccess)
      return hip_fail(e, "occupancy");
    if (nb < 1) return fail(DMALA_ERR_HIP, "a persistent kernel does not fit a CU");
    f.grid = std::min(f.n_items, nb * P->n_cu);
  }
  // heavier families of a stage first
  std::stable_sort(P->fams.begin(), P->fams.end(), [](const Family& a, const Family& b) {
    return a.stage != b.stage ? a.stage < b.stage : a.cost > b.cost;
  });
  const size_t args_bytes = (size_t)nc * (sizeof(SetupArgs) + sizeof(SamplerArgs) + sizeof(EstArgs));
  if ((e = ensure(P->items_dev, P->items_cap, items.size())) != hipSuccess ||
      (e = ensure(P->args_dev, P->args_cap, args_bytes)) != hipSuccess)
    return hip_fail(e, "plan tables");
  if ((int)P->fams.size() * 2 > P->counters_cap) {
    size_t cap = 0;
    if ((e = ensure(P->counters, cap, P->fams.size() * 2)) != hipSuccess) return hip_fail(e, "plan counters");
    P->counters_cap = (int)cap;
    if ((e = hipMemset(P->counters, 0, cap * sizeof(int32_t))) != hipSuccess) return hip_fail(e, "plan counters");
  }
  unsigned char* a_setup = P->args_dev;
  unsigned char* a_samp = a_setup + (size_t)nc * sizeof(SetupArgs);
  unsigned char* a_est = a_samp + (size_t)nc * sizeof(SamplerArgs);
  if ((e = hipMemcpy(P->items_dev, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(a_setup, sa.data(), nc * sizeof(SetupArgs), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(a_samp, ka.data(), nc * sizeof(SamplerArgs), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(a_est, ea.data(), nc * sizeof(EstArgs), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "plan table upload");
  // Branches: the launches of a stage go to the least loaded of kPersBranches streams (longest
  // first), so that a group's tail and the bandwidth-bound large-instance groups overlap other
  // groups of the stage; the stages are joined (every event recorded in the capture is waited on
  // inside it).
  constexpr int kPersBranches = 4;
  while ((int)P->branches.size() < kPersBranches) {
    hipStream_t bs;
    hipEvent_t ev;
    if ((e = hipStreamCreateWithFlags(&bs, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream create");
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event create");
    P->branches.push_back(bs);
    P->joins.push_back(ev);
  }
  const int nstage = est ? 3 : 2;
  while ((int)P->stage_ev.size() < nstage * (1 + kPersBranches)) {
    hipEvent_t ev;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event create");
    P->stage_ev.push_back(ev);
  }
  const int nf = (int)P->fams.size();
  if ((e = hipStreamBeginCapture(P->cap, hipStreamCaptureModeRelaxed)) != hipSuccess) return hip_fail(e, "begin capture");
  dmala_status st = DMALA_OK;
  int fi = 0;
  for (int stage = 0; stage < nstage && st == DMALA_OK; ++stage) {
    int n_st = 0;
    while (fi + n_st < nf && P->fams[fi + n_st].stage == stage) ++n_st;
    const int nbr = std::max(1, std::min(kPersBranches, n_st));
    hipEvent_t* ev = P->stage_ev.data() + stage * (1 + kPersBranches);
    (void)hipEventRecord(ev[0], P->cap);
    for (int b = 0; b < nbr; ++b) (void)hipStreamWaitEvent(P->branches[b], ev[0], 0);
    std::vector<double> load(nbr, 0.0);
    for (int end = fi + n_st; fi < end && st == DMALA_OK; ++fi) {
      const Family& f = P->fams[fi];
      const int br = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[br] += f.cost;
      hipStream_t bs = P->branches[br];
      const int rep = f.cls[0];
      Persist pp{};
      pp.items = P->items_dev + f.item_off;
      pp.n_items = f.n_items;
      pp.lds_off = (int32_t)((f.lds + 15) & ~(size_t)15);
      pp.counter = P->counters + 2 * fi;
      pp.cls = f.stage == 0 ? (const void*)a_setup : (f.stage == 1 ? (const void*)a_samp : (const void*)a_est);
      KernelCfg chk;
      hipError_t le;
      if (f.stage == 0) {
        le = launch_setup(sa[rep], nullptr, nullptr, 0, &chk);
        if (le == hipSuccess && chk.k == f.k) le = launch_setup(sa[rep], bs, &pp, f.grid);
      } else if (f.stage == 1) {
        le = launch_sampler(P->classes[rep].pl.sh, ka[rep], false, nullptr, nullptr, 0, &chk);
        if (le == hipSuccess && chk.k == f.k) le = launch_sampler(P->classes[rep].pl.sh, ka[rep], false, bs, &pp, f.grid);
      } else {
        le = launch_estimate(ea[rep], nullptr, nullptr, 0, &chk);
        if (le == hipSuccess && chk.k == f.k) le = launch_estimate(ea[rep], bs, &pp, f.grid);
      }
      if (le == hipSuccess && chk.k != f.k) le = hipErrorInvalidValue;
      if (le != hipSuccess) st = hip_fail(le, "persistent launch");
    }
    for (int b = 0; b < nbr; ++b) {
      (void)hipEventRecord(ev[1 + b], P->branches[b]);
      (void)hipStreamWaitEvent(P->cap, ev[1 + b], 0);
    }
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(P->cap, &g);
  if (st != DMALA_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  P->graph = g;
  if ((e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0)) != hipSuccess) {
    P->drop_graph();
    return hip_fail(e, "graph instantiate");
  }
  P->persistent = true;
  return DMALA_OK;
}

dmala_status build_graph(dmala_plan_s* P, const void* H, const void* y, const void* sigma2, const dmala_outputs* out,
                         unsigned char* ws) {
  hipError_t e;
  if (!P->cap) {
    if ((e = hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream create");
    if ((e = hipEventCreateWithFlags(&P->fork, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event create");
  }
  while ((int)P->branches.size() < P->n_branches) {
    hipStream_t s;
    hipEvent_t ev;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream create");
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event create");
    P->branches.push_back(s);
    P->joins.push_back(ev);
  }
  P->drop_graph();
  P->persistent = false;
  const dmala_status sp = build_graph_persistent(P, H, y, sigma2, out, ws);
  if (sp != DMALA_ERR_UNSUPPORTED) return sp;
  dmala_outputs o = *out;
  for (int i = 0; i < 4; ++i) o.stage_events[i] = nullptr;
  if ((e = hipStreamBeginCapture(P->cap, hipStreamCaptureModeRelaxed)) != hipSuccess) return hip_fail(e, "begin capture");
  dmala_status st = DMALA_OK;
  (void)hipEventRecord(P->fork, P->cap);
  for (int b = 0; b < P->n_branches; ++b) (void)hipStreamWaitEvent(P->branches[b], P->fork, 0);
  for (auto& c : P->classes) {
    st = enqueue(H, y, sigma2, c.count, c.pl, &P->params, &o, P->desc_dev + c.first, ws + c.ws_off, nullptr, nullptr,
                 nullptr, P->branches[c.branch]);
    if (st != DMALA_OK) break;
  }
  for (int b = 0; b < P->n_branches; ++b) {
    (void)hipEventRecord(P->joins[b], P->branches[b]);
    (void)hipStreamWaitEvent(P->cap, P->joins[b], 0);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(P->cap, &g);
  if (st != DMALA_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  P->graph = g;
  if ((e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0)) != hipSuccess) {
    P->drop_graph();
    return hip_fail(e, "graph instantiate");
  }
  return DMALA_OK;
}

// Minimal reader/writer of the autotune cache:
// {"entries": [{"key": "...", "tile_config": 3, "wg_chain_blocks": 4, "ms": 1.25}, ...]}
struct CacheEntry {
  int tile_config, cbw;
  double ms;
};

std::map<std::string, CacheEntry> read_cache(const char* path) {
  std::map<std::string, CacheEntry> m;
  FILE* f = fopen(path, "rb");
  if (!f) return m;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  fclose(f);
  size_t pos = 0;
  while ((pos = txt.find("\"key\"", pos)) != std::string::npos) {
    const size_t q0 = txt.find('"', txt.find(':', pos) + 1);
    const size_t q1 = txt.find('"', q0 + 1);
    if (q0 == std::string::npos || q1 == std::string::npos) break;
    const std::string key = txt.substr(q0 + 1, q1 - q0 - 1);
    const size_t end = txt.find('}', q1);
    const std::string rest = txt.substr(q1, end - q1);
    CacheEntry ce{0, 4, 0.0};
    const size_t a = rest.find("\"tile_config\""), b = rest.find("\"wg_chain_blocks\""), c = rest.find("\"ms\"");
    if (a != std::string::npos) ce.tile_config = atoi(rest.c_str() + rest.find(':', a) + 1);
    if (b != std::string::npos) ce.cbw = atoi(rest.c_str() + rest.find(':', b) + 1);
    if (c != std::string::npos) ce.ms = atof(rest.c_str() + rest.find(':', c) + 1);
    if (ce.tile_config > 0) m[key] = ce;
    pos = end == std::string::npos ? txt.size() : end;
  }
  return m;
}

bool write_cache(const char* path, const std::map<std::string, CacheEntry>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return false;
  fprintf(f, "{\"entries\": [\n");
  size_t i = 0;
  for (const auto& kv : m) {
    fprintf(f, "  {\"key\": \"%s\", \"tile_config\": %d, \"wg_chain_blocks\": %d, \"ms\": %.6f}%s\n", kv.first.c_str(),
            kv.second.tile_config, kv.second.cbw, kv.second.ms, ++i < m.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  fclose(f);
  return rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" {

dmala_status dmala_plan_create(dmala_plan* plan, const dmala_shape* shapes, int32_t n_inst, const dmala_params* params,
                               size_t* workspace_bytes) {
  if (!plan || !shapes || !params || !workspace_bytes) return fail(DMALA_ERR_ARG, "NULL argument");
  if (n_inst < 1) return fail(DMALA_ERR_ARG, "n_inst must be >= 1");
  *plan = nullptr;
  dmala_plan_s* P = new dmala_plan_s();
  P->params = *params;
  P->n_inst = n_inst;
  // group by shape class; offsets into the caller's packed buffers in instance order
  std::map<std::tuple<int, int, int>, std::vector<int>> groups;
  std::vector<InstDesc> d(n_inst);
  int64_t h = 0, yo = 0, sy = 0, mg = 0, ll = 0, fs = 0;
  for (int b = 0; b < n_inst; ++b) {
    const dmala_shape s = shapes[b];
    if (s.nt < 1 || s.nr < 1 || s.qam_order < 4) {
      delete P;
      return fail(DMALA_ERR_ARG, "instance %d has an invalid shape", b);
    }
    int nb = 0;
    while ((1 << nb) < s.qam_order) ++nb;
    d[b].h_off = h; d[b].y_off = yo; d[b].sym_off = sy; d[b].marg_off = mg; d[b].llr_off = ll; d[b].fs_off = fs;
    d[b].orig = b; d[b].pad_ = 0;
    h += (int64_t)s.nt * s.nr; yo += s.nr; sy += s.nt; mg += (int64_t)s.nt * s.qam_order; ll += (int64_t)s.nt * nb;
    fs += (int64_t)params->n_chains * 2 * s.nt;
    groups[std::make_tuple(s.nt, s.nr, s.qam_order)].push_back(b);
  }
  for (auto& kv : groups) {
    ClassInfo c;
    c.shape = {std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first)};
    c.count = (int)kv.second.size();
    c.cost = class_cost(c.shape, c.count, *params);
    c.tile_config = params->tile_config;
    c.cbw = params->wg_chain_blocks;
    dmala_status st = class_plan(P, c);
    if (st != DMALA_OK) {
      delete P;
      return st;
    }
    P->classes.push_back(c);
  }
  std::sort(P->classes.begin(), P->classes.end(), [](const ClassInfo& a, const ClassInfo& b) { return a.cost > b.cost; });
  std::vector<InstDesc> table;
  table.reserve(n_inst);
  size_t ws = 0;
  for (auto& c : P->classes) {
    c.first = (int)table.size();
    for (int b : groups[std::make_tuple(c.shape.nt, c.shape.nr, c.shape.qam_order)]) table.push_back(d[b]);
    c.ws_off = ws;
    ws = round_up(ws + c.pl.total, 256);
  }
  P->ws_total = ws;
  assign_branches(P);
  hipError_t e = hipMalloc((void**)&P->desc_dev, table.size() * sizeof(InstDesc));
  if (e == hipSuccess) e = hipMemcpy(P->desc_dev, table.data(), table.size() * sizeof(InstDesc), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    delete P;
    return hip_fail(e, "plan table upload");
  }
  *plan = P;
  *workspace_bytes = ws;
  g_err.clear();
  return DMALA_OK;
}

dmala_status dmala_plan_execute(dmala_plan P, const void* H, const void* y, const void* sigma2, const dmala_outputs* out,
                                void* workspace, size_t workspace_bytes, dmala_stream_t stream) {
  if (!P || !out) return fail(DMALA_ERR_ARG, "NULL plan or outputs");
  if (!H || !y || !sigma2) return fail(DMALA_ERR_ARG, "H, y and sigma2 must be non-NULL");
  if (out->train_rows && (P->params.proposal == DMALA_NAIVE || P->params.proposal == DMALA_MHGD ||
                          P->params.precision == DMALA_FP64))
    return fail(DMALA_ERR_UNSUPPORTED, "train_rows needs the PRECOND or LEARNED proposal without DMALA_FP64");
  if (!workspace) return fail(DMALA_ERR_WORKSPACE, "workspace is NULL");
  if (workspace_bytes < P->ws_total)
    return fail(DMALA_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", workspace_bytes, P->ws_total);
  if (((uintptr_t)workspace & 255) != 0) return fail(DMALA_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const std::vector<const void*> key = {H, y, sigma2, out->symbols, out->marginals, out->llrs, out->best_energy,
                                        out->final_state, out->accept_count, out->marginals_mc, out->train_rows,
                                        out->status, out->trace_accept, out->trace_hash, workspace};
  if (!P->exec || key != P->key) {
    const dmala_status st = build_graph(P, H, y, sigma2, out, (unsigned char*)workspace);
    if (st != DMALA_OK) return st;
    P->key = key;
  }
  hipStream_t s = (hipStream_t)stream;
  if (out->stage_events[0]) (void)hipEventRecord((hipEvent_t)out->stage_events[0], s);
  const hipError_t e = hipGraphLaunch(P->exec, s);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  if (out->stage_events[3]) (void)hipEventRecord((hipEvent_t)out->stage_events[3], s);
  g_err.clear();
  return DMALA_OK;
}

dmala_status dmala_plan_autotune(dmala_plan P, const void* H, const void* y, const void* sigma2, void* workspace,
                                 size_t workspace_bytes, const char* cache_path, dmala_stream_t stream) {
  if (!P) return fail(DMALA_ERR_ARG, "NULL plan");
  if (!H || !y || !sigma2) return fail(DMALA_ERR_ARG, "H, y and sigma2 must be non-NULL");
  if (!workspace || workspace_bytes < P->ws_total || ((uintptr_t)workspace & 255) != 0)
    return fail(DMALA_ERR_WORKSPACE, "workspace NULL, unaligned or smaller than %zu bytes", P->ws_total);
  hipStream_t s = (hipStream_t)stream;
  std::map<std::string, CacheEntry> cache;
  if (cache_path) cache = read_cache(cache_path);
  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) return hip_fail(e, "event create");
  dmala_status st = DMALA_OK;
  for (auto& c : P->classes) {
    const std::string k = class_key(c.shape, P->params);
    auto it = cache.find(k);
    if (it != cache.end()) {
      ClassInfo t = c;
      t.tile_config = it->second.tile_config;
      t.cbw = it->second.cbw;
      if (class_plan(P, t) == DMALA_OK) {
        c = t;
        c.tuned_ms = it->second.ms;
        continue;
      }
    }
    double best = INFINITY;
    ClassInfo best_c = c;
    for (int tc = 1; tc <= 10; ++tc) {
      for (int cb : {1, 2, 4}) {
        ClassInfo t = c;
        t.tile_config = tc;
        t.cbw = cb;
        if (class_plan(P, t) != DMALA_OK) continue;
        // the split layouts hold at most 4 / (waves per chain block) blocks per workgroup: skip settings
        // that launch the same configuration
        if ((tc == 5 || tc == 7 || tc == 9) && cb != 4) continue;
        if ((tc == 4 || tc == 6 || tc == 8) && cb == 4) continue;
        double ms_best = INFINITY;
        for (int rep = 0; rep < 3; ++rep) {
          (void)hipEventRecord(e0, s);
          st = enqueue(H, y, sigma2, t.count, t.pl, &P->params, nullptr, P->desc_dev + t.first,
                       (unsigned char*)workspace + t.ws_off, nullptr, nullptr, nullptr, s);
          if (st != DMALA_OK) break;
          (void)hipEventRecord(e1, s);
          if ((e = hipEventSynchronize(e1)) != hipSuccess) { st = hip_fail(e, "autotune run"); break; }
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0) ms_best = std::min(ms_best, (double)ms);
        }
        if (st != DMALA_OK) break;
        if (ms_best < best) {
          best = ms_best;
          best_c = t;
          best_c.tuned_ms = ms_best;
        }
      }
      if (st != DMALA_OK) break;
    }
    if (st != DMALA_OK) break;
    c = best_c;
    cache[k] = CacheEntry{c.tile_config, c.cbw, c.tuned_ms};
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DMALA_OK) return st;
  P->drop_graph();
  if (cache_path && !write_cache(cache_path, cache)) return fail(DMALA_ERR_ARG, "cannot write %s", cache_path);
  g_err.clear();
  return DMALA_OK;
}

int32_t dmala_plan_num_classes(dmala_plan P) { return P ? (int32_t)P->classes.size() : 0; }

dmala_status dmala_plan_class_info(dmala_plan P, int32_t k, dmala_shape* shape, int32_t* n_inst, int32_t* tile_config,
                                   int32_t* wg_chain_blocks, double* tuned_ms) {
  if (!P || k < 0 || k >= (int32_t)P->classes.size()) return fail(DMALA_ERR_ARG, "no such class");
  const ClassInfo& c = P->classes[k];
  if (shape) *shape = c.shape;
  if (n_inst) *n_inst = c.count;
  if (tile_config) *tile_config = c.pl.sh.cfg + 1;
  if (wg_chain_blocks) *wg_chain_blocks = c.pl.sh.cbw;
  if (tuned_ms) *tuned_ms = c.tuned_ms;
  return DMALA_OK;
}

dmala_status dmala_plan_graph_info(dmala_plan P, int32_t* n_kernels, int32_t* persistent) {
  if (!P || !n_kernels || !persistent) return fail(DMALA_ERR_ARG, "NULL argument");
  *n_kernels = -1;
  *persistent = -1;
  if (!P->graph) return DMALA_OK;
  size_t n = 0;
  hipError_t e = hipGraphGetNodes(P->graph, nullptr, &n);
  if (e != hipSuccess) return hip_fail(e, "graph nodes");
  std::vector<hipGraphNode_t> nodes(n);
  if (n && (e = hipGraphGetNodes(P->graph, nodes.data(), &n)) != hipSuccess) return hip_fail(e, "graph nodes");
  int32_t k = 0;
  for (auto nd : nodes) {
    hipGraphNodeType t;
    if (hipGraphNodeGetType(nd, &t) == hipSuccess && t == hipGraphNodeTypeKernel) ++k;
  }
  *n_kernels = k;
  *persistent = P->persistent ? 1 : 0;
  return DMALA_OK;
}

void dmala_plan_destroy(dmala_plan P) { delete P; }

}  // extern "C"
