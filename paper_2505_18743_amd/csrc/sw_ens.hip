// Ensembles of independent members (C ABI in include/sw.h).
//
// Members that share the discretisation (degree, rule, sample counts, RK
// scheme, physical constants) are packed into one batched context, so that one
// launch of each kernel covers every member of the batch; each member keeps
// its own mesh, cell size, bathymetry, Manning field, tide, time and CFL time
// step.  The batches run on their own streams, forked from and joined to the
// caller's stream, so that batches of different degree overlap on the device.
// A step of all batches can be captured once into a hipGraph and replayed.
#include <cstdio>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "sw.h"
#include "sw_internal.h"

using namespace swk;

namespace {
sw_status efail(sw_status s, const std::string& m) { return (sw_status)api_fail(s, m.c_str()); }
}  // namespace

struct sw_ens {
  hipStream_t user = nullptr;   // caller's stream
  hipStream_t cap = nullptr;    // origin stream of the captured graph
  std::vector<sw_ctx*> batch;
  std::vector<hipStream_t> bs;  // one stream per batch
  std::vector<int> mem_batch, mem_index;
  std::vector<int> batch_members;
  hipEvent_t ev_in = nullptr, ev_fork = nullptr, ev_out = nullptr;
  std::vector<hipEvent_t> ev_join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double graph_dt = 0.0;
  int64_t graph_launches = 0;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~sw_ens() {
    if (user) (void)hipStreamSynchronize(user);
    for (auto s : bs) (void)hipStreamSynchronize(s);
    if (cap) (void)hipStreamSynchronize(cap);
    drop_graph();
    for (auto c : batch) sw_destroy(c);
    for (auto s : bs) (void)hipStreamDestroy(s);
    if (cap) (void)hipStreamDestroy(cap);
    for (auto e : ev_join) (void)hipEventDestroy(e);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_out) (void)hipEventDestroy(ev_out);
  }
};

namespace {

#define EHIP(x)                                                                             \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess) return efail(SW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// key of the parameters a batch must share
std::vector<double> batch_key(const sw_params& p) {
  std::vector<double> k = {(double)p.r,   (double)p.rule, (double)p.rk,         (double)p.n_levels,
                           p.g,           p.eps,          p.h_lim,              p.eps0,
                           (double)p.newton_max, (double)p.cfl_mode, (double)(p.tracer != 0),
                           (double)(p.adapt_degree != 0), p.tracer_diff, p.tracer_strain, p.tracer_decay,
                           (double)p.quadrature};
  for (int L = 0; L < 8; ++L) k.push_back(L < p.n_levels ? (double)p.S[L] : 0.0);
  return k;
}

// n steps of every batch on its own stream, forked from / joined to `origin`
sw_status run_forked(sw_ens* e, hipStream_t origin, int32_t n, double dt) {
  EHIP(hipEventRecord(e->ev_fork, origin));
  for (size_t b = 0; b < e->batch.size(); ++b) {
    EHIP(hipStreamWaitEvent(e->bs[b], e->ev_fork, 0));
    hipStream_t old = ctx_swap_stream(e->batch[b], e->bs[b]);
    sw_status st = sw_run(e->batch[b], n, dt);
    ctx_swap_stream(e->batch[b], old);
    if (st != SW_OK) return st;
    EHIP(hipEventRecord(e->ev_join[b], e->bs[b]));
    EHIP(hipStreamWaitEvent(origin, e->ev_join[b], 0));
  }
  return SW_OK;
}

sw_status capture(sw_ens* e, double dt) {
  e->drop_graph();
  std::vector<int64_t> steps(e->batch.size());
  std::vector<bool> prof(e->batch.size());
  for (size_t b = 0; b < e->batch.size(); ++b) {
    steps[b] = ctx_steps(e->batch[b]);
    prof[b] = ctx_set_prof(e->batch[b], false);   // no timing events inside the graph
  }
  EHIP(hipStreamBeginCapture(e->cap, hipStreamCaptureModeRelaxed));
  sw_status st = run_forked(e, e->cap, 1, dt);
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(e->cap, &g);
  for (size_t b = 0; b < e->batch.size(); ++b) {
    ctx_set_steps(e->batch[b], steps[b]);   // capturing ran nothing
    ctx_set_prof(e->batch[b], prof[b]);
  }
  if (st != SW_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (ee != hipSuccess) return efail(SW_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
  e->graph = g;
  EHIP(hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0));
  e->graph_dt = dt;
  return SW_OK;
}

}  // namespace

extern "C" {

sw_status sw_ens_create(sw_ens** out, int32_t n_members, const sw_mesh_desc* meshes, const sw_params* params,
                        void* stream) {
  if (!out || !meshes || !params) return efail(SW_EINVAL, "NULL argument to sw_ens_create");
  *out = nullptr;
  if (n_members < 1) return efail(SW_EINVAL, "n_members must be >= 1");
  // group the members, batches in order of first appearance
  std::map<std::vector<double>, int> bid;
  std::vector<std::vector<int>> groups;
  std::vector<int> mb(n_members), mi(n_members);
  for (int m = 0; m < n_members; ++m) {
    auto k = batch_key(params[m]);
    auto it = bid.find(k);
    int b;
    if (it == bid.end()) {
      b = (int)groups.size();
      bid.emplace(k, b);
      groups.emplace_back();
    } else {
      b = it->second;
    }
    mb[m] = b;
    mi[m] = (int)groups[b].size();
    groups[b].push_back(m);
  }
  auto* e = new sw_ens();
  e->user = (hipStream_t)stream;
  e->mem_batch = mb;
  e->mem_index = mi;
  auto bail = [&](sw_status st, const std::string& msg) {
    delete e;
    return efail(st, msg);
  };
#define ECALL(x)                                                                               \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) return bail(SW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)
  ECALL(hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking));
  ECALL(hipEventCreateWithFlags(&e->ev_in, hipEventDisableTiming));
  ECALL(hipEventCreateWithFlags(&e->ev_fork, hipEventDisableTiming));
  ECALL(hipEventCreateWithFlags(&e->ev_out, hipEventDisableTiming));
  for (auto& g : groups) {
    std::vector<sw_mesh_desc> md;
    std::vector<sw_params> pp;
    for (int m : g) {
      md.push_back(meshes[m]);
      pp.push_back(params[m]);
    }
    sw_ctx* c = nullptr;
    sw_status st = sw_create_batch(&c, (int32_t)g.size(), md.data(), pp.data(), stream);
    if (st != SW_OK) {
      const std::string msg = sw_last_error();
      return bail(st, msg);
    }
    e->batch.push_back(c);
    e->batch_members.push_back((int)g.size());
    hipStream_t s = nullptr;
    ECALL(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    e->bs.push_back(s);
    hipEvent_t ev = nullptr;
    ECALL(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    e->ev_join.push_back(ev);
  }
#undef ECALL
  *out = e;
  return SW_OK;
}

void sw_ens_destroy(sw_ens* e) { delete e; }

sw_status sw_ens_batches(const sw_ens* e, int32_t* n_batches) {
  if (!e || !n_batches) return efail(SW_EINVAL, "NULL argument");
  *n_batches = (int32_t)e->batch.size();
  return SW_OK;
}

sw_status sw_ens_batch(const sw_ens* e, int32_t b, sw_ctx** ctx, int32_t* n_members) {
  if (!e || !ctx) return efail(SW_EINVAL, "NULL argument");
  if (b < 0 || b >= (int32_t)e->batch.size()) return efail(SW_EINVAL, "batch index out of range");
  *ctx = e->batch[b];
  if (n_members) *n_members = e->batch_members[b];
  return SW_OK;
}

sw_status sw_ens_member(const sw_ens* e, int32_t m, int32_t* batch, int32_t* index) {
  if (!e) return efail(SW_EINVAL, "NULL argument");
  if (m < 0 || m >= (int32_t)e->mem_batch.size()) return efail(SW_EINVAL, "member index out of range");
  if (batch) *batch = e->mem_batch[m];
  if (index) *index = e->mem_index[m];
  return SW_OK;
}

sw_status sw_ens_run(sw_ens* e, int32_t n_steps, double dt, int32_t use_graph) {
  if (!e) return efail(SW_EINVAL, "NULL ensemble");
  if (n_steps < 0) return efail(SW_EINVAL, "n_steps must be >= 0");
  if (n_steps == 0) return SW_OK;
  int32_t done = 0;
  bool ready = true;
  for (auto c : e->batch) ready = ready && ctx_graph_ready(c);
  if (!use_graph || !ready) {
    // eager: all steps, or one step that brings every batch to a replayable point
    const int32_t n = use_graph ? 1 : n_steps;
    sw_status st = run_forked(e, e->user, n, dt);
    if (st != SW_OK) return st;
    done = n;
  }
  if (done == n_steps) return SW_OK;
  if (!e->exec || e->graph_dt != dt) {
    // the capture stream must see the caller's prior work before the first replay
    sw_status st = capture(e, dt);
    if (st != SW_OK) return st;
  }
  EHIP(hipEventRecord(e->ev_in, e->user));
  EHIP(hipStreamWaitEvent(e->cap, e->ev_in, 0));
  for (int32_t i = done; i < n_steps; ++i) EHIP(hipGraphLaunch(e->exec, e->cap));
  EHIP(hipEventRecord(e->ev_out, e->cap));
  EHIP(hipStreamWaitEvent(e->user, e->ev_out, 0));
  for (auto c : e->batch) ctx_set_steps(c, ctx_steps(c) + (n_steps - done));
  e->graph_launches += n_steps - done;
  return SW_OK;
}

sw_status sw_ens_step(sw_ens* e, int32_t use_graph) { return sw_ens_run(e, 1, 0.0, use_graph); }

sw_status sw_ens_autotune(sw_ens* e, int32_t steps, const char* cache_path) {
  if (!e) return efail(SW_EINVAL, "NULL ensemble");
  // cache: one line per batch class, "<key> <wavefronts per workgroup> <lanes per face>"
  std::map<std::string, std::pair<int, int>> cache;
  if (cache_path && cache_path[0]) {
    if (FILE* f = fopen(cache_path, "r")) {
      char key[128];
      int w = 0, q = 0;
      while (fscanf(f, "%127s %d %d", key, &w, &q) == 3) cache[key] = {w, q};
      fclose(f);
    }
  }
  bool changed = false;
  for (size_t b = 0; b < e->batch.size(); ++b) {
    sw_ctx* c = e->batch[b];
    int32_t S0 = 0, r = 0;
    ctx_class(c, &r, &S0);
    const std::string key = "r" + std::to_string(r) + "_S" + std::to_string(S0);
    auto it = cache.find(key);
    if (it != cache.end()) {
      sw_status st = sw_set_workgroup(c, -1, 0, it->second.first);
      if (st == SW_OK) st = sw_set_workgroup(c, -1, 1, it->second.second);
      if (st != SW_OK) return st;
      continue;
    }
    int32_t w = 0, q = 0;
    sw_status st = sw_autotune(c, steps, 0.0, &w, &q);
    if (st != SW_OK) return st;
    cache[key] = {w, q};
    changed = true;
  }
  e->drop_graph();   // a captured step holds the old launch shapes
  if (changed && cache_path && cache_path[0]) {
    if (FILE* f = fopen(cache_path, "w")) {
      for (auto& kv : cache) fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.first, kv.second.second);
      fclose(f);
    } else {
      return efail(SW_EINVAL, std::string("cannot write the autotune cache ") + cache_path);
    }
  }
  return SW_OK;
}

sw_status sw_ens_sync(sw_ens* e) {
  if (!e) return efail(SW_EINVAL, "NULL ensemble");
  EHIP(hipStreamSynchronize(e->user));
  for (auto c : e->batch) {
    sw_status st = sw_sync(c);
    if (st != SW_OK) return st;
  }
  return SW_OK;
}

}  // extern "C"
