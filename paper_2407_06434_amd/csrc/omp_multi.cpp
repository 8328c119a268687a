// Host side of the uneven-batch entry points (omp_solve_multi, omp_tune):
// several OMP problems, each with its own prepared dictionary, per-signal
// sparsity caps and tolerances, solved through the slot scheduler.
//
// Each problem owns `slots` workspace columns. The solve kernel retires a
// signal as soon as it stops (writing its outputs) and admits the next waiting
// signal into the freed slot, so finished signals stop costing correlation
// work (the compaction alternative to keeping them in the batch, Section 3.5).
// One iteration is correlation -> solve -> residual per problem; a chunk of
// iterations for all problems, each problem on its own branch, is captured
// once into a hipGraph and replayed until every signal is out. Between chunks
// the host reads the per-problem "finished" counters one chunk behind, so the
// GPU always has the next chunk queued.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <list>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/batched_omp.h"
#include "omp_internal.h"

namespace bomp {
namespace {

constexpr int CTRL_WORDS = 4;      // per problem: next signal, finished, 2 spare
constexpr int DEFAULT_CHUNK = 8;   // iterations per graph replay
constexpr int MAX_CHUNK = 64;
constexpr size_t GRAPH_CACHE = 16;

size_t align_up(size_t x) { return (x + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }

// Everything one problem's launches need; filled with memset first so that the
// raw bytes can key the graph cache.
struct Plan {
  DictView d;
  WorkView w;
  SlotView sv;
  int32_t lanes;
  int32_t pad;
  int64_t B, N, S;
  float *X_out;
  float *coef;
};

int64_t plan_slots(const omp_problem_t &p) {
  const int64_t want = p.slots > 0 ? p.slots : 4096;
  return round_up(std::max<int64_t>(1, std::min<int64_t>(want, p.B)), BPAD);
}

// Per-problem workspace: slot columns, slot table, coefficient staging when
// the caller wants no coefficients.
struct ProbLayout {
  size_t work, sig, coef, total;
};

ProbLayout prob_layout(const omp_problem_t &p, int precision) {
  const omp_dict_t *dd = p.dict;
  const int64_t slots = plan_slots(p);
  ProbLayout L;
  size_t off = 0;
  L.work = off;
  off += align_up(work_bytes(dd->M, dd->N, slots, p.S, precision, p.tile_config));
  L.sig = off;
  off += align_up((size_t)slots * sizeof(int32_t));
  L.coef = off;
  if (!p.coef_out) off += align_up((size_t)p.B * p.S * sizeof(float));
  L.total = off;
  return L;
}

int check_problem(const omp_problem_t &p, int precision) {
  const omp_dict_t *dd = p.dict;
  if (!dd || dd->magic != DICT_MAGIC || dd->precision != precision || !dd->mem) return OMP_EINVAL;
  if (!dims_ok(dd->M, dd->N)) return OMP_EINVAL;
  if (p.B < 0 || p.B > ((int64_t)1 << 26)) return OMP_EINVAL;
  if (p.S < 1 || p.S > dd->M || p.S > dd->N) return OMP_EINVAL;
  if (p.S > OMP_MAX_S) return OMP_ENOTSUPP;
  if (!solve_fits(dd->M, dd->N, plan_slots(p), p.S, precision, p.tile_config)) return OMP_ENOTSUPP;
  if (std::isnan(p.eps)) return OMP_EINVAL;
  if (p.tile_config < 0 || p.tile_config > MAX_TILE_CFG || p.slots < 0) return OMP_EINVAL;
  const int l = p.residual_lanes;
  if (l < 0 || l > 64 || (l & (l - 1))) return OMP_EINVAL;
  if (p.B > 0 && (!p.Y || p.ldy < dd->M || !aligned(p.Y, 4) || !p.support_out)) return OMP_EINVAL;
  return OMP_OK;
}

size_t total_bytes(const omp_problem_t *probs, int nprob, int precision) {
  size_t off = align_up((size_t)nprob * CTRL_WORDS * sizeof(int32_t));
  for (int p = 0; p < nprob; ++p)
    if (probs[p].B > 0) off += prob_layout(probs[p], precision).total;
  return off;
}

// A cached executable graph. `done` is recorded on the launch stream after
// every launch of `exec`, so that an evicted graph is destroyed only once its
// last launch has finished (an asynchronous omp_solve may still have it queued).
struct GraphEntry {
  std::string key;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
};

// Per-device runtime state: internal streams (default priority), events, one
// pinned host buffer for the counters and the graph cache (most recently used
// first).
struct DevState {
  hipStream_t streams[OMP_MAX_PROBLEMS] = {};
  hipEvent_t fork = nullptr, join[OMP_MAX_PROBLEMS] = {}, ready[2] = {};
  int32_t *pinned = nullptr;  // [2][OMP_MAX_PROBLEMS * CTRL_WORDS]
  std::list<GraphEntry> cache;
};

std::mutex g_mu;  // serializes omp_solve_multi / omp_tune across host threads
std::vector<DevState *> g_dev;

hipError_t dev_state(DevState **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1, nullptr);
  if (!g_dev[dev]) {
    DevState *s = new DevState();
    for (int i = 0; i < OMP_MAX_PROBLEMS && e == hipSuccess; ++i)
      e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork, hipEventDisableTiming);
    for (int i = 0; i < OMP_MAX_PROBLEMS && e == hipSuccess; ++i)
      e = hipEventCreateWithFlags(&s->join[i], hipEventDisableTiming);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&s->ready[i], hipEventDisableTiming);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void **>(&s->pinned), 2 * OMP_MAX_PROBLEMS * CTRL_WORDS * sizeof(int32_t),
                        hipHostMallocDefault);
    if (e != hipSuccess) return e;  // the partial state is kept out of the table
    g_dev[dev] = s;
  }
  *out = g_dev[dev];
  return hipSuccess;
}

// Captures `chunk` iterations of every plan: problem p's launches go to
// internal stream p, forked from and joined back into stream 0.
hipError_t capture_chunk(DevState *ds, const std::vector<Plan> &plans, int precision, int chunk,
                         hipGraphExec_t *exec) {
  hipStream_t s0 = ds->streams[0];
  hipError_t e = hipStreamBeginCapture(s0, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return e;
  const int np = (int)plans.size();
  e = hipEventRecord(ds->fork, s0);
  for (int p = 1; p < np && e == hipSuccess; ++p) e = hipStreamWaitEvent(ds->streams[p], ds->fork, 0);
  for (int it = 0; it < chunk && e == hipSuccess; ++it) {
    for (int p = 0; p < np && e == hipSuccess; ++p) {
      const Plan &q = plans[p];
      hipStream_t sp = ds->streams[p];
      e = launch_corr_select(q.d, q.w, precision, sp);
      if (e == hipSuccess) e = launch_solve_slots(q.d, q.w, q.sv, precision, sp);
      if (e == hipSuccess && !q.w.fuse_res)
        e = launch_residual_lp(q.d, q.w, precision, q.lanes, q.w.S, sp);  // slots: any k <= S
    }
  }
  for (int p = 1; p < np && e == hipSuccess; ++p) {
    e = hipEventRecord(ds->join[p], ds->streams[p]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s0, ds->join[p], 0);
  }
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(s0, &graph);  // always ends the capture
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  return e;
}

// Moves the entry under `key` to the front and returns it (nullptr: not cached).
GraphEntry *cache_find(DevState *ds, const std::string &key) {
  for (auto it = ds->cache.begin(); it != ds->cache.end(); ++it) {
    if (it->key == key) {
      ds->cache.splice(ds->cache.begin(), ds->cache, it);
      return &ds->cache.front();
    }
  }
  return nullptr;
}

// Caches a newly instantiated graph under `key`, evicting the least recently
// used entries beyond GRAPH_CACHE: each evicted graph's last launch is waited
// for before the graph is destroyed.
hipError_t cache_insert(DevState *ds, std::string key, hipGraphExec_t g, GraphEntry **out) {
  GraphEntry ent;
  ent.key = std::move(key);
  ent.exec = g;
  hipError_t e = hipEventCreateWithFlags(&ent.done, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipGraphExecDestroy(g);
    return e;
  }
  ds->cache.push_front(std::move(ent));
  while (ds->cache.size() > GRAPH_CACHE) {
    GraphEntry &old = ds->cache.back();
    e = hipEventSynchronize(old.done);  // an event never recorded completes at once
    if (e != hipSuccess) return e;      // kept: it may still be in flight
    (void)hipGraphExecDestroy(old.exec);
    (void)hipEventDestroy(old.done);
    ds->cache.pop_back();
  }
  *out = &ds->cache.front();
  return hipSuccess;
}

// Launches a cached graph on `st` and marks its completion on that stream.
hipError_t cache_launch(GraphEntry *ent, hipStream_t st) {
  hipError_t e = hipGraphLaunch(ent->exec, st);
  if (e == hipSuccess) e = hipEventRecord(ent->done, st);
  return e;
}

// Looks `key` up in the device's graph cache; on a miss, runs `body` under
// stream capture on internal stream 0 and caches the instantiated graph.
hipError_t cached_graph_body(DevState *ds, const std::string &key,
                             const std::function<hipError_t(hipStream_t)> &body, GraphEntry **out) {
  if ((*out = cache_find(ds, key)) != nullptr) return hipSuccess;
  hipStream_t s0 = ds->streams[0];
  hipError_t e = hipStreamBeginCapture(s0, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return e;
  e = body(s0);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(s0, &graph);  // always ends the capture
  if (e == hipSuccess) e = e2;
  hipGraphExec_t g = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  return cache_insert(ds, key, g, out);
}

hipError_t cached_graph(DevState *ds, const std::vector<Plan> &plans, int precision, int chunk, GraphEntry **out) {
  std::string key("M");
  key.append(reinterpret_cast<const char *>(plans.data()), plans.size() * sizeof(Plan));
  key.append(reinterpret_cast<const char *>(&precision), sizeof(precision));
  key.append(reinterpret_cast<const char *>(&chunk), sizeof(chunk));
  // the chunk is captured by capture_chunk (its own fork/join over the problem streams)
  if ((*out = cache_find(ds, key)) != nullptr) return hipSuccess;
  hipGraphExec_t g = nullptr;
  hipError_t e = capture_chunk(ds, plans, precision, chunk, &g);
  if (e != hipSuccess) return e;
  return cache_insert(ds, std::move(key), g, out);
}

int solve_multi_locked(const omp_problem_t *probs, int nprob, const omp_multi_opts_t *opts, void *stream) {
  const int prec = opts->precision;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *ws = static_cast<char *>(opts->workspace);
  int32_t *ctrl = reinterpret_cast<int32_t *>(ws);
  const int chunk = opts->iters_per_graph > 0 ? opts->iters_per_graph : DEFAULT_CHUNK;

  // ---- plans (problems with signals only) ----
  std::vector<Plan> plans;
  std::vector<int> ctrl_of;  // ctrl slot of each plan
  size_t off = align_up((size_t)nprob * CTRL_WORDS * sizeof(int32_t));
  int64_t bound = 0;
  for (int p = 0; p < nprob; ++p) {
    const omp_problem_t &pr = probs[p];
    if (pr.B == 0) continue;
    const omp_dict_t *dd = pr.dict;
    const ProbLayout L = prob_layout(pr, prec);
    const int64_t slots = plan_slots(pr);
    Plan q;
    std::memset(&q, 0, sizeof(q));
    q.d = dict_view(dd->mem, dd->M, dd->N, prec);
    q.w = work_view(ws + off + L.work, dd->M, dd->N, slots, pr.S, prec, pr.tile_config);
    // the same choice as omp_solve on this problem's signals, so results stay bit-identical to it
    q.w.fuse_res = residual_in_solve(q.d, pr.B) ? 1 : 0;
    q.sv.sig = reinterpret_cast<int32_t *>(ws + off + L.sig);
    q.sv.ctrl = ctrl + (size_t)p * CTRL_WORDS;
    q.sv.Y = pr.Y;
    q.sv.ldy = pr.ldy;
    q.sv.M = dd->M;
    q.sv.nsig = pr.B;
    q.sv.S_per = pr.S_per_signal;
    q.sv.eps_per = pr.eps_per_signal;
    q.sv.eps = pr.eps;
    q.sv.support_out = pr.support_out;
    q.sv.coef_out = pr.coef_out ? pr.coef_out : reinterpret_cast<float *>(ws + off + L.coef);
    q.sv.status_out = pr.status_out;
    q.sv.rnorm_out = pr.rnorm_out;
    q.lanes = pr.residual_lanes;
    q.B = pr.B;
    q.N = dd->N;
    q.S = pr.S;
    q.X_out = pr.X_out;
    q.coef = q.sv.coef_out;
    plans.push_back(q);
    ctrl_of.push_back(p);
    off += L.total;
    bound = std::max<int64_t>(bound, (pr.B + slots - 1) / slots * (pr.S + 2) + pr.S + 2);
  }
  if (opts->iterations) *opts->iterations = 0;
  if (opts->elapsed_ms) *opts->elapsed_ms = 0.f;
  if (plans.empty()) return OMP_OK;

  DevState *ds = nullptr;
  hipError_t e = dev_state(&ds);
  if (e != hipSuccess) return device_error(e);
  for (const Plan &q : plans) {
    e = prepare_kernels(q.d, q.w, prec, q.lanes);
    if (e != hipSuccess) return device_error(e);
  }
  GraphEntry *graph = nullptr;
  e = cached_graph(ds, plans, prec, chunk, &graph);
  if (e != hipSuccess) return device_error(e);

  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (opts->elapsed_ms) {
    e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e == hipSuccess) e = hipEventRecord(t0, st);
  }
  for (size_t i = 0; i < plans.size() && e == hipSuccess; ++i) e = launch_init_slots(plans[i].w, plans[i].sv, st);

  // ---- chunks: replay, copy the counters, look at the previous chunk's ----
  const size_t nctrl = (size_t)nprob * CTRL_WORDS;
  int64_t c = 0;
  bool done = false;
  while (e == hipSuccess && !done) {
    e = cache_launch(graph, st);
    int32_t *buf = ds->pinned + (size_t)(c & 1) * OMP_MAX_PROBLEMS * CTRL_WORDS;
    if (e == hipSuccess) e = hipMemcpyAsync(buf, ctrl, nctrl * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(ds->ready[c & 1], st);
    if (e == hipSuccess && c >= 1) {
      e = hipEventSynchronize(ds->ready[(c - 1) & 1]);
      const int32_t *prev = ds->pinned + (size_t)((c - 1) & 1) * OMP_MAX_PROBLEMS * CTRL_WORDS;
      done = true;
      for (size_t i = 0; i < plans.size(); ++i)
        if (prev[(size_t)ctrl_of[i] * CTRL_WORDS + 1] < plans[i].B) done = false;
    }
    ++c;
    if (!done && c * chunk > bound + 2 * chunk) {
      (void)hipStreamSynchronize(st);
      return device_error(hipErrorLaunchTimeOut);  // signals still running past the iteration bound
    }
  }
  for (size_t i = 0; i < plans.size() && e == hipSuccess; ++i)
    if (plans[i].X_out)
      e = launch_densify(plans[i].sv.support_out, plans[i].coef, plans[i].B, (int)plans[i].S, plans[i].N,
                         plans[i].X_out, st);
  if (e == hipSuccess && t1) e = hipEventRecord(t1, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && t1) e = hipEventElapsedTime(opts->elapsed_ms, t0, t1);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (opts->iterations) *opts->iterations = (int32_t)(c * chunk);
  if (e != hipSuccess) return device_error(e);
  return OMP_OK;
}

int validate(const omp_problem_t *probs, int nprob, const omp_multi_opts_t *opts) {
  if (!probs || !opts || nprob < 1 || nprob > OMP_MAX_PROBLEMS) return OMP_EINVAL;
  if (opts->precision != OMP_PREC_FP32 && !is_half(opts->precision)) return OMP_EINVAL;
  if (opts->iters_per_graph < 0 || opts->iters_per_graph > MAX_CHUNK) return OMP_EINVAL;
  for (int p = 0; p < nprob; ++p) {
    const int rc = check_problem(probs[p], opts->precision);
    if (rc != OMP_OK) return rc;
  }
  const size_t need = total_bytes(probs, nprob, opts->precision);
  if (!opts->workspace || opts->workspace_bytes < need || !aligned(opts->workspace, WS_ALIGN)) return OMP_EWORKSPACE;
  return OMP_OK;
}

}  // namespace

hipError_t graph_launch_cached(const std::string &key, const std::function<hipError_t(hipStream_t)> &body,
                               hipStream_t st) {
  std::lock_guard<std::mutex> lock(g_mu);
  DevState *ds = nullptr;
  hipError_t e = dev_state(&ds);
  if (e != hipSuccess) return e;
  GraphEntry *graph = nullptr;
  e = cached_graph_body(ds, "S" + key, body, &graph);
  if (e != hipSuccess) return e;
  return cache_launch(graph, st);
}

}  // namespace bomp

using namespace bomp;

extern "C" {

size_t omp_multi_workspace_size(const omp_problem_t *probs, int32_t nprob, const omp_multi_opts_t *opts) {
  if (!probs || !opts || nprob < 1 || nprob > OMP_MAX_PROBLEMS) return 0;
  if (opts->precision != OMP_PREC_FP32 && !is_half(opts->precision)) return 0;
  for (int p = 0; p < nprob; ++p)
    if (check_problem(probs[p], opts->precision) != OMP_OK) return 0;
  return total_bytes(probs, nprob, opts->precision);
}

int omp_solve_multi(const omp_problem_t *probs, int32_t nprob, const omp_multi_opts_t *opts, void *stream) {
  int rc = validate(probs, nprob, opts);
  if (rc != OMP_OK) return rc;
  bool any = false;
  for (int p = 0; p < nprob; ++p) any |= probs[p].B > 0;
  if (!any) {
    if (opts->iterations) *opts->iterations = 0;
    if (opts->elapsed_ms) *opts->elapsed_ms = 0.f;
    return OMP_OK;
  }
  rc = check_device();
  if (rc != OMP_OK) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  return solve_multi_locked(probs, nprob, opts, stream);
}

int omp_tune(omp_problem_t *probs, int32_t nprob, const omp_multi_opts_t *opts, int64_t sample, void *stream) {
  int rc = validate(probs, nprob, opts);
  if (rc != OMP_OK) return rc;
  if (sample < 0) return OMP_EINVAL;
  rc = check_device();
  if (rc != OMP_OK) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  for (int p = 0; p < nprob; ++p) {
    omp_problem_t &pr = probs[p];
    if (pr.B == 0) continue;
    omp_problem_t trial = pr;
    trial.B = std::min<int64_t>(pr.B, sample > 0 ? sample : 8192);
    const int64_t max_slots =
        round_up(std::max<int64_t>(1, std::min<int64_t>(pr.slots > 0 ? pr.slots : 8192, trial.B)), BPAD);
    omp_multi_opts_t o = *opts;
    float ms = 0.f;
    int32_t iters = 0;
    o.elapsed_ms = &ms;
    o.iterations = &iters;
    // Times one candidate (second run: the first captures its graph); +inf if
    // it does not fit the workspace.
    auto time_one = [&](const omp_problem_t &cand, float *out) -> int {
      *out = INFINITY;
      if (total_bytes(&cand, 1, o.precision) > o.workspace_bytes) return OMP_OK;
      for (int rep = 0; rep < 2; ++rep) {
        const int r = solve_multi_locked(&cand, 1, &o, stream);
        if (r != OMP_OK) return r;
      }
      *out = ms;
      return OMP_OK;
    };
    // Coordinate search: tile configuration, then slots, then residual lanes.
    omp_problem_t best = trial;
    best.slots = (int32_t)std::min<int64_t>(max_slots, 4096);
    float best_ms = INFINITY;
    for (int cfg : {1, 3, 4}) {
      omp_problem_t c = best;
      c.tile_config = cfg;
      float t;
      if ((rc = time_one(c, &t)) != OMP_OK) return rc;
      if (t < best_ms) best_ms = t, best = c;
    }
    for (int64_t sl = 1024; sl <= max_slots; sl *= 2) {
      omp_problem_t c = best;
      c.slots = (int32_t)sl;
      float t;
      if ((rc = time_one(c, &t)) != OMP_OK) return rc;
      if (t < best_ms) best_ms = t, best = c;
    }
    {
      const int64_t Mp = round_up(pr.dict->M, KPAD);
      const int nslice = (round_up(pr.dict->N, NPAD) * Mp * 4 > (int64_t)2 << 20) ? NSLICE_MAX : 1;
      int lp = 1;
      while (lp < Mp / nslice / 4 && lp < 64) lp *= 2;
      for (int l : {lp, std::max(1, lp / 2), std::max(1, lp / 4)}) {
        omp_problem_t c = best;
        c.residual_lanes = l;
        float t;
        if ((rc = time_one(c, &t)) != OMP_OK) return rc;
        if (t < best_ms) best_ms = t, best = c;
      }
    }
    if (!std::isfinite(best_ms)) return OMP_EWORKSPACE;
    pr.tile_config = best.tile_config;
    pr.slots = best.slots;
    pr.residual_lanes = best.residual_lanes;
  }
  return OMP_OK;
}

}  // extern "C"
