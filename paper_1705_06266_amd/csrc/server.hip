// server.hip -- continuous-batching solve server over a pool of graphs.
//
// Requests (graph, right-hand sides, tolerance) arrive at any time.  Worker
// threads, each with its own HIP stream, take the oldest request whose graph
// is idle together with every other queued request for that graph (same
// tolerance and iteration cap, up to max_batch_rhs columns) and solve them as
// one batched lg_solve, so requests that arrive while others run join the
// next batch of their graph and different graphs overlap on the device.
// Hierarchies are built on a graph's first request and stay resident; a
// graph is admitted when its hierarchy fits the HBM budget after evicting
// the least recently used idle ones (one that cannot fit runs alone).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "impl.h"

namespace {

__global__ void k_pack_cols(const double* __restrict__ src, int64_t n, int k,
                            double* __restrict__ dst, int K, int off) {
  const int64_t i = (int64_t)blockIdx.x * lg::kBlock + threadIdx.x;
  if (i >= n * k) return;
  const int64_t row = i / k;
  dst[row * K + off + (i - row * k)] = src[i];
}

__global__ void k_unpack_cols(const double* __restrict__ src, int64_t n, int K, int off,
                              double* __restrict__ dst, int k) {
  const int64_t i = (int64_t)blockIdx.x * lg::kBlock + threadIdx.x;
  if (i >= n * k) return;
  const int64_t row = i / k;
  dst[i] = src[row * K + off + (i - row * k)];
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct GraphEntry {
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  std::vector<double> w;
  lg_hierarchy* h = nullptr;
  size_t bytes = 0;     // measured once built; an estimate before
  size_t reserved = 0;  // admission estimate held while its hierarchy is being built
  uint64_t last_use = 0;
  bool busy = false;
  lg_status failed = LG_OK;  // sticky setup failure (invalid or disconnected graph)
  std::string error;
};

struct Request {
  int64_t id = 0;
  int32_t gid = 0;
  const double* B = nullptr;
  double* X = nullptr;
  int k = 0;
  double rtol = 0.0;
  int max_iter = 0;
  double t_submit = 0.0, t_done = 0.0;
  bool done = false;
  lg_status status = LG_OK;
  std::string error;
  std::vector<lg_rhs_info> info;
};

// Device bytes a hierarchy is expected to take before it is built: the
// finest level's CSR, values and schedules, coarse levels (bounded by the
// finest), and the solve workspace for K columns.
size_t estimate_bytes(int64_t n, int64_t nnz, int K) {
  return (size_t)(48.0 * (double)nnz + (160.0 + 120.0 * K) * (double)n) + ((size_t)64 << 20);
}

}  // namespace

struct lg_server {
  lg_server_opts opts{};
  int device = 0;
  int K = 1;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::vector<std::unique_ptr<GraphEntry>> graphs;
  std::deque<Request*> pending;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_id = 1;
  uint64_t clock = 0;
  size_t resident = 0;  // built hierarchies
  size_t reserved = 0;  // hierarchies being built (admission estimates)
  lg_server_stats st{};
  std::vector<std::thread> workers;

  bool pickable() const {
    for (const Request* r : pending)
      if (!graphs[r->gid]->busy) return true;
    return false;
  }

  // Admission of graph gid (not resident): true if its hierarchy fits the
  // budget after freeing idle hierarchies, least recently used first (then
  // they are freed), or if nothing else is resident or running (a hierarchy
  // larger than the budget runs alone).  Caller holds mu.
  bool admit(int32_t gid) {
    GraphEntry* e = graphs[gid].get();
    const size_t need = e->bytes ? e->bytes : estimate_bytes(e->n, e->nnz, K);
    size_t idle = 0;
    for (size_t g = 0; g < graphs.size(); g++)
      if ((int32_t)g != gid && graphs[g]->h && !graphs[g]->busy) idle += graphs[g]->bytes;
    const bool fits = resident + reserved - idle + need <= budget;
    if (!fits && others_running(gid)) return false;
    while (resident + reserved + need > budget) {
      GraphEntry* victim = nullptr;
      for (size_t g = 0; g < graphs.size(); g++) {
        GraphEntry* v = graphs[g].get();
        if ((int32_t)g == gid || !v->h || v->busy) continue;
        if (!victim || v->last_use < victim->last_use) victim = v;
      }
      if (!victim) break;
      lg_free(victim->h);
      victim->h = nullptr;
      resident -= victim->bytes;
      st.evictions++;
    }
    e->reserved = need;
    reserved += need;
    return true;
  }

  bool others_running(int32_t gid) const {
    for (size_t g = 0; g < graphs.size(); g++)
      if ((int32_t)g != gid && graphs[g]->busy) return true;
    return false;
  }

  void finish(std::vector<Request*>& batch, GraphEntry& G) {
    const double t = now_ms();
    for (Request* r : batch) {
      r->t_done = t;
      r->done = true;
    }
    G.busy = false;
    G.last_use = ++clock;
    st.completed += (int64_t)batch.size();
    cv_done.notify_all();
    cv_work.notify_all();
  }

  void worker() {
    (void)hipSetDevice(device);
    hipStream_t strm = nullptr;
    if (hipStreamCreateWithFlags(&strm, hipStreamNonBlocking) != hipSuccess) strm = nullptr;
    double* stage = nullptr;  // n x K batch input and output
    size_t stage_rows = 0;
    std::vector<lg_rhs_info> info;
    for (;;) {
      std::vector<Request*> batch;
      GraphEntry* G = nullptr;
      int32_t gid = -1;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return (stop && pending.empty()) || pickable(); });
        if (stop && pending.empty()) break;
        // the oldest request whose graph is idle and resident, or admissible
        Request* first = nullptr;
        for (Request* r : pending) {
          GraphEntry* e = graphs[r->gid].get();
          if (e->busy) continue;
          if (e->h || e->failed != LG_OK || admit(r->gid)) {
            first = r;
            break;
          }
        }
        if (!first) {  // every candidate waits for memory held by running batches
          cv_done.wait_for(lk, std::chrono::milliseconds(5));
          continue;
        }
        gid = first->gid;
        G = graphs[gid].get();
        G->busy = true;
        int cols = 0;
        for (auto it = pending.begin(); it != pending.end();) {
          Request* r = *it;
          if (r->gid == gid && r->rtol == first->rtol && r->max_iter == first->max_iter &&
              cols + r->k <= opts.max_batch_rhs) {
            batch.push_back(r);
            cols += r->k;
            it = pending.erase(it);
          } else {
            ++it;
          }
        }
      }
      run_batch(*G, gid, batch, strm, stage, stage_rows, info);
      std::lock_guard<std::mutex> lk(mu);
      finish(batch, *G);
    }
    if (stage) (void)hipFree(stage);
    if (strm) (void)hipStreamDestroy(strm);
  }

  void fail_batch(std::vector<Request*>& batch, lg_status s, const std::string& msg) {
    for (Request* r : batch) {
      r->status = s;
      r->error = msg;
    }
  }

  // Builds the hierarchy if needed, then one batched solve.  Runs without mu
  // except for the bookkeeping of resident bytes.
  void run_batch(GraphEntry& G, int32_t gid, std::vector<Request*>& batch, hipStream_t strm,
                 double*& stage, size_t& stage_rows, std::vector<lg_rhs_info>& info) {
    if (G.failed != LG_OK) {
      fail_batch(batch, G.failed, G.error);
      return;
    }
    if (!G.h) {
      lg_graph g{G.n, G.nnz, G.rp.data(), G.col.data(), G.w.data(), 0};
      lg_setup_opts o = opts.setup;
      o.max_rhs = opts.max_batch_rhs;
      lg_hierarchy* h = nullptr;
      const lg_status s = lg_setup(&g, &o, strm, &h);
      std::lock_guard<std::mutex> lk(mu);
      reserved -= G.reserved;
      G.reserved = 0;
      if (s != LG_OK) {
        G.failed = s;
        G.error = lg_last_error();
        fail_batch(batch, s, G.error);
        return;
      }
      G.h = h;
      G.bytes = lg_hierarchy_bytes(h);
      resident += G.bytes;
      st.setups++;
    }
    int cols = 0;
    for (Request* r : batch) cols += r->k;
    const double* B = batch[0]->B;
    double* X = batch[0]->X;
    const int64_t n = G.n;
    if (batch.size() > 1) {
      if (stage_rows < (size_t)n) {
        if (stage) (void)hipFree(stage);
        stage = nullptr;
        stage_rows = 0;
        if (hipMalloc((void**)&stage, sizeof(double) * (size_t)n * opts.max_batch_rhs * 2) !=
            hipSuccess) {
          stage = nullptr;
          fail_batch(batch, LG_E_NOMEM, "server: staging allocation failed");
          return;
        }
        stage_rows = (size_t)n;
      }
      double* Bs = stage;
      double* Xs = stage + (size_t)n * opts.max_batch_rhs;
      int off = 0;
      for (Request* r : batch) {
        const unsigned blocks = (unsigned)lg::ceil_div(n * r->k, (int64_t)lg::kBlock);
        hipLaunchKernelGGL(k_pack_cols, dim3(blocks), dim3(lg::kBlock), 0, strm, r->B, n, r->k, Bs,
                           cols, off);
        off += r->k;
      }
      B = Bs;
      X = Xs;
    }
    info.assign(cols, lg_rhs_info{});
    const lg_status s = lg_solve(G.h, B, X, cols, batch[0]->rtol, batch[0]->max_iter, strm,
                                 info.data());
    std::string msg = s == LG_OK || s == LG_E_NOT_CONVERGED ? "" : lg_last_error();
    if (s != LG_OK && s != LG_E_NOT_CONVERGED) {
      fail_batch(batch, s, msg);
      return;
    }
    int off = 0;
    for (Request* r : batch) {
      if (batch.size() > 1) {
        const unsigned blocks = (unsigned)lg::ceil_div(n * r->k, (int64_t)lg::kBlock);
        hipLaunchKernelGGL(k_unpack_cols, dim3(blocks), dim3(lg::kBlock), 0, strm, X, n, cols, off,
                           r->X, r->k);
      }
      r->info.assign(info.begin() + off, info.begin() + off + r->k);
      r->status = LG_OK;
      for (const lg_rhs_info& c : r->info)
        if (!(c.rel_residual <= r->rtol)) r->status = LG_E_NOT_CONVERGED;
      off += r->k;
    }
    if (hipStreamSynchronize(strm) != hipSuccess) fail_batch(batch, LG_E_HIP, "server: stream error");
    std::lock_guard<std::mutex> lk(mu);
    st.batches++;
    st.batched_columns += cols;
    (void)gid;
  }
};

namespace {
lg_status server_arg_error(const char* msg) {
  lg::set_last_error(msg);
  return LG_E_ARG;
}
}  // namespace

extern "C" lg_status lg_server_default_opts(lg_server_opts* o) {
  if (!o) return server_arg_error("lg_server_default_opts: null options");
  std::memset(o, 0, sizeof(*o));
  o->workers = 4;
  o->max_batch_rhs = 32;
  o->hbm_budget = 0;
  return lg_default_opts(&o->setup);
}

extern "C" lg_status lg_server_create(const lg_server_opts* o, lg_server** out) {
  if (!out) return server_arg_error("lg_server_create: null output");
  *out = nullptr;
  lg_server_opts opts;
  if (o) opts = *o;
  else lg_server_default_opts(&opts);
  if (opts.workers < 1 || opts.workers > 64) return server_arg_error("workers must be in 1..64");
  if (opts.max_batch_rhs < 1 || opts.max_batch_rhs > 32)
    return server_arg_error("max_batch_rhs must be in 1..32");
  try {
    auto s = std::make_unique<lg_server>();
    s->opts = opts;
    if (hipGetDevice(&s->device) != hipSuccess) {
      lg::set_last_error("lg_server_create: no HIP device");
      return LG_E_HIP;
    }
    int K = 1;
    while (K < opts.max_batch_rhs) K <<= 1;
    s->K = K;
    s->budget = opts.hbm_budget;
    if (s->budget == 0) {
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        lg::set_last_error("lg_server_create: hipMemGetInfo failed");
        return LG_E_HIP;
      }
      s->budget = free_b / 4 * 3;
    }
    lg_server* raw = s.get();
    for (int i = 0; i < opts.workers; i++) s->workers.emplace_back([raw] { raw->worker(); });
    *out = s.release();
    return LG_OK;
  } catch (const std::exception&) {
    lg::set_last_error("lg_server_create: could not start workers");
    return LG_E_NOMEM;
  }
}

extern "C" lg_status lg_server_add_graph(lg_server* s, const lg_graph* g, int32_t* graph_id) {
  if (!s || !g || !graph_id) return server_arg_error("lg_server_add_graph: null argument");
  if (g->n < 1 || g->nnz < 0 || !g->row_ptr || (g->nnz > 0 && (!g->col || !g->w)))
    return server_arg_error("lg_server_add_graph: bad graph");
  try {
    auto e = std::make_unique<GraphEntry>();
    e->n = g->n;
    e->nnz = g->nnz;
    e->rp.resize(g->n + 1);
    e->col.resize(g->nnz);
    e->w.resize(g->nnz);
    const hipMemcpyKind kind = g->on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    if (hipMemcpy(e->rp.data(), g->row_ptr, sizeof(int64_t) * (g->n + 1), kind) != hipSuccess ||
        (g->nnz > 0 &&
         (hipMemcpy(e->col.data(), g->col, sizeof(int32_t) * g->nnz, kind) != hipSuccess ||
          hipMemcpy(e->w.data(), g->w, sizeof(double) * g->nnz, kind) != hipSuccess))) {
      lg::set_last_error("lg_server_add_graph: copy failed");
      return LG_E_HIP;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    *graph_id = (int32_t)s->graphs.size();
    s->graphs.push_back(std::move(e));
    return LG_OK;
  } catch (const std::bad_alloc&) {
    lg::set_last_error("lg_server_add_graph: host allocation failed");
    return LG_E_NOMEM;
  }
}

extern "C" lg_status lg_server_submit(lg_server* s, int32_t graph_id, const double* B, double* X,
                                      int32_t k, double rtol, int32_t max_iter,
                                      int64_t* request_id) {
  if (!s || !B || !X || !request_id) return server_arg_error("lg_server_submit: null argument");
  if (!(rtol > 0.0) || max_iter < 0) return server_arg_error("lg_server_submit: need rtol > 0, max_iter >= 0");
  std::lock_guard<std::mutex> lk(s->mu);
  if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size())
    return server_arg_error("lg_server_submit: unknown graph");
  if (k < 1 || k > s->opts.max_batch_rhs) return server_arg_error("lg_server_submit: k must be in 1..max_batch_rhs");
  if (s->stop) return server_arg_error("lg_server_submit: server is shutting down");
  auto r = std::make_unique<Request>();
  r->id = s->next_id++;
  r->gid = graph_id;
  r->B = B;
  r->X = X;
  r->k = k;
  r->rtol = rtol;
  r->max_iter = max_iter;
  r->t_submit = now_ms();
  *request_id = r->id;
  s->pending.push_back(r.get());
  s->reqs.emplace(r->id, std::move(r));
  s->st.submitted++;
  s->cv_work.notify_one();
  return LG_OK;
}

extern "C" lg_status lg_server_wait(lg_server* s, int64_t request_id, lg_rhs_info* info,
                                    double* latency_ms) {
  if (!s) return server_arg_error("lg_server_wait: null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(request_id);
  if (it == s->reqs.end()) return server_arg_error("lg_server_wait: unknown request");
  Request* r = it->second.get();
  s->cv_done.wait(lk, [&] { return r->done; });
  if (info)
    for (size_t c = 0; c < r->info.size(); c++) info[c] = r->info[c];
  if (latency_ms) *latency_ms = r->t_done - r->t_submit;
  const lg_status st = r->status;
  if (st != LG_OK) lg::set_last_error(r->error.empty() ? lg_status_str(st) : r->error.c_str());
  s->reqs.erase(it);
  return st;
}

extern "C" lg_status lg_server_stats_get(lg_server* s, lg_server_stats* out) {
  if (!s || !out) return server_arg_error("lg_server_stats_get: null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->resident_bytes = s->resident;
  int32_t rg = 0;
  for (auto& g : s->graphs) rg += g->h ? 1 : 0;
  out->resident_graphs = rg;
  out->budget_bytes = s->budget;
  return LG_OK;
}

extern "C" void lg_server_free(lg_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& g : s->graphs)
    if (g->h) lg_free(g->h);
  delete s;
}
