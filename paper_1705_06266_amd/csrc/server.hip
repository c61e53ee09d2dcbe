// server.hip -- continuous-batching solve server over a pool of graphs.
//
// Requests (graph, right-hand sides, tolerance) arrive at any time.  A worker
// thread (each with its own HIP stream) opens a session on the graph of the
// oldest waiting request: one batched CG whose columns are slots.  At every CG
// iteration boundary the columns that have converged leave (their request
// completes once all its columns have), and the freed slots take the next
// queued requests for the same graph, tolerance and iteration cap, so requests
// are admitted as slots free up instead of waiting for a whole batch; sessions
// on different graphs overlap on the device.  Hierarchies are built on a
// graph's first request and stay resident; a graph is admitted when its
// hierarchy fits the HBM budget after evicting the least recently used idle
// ones (one that cannot fit runs alone).
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
  int cols_left = 0;  // columns still in a session's slots
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
  int idle_workers = 0;  // workers waiting for work
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

  // Does request r (for a running session on gid) go ahead of every waiting
  // request of another graph that no worker is free to take?  Keeps one
  // graph's stream of requests from starving the others.  Caller holds mu.
  bool may_join(const Request* r) const {
    if (idle_workers > 0) return true;
    for (const Request* q : pending) {
      if (q == r) return true;
      if (q->gid != r->gid && !graphs[q->gid]->busy) return false;
    }
    return true;
  }

  struct Session;  // the slot feed of one worker's batched solve

  void worker() {
    (void)hipSetDevice(device);
    hipStream_t strm = nullptr;
    if (hipStreamCreateWithFlags(&strm, hipStreamNonBlocking) != hipSuccess) strm = nullptr;
    for (;;) {
      std::vector<Request*> first;
      GraphEntry* G = nullptr;
      int32_t gid = -1;
      int width = 1;
      {
        std::unique_lock<std::mutex> lk(mu);
        idle_workers++;
        cv_work.wait(lk, [&] { return (stop && pending.empty()) || pickable(); });
        if (stop && pending.empty()) {
          idle_workers--;
          break;
        }
        // the oldest request whose graph is idle and resident, or admissible
        Request* head = nullptr;
        for (Request* r : pending) {
          GraphEntry* e = graphs[r->gid].get();
          if (e->busy) continue;
          if (e->h || e->failed != LG_OK || admit(r->gid)) {
            head = r;
            break;
          }
        }
        if (!head) {  // every candidate waits for memory held by running sessions
          idle_workers--;
          cv_done.wait_for(lk, std::chrono::milliseconds(5));
          continue;
        }
        idle_workers--;
        gid = head->gid;
        G = graphs[gid].get();
        G->busy = true;
        // session width: the columns queued for this graph now (at least the
        // head request's), rounded up to a power of two
        int cols = 0;
        for (Request* r : pending)
          if (r->gid == gid && r->rtol == head->rtol && r->max_iter == head->max_iter) cols += r->k;
        cols = std::min(std::max(cols, head->k), opts.max_batch_rhs);
        while (width < cols) width <<= 1;
        first.push_back(head);
        pending.erase(std::find(pending.begin(), pending.end(), head));
      }
      run_session(*G, gid, first, width, strm);
      std::lock_guard<std::mutex> lk(mu);
      G->busy = false;
      G->last_use = ++clock;
      cv_work.notify_all();
    }
    if (strm) (void)hipStreamDestroy(strm);
  }

  void complete(Request* r) {  // caller holds mu
    r->t_done = now_ms();
    r->done = true;
    st.completed++;
    cv_done.notify_all();
  }

  void fail_request(Request* r, lg_status s, const std::string& msg) {  // caller holds mu
    r->status = s;
    r->error = msg;
    r->info.assign(r->k, lg_rhs_info{});
    complete(r);
  }

  // Builds the hierarchy if needed, then one slot-batched solve that keeps
  // taking this graph's requests while it runs.
  void run_session(GraphEntry& G, int32_t gid, std::vector<Request*>& first, int width,
                   hipStream_t strm);
};

struct lg_server::Session : lg::SlotFeed {
  lg_server* s;
  int32_t gid;
  double rtol;
  int max_iter;
  std::vector<Request*> initial;
  std::vector<std::pair<Request*, int>> slot_col;  // request and column in each slot
  int64_t columns = 0;

  void refill(const std::vector<int>& free_slots, std::vector<Col>& out) override {
    std::lock_guard<std::mutex> lk(s->mu);
    size_t next = 0;
    auto place = [&](Request* r) {
      r->cols_left = r->k;
      r->info.assign(r->k, lg_rhs_info{});
      r->status = LG_OK;
      for (int j = 0; j < r->k; j++) {
        const int slot = free_slots[next++];
        slot_col[slot] = {r, j};
        out.push_back(Col{slot, r->B + j, r->k, r->X + j, r->k});
      }
      columns += r->k;
    };
    const bool opening = !initial.empty();
    for (Request* r : initial) place(r);  // the session's first requests
    initial.clear();
    if (s->stop && s->pending.empty()) return;
    for (auto it = s->pending.begin(); it != s->pending.end();) {
      Request* r = *it;
      // opening: every queued request of the graph that fits (batch formation);
      // later, a request joins unless another graph has waited longer with no
      // worker free to take it
      if (r->gid == gid && r->rtol == rtol && r->max_iter == max_iter &&
          (size_t)r->k <= free_slots.size() - next && (opening || s->may_join(r))) {
        it = s->pending.erase(it);
        place(r);
        if (!opening) s->st.refills += r->k;
      } else {
        ++it;
      }
    }
  }

  void finished(int slot, const lg_rhs_info& info) override {
    std::lock_guard<std::mutex> lk(s->mu);
    auto [r, j] = slot_col[slot];
    slot_col[slot] = {nullptr, 0};
    r->info[j] = info;
    if (!(info.rel_residual <= rtol)) r->status = LG_E_NOT_CONVERGED;
    if (--r->cols_left == 0) s->complete(r);
  }
};

void lg_server::run_session(GraphEntry& G, int32_t gid, std::vector<Request*>& first, int width,
                            hipStream_t strm) {
  if (G.failed == LG_OK && !G.h) {
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
    } else {
      G.h = h;
      G.bytes = lg_hierarchy_bytes(h);
      resident += G.bytes;
      st.setups++;
    }
  }
  if (G.failed != LG_OK) {
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : first) fail_request(r, G.failed, G.error);
    return;
  }
  Session sess;
  sess.s = this;
  sess.gid = gid;
  sess.rtol = first[0]->rtol;
  sess.max_iter = first[0]->max_iter;
  sess.initial = first;
  sess.slot_col.assign(width, {nullptr, 0});
  lg_status status = LG_OK;
  std::string msg;
  try {
    status = lg::solve_slots(G.h, width, sess.rtol, sess.max_iter, strm, &sess);
  } catch (const lg::Error& e) {
    status = e.code;
    msg = e.msg;
  } catch (...) {
    status = LG_E_HIP;
    msg = "server: unexpected error in a session";
  }
  std::lock_guard<std::mutex> lk(mu);
  if (status != LG_OK) {  // requests still in slots or never placed fail
    for (auto& [r, j] : sess.slot_col)
      if (r && !r->done) fail_request(r, status, msg);
    for (Request* r : sess.initial) fail_request(r, status, msg);
  }
  st.batches++;
  st.batched_columns += sess.columns;
}

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
