// capi.hip -- extern "C" entry points of liblgmg.so (declared in lgmg.h).
// Internal failures are C++ exceptions (lg::Error); every entry point turns
// them into an lg_status and a per-thread message.
#include <chrono>
#include <cstring>
#include <new>
#include <vector>

#include "impl.h"

using lg::Level;

#define LG_API_BEGIN try {
#define LG_API_END                                                   \
  }                                                                  \
  catch (const lg::Error& e) {                                       \
    lg::set_last_error(e.msg);                                       \
    return e.code;                                                   \
  }                                                                  \
  catch (const std::bad_alloc&) {                                    \
    lg::set_last_error("host allocation failed");                    \
    return LG_E_NOMEM;                                               \
  }                                                                  \
  catch (...) {                                                      \
    lg::set_last_error("unexpected internal error");                 \
    return LG_E_HIP;                                                 \
  }

static lg_status arg_error(const char* msg) {
  lg::set_last_error(msg);
  return LG_E_ARG;
}

extern "C" lg_status lg_default_opts(lg_setup_opts* o) {
  if (!o) return arg_error("lg_default_opts: null options");
  std::memset(o, 0, sizeof(*o));
  o->elim_enable = 1;
  o->elim_max_degree = 4;
  o->elim_min_fraction = 0.05;
  o->agg_iters = 10;
  o->agg_filter_base = 0.5;
  o->seed_votes = 8;
  o->tv_sweeps = 3;
  o->tv_omega = 2.0 / 3.0;
  o->cheb_degree = 2;
  o->cheb_lo = 0.3;
  o->cheb_hi = 1.1;
  o->eig_iters = 10;
  o->coarsest_nnz = 1000;
  o->max_levels = 64;
  o->cycle = LG_CYCLE_V;
  o->hash_mode = 0;
  o->seed = 12345;
  o->precision = LG_FP64;
  o->max_rhs = 1;
  o->keep_setup_data = 0;
  o->validate = 1;
  o->graphs = 1;
  o->autotune = 1;
  o->elim_passes = 1;
  o->merge_path = 0;
  o->row_shift = -1;
  o->reorder = 1;
  o->col_unroll = 0;
  return LG_OK;
}

static const char* check_opts(const lg_setup_opts& o) {
  if (o.max_rhs < 1 || o.max_rhs > 32) return "max_rhs must be in 1..32";
  if (o.precision != LG_FP64 && o.precision != LG_MIXED) return "precision must be LG_FP64 or LG_MIXED";
  if (o.cycle != LG_CYCLE_V && o.cycle != LG_CYCLE_K) return "cycle must be LG_CYCLE_V or LG_CYCLE_K";
  if (o.cheb_degree < 0 || o.cheb_degree > 16) return "cheb_degree must be in 0..16";
  if (!(o.cheb_hi > o.cheb_lo) || !(o.cheb_lo >= 0.0)) return "need 0 <= cheb_lo < cheb_hi";
  if (o.eig_iters < 0 || o.eig_iters > 64) return "eig_iters must be in 0..64";
  if (o.agg_iters < 0 || o.tv_sweeps < 0 || o.seed_votes < 1) return "bad aggregation parameters";
  if (!(o.agg_filter_base > 0.0 && o.agg_filter_base <= 1.0)) return "agg_filter_base must be in (0,1]";
  if (o.hash_mode != 0 && o.hash_mode != 1) return "hash_mode must be 0 or 1";
  if (o.max_levels < 1) return "max_levels must be >= 1";
  if (o.elim_max_degree < 0) return "elim_max_degree must be >= 0";
  if (o.graphs != 0 && o.graphs != 1) return "graphs must be 0 or 1";
  if (o.autotune != 0 && o.autotune != 1) return "autotune must be 0 or 1";
  if (o.elim_passes < 1 || o.elim_passes > 16) return "elim_passes must be in 1..16";
  if (o.merge_path < 0 || o.merge_path > 2) return "merge_path must be 0, 1 or 2";
  if (o.row_shift < -1 || o.row_shift > 2) return "row_shift must be -1, 0, 1 or 2";
  if (o.reorder < 0 || o.reorder > 1) return "reorder must be 0 or 1";
  if (o.col_unroll != 0 && o.col_unroll != 4 && o.col_unroll != 6)
    return "col_unroll must be 0, 4 or 6";
  return nullptr;
}

extern "C" lg_status lg_setup(const lg_graph* g, const lg_setup_opts* o, void* hip_stream,
                              lg_hierarchy** out) {
  if (!out) return arg_error("lg_setup: null output");
  *out = nullptr;
  if (!g || !g->row_ptr) return arg_error("lg_setup: null graph");
  if (g->n < 1 || g->n >= ((int64_t)1 << 30)) return arg_error("lg_setup: need 1 <= n < 2^30");
  if (g->nnz < 0 || g->nnz >= ((int64_t)1 << 31)) return arg_error("lg_setup: need 0 <= nnz < 2^31");
  if (g->nnz > 0 && (!g->col || !g->w)) return arg_error("lg_setup: null col or w");
  lg_setup_opts opts;
  if (o) opts = *o;
  else lg_default_opts(&opts);
  if (const char* m = check_opts(opts)) return arg_error(m);
  lg_hierarchy* h = nullptr;
  LG_API_BEGIN
  hipStream_t st = (hipStream_t)hip_stream;
  auto t0 = std::chrono::steady_clock::now();
  h = new lg_hierarchy();
  h->opts = opts;
  int K = 1;
  while (K < opts.max_rhs) K <<= 1;
  h->K = K;
  LG_HIP(hipGetDevice(&h->device));
  lg::setup_hierarchy(h, g, st);
  lg::alloc_solve_workspace(h, st);
  if (opts.merge_path == 2)
    for (auto& L : h->lev) L.sched.merge = true;
  if (opts.col_unroll > 0)
    for (auto& L : h->lev) L.sched.col_unroll = opts.col_unroll;
  if (opts.row_shift >= 0) {
    for (auto& L : h->lev) L.sched.lane_shift = L.sched.col_shift = opts.row_shift;
  } else if (opts.autotune) {
    lg::autotune(h, st);
  }
  LG_HIP(hipStreamSynchronize(st));
  h->setup_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return LG_OK;
  }
  catch (const lg::Error& e) {
    lg::set_last_error(e.msg);
    delete h;
    return e.code;
  }
  catch (const std::bad_alloc&) {
    lg::set_last_error("host allocation failed");
    delete h;
    return LG_E_NOMEM;
  }
  catch (...) {
    lg::set_last_error("unexpected internal error");
    delete h;
    return LG_E_HIP;
  }
}

extern "C" lg_status lg_solve(lg_hierarchy* h, const double* B, double* X, int32_t k, double rtol,
                              int32_t max_iter, void* hip_stream, lg_rhs_info* info) {
  if (!h || !B || !X) return arg_error("lg_solve: null argument");
  if (k < 1 || k > h->opts.max_rhs) return arg_error("lg_solve: k must be in 1..max_rhs");
  if (!(rtol > 0.0) || max_iter < 0) return arg_error("lg_solve: need rtol > 0 and max_iter >= 0");
  LG_API_BEGIN
  return lg::solve_dispatch(h, B, X, k, rtol, max_iter, (hipStream_t)hip_stream, info);
  LG_API_END
}

extern "C" lg_status lg_eigs(lg_hierarchy* h, int32_t nev, double tol, int32_t max_iter, double* X,
                             double* lambda, int32_t* iters, double* resid, void* hip_stream) {
  if (!h || !X || !lambda) return arg_error("lg_eigs: null argument");
  if (nev < 1 || nev > 7) return arg_error("lg_eigs: nev must be in 1..7");
  if (!(tol > 0.0) || max_iter < 0) return arg_error("lg_eigs: need tol > 0 and max_iter >= 0");
  if (h->lev[0].n < 2 * (nev + 1)) return arg_error("lg_eigs: graph too small for nev");
  LG_API_BEGIN
  return lg::eigs_dispatch(h, nev, tol, max_iter, X, lambda, iters, resid, (hipStream_t)hip_stream);
  LG_API_END
}

extern "C" lg_status lg_eigs_noalloc(lg_hierarchy* h, int32_t nev, double tol, int32_t max_iter,
                                     double* X, double* lambda, int32_t* iters, double* resid,
                                     void* hip_stream) {
  if (!h || !X || !lambda) return arg_error("lg_eigs_noalloc: null argument");
  if (nev < 1 || nev > 7) return arg_error("lg_eigs_noalloc: nev must be in 1..7");
  if (!(tol > 0.0) || max_iter < 0) return arg_error("lg_eigs_noalloc: need tol > 0 and max_iter >= 0");
  if (h->lev[0].n < 2 * (nev + 1)) return arg_error("lg_eigs_noalloc: graph too small for nev");
  LG_API_BEGIN
  return lg::eigs_noalloc_dispatch(h, nev, tol, max_iter, X, lambda, iters, resid,
                                   (hipStream_t)hip_stream);
  LG_API_END
}

extern "C" lg_status lg_cycle(lg_hierarchy* h, const double* B, double* X, int32_t k,
                              void* hip_stream) {
  if (!h || !B || !X) return arg_error("lg_cycle: null argument");
  if (k < 1 || k > h->opts.max_rhs) return arg_error("lg_cycle: k must be in 1..max_rhs");
  LG_API_BEGIN
  lg::cycle_dispatch(h, B, X, k, (hipStream_t)hip_stream);
  LG_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
  return LG_OK;
  LG_API_END
}

extern "C" lg_status lg_spmv(lg_hierarchy* h, int32_t level, const double* X, double* Y, int32_t k,
                             void* hip_stream) {
  if (!h || !X || !Y) return arg_error("lg_spmv: null argument");
  if (level < 0 || level >= (int)h->lev.size()) return arg_error("lg_spmv: bad level");
  LG_API_BEGIN
  lg::spmv_dispatch(h, level, X, Y, k, (hipStream_t)hip_stream);
  return LG_OK;
  LG_API_END
}

extern "C" lg_status lg_hierarchy_stats(const lg_hierarchy* h, lg_level_stats* out, int32_t cap,
                                        int32_t* n_levels) {
  if (!h) return arg_error("lg_hierarchy_stats: null hierarchy");
  const int nl = (int)h->lev.size();
  if (n_levels) *n_levels = nl;
  for (int l = 0; out && l < nl && l < cap; l++) {
    const Level& L = h->lev[l];
    out[l].type = L.type;
    out[l].n = L.n;
    out[l].nnz = L.nnz;
    out[l].nc = L.nc;
    out[l].lmax = L.lmax;
    out[l].n_hub = L.sched.nhub + L.sched.nsplit;
    out[l].lane_shift = L.sched.lane_shift;
    out[l].col_shift = L.sched.col_shift;
    out[l].merge = L.sched.merge ? 1 : 0;
    out[l].reordered = L.perm ? 1 : 0;
    out[l].col_unroll = L.sched.col_unroll;
  }
  return LG_OK;
}

extern "C" lg_status lg_export_level(const lg_hierarchy* h, int32_t level, int64_t* row_ptr,
                                     int32_t* col, double* w, double* d, int32_t* map) {
  if (!h) return arg_error("lg_export_level: null hierarchy");
  if (level < 0 || level >= (int)h->lev.size()) return arg_error("lg_export_level: bad level");
  LG_API_BEGIN
  const Level& L = h->lev[level];
  const int64_t n = L.n;
  const int32_t* src = L.type == LG_LEVEL_AGG ? L.agg : L.type == LG_LEVEL_ELIM ? L.cidx : nullptr;
  if (map && !src) return arg_error("lg_export_level: the coarsest level has no map");
  // Levels stored in the solve-time order are returned in the setup's
  // numbering: row i of the solve order is row perm[i], its entries in
  // their order (column perm[j] for stored column j).
  auto fetch_perm = [](const int32_t* p, int64_t len) {
    std::vector<int32_t> v;
    if (p) {
      v.resize(len);
      LG_HIP(hipMemcpy(v.data(), p, sizeof(int32_t) * len, hipMemcpyDeviceToHost));
    }
    return v;
  };
  const std::vector<int32_t> perm = fetch_perm(L.perm, n);
  std::vector<int32_t> rp(n + 1);
  LG_HIP(hipMemcpy(rp.data(), L.rp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
  if (perm.empty()) {
    if (row_ptr)
      for (int64_t i = 0; i <= n; i++) row_ptr[i] = rp[i];
    if (col && L.nnz) LG_HIP(hipMemcpy(col, L.col, sizeof(int32_t) * L.nnz, hipMemcpyDeviceToHost));
    if (w && L.nnz) LG_HIP(hipMemcpy(w, L.w, sizeof(double) * L.nnz, hipMemcpyDeviceToHost));
    if (d) LG_HIP(hipMemcpy(d, L.d, sizeof(double) * n, hipMemcpyDeviceToHost));
  } else {
    std::vector<int64_t> orp(n + 1, 0);
    for (int64_t i = 0; i < n; i++) orp[perm[i] + 1] = rp[i + 1] - rp[i];
    for (int64_t i = 0; i < n; i++) orp[i + 1] += orp[i];
    if (row_ptr)
      for (int64_t i = 0; i <= n; i++) row_ptr[i] = orp[i];
    if ((col || w) && L.nnz) {
      std::vector<int32_t> cs(L.nnz);
      std::vector<double> ws(L.nnz);
      LG_HIP(hipMemcpy(cs.data(), L.col, sizeof(int32_t) * L.nnz, hipMemcpyDeviceToHost));
      LG_HIP(hipMemcpy(ws.data(), L.w, sizeof(double) * L.nnz, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < n; i++)
        for (int64_t k = 0; k < rp[i + 1] - rp[i]; k++) {
          const int64_t to = orp[perm[i]] + k, from = rp[i] + k;
          if (col) col[to] = perm[cs[from]];
          if (w) w[to] = ws[from];
        }
    }
    if (d) {
      std::vector<double> ds(n);
      LG_HIP(hipMemcpy(ds.data(), L.d, sizeof(double) * n, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < n; i++) d[perm[i]] = ds[i];
    }
  }
  if (map) {
    const std::vector<int32_t> cperm = fetch_perm(h->lev[level + 1].perm, h->lev[level + 1].n);
    std::vector<int32_t> ms(n);
    LG_HIP(hipMemcpy(ms.data(), src, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; i++) {
      const int32_t v = ms[i];
      map[perm.empty() ? i : perm[i]] = (v >= 0 && !cperm.empty()) ? cperm[v] : v;
    }
  }
  return LG_OK;
  LG_API_END
}

extern "C" lg_status lg_export_setup_data(const lg_hierarchy* h, int32_t level, double* X,
                                          double* S, int32_t* state, int32_t* idx, int32_t* votes,
                                          int32_t* z) {
  if (!h) return arg_error("lg_export_setup_data: null hierarchy");
  if (level < 0 || level >= (int)h->lev.size()) return arg_error("lg_export_setup_data: bad level");
  if (!h->opts.keep_setup_data) return arg_error("lg_export_setup_data: setup data not kept");
  LG_API_BEGIN
  const Level& L = h->lev[level];
  if ((X || S || state || idx || votes) && !L.S)
    return arg_error("lg_export_setup_data: no aggregation data on this level");
  if (z && !L.z) return arg_error("lg_export_setup_data: no elimination data on this level");
  if (X) LG_HIP(hipMemcpy(X, L.X, sizeof(double) * 4 * L.n, hipMemcpyDeviceToHost));
  if (S && L.nnz) LG_HIP(hipMemcpy(S, L.S, sizeof(double) * L.nnz, hipMemcpyDeviceToHost));
  if (votes) LG_HIP(hipMemcpy(votes, L.votes, sizeof(int32_t) * L.n, hipMemcpyDeviceToHost));
  if (state || idx) {
    std::vector<int32_t> st(L.n);
    LG_HIP(hipMemcpy(st.data(), L.status, sizeof(int32_t) * L.n, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < L.n; i++) {
      if (state) state[i] = lg::status_state(st[i]);
      if (idx) idx[i] = st[i] & lg::kIdxMask;
    }
  }
  if (z) LG_HIP(hipMemcpy(z, L.z, sizeof(int32_t) * L.n, hipMemcpyDeviceToHost));
  return LG_OK;
  LG_API_END
}

extern "C" lg_status lg_export_coarsest(const lg_hierarchy* h, double* Lplus) {
  if (!h || !Lplus) return arg_error("lg_export_coarsest: null argument");
  LG_API_BEGIN
  const int64_t n = h->lev.back().n;
  LG_HIP(hipMemcpy(Lplus, h->Lplus, sizeof(double) * n * n, hipMemcpyDeviceToHost));
  return LG_OK;
  LG_API_END
}

extern "C" size_t lg_hierarchy_bytes(const lg_hierarchy* h) { return h ? h->mem.bytes() : 0; }

extern "C" double lg_setup_ms(const lg_hierarchy* h) { return h ? h->setup_ms : 0.0; }

extern "C" void lg_free(lg_hierarchy* h) { delete h; }

extern "C" const char* lg_status_str(lg_status s) {
  switch (s) {
    case LG_OK: return "ok";
    case LG_E_ARG: return "invalid argument";
    case LG_E_GRAPH: return "invalid graph";
    case LG_E_DISCONNECTED: return "graph not connected";
    case LG_E_NOMEM: return "out of device memory";
    case LG_E_HIP: return "HIP runtime error";
    case LG_E_NOT_CONVERGED: return "not converged";
    case LG_E_BUSY: return "busy";
    case LG_E_RANGE: return "exact-sum range exceeded";
    default: return "unknown status";
  }
}

extern "C" const char* lg_last_error(void) { return lg::last_error_cstr(); }
