// impl.h -- the device-resident hierarchy behind lg_hierarchy.
#pragma once

#include <vector>

#include "common.h"

namespace lg {

// Packed voting status (Algorithm 3): state in bits 30-31, index in bits 0-29.
// State codes equal their rank in the argmax order: Seed > Undecided > Decided.
constexpr int kDecided = 0, kUndecided = 1, kSeed = 2;
constexpr int32_t kIdxMask = (1 << 30) - 1;
constexpr int32_t kNoStatus = -1;  // "no neighbour" in the argmax (state field 3 never occurs)
__host__ __device__ inline int status_state(int32_t s) { return (int)((uint32_t)s >> 30); }
__host__ __device__ inline int32_t make_status(int state, int64_t idx) {
  return (int32_t)(((uint32_t)state << 30) | (uint32_t)idx);
}

struct Level {
  int type = LG_LEVEL_COARSEST;
  int64_t n = 0, nnz = 0, nc = 0;
  // off-diagonal adjacency (CSR, int32 offsets) and the Laplacian diagonal
  int32_t* rp = nullptr;
  int32_t* col = nullptr;
  double* w = nullptr;
  double* d = nullptr;
  double* dinv = nullptr;
  float* wf = nullptr;  // mixed precision copies
  float* df = nullptr;
  float* dinvf = nullptr;
  Sched sched;
  // aggregation level: aggregate of each vertex and the member lists of R
  int32_t* agg = nullptr;
  int32_t* mptr = nullptr;
  int32_t* mem = nullptr;
  Sched msched;
  // elimination level: coarse index (-1 = eliminated), fine vertex of each
  // coarse vertex, and the F-part of P^T as CSR over coarse rows
  int32_t* cidx = nullptr;
  int32_t* cvert = nullptr;
  int32_t* ptrp = nullptr;
  int32_t* ptf = nullptr;
  double* ptc = nullptr;
  float* ptcf = nullptr;
  Sched ptsched;
  int64_t nF = 0, nnzP = 0;
  // solve-time vertex order (null: the setup's numbering): perm[new] = old
  // and iperm[old] = new; every array above is stored in the new numbering
  int32_t* perm = nullptr;
  int32_t* iperm = nullptr;
  double lmax = 0.0;
  // column-split smoothing from a zero guess: 1 = the first iterate stored by
  // an elementwise pass, then one product (no D^-1 gather per entry); 0 = both
  // steps in one product.  The same arithmetic either way; set by the autotuner.
  bool cheb0_split = false;
  // setup data kept for export
  double* X = nullptr;
  double* S = nullptr;
  int32_t* status = nullptr;
  int32_t* votes = nullptr;
  int32_t* z = nullptr;
  // cycle workspace (precision type, n x K)
  void* vb = nullptr;
  void* vx = nullptr;
  void* vx2 = nullptr;
  void* vr = nullptr;
  // K-cycle workspace (levels whose coarse solve is FCG)
  void* kr = nullptr;
  void* kp1 = nullptr;
  void* kq1 = nullptr;
  void* kz = nullptr;
  void* kx = nullptr;
  double* kscal = nullptr;  // per-column scalars of the inner FCG
};

}  // namespace lg

struct lg_hierarchy {
  lg_setup_opts opts{};
  int device = 0;
  lg::Arena mem{(size_t)64 << 20};
  std::vector<lg::Level> lev;
  double* Lplus = nullptr;  // coarsest pseudo-inverse, fp64
  int K = 1;                // padded right-hand-side capacity
  // outer Krylov workspace, fp64, n0 x K
  double *pb = nullptr, *px = nullptr, *pr = nullptr, *pz = nullptr, *pp = nullptr,
         *pq = nullptr, *pt = nullptr;
  void* cyc_in = nullptr;   // level-0 cycle input in the cycle precision (mixed)
  double* scal = nullptr;   // device scalars, 32 x K
  double* red = nullptr;    // reduction partials
  double* dotp = nullptr;   // partials of the CG product's fused p . q (dot_partials x K)
  int64_t dotp_rows = 0;
  double* host_scal = nullptr;  // pinned mirror of scal
  double setup_ms = 0.0;
  double* lmax_dev = nullptr;
  // The cycle captured as a HIP graph, per width log2(K) (see Engine::cycle):
  // replayed with one launch instead of re-enqueueing every kernel.
  struct CycleGraph {
    hipGraphExec_t exec = nullptr;
    const void* in = nullptr;  // the input buffer the graph reads
    void* out = nullptr;       // the buffer holding its result
    int uses = 0;              // eager applications so far
  };
  CycleGraph cycle_graph[6];
  hipStream_t capture_stream = nullptr;
  bool no_capture = false;  // set during an allocation-free call: replay only, never capture
  ~lg_hierarchy() {
    for (CycleGraph& g : cycle_graph)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    if (host_scal) (void)hipHostFree(host_scal);
  }
};

namespace lg {
constexpr int kRedBlocks = 240;   // grid of the setup's scalar reductions
constexpr int kDotPartials = 2048;  // most workgroups of a column-dot launch
// scalar slots (each K wide) of lg_hierarchy::scal
enum {
  S_BN = 0, S_RZ, S_PQ, S_ALPHA, S_BETA, S_RR, S_PR, S_ZQ, S_ACTIVE, S_MEAN, S_TMP, S_TR,
  S_ZSUM, S_ZY, S_YSUM, S_RESTART, S_FILL,
  S_COUNT = 32
};

// Continuous batching (the solve server): a batched solve whose columns are
// slots.  At each CG iteration boundary the columns that finished are written
// to their destinations and their slots are refilled with queued right-hand
// sides; every column runs its own CG (own iteration count, restarts and
// convergence test), so a column's arithmetic does not depend on what the
// other slots hold.
struct SlotFeed {
  struct Col {
    int slot;
    const double* B;  // right-hand side: B[i * ldb], i < n (device)
    int ldb;
    double* X;        // its solution goes to X[i * ldx] (device)
    int ldx;
  };
  // Columns to load into some of the free slots (at most one per slot).
  virtual void refill(const std::vector<int>& free_slots, std::vector<Col>& out) = 0;
  // The slot's column finished; its solution is in place (stream synchronised).
  virtual void finished(int slot, const lg_rhs_info& info) = 0;
  virtual ~SlotFeed() = default;
};
// Runs until every slot is empty and refill offers nothing.  K: the width
// (a power of two, at most the hierarchy's).
lg_status solve_slots(lg_hierarchy* h, int K, double rtol, int max_iter, hipStream_t st,
                      SlotFeed* feed);

void setup_hierarchy(lg_hierarchy* h, const lg_graph* g, hipStream_t st);
void alloc_solve_workspace(lg_hierarchy* h, hipStream_t st);
lg_status solve_dispatch(lg_hierarchy* h, const double* B, double* X, int k, double rtol,
                         int max_iter, hipStream_t st, lg_rhs_info* info);
void cycle_dispatch(lg_hierarchy* h, const double* B, double* X, int k, hipStream_t st);
void spmv_dispatch(lg_hierarchy* h, int level, const double* X, double* Y, int k, hipStream_t st);
void spmv_ordered(lg_hierarchy* h, int level, const double* X, double* Y, int k, hipStream_t st);
void autotune(lg_hierarchy* h, hipStream_t st);
lg_status eigs_dispatch(lg_hierarchy* h, int nev, double tol, int max_iter, double* X,
                        double* lambda, int* iters, double* resid, hipStream_t st);
lg_status eigs_noalloc_dispatch(lg_hierarchy* h, int nev, double tol, int max_iter, double* X,
                                double* lambda, int* iters, double* resid, hipStream_t st);
}  // namespace lg
