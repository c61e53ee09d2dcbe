/*
 * lgmg_oracle.h -- CPU oracle for the graph-Laplacian multigrid of
 * Konolige & Brown, "A Parallel Solver for Graph Laplacians" (PASC'18).
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load this library.
 * It shares no code with the GPU library.
 *
 * All pointers are host pointers.  Graphs are the CSR of the symmetric
 * adjacency A (both directions, strictly increasing columns, no diagonal,
 * w > 0); the Laplacian is L = D - A with D = diag(row sums of A) (Section 2.1).
 * Status codes: 0 ok, 1 bad argument, 2 invalid graph, 3 disconnected,
 * 4 out of memory, 6 not converged, 8 exact-sum range exceeded.
 */
#ifndef LGMG_ORACLE_H
#define LGMG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LGO_OK = 0, LGO_E_ARG = 1, LGO_E_GRAPH = 2, LGO_E_DISCONNECTED = 3, LGO_E_NOMEM = 4,
       LGO_E_NOT_CONVERGED = 6, LGO_E_RANGE = 8 };
enum { LGO_AGG = 0, LGO_ELIM = 1, LGO_COARSEST = 2 };

typedef struct {
  int32_t elim_enable;        /* low-degree elimination on/off (Section 3.4) */
  int32_t elim_max_degree;    /* candidates have degree <= this (4) */
  double elim_min_fraction;   /* apply only if |F| > fraction * n (0.05) */
  int32_t agg_iters;          /* voting iterations (10) */
  double agg_filter_base;     /* iteration t keeps S >= base^t (0.5) */
  int32_t seed_votes;         /* Undecided vertex with >= this many votes becomes a Seed (8) */
  int32_t tv_sweeps;          /* Jacobi sweeps on the 4 test vectors (3) */
  double tv_omega;            /* Jacobi damping (2/3) */
  int32_t cheb_degree;        /* Chebyshev degree (2) */
  double cheb_lo, cheb_hi;    /* bounds as fractions of the estimated lambda_max (0.3, 1.1) */
  int32_t eig_iters;          /* Lanczos steps for lambda_max (10) */
  int64_t coarsest_nnz;       /* stop when nnz(L) = n + nnz(A) <= this (1000) */
  int32_t max_levels;         /* hard cap on levels (64) */
  int32_t cycle;              /* 1 = V-cycle inside CG, 2 = K-cycle inside FCG */
  int32_t hash_mode;          /* 0 = mixed hash of the id, 1 = identity (test hook) */
  uint64_t seed;              /* seed of the counter-based generator */
  int32_t elim_passes;        /* elimination passes before each aggregation (1: Section 3.4) */
} lgo_opts;

void lgo_default_opts(lgo_opts* o);
/* Threads of the row-parallel loops (1 unless built with -fopenmp). */
int32_t lgo_threads(void);

/* ---- primitives (pinned individually by the tests) ---- */
uint64_t lgo_mix64(uint64_t z);
uint64_t lgo_hash(int64_t i, int32_t mode);
double lgo_tv(uint64_t seed, int32_t level, int32_t k, int64_t i);
int lgo_xs_term(double v, int64_t* hi, uint64_t* lo);
double lgo_xs_round(int64_t hi, uint64_t lo);
int lgo_xsum(const double* t, int64_t n, double* out);

/* ---- single steps on caller-provided graphs ---- */
int lgo_validate(int64_t n, const int64_t* rp, const int32_t* col, const double* w);
int lgo_diag(int64_t n, const int64_t* rp, const int32_t* col, const double* w, double* d);
int64_t lgo_elim_select(int64_t n, const int64_t* rp, const int32_t* col, int32_t max_degree,
                        int32_t hash_mode, int32_t* z, uint8_t* F);
int64_t lgo_elim_build(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                       const double* d, const uint8_t* F, int32_t* cidx, int64_t* crp,
                       int32_t* ccol, double* cw, double* cd, int64_t cap);
int lgo_soc(int64_t n, const int64_t* rp, const int32_t* col, const double* w, const double* d,
            const lgo_opts* o, int32_t level, double* X, double* S);
int64_t lgo_aggregate(int64_t n, const int64_t* rp, const int32_t* col, const double* S,
                      const lgo_opts* o, int32_t* state, int32_t* idx, int32_t* votes,
                      int32_t* agg);
int64_t lgo_galerkin(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                     const int32_t* agg, int64_t nc, int64_t* crp, int32_t* ccol, double* cw,
                     double* cd, int64_t cap);
double lgo_lanczos_lmax(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                        const double* d, int32_t steps, uint64_t seed, int32_t level);
double lgo_tridiag_max(const double* alpha, const double* beta, int32_t m);
int lgo_pinv_dense(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                   const double* d, double* out);
int lgo_cheb_apply(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                   const double* d, double lmax, const lgo_opts* o, double* x, const double* b,
                   int32_t x_is_zero);

/* ---- full hierarchy ---- */
typedef struct lgo_hier lgo_hier;
int lgo_setup(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
              const lgo_opts* o, lgo_hier** out);
void lgo_free(lgo_hier* h);
int32_t lgo_num_levels(const lgo_hier* h);
int lgo_level_info(const lgo_hier* h, int32_t l, int32_t* type, int64_t* n, int64_t* nnz,
                   int64_t* nc, double* lmax);
int lgo_level_csr(const lgo_hier* h, int32_t l, int64_t* rp, int32_t* col, double* w, double* d);
int lgo_level_map(const lgo_hier* h, int32_t l, int32_t* map); /* agg (AGG) or cidx (ELIM) */
int lgo_level_elim(const lgo_hier* h, int32_t l, int32_t* z);
int lgo_level_soc(const lgo_hier* h, int32_t l, double* X, double* S);
int lgo_level_votes(const lgo_hier* h, int32_t l, int32_t* state, int32_t* idx, int32_t* votes);
int lgo_coarsest_pinv(const lgo_hier* h, double* out);
double lgo_cycle_work(const lgo_hier* h);
int lgo_cycle(const lgo_hier* h, const double* b, double* x);
int lgo_level_cycle(const lgo_hier* h, int32_t l, const double* b, double* x);
int lgo_level_fcg2(const lgo_hier* h, int32_t l, const double* b, double* x);
int lgo_spmv(const lgo_hier* h, int32_t l, const double* x, double* y);
int lgo_solve(const lgo_hier* h, const double* b, double* x, double rtol, int32_t max_iter,
              int32_t* iters, double* rel_residual, double* work_units);

#ifdef __cplusplus
}
#endif
#endif
