/*
 * lgmg.h -- C ABI of liblgmg.so: unsmoothed-aggregation multigrid for graph
 * Laplacians (Konolige & Brown, "A Parallel Solver for Graph Laplacians",
 * PASC'18) on one AMD Instinct MI355X (gfx950).
 *
 * The problem (Section 2.1): a connected, undirected graph with positive edge
 * weights w_ij defines L = D - A with D_ii = sum_j w_ij.  L is symmetric
 * positive semi-definite with null space span{1}; lg_solve returns the
 * mean-zero x with L x = b - mean(b).
 *
 * Conventions for every entry point:
 *  - Every function returns lg_status; no C++ exception crosses the boundary.
 *    On failure lg_last_error() (per thread) describes the cause.
 *  - Graph arrays are the CSR of the symmetric adjacency A: both directions
 *    stored, column indices strictly increasing within a row, no diagonal
 *    entries, weights > 0.  row_ptr is int64[n+1], col int32[nnz],
 *    w float64[nnz].  nnz must be below 2^31.
 *  - "device" pointers are HIP device allocations (e.g. torch tensors'
 *    data_ptr on cuda:0), used on the caller's stream.  Host pointers are
 *    ordinary memory.  The library never frees caller memory.
 *  - Multi-vector layout: n x k row-major (entry (i, c) at [i*k + c]).
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Calls are
 *    asynchronous with respect to the host only where stated; setup and
 *    solve synchronise the stream before returning.
 *  - A hierarchy may be used by one call at a time (solves on one hierarchy
 *    share its workspace).
 */
#ifndef LGMG_H
#define LGMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lg_status;
enum {
  LG_OK = 0,
  LG_E_ARG = 1,           /* invalid argument or unsupported size */
  LG_E_GRAPH = 2,         /* not a valid weighted undirected graph (asymmetric, w <= 0, loop, unsorted) */
  LG_E_DISCONNECTED = 3,  /* graph not connected (Section 2.1 assumes connectivity) */
  LG_E_NOMEM = 4,         /* device allocation failed */
  LG_E_HIP = 5,           /* HIP runtime error */
  LG_E_NOT_CONVERGED = 6, /* max_iter reached or breakdown; X and info are still filled */
  LG_E_BUSY = 7,          /* reserved */
  LG_E_RANGE = 8          /* total edge weight >= 2^62: outside the exact-sum range */
};

enum { LG_LEVEL_AGG = 0, LG_LEVEL_ELIM = 1, LG_LEVEL_COARSEST = 2 };
enum { LG_CYCLE_V = 1, LG_CYCLE_K = 2 };
enum { LG_FP64 = 0, LG_MIXED = 1 };

typedef struct {
  int64_t n;               /* vertices, >= 1 */
  int64_t nnz;             /* stored adjacency entries (2 x undirected edges) */
  const int64_t* row_ptr;  /* [n+1] */
  const int32_t* col;      /* [nnz] */
  const double* w;         /* [nnz] */
  int32_t on_device;       /* 1: the three arrays are device pointers, 0: host pointers */
} lg_graph;

/* Method parameters; lg_default_opts fills the paper's values. */
typedef struct {
  int32_t elim_enable;      /* low-degree elimination before each aggregation (Section 3.4) */
  int32_t elim_max_degree;  /* candidates: degree <= this (4, Section 3.4) */
  double elim_min_fraction; /* apply only if more than this fraction is eliminated (0.05) */
  int32_t agg_iters;        /* voting iterations (10, Section 3.5) */
  double agg_filter_base;   /* iteration t keeps strengths >= base^t (0.5, Algorithm 3) */
  int32_t seed_votes;       /* votes that make an Undecided vertex a Seed (8, Section 3.5) */
  int32_t tv_sweeps;        /* Jacobi sweeps on the 4 test vectors (3, Section 3.5) */
  double tv_omega;          /* their damping; the paper gives none (2/3) */
  int32_t cheb_degree;      /* Chebyshev smoother degree (2, Section 4) */
  double cheb_lo, cheb_hi;  /* interval as fractions of lambda_max (0.3, 1.1, Section 3.6) */
  int32_t eig_iters;        /* Lanczos steps for lambda_max (10, Section 3.6) */
  int64_t coarsest_nnz;     /* stop coarsening once n + nnz(A) <= this (1000, Section 4) */
  int32_t max_levels;       /* cap on hierarchy depth (64) */
  int32_t cycle;            /* LG_CYCLE_V (CG outside) or LG_CYCLE_K (FCG outside, Section 3.7) */
  int32_t hash_mode;        /* elimination hash: 0 = mixed id, 1 = identity (testing) */
  uint64_t seed;            /* seed of the counter-based generator for test and start vectors */
  int32_t precision;        /* LG_FP64, or LG_MIXED: fp32 hierarchy values and cycle inside fp64 CG */
  int32_t max_rhs;          /* largest k passed to lg_solve (1..32); sizes the solve workspace */
  int32_t keep_setup_data;  /* 1: keep strengths, test vectors, votes and elimination choices for export */
  int32_t validate;         /* 1: check symmetry, weights and connectivity on the device */
  int32_t graphs;           /* 1: after its first use, replay the cycle as a captured HIP graph */
  int32_t autotune;         /* 1: choose lanes per row of each large level by timing (cached per
                               structure; summation order, hence rounding, follows the choice) */
  int32_t elim_passes;      /* elimination passes before each aggregation, 1..16 (1: Section 3.4;
                               more repeat it on its own result while it removes enough) */
  int32_t merge_path;       /* one-column Laplacian products: 0 degree-class rows only (default),
                               1 the autotuner may pick a merge-path traversal per level, 2 every
                               level uses it (the autotuner then leaves one-column levels alone) */
  int32_t row_shift;        /* -1: lanes per row chosen by the autotuner (shift 1 without it);
                               0, 1, 2: every level's row products use 2^(class - row_shift)
                               lanes and the autotuner is not run.  The shift fixes the
                               summation order inside a row, so a solve is bit-reproducible
                               given the shifts in lg_level_stats (and col_unroll), and a tuned
                               run can differ from another process's in the last bits */
  int32_t reorder;          /* 1: after setup, aggregation levels (and an elimination level 0
                               when max_rhs >= 4) of at least 2^14 vertices whose largest
                               degree is at least 8x their mean, and whose mean degree is at
                               most 128, are stored in a solve-time
                               vertex order (higher degree classes first, the setup's order
                               kept within a class), so that the rows most entries gather
                               share cache lines.  Every row keeps its entries in order, so
                               each row's sum is unchanged; inputs, outputs and exports use
                               the setup's numbering.  0: the setup's numbering throughout */
  int32_t col_unroll;       /* column-split products (k columns of at least 32 bytes per row):
                               entries each lane group loads per trip, 4 or 6 on every level's
                               Laplacian products; 0 (default): by width, 4 for products of
                               at most 16 columns and 6 for 32.  A row's entries
                               are added in the same order at either value, so products and
                               cycles keep their bits; the CG product's fused p . q sums per
                               workgroup, and the workgroup count follows the kernel's
                               occupancy, so a solve is bit-reproducible given this option */
} lg_setup_opts;

typedef struct lg_hierarchy lg_hierarchy;

typedef struct {
  int32_t type;    /* LG_LEVEL_* */
  int64_t n;       /* vertices on this level */
  int64_t nnz;     /* stored off-diagonal entries */
  int64_t nc;      /* vertices on the next level (0 for the coarsest) */
  double lmax;     /* lambda_max estimate of D^-1 L (aggregation levels) */
  int64_t n_hub;   /* rows split across workgroups by the row scheduler */
  int32_t lane_shift, col_shift; /* row lanes 2^(class - shift) in use (set by the autotuner) */
  int32_t merge;                 /* 1: one-column products use the merge-path traversal */
  int32_t reordered;             /* 1: stored in the solve-time vertex order (reorder option) */
  int32_t col_unroll;            /* col_unroll in use on the level's Laplacian products (0: by width) */
} lg_level_stats;

typedef struct {
  int32_t iters;        /* CG / FCG iterations */
  double rel_residual;  /* final true ||b - L x|| / ||b|| (b projected to mean zero) */
  double work_units;    /* work in finest-level residual evaluations (Section 2.3.1) */
  double wda;           /* work per digit of accuracy, -work / log10(rel_residual) */
} lg_rhs_info;

/* Fill o with the paper's parameters (Sections 3.4-3.6, 4). */
lg_status lg_default_opts(lg_setup_opts* o);

/* Build the multigrid hierarchy of L = D - A (Sections 3.4-3.6): per level an
 * optional low-degree elimination (Algorithm 2 and the Schur complement), the
 * affinity strength of connection, voting aggregation (Algorithm 3), the
 * Galerkin operator R L P and a Lanczos lambda_max estimate; the last level
 * gets a dense pseudo-inverse.  g's arrays are only read during the call.
 * On success *out owns device memory until lg_free.  Errors: LG_E_ARG,
 * LG_E_GRAPH, LG_E_DISCONNECTED, LG_E_RANGE, LG_E_NOMEM, LG_E_HIP. */
lg_status lg_setup(const lg_graph* g, const lg_setup_opts* o, void* hip_stream,
                   lg_hierarchy** out);

/* Solve L X = B - mean(B) for k right-hand sides at once (Section 4: CG
 * preconditioned by one V-cycle, or FCG with a K-cycle; relative tolerance
 * rtol on the true residual).  B and X are device n x k row-major fp64; B is
 * not modified; X receives mean-zero solutions.  info (host, k entries, may
 * be NULL) receives per-column statistics.  1 <= k <= max_rhs of setup.  The
 * columns run together at width next_pow2(k); each column's arithmetic is
 * independent of the others, so at one width a column's result does not
 * depend on what the other columns hold.  Returns LG_E_NOT_CONVERGED (X and
 * info filled) if a column misses rtol. */
lg_status lg_solve(lg_hierarchy* h, const double* B, double* X, int32_t k, double rtol,
                   int32_t max_iter, void* hip_stream, lg_rhs_info* info);

/* The nev smallest nonzero eigenvalues of L (ascending, host lambda[nev])
 * and unit eigenvectors (device X, n x nev row-major, mean zero) -- the
 * Fiedler vector first (Section 2.1: spectral partitioning and drawing).
 * Block inverse subspace iteration on the mean-zero space, each block solved
 * with lg_solve's preconditioned CG; stops when every pair has
 * ||L x - lambda x|| <= tol * lambda (resid, host nev, may be NULL) or after
 * max_iter blocks (*iters, may be NULL).  The block is next_pow2(nev + 1)
 * columns: 1 <= nev <= 7 and that block at most max_rhs of setup.  Returns
 * LG_E_NOT_CONVERGED (outputs filled) if a pair misses tol. */
lg_status lg_eigs(lg_hierarchy* h, int32_t nev, double tol, int32_t max_iter, double* X,
                  double* lambda, int32_t* iters, double* resid, void* hip_stream);

/* lg_eigs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * same computation and results as lg_eigs, but its per-call buffers (the
 * block vectors and Gram matrices) live in a static 64 MiB device array of
 * the library, one per GPU, held until the process ends; the call allocates
 * no device memory and captures no HIP graph (it replays one the hierarchy
 * already has).  Needs 8 * (3 * n * K + small) bytes for a block of
 * K = next_pow2(nev + 1) columns on the finest level's n vertices (n up to
 * about 340,000 at K = 8, 2.7M at K = 2); larger problems return LG_E_ARG
 * naming the size.  Calls on one GPU share the array: calls that overlap in
 * time on the same GPU race and must not be made.  The hierarchy must live on
 * the current device (else LG_E_ARG). */
lg_status lg_eigs_noalloc(lg_hierarchy* h, int32_t nev, double tol, int32_t max_iter, double* X,
                          double* lambda, int32_t* iters, double* resid, void* hip_stream);

/* One application of the preconditioner (Algorithm 1 from the finest level
 * with zero initial guess; V- or K-cycle and precision as in setup):
 * X = M B for device n x k fp64 arrays.  No projection.  The columns of B
 * should have zero mean, as every vector the solver preconditions does: the
 * K-cycle's inner Krylov steps are otherwise inconsistent singular systems. */
lg_status lg_cycle(lg_hierarchy* h, const double* B, double* X, int32_t k, void* hip_stream);

/* Y = L_l X on hierarchy level l for device n_l x k fp64 arrays (fp64
 * values), with L_l = D_l - A_l the level's Laplacian (Section 2.1; coarse
 * levels are the Galerkin and Schur-complement operators of Sections 3.4-3.5).
 * k must be 1, 2, 4, 8, 16 or 32.  X and Y are caller-owned; the call only
 * queues work on hip_stream (asynchronous).  Errors: LG_E_ARG for a bad level
 * or k. */
lg_status lg_spmv(lg_hierarchy* h, int32_t level, const double* X, double* Y, int32_t k,
                  void* hip_stream);

/* Level statistics into out[0 .. min(cap, levels)) (host), *n_levels = depth
 * (host): the level sequence of the setup loop (Section 4: elimination and
 * aggregation levels down to a coarsest level of at most coarsest_nnz
 * entries) and the lambda_max estimates of Section 3.6.  Errors: LG_E_ARG for
 * a null h or n_levels. */
lg_status lg_hierarchy_stats(const lg_hierarchy* h, lg_level_stats* out, int32_t cap,
                             int32_t* n_levels);

/* Parity hook.  Copy level l's operator (its Laplacian as adjacency plus
 * diagonal, Section 2.1) and its transfer map (the aggregates of Algorithm 3,
 * or the kept vertices of Algorithm 2's elimination) to host buffers sized from
 * lg_hierarchy_stats:
 * row_ptr int64[n+1], col int32[nnz], w float64[nnz], d float64[n] (any may
 * be NULL).  map (int32[n], may be NULL) receives the aggregate of each vertex
 * (aggregation level) or its coarse index, -1 if eliminated (elimination
 * level).  Returns LG_E_ARG for a bad level. */
lg_status lg_export_level(const lg_hierarchy* h, int32_t level, int64_t* row_ptr, int32_t* col,
                          double* w, double* d, int32_t* map);

/* Parity hook: setup intermediates of level l (the smoothed test vectors and
 * affinity strengths of Section 3.5, the voting state of Algorithm 3 and the
 * elimination product of Algorithm 2), kept only when keep_setup_data was set
 * (else LG_E_ARG); any pointer may be NULL.  Host buffers:
 * X float64[n*4] (test vectors after smoothing), S float64[nnz] (strength per
 * stored edge), state int32[n] (0 Decided, 1 Undecided, 2 Seed), idx int32[n]
 * (root named by each vertex), votes int32[n], z int32[n] (elimination
 * semiring product, -1 for none). */
lg_status lg_export_setup_data(const lg_hierarchy* h, int32_t level, double* X, double* S,
                               int32_t* state, int32_t* idx, int32_t* votes, int32_t* z);

/* Parity hook: the dense pseudo-inverse used as the coarsest-level solve
 * (Algorithm 1's direct solve at the bottom of the cycle), host
 * float64[nc*nc] row-major.  Errors: LG_E_ARG for a null argument. */
lg_status lg_export_coarsest(const lg_hierarchy* h, double* Lplus);

/* Device bytes held by the hierarchy, including the solve workspace; the
 * serving loop admits hierarchies by this figure.  No passage of the paper
 * defines it.  0 for NULL. */
size_t lg_hierarchy_bytes(const lg_hierarchy* h);

/* Milliseconds the lg_setup call that built h took (host wall clock, for
 * measurement; no passage of the paper defines it).  0 for NULL. */
double lg_setup_ms(const lg_hierarchy* h);

/* Release h (memory management only; no passage of the paper applies).
 * Waits for the work queued on the device (as hipFree would),
 * then keeps its device blocks, up to 4 GiB per process, in a per-device
 * cache that later lg_setup calls draw from before allocating; blocks beyond
 * that are freed.  NULL is ignored. */
void lg_free(lg_hierarchy* h);

/* Kernel timing with HIP events for kernel families (one name as listed by
 * lg_profile_names, or several separated by commas), recorded around each of
 * their launches on the launch stream while enabled.  Families of the sparse
 * products time the row kernel alone: "spmv" the CG iteration's fp64 L x,
 * "lanczos" the exact-sum L x of setup's Lanczos steps,
 * "spmm" lg_spmv's own launches, "cheb0" the zero-start smoother steps, "cheb1"
 * the coarse correction with the first post-smoothing step (or that step
 * alone), "cheb" the later steps, "resid" the cycle's residual, "resid64" the
 * CG's true residual (in FP64 the same kernel instance as "resid"), "spmm_inner" the
 * K-cycle's coarse-level FCG products, "cg_update" the CG's residual update
 * (a vector pass); "restrict", "prolong" and "coarse" time those
 * cycle steps.  "hubs" times the hub and split rows of every row kernel: while
 * it is enabled their workgroups run as a launch of their own before the
 * other rows' (each row is reduced as in the single launch; the other
 * families then exclude them).  The setup families ("jacobi_xsum", "row_xsum", "affinity",
 * "vote", "elim_select", "galerkin_reduce") time the span of each call of
 * that setup step, "radix" each radix sort.  lg_profile_read returns
 * the launch count, the summed event time and the summed algorithmic bytes of
 * those launches, then resets the counters.  Disabled by default (NULL). */
lg_status lg_profile_enable(const char* family);
lg_status lg_profile_read(int64_t* launches, double* total_ms, double* total_bytes);
const char* lg_profile_names(void);

const char* lg_status_str(lg_status s);
const char* lg_last_error(void);

/* ------------------------------------------------------------------------
 * Solve server: continuous batching over a pool of graphs (a serving layer
 * over lg_setup / lg_solve; no passage of the paper describes it).  Requests
 * (graph, right-hand sides, tolerance) may arrive at any time from any thread.
 * A worker thread, each with its own HIP stream, opens a session on the graph
 * of the oldest waiting request: one batched CG (as lg_solve) whose columns
 * are slots, as wide as the columns then queued for that graph (a power of
 * two, at most max_batch_rhs), opened with every queued request of the graph
 * that fits.  At every CG iteration boundary the columns that have converged
 * leave, a request completes when all its columns have, and freed or idle
 * slots take the next queued requests for the same graph, tolerance and
 * iteration cap (a request's columns enter together), unless a request of
 * another graph has waited longer and no worker is free.  Each
 * column runs its own CG (iteration cap, restarts, convergence test).
 * Sessions on different graphs overlap on the device.  A graph's hierarchy is
 * built on its first request and cached; it is admitted when it fits
 * hbm_budget after freeing the least recently used idle hierarchies (a
 * hierarchy larger than the budget runs alone).  A column's result depends on
 * the session's width and its slot only through summation orders, so it
 * agrees with the same request solved alone within the solver tolerance.
 * ------------------------------------------------------------------------ */
typedef struct lg_server lg_server;

typedef struct {
  int32_t workers;        /* worker threads / HIP streams, 1..64 (default 4) */
  int32_t max_batch_rhs;  /* columns per batched solve, 1..32 (default 32) */
  size_t hbm_budget;      /* bytes of cached hierarchies; 0 = 3/4 of free device memory */
  lg_setup_opts setup;    /* options of every hierarchy (max_rhs is taken from max_batch_rhs) */
} lg_server_opts;

typedef struct {
  int64_t submitted, completed; /* requests */
  int64_t batches;              /* sessions (slot-batched solves) run */
  int64_t batched_columns;      /* right-hand sides solved in them */
  int64_t setups, evictions;    /* hierarchies built and freed for room */
  size_t resident_bytes;        /* device bytes of the cached hierarchies */
  size_t budget_bytes;          /* the admission budget in effect */
  int32_t resident_graphs;
  int64_t refills;              /* right-hand sides admitted into a session already running */
} lg_server_stats;

/* Fill o with the defaults (4 workers, 32 columns, budget from free memory,
 * the paper's setup parameters). */
lg_status lg_server_default_opts(lg_server_opts* o);

/* Start a server on the current HIP device (o may be NULL for defaults). */
lg_status lg_server_create(const lg_server_opts* o, lg_server** out);

/* Register a graph (lg_graph as for lg_setup, host or device arrays, copied
 * to host memory during the call); *graph_id identifies it in submits.
 * Invalid or disconnected graphs are reported by the requests on them. */
lg_status lg_server_add_graph(lg_server* s, const lg_graph* g, int32_t* graph_id);

/* Queue a solve of L X = B - mean(B) for k columns (1..max_batch_rhs).  B and
 * X are device n x k row-major fp64 arrays owned by the caller: B must hold
 * its values when this is called, and both must stay valid until
 * lg_server_wait returns for *request_id.  Never blocks on the solve. */
lg_status lg_server_submit(lg_server* s, int32_t graph_id, const double* B, double* X, int32_t k,
                           double rtol, int32_t max_iter, int64_t* request_id);

/* Block until the request is done; fills info (host, k entries, may be NULL)
 * and *latency_ms (submit to completion, may be NULL), forgets the request
 * and returns its status (LG_OK, LG_E_NOT_CONVERGED, or the setup error of
 * its graph).  Each request is waited for once. */
lg_status lg_server_wait(lg_server* s, int64_t request_id, lg_rhs_info* info, double* latency_ms);

lg_status lg_server_stats_get(lg_server* s, lg_server_stats* out);

/* Finish all queued requests, stop the workers and free every hierarchy. */
void lg_server_free(lg_server* s);

#ifdef __cplusplus
}
#endif
#endif
