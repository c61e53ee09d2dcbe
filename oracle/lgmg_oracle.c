/*
 * lgmg_oracle.c -- plain CPU oracle for the unsmoothed-aggregation multigrid
 * for graph Laplacians of Konolige & Brown, "A Parallel Solver for Graph
 * Laplacians" (PASC'18).
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load this library.
 * It shares no code with the GPU library; both are written independently from
 * the paper and from the conventions listed below.
 *
 * Slow and obvious on purpose: fp64, loops in the order the paper states the
 * steps.  Compile with -ffp-contract=off (no fused multiply-add) so every
 * product and sum is rounded on its own.  The tests use a single-threaded
 * build.  A second build with -fopenmp (for the CPU timing baseline only) runs
 * the loops whose iterations each write their own row in parallel; every
 * floating-point reduction, and every loop that adds into shared entries in
 * floating point, stays serial, so both builds compute identical bits.
 *
 * Conventions where the paper leaves the arithmetic open (each is a reading):
 *  - Exact sums ("XSUM").  Every sum that feeds a decision or a stored
 *    hierarchy value (row sums, the Jacobi sums of the test vectors, Galerkin
 *    and Schur-complement entries) is order independent: each fp64 term is
 *    rounded to the nearest multiple of 2^-64 (ties to even), the integers are
 *    added exactly, and the total is rounded once to the nearest fp64 (ties to
 *    even).  Graphs whose total edge weight is 2^62 or more are rejected.
 *  - Counter-based randomness: the SplitMix64 output function (Steele, Lea &
 *    Flood, OOPSLA 2014) applied to multiples of its golden-ratio increment.
 *  - The elimination hash is that generator's i-th output, a bijection.
 *  - Voting uses the total order (state, strength, -index) for its argmax.
 */
#include "lgmg_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;
typedef unsigned __int128 u128;

#define GOLDEN 0x9e3779b97f4a7c15ULL
#define MAXLEV 128
#define ST_DECIDED 0
#define ST_UNDECIDED 1
#define ST_SEED 2
#define TV_LANCZOS_STREAM 64

/* Threads the row-parallel loops use: 1 in the single-threaded build. */
int32_t lgo_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

void lgo_default_opts(lgo_opts* o) {
  memset(o, 0, sizeof(*o));
  o->elim_enable = 1;
  o->elim_max_degree = 4;      /* Section 3.4: degree 4 or less */
  o->elim_min_fraction = 0.05; /* Section 3.4: only if more than 5% eliminated */
  o->agg_iters = 10;           /* Section 3.5: 10 voting iterations */
  o->agg_filter_base = 0.5;    /* Algorithm 3: filter factor 0.5^iter */
  o->seed_votes = 8;           /* Section 3.5: 8 or more votes */
  o->tv_sweeps = 3;            /* Section 3.5: four vectors, three Jacobi sweeps */
  o->tv_omega = 2.0 / 3.0;     /* damping: not stated in the paper (a reading) */
  o->cheb_degree = 2;          /* Section 4: degree-2 Chebyshev */
  o->cheb_lo = 0.3;            /* Section 3.6: 0.3 and 1.1 times lambda_max */
  o->cheb_hi = 1.1;
  o->eig_iters = 10;           /* Section 3.6: 10 iterations for lambda_max */
  o->coarsest_nnz = 1000;      /* Section 4: coarsest L has at most 1000 nonzeros */
  o->max_levels = 64;
  o->cycle = 1;
  o->hash_mode = 0;
  o->seed = 12345;
  o->elim_passes = 1;  /* one pass, as the paper applies; more repeat it on the result */
}

/* ---------------------------------------------------------------- RNG ---- */

/* SplitMix64 output function (Steele, Lea & Flood 2014). */
uint64_t lgo_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* Hash of a vertex id for elimination (Section 3.4): the id-th output of
 * SplitMix64 seeded with 0; mode 1 is the identity (tests of the chain cases). */
uint64_t lgo_hash(int64_t i, int32_t mode) {
  if (mode == 1) return (uint64_t)i;
  return lgo_mix64((uint64_t)(i + 1) * GOLDEN);
}

/* Test-vector entry k of vertex i on hierarchy level `level`, uniform in [-1, 1). */
double lgo_tv(uint64_t seed, int32_t level, int32_t k, int64_t i) {
  uint64_t key = lgo_mix64((seed + 1) * GOLDEN);
  uint64_t ctr = key ^ (((uint64_t)level << 56) | ((uint64_t)k << 48) | (uint64_t)i);
  uint64_t u = lgo_mix64((ctr + 1) * GOLDEN) >> 11;
  return 2.0 * ((double)u * 0x1p-53) - 1.0;
}

/* -------------------------------------------------------- exact sums ---- */

/* Nearest integer to v * 2^64, ties to even.  Nonzero return = out of range. */
static int xs_term(double v, i128* out) {
  if (!isfinite(v)) return 1;
  double y = ldexp(v, 64); /* exact scaling */
  if (fabs(y) >= 0x1p126) return 1;
  double ip = trunc(y);
  double fr = y - ip; /* exact: the fractional part of a double */
  i128 t = (i128)ip;  /* exact: ip is an integer below 2^126 */
  double afr = fabs(fr);
  int up = 0;
  if (afr > 0.5) up = 1;
  else if (afr == 0.5) up = (int)(t & 1);
  if (up) t += (v < 0) ? -1 : 1;
  *out = t;
  return 0;
}

/* Nearest fp64 to s * 2^-64, ties to even (libgcc's int128 -> double is
 * correctly rounded; the scaling by 2^-64 is exact). */
static double xs_round(i128 s) {
  if (s == 0) return 0.0;
  return ldexp((double)s, -64);
}

int lgo_xs_term(double v, int64_t* hi, uint64_t* lo) {
  i128 t = 0;
  int st = xs_term(v, &t);
  *hi = (int64_t)(t >> 64);
  *lo = (uint64_t)t;
  return st ? LGO_E_RANGE : LGO_OK;
}

double lgo_xs_round(int64_t hi, uint64_t lo) {
  u128 u = ((u128)(uint64_t)hi << 64) | (u128)lo;
  return xs_round((i128)u);
}

typedef struct {
  u128 s; /* wraps mod 2^128; the final value is in range by the weight guard */
  int bad;
} xacc;

static void xa_init(xacc* a) { a->s = 0; a->bad = 0; }
static void xa_add(xacc* a, double v) {
  i128 t;
  if (xs_term(v, &t)) a->bad = 1;
  else a->s += (u128)t;
}
static double xa_value(const xacc* a) { return xs_round((i128)a->s); }

int lgo_xsum(const double* t, int64_t n, double* out) {
  xacc a;
  xa_init(&a);
  for (int64_t i = 0; i < n; i++) xa_add(&a, t[i]);
  *out = xa_value(&a);
  return a.bad ? LGO_E_RANGE : LGO_OK;
}

/* ----------------------------------------------------- graph basics ---- */

typedef struct {
  int64_t n, nnz;
  int64_t* rp;
  int32_t* col;
  double* w;
  double* d;
} ocsr;

static void* xmalloc(size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p) {
    fprintf(stderr, "lgmg_oracle: out of memory (%zu bytes)\n", bytes);
    abort();
  }
  return p;
}
static void* xcalloc(size_t n, size_t sz) {
  void* p = calloc(n ? n : 1, sz ? sz : 1);
  if (!p) {
    fprintf(stderr, "lgmg_oracle: out of memory\n");
    abort();
  }
  return p;
}

/* Position of column j in row i, or -1. */
static int64_t find_entry(const int64_t* rp, const int32_t* col, int64_t i, int64_t j) {
  int64_t lo = rp[i], hi = rp[i + 1] - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] == j) return mid;
    if (col[mid] < j) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

/* Input checks of Section 2.1: undirected (symmetric weights), w > 0, no
 * self-loops, connected; plus the CSR layout rules and the weight guard. */
int lgo_validate(int64_t n, const int64_t* rp, const int32_t* col, const double* w) {
  if (n < 1 || !rp) return LGO_E_ARG;
  if (rp[0] != 0) return LGO_E_GRAPH;
  for (int64_t i = 0; i < n; i++)
    if (rp[i + 1] < rp[i]) return LGO_E_GRAPH;
  if (rp[n] > 0 && (!col || !w)) return LGO_E_ARG;
  if (rp[n] >= ((int64_t)1 << 31)) return LGO_E_ARG;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : bad)
  for (int64_t i = 0; i < n; i++) {
    for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
      int64_t j = col[e];
      if (j < 0 || j >= n || j == i) { bad = 1; break; }
      if (e > rp[i] && col[e - 1] >= j) { bad = 1; break; }
      if (!(w[e] > 0.0) || !isfinite(w[e])) { bad = 1; break; }
      int64_t back = find_entry(rp, col, j, i);
      if (back < 0 || w[back] != w[e]) { bad = 1; break; }
    }
  }
  if (bad) return LGO_E_GRAPH;
  double total = 0.0;
  for (int64_t e = 0; e < rp[n]; e++) total += w[e];
  if (!(total < 0x1p62)) return LGO_E_RANGE;
  /* connectivity by breadth-first search from vertex 0 */
  int32_t* queue = (int32_t*)xmalloc(sizeof(int32_t) * n);
  uint8_t* seen = (uint8_t*)xcalloc(n, 1);
  int64_t head = 0, tail = 0;
  queue[tail++] = 0;
  seen[0] = 1;
  while (head < tail) {
    int64_t i = queue[head++];
    for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
      int32_t j = col[e];
      if (!seen[j]) {
        seen[j] = 1;
        queue[tail++] = j;
      }
    }
  }
  free(queue);
  free(seen);
  return tail == n ? LGO_OK : LGO_E_DISCONNECTED;
}

/* D_ii = sum_j A_ij (Section 2.1), as an exact sum. */
int lgo_diag(int64_t n, const int64_t* rp, const int32_t* col, const double* w, double* d) {
  (void)col;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : bad)
  for (int64_t i = 0; i < n; i++) {
    xacc a;
    xa_init(&a);
    for (int64_t e = rp[i]; e < rp[i + 1]; e++) xa_add(&a, w[e]);
    d[i] = xa_value(&a);
    bad |= a.bad;
  }
  return bad ? LGO_E_RANGE : LGO_OK;
}

/* y = L x = D x - A x, plain fp64 in row order. */
static void spmv(const ocsr* A, const double* x, double* y) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < A->n; i++) {
    double s = 0.0;
    for (int64_t e = A->rp[i]; e < A->rp[i + 1]; e++) s += A->w[e] * x[A->col[e]];
    y[i] = A->d[i] * x[i] - s;
  }
}

/* ------------------------------------------ low-degree elimination ---- */

/* Algorithm 2 (Section 3.4).  candidates_i = i if deg(i) <= max_degree, else
 * empty.  z = L (min-by-hash).(filter) candidates: z_i is the candidate with
 * the smallest hash among i and its neighbours (L's diagonal puts i in its own
 * neighbourhood), or -1 when there is none.  i is eliminated when z_i = i.
 * Returns |F|. */
int64_t lgo_elim_select(int64_t n, const int64_t* rp, const int32_t* col, int32_t max_degree,
                        int32_t hash_mode, int32_t* z, uint8_t* F) {
  int64_t count = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : count)
  for (int64_t i = 0; i < n; i++) {
    int64_t best = -1;
    uint64_t best_h = UINT64_MAX; /* hash of "no candidate" is infinity */
    if (rp[i + 1] - rp[i] <= max_degree) {
      best = i;
      best_h = lgo_hash(i, hash_mode);
    }
    for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
      int64_t j = col[e];
      if (rp[j + 1] - rp[j] > max_degree) continue;
      uint64_t h = lgo_hash(j, hash_mode);
      if (h < best_h) {
        best_h = h;
        best = j;
      }
    }
    z[i] = (int32_t)best;
    F[i] = (uint8_t)(best == i);
    count += F[i];
  }
  return count;
}

typedef struct {
  int32_t j;
  double v;
} entry;

static int cmp_entry(const void* a, const void* b) {
  int32_t x = ((const entry*)a)->j, y = ((const entry*)b)->j;
  return (x > y) - (x < y);
}

/* Sort (column, value) entries and add equal columns exactly.  Appends the
 * merged row at ccol/cw[*pos]; returns nonzero on overflow of cap or range. */
static int merge_row(entry* ent, int64_t cnt, int32_t* ccol, double* cw, int64_t* pos,
                     int64_t cap) {
  qsort(ent, (size_t)cnt, sizeof(entry), cmp_entry);
  int bad = 0;
  int64_t k = 0;
  while (k < cnt) {
    int64_t k2 = k;
    xacc a;
    xa_init(&a);
    while (k2 < cnt && ent[k2].j == ent[k].j) xa_add(&a, ent[k2++].v);
    if (*pos >= cap) return 1;
    ccol[*pos] = ent[k].j;
    cw[*pos] = xa_value(&a);
    bad |= a.bad;
    (*pos)++;
    k = k2;
  }
  return bad ? 2 : 0;
}

/* Elimination level (Section 3.4): C = V \ F numbered in increasing id, and the
 * Schur complement L_CC - L_FC^T L_FF^-1 L_FC.  With L_FF = diag(d_F), the
 * off-diagonal weight between a, b in C is
 *     w_ab + sum over f in F adjacent to both of (w_fa * w_fb) / d_f,
 * and the coarse diagonal is recomputed as the exact row sum so that the
 * coarse matrix keeps zero row sums.  Returns the coarse nnz (< 0: error). */
int64_t lgo_elim_build(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                       const double* d, const uint8_t* F, int32_t* cidx, int64_t* crp,
                       int32_t* ccol, double* cw, double* cd, int64_t cap) {
  int64_t nc = 0;
  for (int64_t i = 0; i < n; i++) cidx[i] = F[i] ? -1 : (int32_t)nc++;
  crp[0] = 0;
  int64_t pos = 0;
  int bad = 0;
  for (int64_t a = 0; a < n; a++) {
    if (F[a]) continue;
    int64_t cnt = 0;
    for (int64_t e = rp[a]; e < rp[a + 1]; e++) {
      int64_t f = col[e];
      cnt += F[f] ? (rp[f + 1] - rp[f] - 1) : 1;
    }
    entry* ent = (entry*)xmalloc(sizeof(entry) * (size_t)(cnt ? cnt : 1));
    int64_t k = 0;
    for (int64_t e = rp[a]; e < rp[a + 1]; e++) {
      int64_t b = col[e];
      if (!F[b]) {
        ent[k].j = cidx[b];
        ent[k].v = w[e];
        k++;
        continue;
      }
      int64_t f = b;
      double w_fa = w[e];
      for (int64_t e2 = rp[f]; e2 < rp[f + 1]; e2++) {
        int64_t c = col[e2];
        if (c == a) continue;
        if (F[c]) {
          free(ent);
          return -LGO_E_GRAPH; /* F must be independent */
        }
        ent[k].j = cidx[c];
        ent[k].v = (w_fa * w[e2]) / d[f];
        k++;
      }
    }
    int r = merge_row(ent, k, ccol, cw, &pos, cap);
    free(ent);
    if (r == 1) return -LGO_E_ARG;
    if (r == 2) bad = 1;
    crp[cidx[a] + 1] = pos;
  }
  for (int64_t a = 0; a < nc; a++) {
    xacc s;
    xa_init(&s);
    for (int64_t e = crp[a]; e < crp[a + 1]; e++) xa_add(&s, cw[e]);
    cd[a] = xa_value(&s);
    bad |= s.bad;
  }
  return bad ? -LGO_E_RANGE : pos;
}

/* ------------------------------------------------ strength of connection ---- */

/* Affinity strength of connection (Section 3.5).  Four random vectors get
 * tv_sweeps weighted-Jacobi sweeps on L y = 0,
 *     x_i <- (1 - omega) x_i + omega * (sum_j w_ij x_j) / d_i,
 * then per edge C_ij = (sum_k x_ik x_jk)^2 / ((sum_k x_ik^2)(sum_k x_jk^2))
 * (the reading of the printed formula: squares in the numerator only, which
 * keeps C in [0, 1]) and S_ij = C_ij / max(max_s C_is, max_s C_sj); S has a
 * zero diagonal because only off-diagonal entries are stored.  X is n x 4
 * row-major (the smoothed vectors), S is per stored edge. */
int lgo_soc(int64_t n, const int64_t* rp, const int32_t* col, const double* w, const double* d,
            const lgo_opts* o, int32_t level, double* X, double* S) {
  double* Y = (double*)xmalloc(sizeof(double) * 4 * (size_t)n);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; i++)
    for (int k = 0; k < 4; k++) X[i * 4 + k] = lgo_tv(o->seed, level, k, i);
  const double omega = o->tv_omega;
  const double keep = 1.0 - omega;
  for (int sweep = 0; sweep < o->tv_sweeps; sweep++) {
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : bad)
    for (int64_t i = 0; i < n; i++) {
      for (int k = 0; k < 4; k++) {
        xacc a;
        xa_init(&a);
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) xa_add(&a, w[e] * X[(int64_t)col[e] * 4 + k]);
        bad |= a.bad;
        double t = xa_value(&a) / d[i];
        Y[i * 4 + k] = keep * X[i * 4 + k] + omega * t;
      }
    }
    memcpy(X, Y, sizeof(double) * 4 * (size_t)n);
  }
  free(Y);
  double* sq = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* M = (double*)xmalloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; i++) {
    const double* xi = X + i * 4;
    sq[i] = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2] + xi[3] * xi[3];
  }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; i++) {
    const double* xi = X + i * 4;
    double m = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
      const double* xj = X + (int64_t)col[e] * 4;
      double p = xi[0] * xj[0] + xi[1] * xj[1] + xi[2] * xj[2] + xi[3] * xj[3];
      double den = sq[i] * sq[col[e]];
      double c = den > 0.0 ? (p * p) / den : 0.0;
      S[e] = c; /* C for now */
      if (c > m) m = c;
    }
    M[i] = m;
  }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; i++) {
    for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
      double mx = M[i] > M[col[e]] ? M[i] : M[col[e]];
      S[e] = mx > 0.0 ? S[e] / mx : 0.0;
    }
  }
  free(sq);
  free(M);
  return bad ? LGO_E_RANGE : LGO_OK;
}

/* ------------------------------------------------------- aggregation ---- */

/* Is (s1, w1, j1) ahead of (s2, w2, j2) in the argmax order: state first
 * (Seed > Undecided > Decided), then strength, then the smaller index. */
static int agg_better(int s1, double w1, int64_t j1, int s2, double w2, int64_t j2) {
  if (s1 != s2) return s1 > s2;
  if (w1 != w2) return w1 > w2;
  return j1 < j2;
}

/* Algorithm 3 (Section 3.5).  Per iteration t with filter tau = base^t:
 * each Undecided vertex takes the best kept neighbour (S_ij >= tau) under the
 * argmax order above; if that neighbour is a Seed it joins the Seed's
 * aggregate, if it is Undecided it votes for it.  All choices use the status
 * at the start of the iteration.  Votes persist; afterwards any vertex still
 * (Undecided, itself) with at least seed_votes votes becomes a Seed.  At the
 * end every vertex's index names its root; roots (Seeds and leftover
 * Undecided vertices) are numbered in increasing vertex id.  Returns the
 * number of aggregates; state/idx/votes hold the final status. */
int64_t lgo_aggregate(int64_t n, const int64_t* rp, const int32_t* col, const double* S,
                      const lgo_opts* o, int32_t* state, int32_t* idx, int32_t* votes,
                      int32_t* agg) {
  int32_t* nstate = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n);
  int32_t* nidx = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n);
  int32_t* lv = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n);
  for (int64_t i = 0; i < n; i++) {
    state[i] = ST_UNDECIDED;
    idx[i] = (int32_t)i;
    votes[i] = 0;
  }
  double tau = 1.0;
  for (int it = 1; it <= o->agg_iters; it++) {
    tau *= o->agg_filter_base;
    memcpy(nstate, state, sizeof(int32_t) * (size_t)n);
    memcpy(nidx, idx, sizeof(int32_t) * (size_t)n);
    memset(lv, 0, sizeof(int32_t) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; i++) {
      if (state[i] != ST_UNDECIDED) continue;
      int have = 0, bs = 0;
      double bw = 0.0;
      int64_t bj = 0;
      for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
        if (!(S[e] >= tau)) continue;
        int64_t j = col[e];
        if (!have || agg_better(state[j], S[e], idx[j], bs, bw, bj)) {
          have = 1;
          bs = state[j];
          bw = S[e];
          bj = idx[j];
        }
      }
      if (!have) continue;
      if (bs == ST_SEED) {
        nstate[i] = ST_DECIDED;
        nidx[i] = (int32_t)bj;
      } else if (bs == ST_UNDECIDED) {
#pragma omp atomic
        lv[bj] += 1; /* integer tally: the same total in any order */
      }
    }
    for (int64_t i = 0; i < n; i++) votes[i] += lv[i];
    for (int64_t i = 0; i < n; i++)
      if (nstate[i] == ST_UNDECIDED && nidx[i] == i && votes[i] >= o->seed_votes)
        nstate[i] = ST_SEED;
    memcpy(state, nstate, sizeof(int32_t) * (size_t)n);
    memcpy(idx, nidx, sizeof(int32_t) * (size_t)n);
  }
  free(nstate);
  free(nidx);
  free(lv);
  /* global renumbering of the roots (Section 3.5) */
  int32_t* rank = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n);
  int64_t nc = 0;
  for (int64_t i = 0; i < n; i++) rank[i] = (idx[i] == i) ? (int32_t)nc++ : -1;
  for (int64_t i = 0; i < n; i++) agg[i] = rank[idx[i]];
  free(rank);
  return nc;
}

/* Galerkin coarse operator L_c = R L P with R_{v_j j} = 1, P = R^T
 * (Section 3.5).  For aggregates I != J the coarse off-diagonal weight is the
 * exact sum of the fine weights between them; weight inside an aggregate
 * cancels from the coarse Laplacian, whose diagonal is again the exact row
 * sum.  Returns the coarse nnz (< 0: error). */
int64_t lgo_galerkin(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                     const int32_t* agg, int64_t nc, int64_t* crp, int32_t* ccol, double* cw,
                     double* cd, int64_t cap) {
  /* members of each aggregate (counting sort, increasing vertex id) */
  int64_t* mp = (int64_t*)xcalloc((size_t)nc + 1, sizeof(int64_t));
  int64_t* mem = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < n; i++) mp[agg[i] + 1]++;
  for (int64_t I = 0; I < nc; I++) mp[I + 1] += mp[I];
  int64_t* fill = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(nc ? nc : 1));
  for (int64_t I = 0; I < nc; I++) fill[I] = mp[I];
  for (int64_t i = 0; i < n; i++) mem[fill[agg[i]]++] = i;
  free(fill);
  crp[0] = 0;
  int64_t pos = 0;
  int bad = 0;
  for (int64_t I = 0; I < nc; I++) {
    int64_t cnt = 0;
    for (int64_t k = mp[I]; k < mp[I + 1]; k++) cnt += rp[mem[k] + 1] - rp[mem[k]];
    entry* ent = (entry*)xmalloc(sizeof(entry) * (size_t)(cnt ? cnt : 1));
    int64_t m = 0;
    for (int64_t k = mp[I]; k < mp[I + 1]; k++) {
      int64_t i = mem[k];
      for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
        int32_t J = agg[col[e]];
        if (J == I) continue;
        ent[m].j = J;
        ent[m].v = w[e];
        m++;
      }
    }
    int r = merge_row(ent, m, ccol, cw, &pos, cap);
    free(ent);
    if (r == 1) {
      free(mp);
      free(mem);
      return -LGO_E_ARG;
    }
    if (r == 2) bad = 1;
    crp[I + 1] = pos;
  }
  for (int64_t I = 0; I < nc; I++) {
    xacc s;
    xa_init(&s);
    for (int64_t e = crp[I]; e < crp[I + 1]; e++) xa_add(&s, cw[e]);
    cd[I] = xa_value(&s);
    bad |= s.bad;
  }
  free(mp);
  free(mem);
  return bad ? -LGO_E_RANGE : pos;
}

/* ------------------------------------------------- eigenvalue estimate ---- */

/* Number of eigenvalues of the symmetric tridiagonal (alpha, beta) below x
 * (Sturm sequence of the LDL^T pivots). */
static int sturm_below(const double* a, const double* b, int m, double x) {
  int c = 0;
  double q = 1.0;
  for (int i = 0; i < m; i++) {
    q = (a[i] - x) - (i > 0 ? (b[i - 1] * b[i - 1]) / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) c++;
  }
  return c;
}

/* Largest eigenvalue of the m x m symmetric tridiagonal matrix with diagonal
 * alpha[0..m) and off-diagonal beta[0..m-1), by bisection. */
double lgo_tridiag_max(const double* alpha, const double* beta, int32_t m) {
  if (m <= 0) return 0.0;
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < m; i++) {
    double r = (i > 0 ? fabs(beta[i - 1]) : 0.0) + (i < m - 1 ? fabs(beta[i]) : 0.0);
    if (alpha[i] - r < lo) lo = alpha[i] - r;
    if (alpha[i] + r > hi) hi = alpha[i] + r;
  }
  hi += 1e-12 * fabs(hi) + 1e-300;
  lo -= 1e-12 * fabs(lo) + 1e-300;
  for (int it = 0; it < 400; it++) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_below(alpha, beta, m, mid) == m) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

/* Exact (order-free) sums for the Lanczos estimate: like every other sum that
 * feeds a stored hierarchy value, they are XSUM accumulations (lambda_max
 * sets the smoother's interval).  xdot: sum of a_i b_i, or of (d_i a_i) a_i
 * when d is given, or of a_i when b and d are NULL. */
static double xdot(const double* a, const double* b, const double* d, int64_t n, int* bad) {
  xacc s;
  xa_init(&s);
  for (int64_t i = 0; i < n; i++)
    xa_add(&s, d ? (d[i] * a[i]) * a[i] : b ? a[i] * b[i] : a[i]);
  *bad |= s.bad;
  return xa_value(&s);
}

/* y = L x with each row's sum of w_ij x_j exact. */
static void spmv_exact(const ocsr* A, const double* x, double* y, int* bad) {
  int b = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : b)
  for (int64_t i = 0; i < A->n; i++) {
    xacc s;
    xa_init(&s);
    for (int64_t e = A->rp[i]; e < A->rp[i + 1]; e++) xa_add(&s, A->w[e] * x[A->col[e]]);
    b |= s.bad;
    y[i] = A->d[i] * x[i] - xa_value(&s);
  }
  *bad |= b;
}

/* lambda_max of D^-1 L by `steps` Lanczos steps in the D inner product
 * (equivalent to Arnoldi for this D-self-adjoint operator; Section 3.6 uses
 * 10 Arnoldi iterations).  Start vector: the counter generator's stream 64 at
 * this level, mean-projected.  Every sum is exact, so the Ritz values do not
 * depend on summation order (a clustered spectrum makes ten steps sensitive
 * to it).  Returns the largest Ritz value. */
double lgo_lanczos_lmax(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                        const double* d, int32_t steps, uint64_t seed, int32_t level) {
  if (n < 2 || steps < 1) return 0.0;
  ocsr A = {n, rp[n], (int64_t*)rp, (int32_t*)col, (double*)w, (double*)d};
  double* q = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* qp = (double*)xcalloc((size_t)n, sizeof(double));
  double* u = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* al = (double*)xcalloc((size_t)steps, sizeof(double));
  double* be = (double*)xcalloc((size_t)steps, sizeof(double));
  int bad = 0;
  for (int64_t i = 0; i < n; i++) q[i] = lgo_tv(seed, level, TV_LANCZOS_STREAM, i);
  double mean = xdot(q, NULL, NULL, n, &bad);
  for (int64_t i = 0; i < n; i++) q[i] -= mean / (double)n;
  double nrm = sqrt(xdot(q, NULL, d, n, &bad));
  for (int64_t i = 0; i < n; i++) q[i] /= nrm;
  double bprev = 0.0, scale = 0.0;
  int m = 0;
  for (int j = 0; j < steps; j++) {
    spmv_exact(&A, q, u, &bad); /* u = L q */
    double a = xdot(q, u, NULL, n, &bad);
    al[j] = a;
    m = j + 1;
    for (int64_t i = 0; i < n; i++) u[i] = u[i] / d[i] - a * q[i] - bprev * qp[i];
    double b = sqrt(xdot(u, NULL, d, n, &bad));
    if (fabs(a) + bprev > scale) scale = fabs(a) + bprev;
    if (j == steps - 1 || b <= 1e-12 * scale) break;
    be[j] = b;
    for (int64_t i = 0; i < n; i++) {
      qp[i] = q[i];
      q[i] = u[i] / b;
    }
    bprev = b;
  }
  double lmax = lgo_tridiag_max(al, be, m);
  free(q);
  free(qp);
  free(u);
  free(al);
  free(be);
  return lmax;
}

/* ---------------------------------------------------------- smoother ---- */

/* One application of degree-k Chebyshev iteration on D^-1 L for the interval
 * [cheb_lo, cheb_hi] * lmax (Section 3.6), in the three-term form of Saad,
 * Iterative Methods for Sparse Linear Systems, Algorithm 12.1, with the
 * Jacobi-preconditioned residual r = D^-1 (b - L x). */
static void cheb(const ocsr* A, double lmax, const lgo_opts* o, double* x, const double* b,
                 int x_is_zero, double* r, double* p, double* t) {
  int64_t n = A->n;
  if (o->cheb_degree < 1 || !(lmax > 0.0)) return;
  double lo = o->cheb_lo * lmax, hi = o->cheb_hi * lmax;
  double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
  double sigma = theta / delta;
  double rho = 1.0 / sigma;
  if (x_is_zero) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) r[i] = b[i] / A->d[i];
  } else {
    spmv(A, x, t);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) r[i] = (b[i] - t[i]) / A->d[i];
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    p[i] = r[i] / theta;
    x[i] = (x_is_zero ? 0.0 : x[i]) + p[i];
  }
  for (int k = 1; k < o->cheb_degree; k++) {
    double rho1 = 1.0 / (2.0 * sigma - rho);
    double c1 = rho1 * rho, c2 = 2.0 * rho1 / delta;
    spmv(A, x, t);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
      r[i] = (b[i] - t[i]) / A->d[i];
      p[i] = c1 * p[i] + c2 * r[i];
      x[i] += p[i];
    }
    rho = rho1;
  }
}

int lgo_cheb_apply(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                   const double* d, double lmax, const lgo_opts* o, double* x, const double* b,
                   int32_t x_is_zero) {
  ocsr A = {n, rp[n], (int64_t*)rp, (int32_t*)col, (double*)w, (double*)d};
  double* r = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* p = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* t = (double*)xmalloc(sizeof(double) * (size_t)n);
  cheb(&A, lmax, o, x, b, x_is_zero, r, p, t);
  free(r);
  free(p);
  free(t);
  return LGO_OK;
}

/* --------------------------------------------------------- coarsest ---- */

/* Dense pseudo-inverse of a connected graph's Laplacian, the coarsest
 * level's direct solve (Algorithm 1):
 *     L^+ = (L + (s/n) 11^T)^-1 - 11^T/(s n)    for any s > 0,
 * because 1 spans the null space and is an eigenvector of L + (s/n)11^T with
 * eigenvalue s.  s = max_i d_i (an order-free choice) puts that eigenvalue
 * inside the range of L's other eigenvalues, so the matrix inverted is no worse
 * conditioned than L is on the mean-zero space; s = 1 would not be when the
 * weights are far from 1.  Inverted by Cholesky in fp64. */
int lgo_pinv_dense(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
                   const double* d, double* out) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++)
    if (d[i] > s) s = d[i];
  if (!(s > 0.0)) s = 1.0; /* one vertex: L = 0 */
  double shift = s / (double)n, inv_sn = 1.0 / (s * (double)n);
  double* M = (double*)xmalloc(sizeof(double) * (size_t)(n * n));
  for (int64_t i = 0; i < n * n; i++) M[i] = shift;
  for (int64_t i = 0; i < n; i++) {
    M[i * n + i] += d[i];
    for (int64_t e = rp[i]; e < rp[i + 1]; e++) M[i * n + col[e]] -= w[e];
  }
  /* Cholesky M = G G^T, G lower (stored in M's lower triangle) */
  for (int64_t j = 0; j < n; j++) {
    double s = M[j * n + j];
    for (int64_t k = 0; k < j; k++) s -= M[j * n + k] * M[j * n + k];
    if (!(s > 0.0)) {
      free(M);
      return LGO_E_GRAPH;
    }
    double gjj = sqrt(s);
    M[j * n + j] = gjj;
    for (int64_t i = j + 1; i < n; i++) {
      double t = M[i * n + j];
      for (int64_t k = 0; k < j; k++) t -= M[i * n + k] * M[j * n + k];
      M[i * n + j] = t / gjj;
    }
  }
  /* columns of M^-1 by forward and back substitution */
  double* y = (double*)xmalloc(sizeof(double) * (size_t)n);
  for (int64_t c = 0; c < n; c++) {
    for (int64_t i = 0; i < n; i++) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int64_t k = 0; k < i; k++) t -= M[i * n + k] * y[k];
      y[i] = t / M[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; i--) {
      double t = y[i];
      for (int64_t k = i + 1; k < n; k++) t -= M[k * n + i] * y[k];
      y[i] = t / M[i * n + i];
    }
    for (int64_t i = 0; i < n; i++) out[i * n + c] = y[i] - inv_sn;
  }
  free(y);
  free(M);
  return LGO_OK;
}

/* -------------------------------------------------------- hierarchy ---- */

typedef struct {
  int32_t type;
  ocsr A;
  int64_t nc;
  int32_t* map; /* AGG: aggregate of each vertex; ELIM: coarse index or -1 */
  int32_t* z;
  double* X;
  double* S;
  int32_t *state, *idx, *votes;
  double lmax;
  int64_t nnzP; /* ELIM: nnz of the prolongation (|C| + sum of F degrees) */
} olevel;

struct lgo_hier {
  int32_t nlev;
  olevel lev[MAXLEV];
  double* Lplus;
  lgo_opts o;
  double work; /* work counter of the current solve, in finest-residual units */
};

static void free_csr(ocsr* A) {
  free(A->rp);
  free(A->col);
  free(A->w);
  free(A->d);
  memset(A, 0, sizeof(*A));
}

void lgo_free(lgo_hier* h) {
  if (!h) return;
  for (int l = 0; l < h->nlev; l++) {
    olevel* L = &h->lev[l];
    free_csr(&L->A);
    free(L->map);
    free(L->z);
    free(L->X);
    free(L->S);
    free(L->state);
    free(L->idx);
    free(L->votes);
  }
  free(h->Lplus);
  free(h);
}

static int shrink_csr(ocsr* C, int64_t n, int64_t nnz) {
  C->n = n;
  C->nnz = nnz;
  C->col = (int32_t*)realloc(C->col, sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
  C->w = (double*)realloc(C->w, sizeof(double) * (size_t)(nnz ? nnz : 1));
  return (C->col && C->w) ? 0 : 1;
}

/* Level loop (Section 3.4, 3.5, 4): while nnz(L) = n + nnz(A) exceeds
 * coarsest_nnz, try one elimination pass (applied when more than
 * elim_min_fraction of the vertices go), then aggregate.  The last level is
 * solved exactly with a dense pseudo-inverse. */
int lgo_setup(int64_t n, const int64_t* rp, const int32_t* col, const double* w,
              const lgo_opts* o, lgo_hier** out) {
  *out = NULL;
  int st = lgo_validate(n, rp, col, w);
  if (st) return st;
  lgo_hier* h = (lgo_hier*)xcalloc(1, sizeof(lgo_hier));
  h->o = *o;
  int64_t nnz = rp[n];
  olevel* L0 = &h->lev[0];
  L0->A.n = n;
  L0->A.nnz = nnz;
  L0->A.rp = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(n + 1));
  L0->A.col = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
  L0->A.w = (double*)xmalloc(sizeof(double) * (size_t)(nnz ? nnz : 1));
  L0->A.d = (double*)xmalloc(sizeof(double) * (size_t)n);
  memcpy(L0->A.rp, rp, sizeof(int64_t) * (size_t)(n + 1));
  if (nnz) {
    memcpy(L0->A.col, col, sizeof(int32_t) * (size_t)nnz);
    memcpy(L0->A.w, w, sizeof(double) * (size_t)nnz);
  }
  h->nlev = 1;
  st = lgo_diag(n, rp, col, w, L0->A.d);
  if (st) goto fail;
  int l = 0;
  for (;;) {
    olevel* cur = &h->lev[l];
    int64_t nl = cur->A.n;
    if (nl + cur->A.nnz <= o->coarsest_nnz || l + 1 >= o->max_levels || l + 2 >= MAXLEV) break;
    /* Section 3.4's elimination, repeated on its own result while it still
       removes more than the minimum fraction (elim_passes > 1) */
    int stop = 0;
    for (int pass = 0; o->elim_enable && pass < o->elim_passes; pass++) {
      int32_t* z = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nl);
      uint8_t* F = (uint8_t*)xmalloc((size_t)nl);
      int64_t nf = lgo_elim_select(nl, cur->A.rp, cur->A.col, o->elim_max_degree, o->hash_mode,
                                   z, F);
      if ((double)nf > o->elim_min_fraction * (double)nl) {
        olevel* nxt = &h->lev[l + 1];
        /* an eliminated vertex of degree k adds at most k (k - 1) fill entries */
        const int64_t kmax = o->elim_max_degree > 1 ? o->elim_max_degree : 1;
        int64_t cap = cur->A.nnz + kmax * (kmax - 1) * nf + 1;
        nxt->A.rp = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(nl - nf + 1));
        nxt->A.col = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)cap);
        nxt->A.w = (double*)xmalloc(sizeof(double) * (size_t)cap);
        nxt->A.d = (double*)xmalloc(sizeof(double) * (size_t)(nl - nf));
        cur->map = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nl);
        int64_t cn = lgo_elim_build(nl, cur->A.rp, cur->A.col, cur->A.w, cur->A.d, F, cur->map,
                                    nxt->A.rp, nxt->A.col, nxt->A.w, nxt->A.d, cap);
        if (cn < 0) {
          free(z);
          free(F);
          h->nlev = l + 2;
          st = (int)-cn;
          goto fail;
        }
        shrink_csr(&nxt->A, nl - nf, cn);
        cur->type = LGO_ELIM;
        cur->nc = nl - nf;
        cur->z = z;
        int64_t nnzP = cur->nc;
        for (int64_t i = 0; i < nl; i++)
          if (F[i]) nnzP += cur->A.rp[i + 1] - cur->A.rp[i];
        cur->nnzP = nnzP;
        free(F);
        h->nlev = l + 2;
        l++;
        cur = &h->lev[l];
        nl = cur->A.n;
        if (nl + cur->A.nnz <= o->coarsest_nnz || l + 1 >= o->max_levels || l + 2 >= MAXLEV) {
          stop = 1;
          break;
        }
      } else {
        free(z);
        free(F);
        break;
      }
    }
    if (stop) break;
    /* aggregation level */
    cur->X = (double*)xmalloc(sizeof(double) * 4 * (size_t)nl);
    cur->S = (double*)xmalloc(sizeof(double) * (size_t)(cur->A.nnz ? cur->A.nnz : 1));
    st = lgo_soc(nl, cur->A.rp, cur->A.col, cur->A.w, cur->A.d, o, l, cur->X, cur->S);
    if (st) goto fail;
    cur->state = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nl);
    cur->idx = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nl);
    cur->votes = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nl);
    cur->map = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nl);
    int64_t nc = lgo_aggregate(nl, cur->A.rp, cur->A.col, cur->S, o, cur->state, cur->idx,
                               cur->votes, cur->map);
    if (nc >= nl) { /* no progress: this level becomes the coarsest */
      free(cur->map);
      cur->map = NULL;
      break;
    }
    olevel* nxt = &h->lev[l + 1];
    int64_t cap = cur->A.nnz + 1;
    nxt->A.rp = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(nc + 1));
    nxt->A.col = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)cap);
    nxt->A.w = (double*)xmalloc(sizeof(double) * (size_t)cap);
    nxt->A.d = (double*)xmalloc(sizeof(double) * (size_t)nc);
    int64_t cn = lgo_galerkin(nl, cur->A.rp, cur->A.col, cur->A.w, cur->map, nc, nxt->A.rp,
                              nxt->A.col, nxt->A.w, nxt->A.d, cap);
    h->nlev = l + 2;
    if (cn < 0) {
      st = (int)-cn;
      goto fail;
    }
    shrink_csr(&nxt->A, nc, cn);
    cur->type = LGO_AGG;
    cur->nc = nc;
    cur->lmax = lgo_lanczos_lmax(nl, cur->A.rp, cur->A.col, cur->A.w, cur->A.d, o->eig_iters,
                                 o->seed, l);
    l++;
  }
  h->nlev = l + 1;
  olevel* last = &h->lev[l];
  last->type = LGO_COARSEST;
  if (last->A.n > 2048) {
    st = LGO_E_ARG; /* coarsening stalled far above a dense-solvable size */
    goto fail;
  }
  h->Lplus = (double*)xmalloc(sizeof(double) * (size_t)(last->A.n * last->A.n));
  st = lgo_pinv_dense(last->A.n, last->A.rp, last->A.col, last->A.w, last->A.d, h->Lplus);
  if (st) goto fail;
  *out = h;
  return LGO_OK;
fail:
  lgo_free(h);
  return st;
}

int32_t lgo_num_levels(const lgo_hier* h) { return h->nlev; }

int lgo_level_info(const lgo_hier* h, int32_t l, int32_t* type, int64_t* n, int64_t* nnz,
                   int64_t* nc, double* lmax) {
  if (l < 0 || l >= h->nlev) return LGO_E_ARG;
  const olevel* L = &h->lev[l];
  *type = L->type;
  *n = L->A.n;
  *nnz = L->A.nnz;
  *nc = L->nc;
  *lmax = L->lmax;
  return LGO_OK;
}

int lgo_level_csr(const lgo_hier* h, int32_t l, int64_t* rp, int32_t* col, double* w, double* d) {
  if (l < 0 || l >= h->nlev) return LGO_E_ARG;
  const ocsr* A = &h->lev[l].A;
  memcpy(rp, A->rp, sizeof(int64_t) * (size_t)(A->n + 1));
  if (A->nnz) {
    memcpy(col, A->col, sizeof(int32_t) * (size_t)A->nnz);
    memcpy(w, A->w, sizeof(double) * (size_t)A->nnz);
  }
  memcpy(d, A->d, sizeof(double) * (size_t)A->n);
  return LGO_OK;
}

int lgo_level_map(const lgo_hier* h, int32_t l, int32_t* map) {
  if (l < 0 || l >= h->nlev || !h->lev[l].map) return LGO_E_ARG;
  memcpy(map, h->lev[l].map, sizeof(int32_t) * (size_t)h->lev[l].A.n);
  return LGO_OK;
}

int lgo_level_elim(const lgo_hier* h, int32_t l, int32_t* z) {
  if (l < 0 || l >= h->nlev || !h->lev[l].z) return LGO_E_ARG;
  memcpy(z, h->lev[l].z, sizeof(int32_t) * (size_t)h->lev[l].A.n);
  return LGO_OK;
}

int lgo_level_soc(const lgo_hier* h, int32_t l, double* X, double* S) {
  if (l < 0 || l >= h->nlev || !h->lev[l].S) return LGO_E_ARG;
  const olevel* L = &h->lev[l];
  memcpy(X, L->X, sizeof(double) * 4 * (size_t)L->A.n);
  if (L->A.nnz) memcpy(S, L->S, sizeof(double) * (size_t)L->A.nnz);
  return LGO_OK;
}

int lgo_level_votes(const lgo_hier* h, int32_t l, int32_t* state, int32_t* idx, int32_t* votes) {
  if (l < 0 || l >= h->nlev || !h->lev[l].state) return LGO_E_ARG;
  const olevel* L = &h->lev[l];
  memcpy(state, L->state, sizeof(int32_t) * (size_t)L->A.n);
  memcpy(idx, L->idx, sizeof(int32_t) * (size_t)L->A.n);
  memcpy(votes, L->votes, sizeof(int32_t) * (size_t)L->A.n);
  return LGO_OK;
}

int lgo_coarsest_pinv(const lgo_hier* h, double* out) {
  int64_t n = h->lev[h->nlev - 1].A.n;
  memcpy(out, h->Lplus, sizeof(double) * (size_t)(n * n));
  return LGO_OK;
}

int lgo_spmv(const lgo_hier* h, int32_t l, const double* x, double* y) {
  if (l < 0 || l >= h->nlev) return LGO_E_ARG;
  spmv(&h->lev[l].A, x, y);
  return LGO_OK;
}

/* ------------------------------------------------------------ cycles ---- */

static double unit_cost(const lgo_hier* h) {
  return (double)(h->lev[0].A.n + h->lev[0].A.nnz);
}
static void add_work(lgo_hier* h, double units) { h->work += units / unit_cost(h); }
static double L_nnz(const olevel* L) { return (double)(L->A.n + L->A.nnz); }

static void precond(lgo_hier* h, int l, const double* b, double* x);

/* Two flexible-CG iterations on L_l x = b with the cycle from level l as
 * preconditioner (the coarse solve of a K-cycle, Section 3.7, after Notay &
 * Vassilevski; FCG after Notay 2000). */
static void fcg2(lgo_hier* h, int l, const double* b, double* x) {
  const olevel* L = &h->lev[l];
  int64_t n = L->A.n;
  double* r = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* z = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* p1 = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* q1 = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* q2 = (double*)xmalloc(sizeof(double) * (size_t)n);
  memcpy(r, b, sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; i++) x[i] = 0.0;
  precond(h, l, r, p1);
  spmv(&L->A, p1, q1);
  add_work(h, L_nnz(L));
  double d1 = 0.0, a1 = 0.0;
  for (int64_t i = 0; i < n; i++) {
    d1 += p1[i] * q1[i];
    a1 += p1[i] * r[i];
  }
  if (d1 > 0.0) {
    a1 /= d1;
    for (int64_t i = 0; i < n; i++) {
      x[i] = a1 * p1[i];
      r[i] -= a1 * q1[i];
    }
    precond(h, l, r, z);
    double g = 0.0;
    for (int64_t i = 0; i < n; i++) g += z[i] * q1[i];
    g /= d1;
    for (int64_t i = 0; i < n; i++) z[i] -= g * p1[i]; /* p2 */
    spmv(&L->A, z, q2);
    add_work(h, L_nnz(L));
    double d2 = 0.0, a2 = 0.0;
    for (int64_t i = 0; i < n; i++) {
      d2 += z[i] * q2[i];
      a2 += z[i] * r[i];
    }
    if (d2 > 0.0) {
      a2 /= d2;
      for (int64_t i = 0; i < n; i++) x[i] += a2 * z[i];
    }
  }
  free(r);
  free(z);
  free(p1);
  free(q1);
  free(q2);
}

/* Algorithm 1 from level l with zero initial guess: x approximates L_l^+ b. */
static void precond(lgo_hier* h, int l, const double* b, double* x) {
  olevel* L = &h->lev[l];
  int64_t n = L->A.n;
  if (L->type == LGO_COARSEST) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
      double s = 0.0;
      for (int64_t j = 0; j < n; j++) s += h->Lplus[i * n + j] * b[j];
      x[i] = s;
    }
    add_work(h, (double)n * (double)n);
    return;
  }
  int64_t nc = L->nc;
  double* bc = (double*)xcalloc((size_t)nc, sizeof(double));
  double* xc = (double*)xcalloc((size_t)nc, sizeof(double));
  const ocsr* A = &L->A;
  if (L->type == LGO_ELIM) {
    /* b_c = P^T b with P = Pi [ -L_FF^-1 L_FC ; I ] (Section 3.4) */
    for (int64_t a = 0; a < n; a++)
      if (L->map[a] >= 0) bc[L->map[a]] = b[a];
    for (int64_t f = 0; f < n; f++) {
      if (L->map[f] >= 0) continue;
      for (int64_t e = A->rp[f]; e < A->rp[f + 1]; e++)
        bc[L->map[A->col[e]]] += (A->w[e] / A->d[f]) * b[f];
    }
    add_work(h, (double)L->nnzP);
    precond(h, l + 1, bc, xc); /* no Krylov acceleration on elimination levels */
    /* x = P x_c + F-smoother (additive two-level form) */
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t a = 0; a < n; a++) {
      if (L->map[a] >= 0) {
        x[a] = xc[L->map[a]];
        continue;
      }
      double s = 0.0;
      for (int64_t e = A->rp[a]; e < A->rp[a + 1]; e++)
        s += (A->w[e] / A->d[a]) * xc[L->map[A->col[e]]];
      x[a] = s + b[a] / A->d[a];
    }
    add_work(h, (double)L->nnzP + (double)(n - nc));
  } else {
    double* r = (double*)xmalloc(sizeof(double) * (size_t)n);
    double* p = (double*)xmalloc(sizeof(double) * (size_t)n);
    double* t = (double*)xmalloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; i++) x[i] = 0.0;
    cheb(A, L->lmax, &h->o, x, b, 1, r, p, t); /* pre-smoothing */
    add_work(h, (h->o.cheb_degree - 1) * L_nnz(L));
    spmv(A, x, t); /* residual */
    add_work(h, L_nnz(L));
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - t[i];
    for (int64_t i = 0; i < n; i++) bc[L->map[i]] += r[i]; /* restriction R r */
    add_work(h, (double)n);
    const olevel* C = &h->lev[l + 1];
    if (h->o.cycle == 2 && C->type != LGO_COARSEST) fcg2(h, l + 1, bc, xc);
    else precond(h, l + 1, bc, xc);
    for (int64_t i = 0; i < n; i++) x[i] += xc[L->map[i]]; /* prolongation */
    add_work(h, (double)n);
    cheb(A, L->lmax, &h->o, x, b, 0, r, p, t); /* post-smoothing */
    add_work(h, h->o.cheb_degree * L_nnz(L));
    free(r);
    free(p);
    free(t);
  }
  free(bc);
  free(xc);
}

double lgo_cycle_work(const lgo_hier* h) {
  /* work of one cycle in finest-residual units (Section 2.3.1: operator
     applications weighted by their nonzeros), counted while the cycle runs on
     the nonzero mean-zero vector b_i = i - (n-1)/2, so that a K-cycle's inner
     FCG takes both of its steps as it does on any residual the solver hands it */
  lgo_hier* hh = (lgo_hier*)h;
  int64_t n = h->lev[0].A.n;
  double* b = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* x = (double*)xmalloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; i++) b[i] = (double)i - 0.5 * (double)(n - 1);
  double saved = hh->work;
  hh->work = 0.0;
  precond(hh, 0, b, x);
  double w = hh->work;
  hh->work = saved;
  free(b);
  free(x);
  return w;
}

int lgo_cycle(const lgo_hier* h, const double* b, double* x) {
  precond((lgo_hier*)h, 0, b, x);
  return LGO_OK;
}

/* Test hooks: Algorithm 1 started on level l (zero initial guess), and the
 * K-cycle's inner solve on level l (two FCG steps preconditioned by that
 * cycle, Section 3.7).  Both leave the work counter as it was. */
int lgo_level_cycle(const lgo_hier* h, int32_t l, const double* b, double* x) {
  if (l < 0 || l >= h->nlev) return LGO_E_ARG;
  lgo_hier* hh = (lgo_hier*)h;
  double saved = hh->work;
  precond(hh, l, b, x);
  hh->work = saved;
  return LGO_OK;
}

int lgo_level_fcg2(const lgo_hier* h, int32_t l, const double* b, double* x) {
  if (l < 0 || l >= h->nlev || h->lev[l].type == LGO_COARSEST) return LGO_E_ARG;
  lgo_hier* hh = (lgo_hier*)h;
  double saved = hh->work;
  fcg2(hh, l, b, x);
  hh->work = saved;
  return LGO_OK;
}

static void project_mean(double* v, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s += v[i];
  s /= (double)n;
  for (int64_t i = 0; i < n; i++) v[i] -= s;
}

static double dot(const double* a, const double* b, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

/* Conjugate gradients preconditioned by one V-cycle (cycle = 1), or flexible
 * CG with one previous direction preconditioned by one K-cycle (cycle = 2)
 * (Section 2.3.2, 3.7, 4).  The right-hand side and every preconditioned
 * residual are projected to mean zero (the constant vector spans the null
 * space of a connected graph's Laplacian).  Stops when the relative residual
 * ||b - L x|| / ||b|| is at most rtol, confirmed on the true residual. */
int lgo_solve(const lgo_hier* hc, const double* b_in, double* x, double rtol, int32_t max_iter,
              int32_t* iters, double* rel_residual, double* work_units) {
  lgo_hier* h = (lgo_hier*)hc;
  const ocsr* A = &h->lev[0].A;
  int64_t n = A->n;
  double* b = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* r = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* z = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* p = (double*)xmalloc(sizeof(double) * (size_t)n);
  double* q = (double*)xmalloc(sizeof(double) * (size_t)n);
  memcpy(b, b_in, sizeof(double) * (size_t)n);
  project_mean(b, n);
  double bn = sqrt(dot(b, b, n));
  h->work = 0.0;
  int it = 0, st = LGO_E_NOT_CONVERGED;
  for (int64_t i = 0; i < n; i++) x[i] = 0.0;
  double rel = 0.0;
  if (bn == 0.0) {
    st = LGO_OK;
    goto done;
  }
  memcpy(r, b, sizeof(double) * (size_t)n);
  precond(h, 0, r, z);
  project_mean(z, n);
  memcpy(p, z, sizeof(double) * (size_t)n);
  double rz = dot(r, z, n);
  rel = 1.0;
  while (it < max_iter) {
    spmv(A, p, q);
    add_work(h, L_nnz(&h->lev[0]));
    it++;
    double pq = dot(p, q, n);
    if (!(pq > 0.0)) break;
    double alpha = (h->o.cycle == 2 ? dot(p, r, n) : rz) / pq;
    for (int64_t i = 0; i < n; i++) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    if (sqrt(dot(r, r, n)) / bn <= rtol) {
      spmv(A, x, q); /* confirm on the true residual */
      add_work(h, L_nnz(&h->lev[0]));
      for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
      rel = sqrt(dot(r, r, n)) / bn;
      if (rel <= rtol) {
        st = LGO_OK;
        break;
      }
      precond(h, 0, r, z); /* restart from the true residual */
      project_mean(z, n);
      memcpy(p, z, sizeof(double) * (size_t)n);
      rz = dot(r, z, n);
      continue;
    }
    precond(h, 0, r, z);
    project_mean(z, n);
    if (h->o.cycle == 2) {
      double beta = -dot(z, q, n) / pq;
      for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
    } else {
      double rz2 = dot(r, z, n);
      double beta = rz2 / rz;
      rz = rz2;
      for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
    }
  }
  if (st != LGO_OK) {
    spmv(A, x, q);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
    rel = sqrt(dot(r, r, n)) / bn;
  }
done:
  project_mean(x, n);
  *iters = it;
  *rel_residual = rel;
  *work_units = h->work;
  free(b);
  free(r);
  free(z);
  free(p);
  free(q);
  return st;
}
