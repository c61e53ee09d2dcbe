// setup.hip -- hierarchy construction on the device (Sections 3.4-3.6, 4).
//
// Decisions (which vertices are eliminated, which aggregates form) must not
// depend on thread scheduling.  All sums that feed them or a stored level are
// exact and order free (xs_limbs_add/xs_value in common.h); products, quotients
// and the per-edge affinity use a fixed operand order, and the argmin/argmax
// reductions use total orders.  Integer atomics only count.
#include <algorithm>
#include <cmath>
#include <string>

#include "impl.h"
#include "ops.h"

namespace lg {

enum {
  F_ROWPTR = 1, F_COL = 2, F_LOOP = 4, F_ORDER = 8, F_WEIGHT = 16, F_ASYM = 32, F_XSUM = 64,
  F_SPLIT = 128
};

constexpr int kMaxLevelCap = 128;
constexpr int64_t kDenseLimit = 2048;

static inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)ceil_div(n, b); }

// --------------------------------------------------------------- input
__global__ void k_rowptr_to32(const int64_t* __restrict__ rp64, int32_t* __restrict__ rp,
                              int64_t n, int64_t nnz, int* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i > n) return;
  const int64_t v = rp64[i];
  int f = 0;
  if (v < 0 || v > nnz) f = F_ROWPTR;
  if (i == 0 && v != 0) f = F_ROWPTR;
  if (i == n && v != nnz) f = F_ROWPTR;
  if (i < n && rp64[i + 1] < v) f = F_ROWPTR;
  if (f) atomicOr(flags, f);
  rp[i] = (int32_t)v;
}

struct NoAcc {
  int v;
};

// Section 2.1: weights positive, undirected (w_ij = w_ji), no self-loops;
// plus the CSR rules (columns in range, strictly increasing).  One thread per
// stored entry.  Symmetry: of the two entries (i, j) and (j, i) of a pair only
// the one whose partner lies in the shorter row (ties by index) searches for
// it, and counts itself.  With strictly increasing rows and no self-loops the
// searching entries map one-to-one onto distinct non-searching partners, so
// the matrix is symmetric iff every search succeeds with an equal weight and
// exactly half of the entries search (k_validate_pairs).
__global__ void k_validate(const int32_t* __restrict__ rowidx, const int32_t* __restrict__ rp,
                           const int32_t* __restrict__ col, const double* __restrict__ w,
                           int64_t n, int64_t nnz, int* __restrict__ flags,
                           int32_t* __restrict__ searched) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int f = 0;
  bool srch = false;
  if (e < nnz) {
    const int row = rowidx[e];
    const int j = col[e];
    if (j < 0 || j >= n) {
      f = F_COL;
    } else {
      if (j == row) f |= F_LOOP;
      const int r0 = rp[row];
      if (e > r0 && col[e - 1] >= j) f |= F_ORDER;
      const double we = w[e];
      if (!(we > 0.0) || !__builtin_isfinite(we)) f |= F_WEIGHT;
      int lo = rp[j], hi = rp[j + 1] - 1;
      const int dj = hi + 1 - lo, di = rp[row + 1] - r0;
      srch = dj < di || (dj == di && j < row);
      if (srch && dj <= 32) {
        // short row: independent loads, one round trip
        int found = -1;
#pragma unroll 8
        for (int k = 0; k < dj; k++)
          if (col[lo + k] == row) found = lo + k;
        if (found < 0 || w[found] != we) f |= F_ASYM;
      } else if (srch) {
        int found = -1;
        while (lo <= hi) {
          const int mid = lo + ((hi - lo) >> 1);
          const int c = col[mid];
          if (c == row) {
            found = mid;
            break;
          }
          if (c < row) lo = mid + 1;
          else hi = mid - 1;
        }
        if (found < 0 || w[found] != we) f |= F_ASYM;
      }
    }
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) f |= __shfl_xor(f, m);
  __shared__ int wcnt[kBlock / 64];
  const int cnt = __popcll(__ballot(srch));  // the whole wavefront's searches
  if ((threadIdx.x & 63) == 0) {
    if (f) atomicOr(flags, f);
    wcnt[threadIdx.x >> 6] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; k++) c += wcnt[k];
    searched[blockIdx.x] = c;  // one slot per workgroup: no contended atomics
  }
}

// Total of the per-workgroup search counts against nnz / 2.
constexpr int kPairThreads = 1024;
__global__ __launch_bounds__(kPairThreads) void k_validate_pairs(const int32_t* __restrict__ searched,
                                                                 int64_t nb, int64_t nnz,
                                                                 int* __restrict__ flags) {
  __shared__ unsigned long long sm[kPairThreads];
  unsigned long long v = 0;
  for (int64_t i = threadIdx.x; i < nb; i += kPairThreads) v += (unsigned long long)searched[i];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int m = kPairThreads / 2; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m) sm[threadIdx.x] += sm[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0 && 2 * sm[0] != (unsigned long long)nnz) atomicOr(flags, F_ASYM);
}

// ------------------------------------------------------------ connectivity
// Elimination and aggregation keep the connected components of a graph, except
// that an isolated vertex disappears when it is eliminated.  So the input is
// connected iff no level with more than one vertex has an isolated vertex and
// the coarsest level is connected; the latter is checked here by a
// breadth-first search in one workgroup (the coarsest level is small).
// flags: F_SPLIT is raised when the search does not reach every vertex.
__global__ __launch_bounds__(1024) void k_coarse_connected(const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col, int n,
                                                           int* __restrict__ seen, int* qa, int* qb,
                                                           int* __restrict__ flags) {
  __shared__ int nq, nnext, total;
  for (int i = threadIdx.x; i < n; i += blockDim.x) seen[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    seen[0] = 1;
    qa[0] = 0;
    nq = 1;
    total = 1;
  }
  __syncthreads();
  for (int it = 0; it < n; it++) {
    if (nq == 0) break;
    if (threadIdx.x == 0) nnext = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < nq; k += blockDim.x) {
      const int v = qa[k];
      for (int e = rp[v]; e < rp[v + 1]; e++) {
        const int j = col[e];
        if (atomicExch(&seen[j], 1) == 0) qb[atomicAdd(&nnext, 1)] = j;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      total += nnext;
      nq = nnext;
    }
    __syncthreads();
    int* t = qa;
    qa = qb;
    qb = t;
  }
  if (threadIdx.x == 0 && total != n) atomicOr(flags, F_SPLIT);
}

// ------------------------------------------------------ exact row sums
// one sum in limb form (xs_limbs_add)
struct XLAcc {
  uint64_t l[4];
  int bad;
  int pad[3];
};
#define XSUM_ACC_OPS                                                         \
  __device__ Acc identity() const { return {{0, 0, 0, 0}, 0, {0, 0, 0}}; } \
  __device__ static void add(Acc& a, double v) { xs_limbs_add(v, a.l, a.bad); } \
  __device__ void combine(Acc& a, const Acc& o) const {                     \
    for (int q = 0; q < 4; q++) a.l[q] += o.l[q];                           \
    a.bad |= o.bad;                                                         \
  }                                                                         \
  __device__ static double total(const Acc& a) { return xs_value(xs_limbs_total(a.l)); }

// out[row] = exact sum of val over the row; outinv[row] = 1 / out[row].
struct RowXsumOp {
  using Acc = XLAcc;
  const double* __restrict__ val;
  double* __restrict__ out;
  double* __restrict__ outinv;
  int* flags;
  XSUM_ACC_OPS
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc& a, int64_t, int e) const { add(a, val[e]); }
  __device__ void finish(int64_t row, const Acc& a, int lane, int) const {
    if (lane) return;
    const double v = total(a);
    out[row] = v;
    if (outinv) outinv[row] = v > 0.0 ? 1.0 / v : 0.0;
    if (a.bad) atomicOr(flags, F_XSUM);
  }
};

// Runs of equal (row, col) keys after sorting: one exact sum per run.
struct RunXsumOp {
  using Acc = XLAcc;
  const double* __restrict__ val;
  const uint64_t* __restrict__ keys;
  const int32_t* __restrict__ start;
  int32_t* __restrict__ ocol;
  double* __restrict__ ow;
  int* flags;
  XSUM_ACC_OPS
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc& a, int64_t, int e) const { add(a, val[e]); }
  __device__ void finish(int64_t run, const Acc& a, int lane, int) const {
    if (lane) return;
    ow[run] = total(a);
    ocol[run] = (int32_t)(keys[start[run]] & 0xffffffffULL);
    if (a.bad) atomicOr(flags, F_XSUM);
  }
};

// u[row] = (L q)_row = d_row q_row - exact sum of w q over the row (the
// Lanczos product: its sums are order free, so the estimate does not depend
// on how rows are split among lanes).
struct LzXsumOp {
  using Acc = XLAcc;
  const int32_t* __restrict__ col;
  const double* __restrict__ w;
  const double* __restrict__ d;
  const double* __restrict__ q;
  double* __restrict__ u;
  int* flags;
  XSUM_ACC_OPS
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc& a, int64_t, int e) const { add(a, w[e] * q[col[e]]); }
  __device__ void finish(int64_t row, const Acc& a, int lane, int) const {
    if (lane) return;
    u[row] = d[row] * q[row] - total(a);
    if (a.bad) atomicOr(flags, F_XSUM);
  }
};

// --------------------------------------- Algorithm 2: elimination choice
struct MinAcc {
  uint64_t h;
  int32_t id;
  int32_t pad;
};

// z_i = candidate of least hash among i and its neighbours (-1 if none);
// candidates have degree <= maxdeg.  flagC[i] = 1 unless z_i = i.
struct ElimSelectOp {
  using Acc = MinAcc;
  const int32_t* __restrict__ rp;
  const int32_t* __restrict__ col;
  int maxdeg, hash_mode;
  int32_t* __restrict__ z;
  int32_t* __restrict__ keepC;
  __device__ Acc identity() const { return {~0ULL, -1, 0}; }
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc& a, int64_t, int e) const {
    const int j = col[e];
    if (rp[j + 1] - rp[j] > maxdeg) return;
    const uint64_t h = vertex_hash(j, hash_mode);
    if (h < a.h) {
      a.h = h;
      a.id = j;
    }
  }
  __device__ void combine(Acc& a, const Acc& o) const {
    if (o.h < a.h) a = o;
  }
  __device__ void finish(int64_t row, const Acc& acc, int lane, int) const {
    if (lane) return;
    Acc a = acc;
    if (rp[row + 1] - rp[row] <= maxdeg) {
      const uint64_t h = vertex_hash(row, hash_mode);
      if (h < a.h) {
        a.h = h;
        a.id = (int32_t)row;
      }
    }
    z[row] = a.id;
    keepC[row] = (a.id == row) ? 0 : 1;
  }
};

// ----------------------------------------------------- per-entry helpers
struct RowIdxOp {
  using Acc = NoAcc;
  int32_t* __restrict__ rowidx;
  __device__ Acc identity() const { return {0}; }
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc&, int64_t row, int e) const { rowidx[e] = (int32_t)row; }
  __device__ void combine(Acc&, const Acc&) const {}
  __device__ void finish(int64_t, const Acc&, int, int) const {}
};

__global__ void k_cidx(const int32_t* __restrict__ keepC, const int64_t* __restrict__ pos,
                       int64_t n, int32_t* __restrict__ cidx, int32_t* __restrict__ cvert) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  if (keepC[i]) {
    cidx[i] = (int32_t)pos[i];
    cvert[pos[i]] = (int32_t)i;
  } else {
    cidx[i] = -1;
  }
}

// Entries contributed to the Schur complement by stored entry e = (a, b):
// 1 if b stays, deg(b) - 1 fill entries if b is eliminated, 0 if a is.
__global__ void k_elim_count(const int32_t* __restrict__ rowidx, const int32_t* __restrict__ col,
                             const int32_t* __restrict__ rp, const int32_t* __restrict__ cidx,
                             int64_t nnz, int32_t* __restrict__ direct, int32_t* __restrict__ fill,
                             int32_t* __restrict__ ptflag) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= nnz) return;
  const int a = rowidx[e], b = col[e];
  int c = 0, f = 0, fl = 0;
  if (cidx[a] >= 0) {
    if (cidx[b] >= 0) {
      c = 1;
    } else {
      fl = rp[b + 1] - rp[b] - 1;
      f = 1;
    }
  }
  direct[e] = c;
  fill[e] = fl;
  ptflag[e] = f;
}

// Schur complement entries (Section 3.4) in two streams: the kept edges
// (a', b') <- w_ab, in CSR order, which is already (a', b') order because C
// keeps increasing ids; and the fill (a', c') <- (w_fa * w_fc) / d_f for each
// eliminated neighbour f of a and each other neighbour c of f.
__global__ void k_elim_emit(const int32_t* __restrict__ rowidx, const int32_t* __restrict__ rp,
                            const int32_t* __restrict__ col, const double* __restrict__ w,
                            const double* __restrict__ d, const int32_t* __restrict__ cidx,
                            const int64_t* __restrict__ offd, const int64_t* __restrict__ offf,
                            int64_t nnz, uint64_t* __restrict__ dkeys, double* __restrict__ dvals,
                            uint64_t* __restrict__ fkeys, double* __restrict__ fvals) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= nnz) return;
  const int a = rowidx[e];
  const int ca = cidx[a];
  if (ca < 0) return;
  const int b = col[e];
  const uint64_t hi = (uint64_t)ca << 32;
  if (cidx[b] >= 0) {
    dkeys[offd[e]] = hi | (uint32_t)cidx[b];
    dvals[offd[e]] = w[e];
    return;
  }
  int64_t pos = offf[e];
  const double w_fa = w[e];
  const double d_f = d[b];
  for (int e2 = rp[b]; e2 < rp[b + 1]; e2++) {
    const int c = col[e2];
    if (c == a) continue;
    fkeys[pos] = hi | (uint32_t)cidx[c];
    fvals[pos] = (w_fa * w[e2]) / d_f;
    pos++;
  }
}

// Merge of a sorted stream A with a sorted stream B into out (ties: A first).
// B entries find their slot by binary search in A and flag it; A entries then
// fill the unflagged slots in order (k_merge_a, after a scan of the flags).
__global__ void k_merge_b(const uint64_t* __restrict__ ak, int64_t na, const uint64_t* __restrict__ bk,
                          const double* __restrict__ bv, int64_t nb, uint64_t* __restrict__ ok,
                          double* __restrict__ ov, int32_t* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= nb) return;
  const uint64_t k = bk[j];
  int64_t lo = 0, hi = na;  // first A entry > k
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (ak[mid] <= k) lo = mid + 1;
    else hi = mid;
  }
  const int64_t p = j + lo;
  ok[p] = k;
  ov[p] = bv[j];
  flag[p] = 1;
}

__global__ void k_merge_a(const uint64_t* __restrict__ ak, const double* __restrict__ av,
                          const int32_t* __restrict__ flag, const int64_t* __restrict__ before,
                          int64_t m, uint64_t* __restrict__ ok, double* __restrict__ ov) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= m || flag[p]) return;
  const int64_t i = p - before[p];
  ok[p] = ak[i];
  ov[p] = av[i];
}

// F-part of P^T: coarse row of a lists (f, w_af / d_f) for eliminated neighbours f.
__global__ void k_pt_emit(const int32_t* __restrict__ rowidx, const int32_t* __restrict__ col,
                          const double* __restrict__ w, const double* __restrict__ d,
                          const int32_t* __restrict__ ptflag, const int64_t* __restrict__ off,
                          int64_t nnz, int32_t* __restrict__ ptf, double* __restrict__ ptc) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= nnz || !ptflag[e]) return;
  const int f = col[e];
  ptf[off[e]] = f;
  ptc[off[e]] = w[e] / d[f];
}

__global__ void k_pt_rowptr(const int32_t* __restrict__ rp, const int32_t* __restrict__ cidx,
                            const int64_t* __restrict__ off, int64_t n, int64_t total,
                            int64_t nc, int32_t* __restrict__ ptrp) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n && cidx[i] >= 0) ptrp[cidx[i]] = (int32_t)off[rp[i]];
  if (i == 0) ptrp[nc] = (int32_t)total;
}

// ------------------------------------ Section 3.5: strength of connection
__global__ void k_tv_init(double* __restrict__ X, int64_t n, uint64_t key, int level) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int k = 0; k < 4; k++) X[i * 4 + k] = counter_uniform(key, level, k, i);
}

// four sums in limb form (xs_limbs_add)
struct X4LAcc {
  uint64_t l[4][4];
  int bad;
  int pad[3];
};

// One weighted-Jacobi sweep on L y = 0 for the four test vectors:
// Y_i = (1 - omega) X_i + omega * (exact sum_j w_ij X_j) / d_i.
struct JacobiOp {
  using Acc = X4LAcc;
  // one entry per lane step: the 16 limb accumulators already hold 132 VGPRs
  static constexpr int kUnroll = 1;
  const int32_t* __restrict__ col;
  const double* __restrict__ w;
  const double* __restrict__ d;
  const double* __restrict__ X;
  double* __restrict__ Y;
  double keep, omega;
  int* flags;
  __device__ Acc identity() const {
    Acc a;
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
      for (int q = 0; q < 4; q++) a.l[k][q] = 0;
    a.bad = 0;
    return a;
  }
  __device__ void accum(Acc& a, int64_t, int e) const {
    const double we = w[e];
    const double* xj = X + (int64_t)col[e] * 4;
#pragma unroll
    for (int k = 0; k < 4; k++) xs_limbs_add(we * xj[k], a.l[k], a.bad);
  }
  __device__ void combine(Acc& a, const Acc& o) const {
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
      for (int q = 0; q < 4; q++) a.l[k][q] += o.l[k][q];
    a.bad |= o.bad;
  }
  __device__ static u128 total(const Acc& a, int k) { return xs_limbs_total(a.l[k]); }
  __device__ bool active(int64_t) const { return true; }
  __device__ void finish(int64_t row, const Acc& a, int lane, int G) const {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      if (k % G != lane) continue;
      const double t = xs_value(total(a, k)) / d[row];
      Y[row * 4 + k] = keep * X[row * 4 + k] + omega * t;
    }
    if (lane == 0 && a.bad) atomicOr(flags, F_XSUM);
  }
};

__device__ __forceinline__ double sq4(const double* x) {
  return x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3];
}

// Affinity C_ij = (x_i . x_j)^2 / (|x_i|^2 |x_j|^2) per stored edge, written to S.
struct AffinityOp {
  using Acc = NoAcc;
  const int32_t* __restrict__ col;
  const double* __restrict__ X;
  double* __restrict__ S;
  __device__ Acc identity() const { return {0}; }
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc&, int64_t row, int e) const {
    const double* xi = X + row * 4;
    const double* xj = X + (int64_t)col[e] * 4;
    const double p = xi[0] * xj[0] + xi[1] * xj[1] + xi[2] * xj[2] + xi[3] * xj[3];
    const double den = sq4(xi) * sq4(xj);
    S[e] = den > 0.0 ? (p * p) / den : 0.0;
  }
  __device__ void combine(Acc&, const Acc&) const {}
  __device__ void finish(int64_t, const Acc&, int, int) const {}
};

// Row maximum of non-negative doubles (exact, order free).
struct RowMaxOp {
  using Acc = VecAcc<double, 1>;
  const double* __restrict__ val;
  double* __restrict__ out;
  __device__ Acc identity() const { return {{0.0}}; }
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc& a, int64_t, int e) const {
    const double v = val[e];
    if (v > a.v[0]) a.v[0] = v;
  }
  __device__ void combine(Acc& a, const Acc& o) const {
    if (o.v[0] > a.v[0]) a.v[0] = o.v[0];
  }
  __device__ void finish(int64_t row, const Acc& a, int lane, int) const {
    if (lane == 0) out[row] = a.v[0];
  }
};

// S_ij = C_ij / max(M_i, M_j), 0 when that maximum is 0.
struct NormalizeOp {
  using Acc = NoAcc;
  const int32_t* __restrict__ col;
  const double* __restrict__ M;
  double* __restrict__ S;
  __device__ Acc identity() const { return {0}; }
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc&, int64_t row, int e) const {
    const double mi = M[row], mj = M[col[e]];
    const double mx = mi > mj ? mi : mj;
    S[e] = mx > 0.0 ? S[e] / mx : 0.0;
  }
  __device__ void combine(Acc&, const Acc&) const {}
  __device__ void finish(int64_t, const Acc&, int, int) const {}
};

// ------------------------------------------ Algorithm 3: voting aggregation
struct VoteAcc {
  double s;
  int32_t st;  // packed status of the best neighbour, -1 = none
  int32_t pad;
};

__device__ __forceinline__ bool vote_better(const VoteAcc& x, const VoteAcc& y) {
  if (x.st == kNoStatus) return false;
  if (y.st == kNoStatus) return true;
  const int rx = status_state(x.st), ry = status_state(y.st);
  if (rx != ry) return rx > ry;
  if (x.s != y.s) return x.s > y.s;
  return (x.st & kIdxMask) < (y.st & kIdxMask);
}

// d_i = S_filt (+)agg.(x)agg status for Undecided i; a Seed neighbour is
// joined, an Undecided neighbour gets a vote.  Reads `status`, writes `next`.
struct VoteOp {
  using Acc = VoteAcc;
  const int32_t* __restrict__ col;
  const double* __restrict__ S;
  const int32_t* __restrict__ status;
  int32_t* __restrict__ next;
  int32_t* __restrict__ votes;
  double tau;
  __device__ Acc identity() const { return {-1.0, kNoStatus, 0}; }
  __device__ bool active(int64_t row) const { return status_state(status[row]) == kUndecided; }
  __device__ void accum(Acc& a, int64_t, int e) const {
    const double s = S[e];
    if (!(s >= tau)) return;
    const VoteAcc c{s, status[col[e]], 0};
    if (vote_better(c, a)) a = c;
  }
  __device__ void combine(Acc& a, const Acc& o) const {
    if (vote_better(o, a)) a = o;
  }
  __device__ void finish(int64_t row, const Acc& a, int lane, int) const {
    if (lane) return;
    const int32_t st = status[row];
    int32_t out = st;
    if (status_state(st) == kUndecided && a.st != kNoStatus) {
      const int r = status_state(a.st);
      if (r == kSeed) out = make_status(kDecided, a.st & kIdxMask);
      else if (r == kUndecided) atomicAdd(&votes[a.st & kIdxMask], 1);
    }
    next[row] = out;
  }
};

__global__ void k_status_init(int32_t* __restrict__ status, int32_t* __restrict__ votes,
                              int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  status[i] = make_status(kUndecided, i);
  votes[i] = 0;
}

__global__ void k_promote(int32_t* __restrict__ next, const int32_t* __restrict__ votes,
                          int64_t n, int seed_votes) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  if (next[i] == make_status(kUndecided, i) && votes[i] >= seed_votes)
    next[i] = make_status(kSeed, i);
}

__global__ void k_root_flags(const int32_t* __restrict__ status, int64_t n,
                             int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) flag[i] = (status[i] & kIdxMask) == i;
}

__global__ void k_agg_from_roots(const int32_t* __restrict__ status,
                                 const int64_t* __restrict__ rank, int64_t n,
                                 int32_t* __restrict__ agg) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) agg[i] = (int32_t)rank[status[i] & kIdxMask];
}

// --------------------------------------------------- Galerkin assembly
__global__ void k_gal_flags(const int32_t* __restrict__ rowidx, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ agg, int64_t nnz,
                            int32_t* __restrict__ flag) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < nnz) flag[e] = agg[rowidx[e]] != agg[col[e]];
}

__global__ void k_gal_emit(const int32_t* __restrict__ rowidx, const int32_t* __restrict__ col,
                           const double* __restrict__ w, const int32_t* __restrict__ agg,
                           const int32_t* __restrict__ flag, const int64_t* __restrict__ off,
                           int64_t nnz, uint64_t* __restrict__ keys, double* __restrict__ vals) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= nnz || !flag[e]) return;
  keys[off[e]] = ((uint64_t)agg[rowidx[e]] << 32) | (uint32_t)agg[col[e]];
  vals[off[e]] = w[e];
}

__global__ void k_run_heads(const uint64_t* __restrict__ keys, int64_t m,
                            int32_t* __restrict__ head) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < m) head[e] = (e == 0 || keys[e] != keys[e - 1]);
}

// R: the number of runs (on the device, ridx[m] after the scan).
__global__ void k_run_starts(const int32_t* __restrict__ head, const int64_t* __restrict__ ridx,
                             int64_t m, const int64_t* __restrict__ R, int32_t* __restrict__ start) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < m && head[e]) start[ridx[e]] = (int32_t)e;
  if (e == 0) start[*R] = (int32_t)m;
}

// Row pointer of a matrix whose entries are sorted by row = key >> shift:
// ptr[r] = index of the first entry with row >= r.
__global__ void k_rowptr_sorted(const uint64_t* __restrict__ keys, const int32_t* __restrict__ at,
                                int64_t m, int shift, int64_t nrows, int32_t* __restrict__ ptr) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= m) return;
  const int64_t r = (int64_t)(keys[at ? at[e] : e] >> shift);
  const int64_t rprev = e == 0 ? -1 : (int64_t)(keys[at ? at[e - 1] : e - 1] >> shift);
  for (int64_t q = rprev + 1; q <= r; q++) ptr[q] = (int32_t)e;
  if (e == m - 1)
    for (int64_t q = r + 1; q <= nrows; q++) ptr[q] = (int32_t)m;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_u64_to_i32(const uint64_t* __restrict__ in, int64_t n, int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (int32_t)in[i];
}

__global__ void k_members_keys(const int32_t* __restrict__ agg, int64_t n,
                               uint64_t* __restrict__ keys, uint64_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  keys[i] = (uint64_t)agg[i];
  vals[i] = (uint64_t)i;
}

// -------------------------------------------- reductions (deterministic)
enum { RED_SUM = 0, RED_DOT = 1, RED_DDOT = 2 };

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_red1(const double* __restrict__ a,
                                                 const double* __restrict__ b,
                                                 const double* __restrict__ d, int64_t n,
                                                 double* __restrict__ partial) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    if (MODE == RED_SUM) s += a[i];
    else if (MODE == RED_DOT) s += a[i] * b[i];
    else s += d[i] * a[i] * a[i];
  }
  __shared__ double sm[kBlock];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int m = kBlock / 2; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m) sm[threadIdx.x] += sm[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

__global__ void k_red2(const double* __restrict__ partial, int nb, double* __restrict__ out) {
  __shared__ double sm[kBlock];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) s += partial[i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int m = kBlock / 2; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m) sm[threadIdx.x] += sm[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

template <int MODE>
static void reduce_dev(const double* a, const double* b, const double* d, int64_t n,
                       double* partial, double* out, hipStream_t st) {
  const int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, ceil_div(n, kBlock)));
  hipLaunchKernelGGL((k_red1<MODE>), dim3(nb), dim3(kBlock), 0, st, a, b, d, n, partial);
  hipLaunchKernelGGL(k_red2, dim3(1), dim3(kBlock), 0, st, partial, nb, out);
}

// ------------------------------------------ exact reductions over n entries
// Terms of a sum, an inner product a.b or a D-weighted square (d a) a, added
// exactly in limb form by every thread of a fixed grid; each workgroup folds
// its threads' limbs (integer adds: order free) into partial[block].  Any
// workgroup can then form the same total from the partials.
struct XPartial {
  uint64_t l[4];
  int bad;
  int pad[3];
};

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_xred(const double* __restrict__ a,
                                                 const double* __restrict__ b,
                                                 const double* __restrict__ d, int64_t n,
                                                 XPartial* __restrict__ partial) {
  uint64_t acc[4] = {0, 0, 0, 0};
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double t = MODE == RED_SUM ? a[i] : MODE == RED_DOT ? a[i] * b[i] : (d[i] * a[i]) * a[i];
    xs_limbs_add(t, acc, bad);
  }
  __shared__ uint64_t sm[4][kBlock];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  for (int q = 0; q < 4; q++) sm[q][threadIdx.x] = acc[q];
  __syncthreads();
  if (bad) atomicOr(&sbad, 1);
  for (int m = kBlock / 2; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m)
      for (int q = 0; q < 4; q++) sm[q][threadIdx.x] += sm[q][threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int q = 0; q < 4; q++) partial[blockIdx.x].l[q] = sm[q][0];
    partial[blockIdx.x].bad = sbad;
  }
}

// The exact total of nb partials, rounded once (every workgroup that calls it
// obtains the same bits); raises F_XSUM for terms outside the range.
__device__ __forceinline__ double xred_total(const XPartial* __restrict__ partial, int nb,
                                             int* flags) {
  __shared__ uint64_t sm[4][kBlock];
  uint64_t acc[4] = {0, 0, 0, 0};
  int bad = 0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    for (int q = 0; q < 4; q++) acc[q] += partial[i].l[q];
    bad |= partial[i].bad;
  }
  for (int q = 0; q < 4; q++) sm[q][threadIdx.x] = acc[q];
  if (bad) atomicOr(flags, F_XSUM);
  __syncthreads();
  for (int m = kBlock / 2; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m)
      for (int q = 0; q < 4; q++) sm[q][threadIdx.x] += sm[q][threadIdx.x + m];
    __syncthreads();
  }
  uint64_t tot[4];
  for (int q = 0; q < 4; q++) tot[q] = sm[q][0];
  __syncthreads();
  return xs_value(xs_limbs_total(tot));
}

__global__ __launch_bounds__(kBlock) void k_xred_final(const XPartial* __restrict__ partial, int nb,
                                                       double* __restrict__ out, int* flags) {
  const double v = xred_total(partial, nb, flags);
  if (threadIdx.x == 0) *out = v;
}

// ---------------------------------------------- Lanczos (Section 3.6)
// Every sum of the estimate (the products' rows, the inner products and
// norms) is exact and order free, like the other sums that feed stored
// hierarchy values: lambda_max is reproducible bit for bit whatever the row
// schedule, and equal to a sequential evaluation of the same steps.
enum { LZ_AL = 0, LZ_BE = 64, LZ_B2 = 128, LZ_SCALE = 129, LZ_M = 130, LZ_STOP = 131,
       LZ_SUM = 132, LZ_SIZE = 136 };

__global__ void k_lz_start(double* __restrict__ q, double* __restrict__ qp, int64_t n,
                           uint64_t key, int level) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  q[i] = counter_uniform(key, level, kLanczosStream, i);
  qp[i] = 0.0;
}

__global__ void k_lz_center(double* __restrict__ q, int64_t n, const double* __restrict__ lz) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) q[i] -= lz[LZ_SUM] / (double)n;
}

__global__ void k_lz_scale(double* __restrict__ q, int64_t n, const double* __restrict__ lz) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) q[i] /= sqrt(lz[LZ_B2]);
}

__global__ void k_lz_init_scalars(double* lz) {
  for (int i = threadIdx.x; i < LZ_SIZE; i += blockDim.x) lz[i] = 0.0;
}

__global__ void k_lz_next(double* __restrict__ u, double* __restrict__ q, double* __restrict__ qp,
                          int64_t n, const double* __restrict__ lz, int j) {
  if (lz[LZ_STOP] != 0.0) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double b = lz[LZ_BE + j];
  qp[i] = q[i];
  q[i] = u[i] / b;
}

// One Lanczos step after u = L q and the partials of q . u: alpha from those
// partials (exact, the same bits in every workgroup),
// u <- D^-1 u - alpha q - beta_{j-1} q_prev, and the partials of (d u) u for
// beta.
__global__ __launch_bounds__(kBlock) void k_lz_update_x(
    double* __restrict__ u, const double* __restrict__ q, const double* __restrict__ qp,
    const double* __restrict__ d, int64_t n, double* __restrict__ lz, int j,
    const XPartial* __restrict__ dot_part, int nb_dot, XPartial* __restrict__ dd_part,
    int* flags) {
  if (lz[LZ_STOP] != 0.0) return;  // uniform: every workgroup reads the same flag
  const double a = xred_total(dot_part, nb_dot, flags);
  if (blockIdx.x == 0 && threadIdx.x == 0) lz[LZ_AL + j] = a;
  const double bp = j > 0 ? lz[LZ_BE + j - 1] : 0.0;
  uint64_t acc[4] = {0, 0, 0, 0};
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double v = u[i] / d[i] - a * q[i] - bp * qp[i];
    u[i] = v;
    xs_limbs_add((d[i] * v) * v, acc, bad);
  }
  __shared__ uint64_t sm[4][kBlock];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  for (int q2 = 0; q2 < 4; q2++) sm[q2][threadIdx.x] = acc[q2];
  __syncthreads();
  if (bad) atomicOr(&sbad, 1);
  for (int m = kBlock / 2; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m)
      for (int q2 = 0; q2 < 4; q2++) sm[q2][threadIdx.x] += sm[q2][threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int q2 = 0; q2 < 4; q2++) dd_part[blockIdx.x].l[q2] = sm[q2][0];
    dd_part[blockIdx.x].bad = sbad;
  }
}

// beta_j from the partials of (d u) u, then the stopping test.
__global__ __launch_bounds__(kBlock) void k_lz_beta_x(const XPartial* __restrict__ dd_part, int nb,
                                                      double* lz, int j, int steps, int* flags) {
  if (lz[LZ_STOP] != 0.0) return;
  const double b2 = xred_total(dd_part, nb, flags);
  if (threadIdx.x != 0) return;
  const double a = lz[LZ_AL + j];
  const double bp = j > 0 ? lz[LZ_BE + j - 1] : 0.0;
  const double b = sqrt(b2);
  double scale = lz[LZ_SCALE];
  if (fabs(a) + bp > scale) scale = fabs(a) + bp;
  lz[LZ_SCALE] = scale;
  lz[LZ_M] = (double)(j + 1);
  if (j == steps - 1 || b <= 1e-12 * scale) lz[LZ_STOP] = 1.0;
  else lz[LZ_BE + j] = b;
}

__device__ int sturm_below(const double* a, const double* b, int m, double x) {
  int c = 0;
  double q = 1.0;
  for (int i = 0; i < m; i++) {
    q = (a[i] - x) - (i > 0 ? (b[i - 1] * b[i - 1]) / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) c++;
  }
  return c;
}

// Largest eigenvalue of the Lanczos tridiagonal: multisection with one
// wavefront, 64 Sturm counts per step, inside the Gershgorin interval.
__global__ __launch_bounds__(64) void k_lz_eig(const double* __restrict__ lz,
                                               double* __restrict__ out) {
  const int m = (int)lz[LZ_M];
  const double* a = lz + LZ_AL;
  const double* b = lz + LZ_BE;
  const int lane = threadIdx.x;
  if (m <= 0) {
    if (lane == 0) *out = 0.0;
    return;
  }
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; i++) {
    const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i < m - 1 ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
  }
  hi += 1e-12 * fabs(hi) + 1e-300;
  lo -= 1e-12 * fabs(lo) + 1e-300;
  for (int it = 0; it < 16; it++) {
    const double step = (hi - lo) / 65.0;
    if (!(step > 0.0)) break;
    const double x = lo + step * (lane + 1);
    const bool above = x < hi && sturm_below(a, b, m, x) == m;  // every eigenvalue below x
    const uint64_t mask = __ballot(above);
    const int first = mask ? (int)__ffsll((unsigned long long)mask) - 1 : 64;
    const double nlo = lo + step * first;
    const double nhi = first == 64 ? hi : lo + step * (first + 1);
    if (!(nhi > nlo) || (nlo == lo && nhi == hi)) break;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) *out = 0.5 * (lo + hi);
}

// --------------------------------------------- coarsest pseudo-inverse
// L^+ = (L + (s/n) 11^T)^-1 - 11^T/(s n) for any s > 0 on a connected graph:
// 1 is an eigenvector of the shifted matrix with eigenvalue s.  With
// s = max_i d_i that eigenvalue lies inside the range of L's others, so the
// inverted matrix is as well conditioned as L on the mean-zero space (a fixed
// s = 1 is not when the weights are far from 1).

// s = max_i d_i (1 for a single vertex, whose L is 0), one workgroup.
__global__ __launch_bounds__(kBlock) void k_coarse_shift(const double* __restrict__ d, int64_t n,
                                                         double* __restrict__ s_out) {
  __shared__ double red[kBlock];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) m = fmax(m, d[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *s_out = red[0] > 0.0 ? red[0] : 1.0;
}

__global__ void k_dense_lap(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const double* __restrict__ w, const double* __restrict__ d, int64_t n,
                            const double* __restrict__ s, double* __restrict__ M) {
  const int64_t i = blockIdx.x;
  const double shift = *s / (double)n;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) M[i * n + j] = shift + (i == j ? d[i] : 0.0);
  __syncthreads();
  for (int e = rp[i] + threadIdx.x; e < rp[i + 1]; e += blockDim.x) M[i * n + col[e]] -= w[e];
}

// In-place Gauss-Jordan inversion of the SPD matrix L + (s/n) 11^T (no pivoting),
// one workgroup, for the small coarsest level.
__global__ __launch_bounds__(1024) void k_gauss_jordan(double* __restrict__ M, int n,
                                                       double* __restrict__ colbuf) {
  for (int k = 0; k < n; k++) {
    __syncthreads();
    const double inv = 1.0 / M[(int64_t)k * n + k];
    for (int i = threadIdx.x; i < n; i += blockDim.x) colbuf[i] = M[(int64_t)i * n + k];
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x)
      M[(int64_t)k * n + j] = (j == k ? 1.0 : M[(int64_t)k * n + j]) * inv;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += blockDim.x) {
      const int i = (int)(t / n), j = (int)(t % n);
      if (i == k) continue;
      const double mkj = M[(int64_t)k * n + j];
      M[t] = (j == k ? 0.0 : M[t]) - colbuf[i] * mkj;
    }
  }
}

__global__ void k_sub_shift(double* __restrict__ M, int64_t nn, int64_t n,
                            const double* __restrict__ s) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < nn) M[t] -= 1.0 / (*s * (double)n);
}

__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

__global__ void k_copy_f64(const double* __restrict__ in, double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = in[i];
}


// ------------------------------------------------ solve-time vertex order
// Key of a row in the solve order: split rows, hub rows, then degree classes
// from the highest down (ties keep the setup's order: the sort is stable).
__global__ void k_order_keys(const int32_t* __restrict__ rp, int64_t n, int hub_deg,
                             uint64_t* __restrict__ keys, uint64_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int d = rp[i + 1] - rp[i];
  const int c = degree_class(d, hub_deg);
  keys[i] = c >= kClasses ? (d > kSplitDeg ? 0u : 1u) : (uint64_t)(2 + (kClasses - 1 - c));
  vals[i] = (uint64_t)i;
}

// perm[new] = old from the sorted pairs, and iperm[old] = new.
__global__ void k_order_perm(const uint64_t* __restrict__ vals, int64_t n, int32_t* __restrict__ perm,
                             int32_t* __restrict__ iperm) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t o = (int32_t)vals[i];
  perm[i] = o;
  iperm[o] = (int32_t)i;
}

// deg[new] = length of old row perm[new].
__global__ void k_perm_degrees(const int32_t* __restrict__ ptr, const int32_t* __restrict__ perm,
                               int64_t nr, int32_t* __restrict__ deg) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nr) return;
  const int64_t r = perm ? perm[i] : i;
  deg[i] = ptr[r + 1] - ptr[r];
}

__global__ void k_i64_to_i32(const int64_t* __restrict__ in, int64_t n, int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (int32_t)in[i];
}

// Entry e of old row r moves to new row rmap[r] at the same offset; its index
// maps through emap and its value follows (run over the old rows).
struct PermEntriesOp {
  using Acc = NoAcc;
  const int32_t* __restrict__ ptr0;
  const int32_t* __restrict__ idx0;
  const double* __restrict__ val0;
  const int32_t* __restrict__ rmap;
  const int32_t* __restrict__ emap;
  const int32_t* __restrict__ ptr;
  int32_t* __restrict__ idx;
  double* __restrict__ val;
  __device__ Acc identity() const { return {0}; }
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc&, int64_t row, int e) const {
    const int64_t dst = (int64_t)ptr[rmap ? rmap[row] : row] + (e - ptr0[row]);
    const int32_t j = idx0[e];
    idx[dst] = emap ? emap[j] : j;
    if (val) val[dst] = val0[e];
  }
  __device__ void combine(Acc&, const Acc&) const {}
  __device__ void finish(int64_t, const Acc&, int, int) const {}
};

// dst[new] = src[perm[new]], mapped through map where it is an index (>= 0).
__global__ void k_perm_index(const int32_t* __restrict__ src, const int32_t* __restrict__ perm,
                             const int32_t* __restrict__ map, int64_t n, int32_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t v = src[perm ? perm[i] : i];
  dst[i] = (v >= 0 && map) ? map[v] : v;
}

__global__ void k_perm_f64(const double* __restrict__ src, const int32_t* __restrict__ perm, int64_t n,
                           double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

// ===================================================================== host
namespace {

// A second stream for work that only reads finished levels (Lanczos), so it
// fills the gaps of the level construction.  Its destructor waits for it, so
// an error thrown mid-setup cannot release memory the stream still reads.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t ready = nullptr, done = nullptr;
  std::vector<hipEvent_t> level_done;  // per level: its Lanczos steps are done
  SideStream() = default;
  SideStream(const SideStream&) = delete;
  SideStream& operator=(const SideStream&) = delete;
  ~SideStream() {
    if (s) (void)hipStreamSynchronize(s);
    if (ready) (void)hipEventDestroy(ready);
    if (done) (void)hipEventDestroy(done);
    for (hipEvent_t e : level_done)
      if (e) (void)hipEventDestroy(e);
  }
};

struct Ctx {
  lg_hierarchy* h;
  hipStream_t st;
  TempArena lease;
  Arena& tmp = *lease.a;
  TempArena side_lease;  // side-stream temporaries, kept until setup ends
  Arena& side_tmp = *side_lease.a;
  SideStream side;  // declared after the arenas: joined before they are released
  int* flags = nullptr;  // device error flags
  uint64_t key = 0;
};

void raise_flags(int f) {
  if (f & F_ROWPTR) fail(LG_E_GRAPH, "row pointers are not a valid CSR offset array");
  if (f & F_COL) fail(LG_E_GRAPH, "column index out of range");
  if (f & F_LOOP) fail(LG_E_GRAPH, "self-loop (diagonal entry) in the adjacency");
  if (f & F_ORDER) fail(LG_E_GRAPH, "row columns not strictly increasing (unsorted or duplicate)");
  if (f & F_WEIGHT) fail(LG_E_GRAPH, "edge weight not finite and positive");
  if (f & F_ASYM) fail(LG_E_GRAPH, "adjacency not symmetric");
  if (f & F_XSUM) fail(LG_E_RANGE, "sum outside the exact-sum range (total weight too large)");
  if (f & F_SPLIT) fail(LG_E_DISCONNECTED, "graph is not connected (coarsest level splits)");
}

void check_flags(Ctx& c) {
  int f = 0;
  read_dev(&f, c.flags, sizeof(int), c.st);
  raise_flags(f);
}

// A level with more than one vertex and an isolated vertex: the input graph
// has more than one connected component (Section 2.1 assumes one).
void check_isolated(const Level& L) {
  if (L.n > 1 && L.sched.min_deg == 0)
    fail(LG_E_DISCONNECTED, "graph is not connected (isolated vertex on a level with " +
                                std::to_string(L.n) + " vertices)");
}

// Row sums and reciprocals of a level's adjacency.
void level_diag(Ctx& c, Level& L) {
  L.d = c.h->mem.get<double>(L.n);
  L.dinv = c.h->mem.get<double>(L.n);
  ProfScope ps("row_xsum", c.st, 4.0 * (L.n + 1) + 8.0 * L.nnz + 16.0 * L.n);
  run_rows(L.sched, L.rp, RowXsumOp{L.w, L.d, L.dinv, c.flags}, c.st);
}

// Sorted (row << 32 | col, value) pairs -> CSR of `out` with exact sums of
// equal keys (rows 0..nrows-1), then its schedule and diagonal.
// A schedule whose statistics are on the device, to be read back with the
// next values the host waits for.
struct PendingSched {
  Sched* s;
  const int* stats;
  const int32_t* rp;
  int64_t n, nnz;
};

// Coarse matrix from sorted (row << 32 | col, value) pairs: one exact sum per
// run of equal keys.  pend: a schedule laid out after the same read back.
void assemble(Ctx& c, uint64_t* keys, double* vals, int64_t m, int64_t nrows, Level& out,
              const PendingSched* pend = nullptr) {
  Arena& tmp = c.tmp;
  lg_hierarchy* h = c.h;
  out.n = nrows;
  out.rp = h->mem.get<int32_t>(nrows + 1);
  int pt[kStat] = {};
  if (m == 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk(nrows + 1)), dim3(kBlock), 0, c.st, out.rp,
                       nrows + 1, 0);
    out.nnz = 0;
    out.col = h->mem.get<int32_t>(1);
    out.w = h->mem.get<double>(1);
    if (pend && pend->n) read_dev(pt, pend->stats, sizeof(pt), c.st);
  } else {
    int32_t* head = tmp.get<int32_t>(m);
    int64_t* ridx = tmp.get<int64_t>(m + 1);
    hipLaunchKernelGGL(k_run_heads, dim3(nblk(m)), dim3(kBlock), 0, c.st, keys, m, head);
    scan_i32_to_i64(head, ridx, m, tmp, c.st, false);
    // the runs are the rows of a CSR over the pairs; R <= m is still on the device
    int32_t* start = tmp.get<int32_t>(m + 1);
    hipLaunchKernelGGL(k_run_starts, dim3(nblk(m)), dim3(kBlock), 0, c.st, head, ridx, m,
                       (const int64_t*)(ridx + m), start);
    const int* rstats = sched_stats(start, m, ridx + m, tmp, c.st);
    int64_t R = 0;
    int rt[kStat];
    DevRead rd[3] = {{&R, ridx + m, sizeof(R)}, {rt, rstats, sizeof(rt)}, {pt, nullptr, 0}};
    int nread = 2;
    if (pend && pend->n) rd[nread++] = {pt, pend->stats, sizeof(pt)};
    read_dev_n(rd, nread, c.st);
    out.nnz = R;
    out.col = h->mem.get<int32_t>(R);
    out.w = h->mem.get<double>(R);
    Sched rs;
    sched_layout(rs, rt, start, R, m, false, tmp, tmp, c.st);
    {
      ProfScope ps("galerkin_reduce", c.st, (double)m * 16.0 + (double)R * 12.0);
      run_rows(rs, start, RunXsumOp{vals, keys, start, out.col, out.w, c.flags}, c.st);
    }
    hipLaunchKernelGGL(k_rowptr_sorted, dim3(nblk(R)), dim3(kBlock), 0, c.st, keys, start, R, 32,
                       nrows, out.rp);
    LG_LAUNCH_CHECK();
  }
  if (pend) sched_layout(*pend->s, pt, pend->rp, pend->n, pend->nnz, false, h->mem, tmp, c.st);
  build_sched(out.sched, out.rp, out.n, out.nnz, h->mem, tmp, c.st, h->opts.merge_path != 0);
  check_isolated(out);
  level_diag(c, out);
}

void row_index(Ctx& c, const Level& L, int32_t* rowidx) {
  run_rows(L.sched, L.rp, RowIdxOp{rowidx}, c.st);
}

// Algorithm 2 on level l; returns |F| and leaves keepC / pos (scan) in tmp.
struct ElimChoice {
  int64_t nf = 0, nc = 0;
  int32_t* keepC = nullptr;
  int64_t* pos = nullptr;
  int32_t* z = nullptr;
};

ElimChoice elim_select(Ctx& c, Level& L) {
  const lg_setup_opts& o = c.h->opts;
  ElimChoice ch;
  ch.keepC = c.tmp.get<int32_t>(L.n);
  ch.pos = c.tmp.get<int64_t>(L.n + 1);
  ch.z = o.keep_setup_data ? c.h->mem.get<int32_t>(L.n) : c.tmp.get<int32_t>(L.n);
  {
    ProfScope ps("elim_select", c.st, 4.0 * (L.n + 1) + 4.0 * L.nnz + 8.0 * L.n);
    run_rows(L.sched, L.rp, ElimSelectOp{L.rp, L.col, o.elim_max_degree, o.hash_mode, ch.z, ch.keepC},
             c.st);
  }
  ch.nc = scan_i32_to_i64(ch.keepC, ch.pos, L.n, c.tmp, c.st, true);
  ch.nf = L.n - ch.nc;
  return ch;
}

// Elimination level (Section 3.4): Schur complement onto C and the transfer data.
void build_elim(Ctx& c, Level& L, const ElimChoice& ch, Level& out) {
  lg_hierarchy* h = c.h;
  Arena& tmp = c.tmp;
  const int64_t n = L.n, nnz = L.nnz, nc = ch.nc;
  L.type = LG_LEVEL_ELIM;
  L.nc = nc;
  L.nF = ch.nf;
  if (h->opts.keep_setup_data) L.z = ch.z;
  L.cidx = h->mem.get<int32_t>(n);
  L.cvert = h->mem.get<int32_t>(nc);
  hipLaunchKernelGGL(k_cidx, dim3(nblk(n)), dim3(kBlock), 0, c.st, ch.keepC, ch.pos, n, L.cidx,
                     L.cvert);
  int32_t* rowidx = tmp.get<int32_t>(nnz);
  row_index(c, L, rowidx);
  int32_t* dcnt = tmp.get<int32_t>(nnz);
  int32_t* fcnt = tmp.get<int32_t>(nnz);
  int32_t* ptflag = tmp.get<int32_t>(nnz);
  hipLaunchKernelGGL(k_elim_count, dim3(nblk(nnz)), dim3(kBlock), 0, c.st, rowidx, L.col, L.rp,
                     L.cidx, nnz, dcnt, fcnt, ptflag);
  int64_t* offd = tmp.get<int64_t>(nnz + 1);
  int64_t* offf = tmp.get<int64_t>(nnz + 1);
  int64_t* off2 = tmp.get<int64_t>(nnz + 1);
  scan_i32_to_i64(dcnt, offd, nnz, tmp, c.st, false);
  scan_i32_to_i64(fcnt, offf, nnz, tmp, c.st, false);
  scan_i32_to_i64(ptflag, off2, nnz, tmp, c.st, false);
  int64_t na = 0, nfill = 0, npt = 0;
  {
    const DevRead rd[3] = {{&na, offd + nnz, sizeof(na)},
                           {&nfill, offf + nnz, sizeof(nfill)},
                           {&npt, off2 + nnz, sizeof(npt)}};
    read_dev_n(rd, 3, c.st);  // all three totals, one round trip
  }
  const int64_t m = na + nfill;
  uint64_t* dkeys = tmp.get<uint64_t>(na);
  double* dvals = tmp.get<double>(na);
  uint64_t* fkeys = tmp.get<uint64_t>(nfill);
  double* fvals = tmp.get<double>(nfill);
  hipLaunchKernelGGL(k_elim_emit, dim3(nblk(nnz)), dim3(kBlock), 0, c.st, rowidx, L.rp, L.col, L.w,
                     L.d, L.cidx, offd, offf, nnz, dkeys, dvals, fkeys, fvals);
  LG_LAUNCH_CHECK();
  const int b = bits_for(nc > 0 ? nc - 1 : 0);
  {
    const SortedPairs sp =
        radix_sort_pairs(fkeys, (uint64_t*)fvals, nfill, pair_shifts(b), tmp, c.st, b);
    fkeys = sp.keys;
    fvals = (double*)sp.vals;
  }
  uint64_t* keys = tmp.get<uint64_t>(m);
  double* vals = tmp.get<double>(m);
  {
    Arena::Mark mm = tmp.mark();
    int32_t* flag = tmp.get<int32_t>(m);
    int64_t* before = tmp.get<int64_t>(m + 1);
    if (m > 0) {
      hipLaunchKernelGGL(k_fill_i32, dim3(nblk(m)), dim3(kBlock), 0, c.st, flag, m, 0);
      if (nfill > 0)
        hipLaunchKernelGGL(k_merge_b, dim3(nblk(nfill)), dim3(kBlock), 0, c.st,
                           (const uint64_t*)dkeys, na, (const uint64_t*)fkeys, (const double*)fvals,
                           nfill, keys, vals, flag);
      scan_i32_to_i64(flag, before, m, tmp, c.st, false);
      hipLaunchKernelGGL(k_merge_a, dim3(nblk(m)), dim3(kBlock), 0, c.st, (const uint64_t*)dkeys,
                         (const double*)dvals, (const int32_t*)flag, (const int64_t*)before, m, keys,
                         vals);
      LG_LAUNCH_CHECK();
    }
    tmp.rewind(mm);
  }
  // transfer data: F-part of P^T
  L.ptrp = h->mem.get<int32_t>(nc + 1);
  L.ptf = h->mem.get<int32_t>(npt);
  L.ptc = h->mem.get<double>(npt);
  hipLaunchKernelGGL(k_pt_emit, dim3(nblk(nnz)), dim3(kBlock), 0, c.st, rowidx, L.col, L.w, L.d,
                     ptflag, off2, nnz, L.ptf, L.ptc);
  hipLaunchKernelGGL(k_pt_rowptr, dim3(nblk(n)), dim3(kBlock), 0, c.st, L.rp, L.cidx, off2, n, npt,
                     nc, L.ptrp);
  LG_LAUNCH_CHECK();
  const PendingSched pend{&L.ptsched, nc ? sched_stats(L.ptrp, nc, nullptr, tmp, c.st) : nullptr,
                          L.ptrp, nc, npt};
  L.nnzP = nc + npt;  // each eliminated vertex's entries appear once in P^T
  assemble(c, keys, vals, m, nc, out, &pend);
}

// Section 3.5: four smoothed test vectors and the normalised affinity S.
void strength(Ctx& c, Level& L, int level, double* S, double* X) {
  const lg_setup_opts& o = c.h->opts;
  Arena& tmp = c.tmp;
  double* Y = tmp.get<double>(4 * L.n);
  hipLaunchKernelGGL(k_tv_init, dim3(nblk(L.n)), dim3(kBlock), 0, c.st, X, L.n, c.key, level);
  const double omega = o.tv_omega, keep = 1.0 - o.tv_omega;
  double* src = X;
  double* dst = Y;
  for (int s = 0; s < o.tv_sweeps; s++) {
    ProfScope ps("jacobi_xsum", c.st, 4.0 * (L.n + 1) + 12.0 * L.nnz + 8.0 * L.n + 64.0 * L.n);
    run_rows(L.sched, L.rp, JacobiOp{L.col, L.w, L.d, src, dst, keep, omega, c.flags}, c.st);
    std::swap(src, dst);
  }
  if (src != X)
    hipLaunchKernelGGL(k_copy_f64, dim3(nblk(4 * L.n)), dim3(kBlock), 0, c.st, src, X, 4 * L.n);
  double* M = tmp.get<double>(L.n);
  {
    ProfScope ps("affinity", c.st, 4.0 * (L.n + 1) + 12.0 * L.nnz + 32.0 * L.n);
    run_rows(L.sched, L.rp, AffinityOp{L.col, X, S}, c.st);
    run_rows(L.sched, L.rp, RowMaxOp{S, M}, c.st);
    run_rows(L.sched, L.rp, NormalizeOp{L.col, M, S}, c.st);
  }
  LG_LAUNCH_CHECK();
}

// Algorithm 3; returns the number of aggregates and fills L.agg.
int64_t aggregate(Ctx& c, Level& L, const double* S, int32_t** status_out, int32_t** votes_out) {
  const lg_setup_opts& o = c.h->opts;
  Arena& tmp = c.tmp;
  const int64_t n = L.n;
  const bool keep = o.keep_setup_data != 0;
  int32_t* status = tmp.get<int32_t>(n);
  int32_t* next = tmp.get<int32_t>(n);
  int32_t* votes = keep ? c.h->mem.get<int32_t>(n) : tmp.get<int32_t>(n);
  hipLaunchKernelGGL(k_status_init, dim3(nblk(n)), dim3(kBlock), 0, c.st, status, votes, n);
  double tau = 1.0;
  for (int it = 1; it <= o.agg_iters; it++) {
    tau *= o.agg_filter_base;
    {
      ProfScope ps("vote", c.st, 4.0 * (n + 1) + 12.0 * L.nnz + 8.0 * n);
      run_rows(L.sched, L.rp, VoteOp{L.col, S, status, next, votes, tau}, c.st);
    }
    hipLaunchKernelGGL(k_promote, dim3(nblk(n)), dim3(kBlock), 0, c.st, next, votes, n,
                       o.seed_votes);
    std::swap(status, next);
  }
  LG_LAUNCH_CHECK();
  int32_t* flag = tmp.get<int32_t>(n);
  int64_t* rank = tmp.get<int64_t>(n + 1);
  hipLaunchKernelGGL(k_root_flags, dim3(nblk(n)), dim3(kBlock), 0, c.st, status, n, flag);
  const int64_t nc = scan_i32_to_i64(flag, rank, n, tmp, c.st, true);
  L.agg = c.h->mem.get<int32_t>(n);
  hipLaunchKernelGGL(k_agg_from_roots, dim3(nblk(n)), dim3(kBlock), 0, c.st, status, rank, n, L.agg);
  if (keep) {
    int32_t* st_keep = c.h->mem.get<int32_t>(n);
    LG_HIP(hipMemcpyAsync(st_keep, status, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c.st));
    *status_out = st_keep;
    *votes_out = votes;
  }
  LG_LAUNCH_CHECK();
  return nc;
}

// Members of each aggregate (CSR of R, increasing vertex id) and the
// Galerkin product R L P as the exact inter-aggregate weight sums.
void galerkin(Ctx& c, Level& L, int64_t nc, Level& out) {
  lg_hierarchy* h = c.h;
  Arena& tmp = c.tmp;
  const int64_t n = L.n, nnz = L.nnz;
  const int b = bits_for(nc > 0 ? nc - 1 : 0);
  {
    uint64_t* mk = tmp.get<uint64_t>(n);
    uint64_t* mv = tmp.get<uint64_t>(n);
    hipLaunchKernelGGL(k_members_keys, dim3(nblk(n)), dim3(kBlock), 0, c.st, L.agg, n, mk, mv);
    const SortedPairs sp = radix_sort_pairs(mk, mv, n, digit_shifts(b, 0), tmp, c.st);
    mk = sp.keys;
    mv = sp.vals;
    L.mem = h->mem.get<int32_t>(n);
    L.mptr = h->mem.get<int32_t>(nc + 1);
    hipLaunchKernelGGL(k_u64_to_i32, dim3(nblk(n)), dim3(kBlock), 0, c.st, mv, n, L.mem);
    hipLaunchKernelGGL(k_rowptr_sorted, dim3(nblk(n)), dim3(kBlock), 0, c.st, mk,
                       (const int32_t*)nullptr, n, 0, nc, L.mptr);
    LG_LAUNCH_CHECK();
  }
  // the member schedule's statistics come back with the pair count below
  const int* mstats = nc ? sched_stats(L.mptr, nc, nullptr, tmp, c.st) : nullptr;
  int32_t* rowidx = tmp.get<int32_t>(nnz);
  row_index(c, L, rowidx);
  int32_t* flag = tmp.get<int32_t>(nnz);
  hipLaunchKernelGGL(k_gal_flags, dim3(nblk(nnz)), dim3(kBlock), 0, c.st, rowidx, L.col, L.agg,
                     nnz, flag);
  int64_t* off = tmp.get<int64_t>(nnz + 1);
  scan_i32_to_i64(flag, off, nnz, tmp, c.st, false);
  int64_t m = 0;
  int mt[kStat] = {};
  {
    const DevRead rd[2] = {{&m, off + nnz, sizeof(m)}, {mt, mstats, sizeof(mt)}};
    read_dev_n(rd, mstats ? 2 : 1, c.st);
  }
  sched_layout(L.msched, mt, L.mptr, nc, n, false, h->mem, tmp, c.st);
  uint64_t* keys = tmp.get<uint64_t>(m);
  double* vals = tmp.get<double>(m);
  hipLaunchKernelGGL(k_gal_emit, dim3(nblk(nnz)), dim3(kBlock), 0, c.st, rowidx, L.col, L.w, L.agg,
                     flag, off, nnz, keys, vals);
  LG_LAUNCH_CHECK();
  const SortedPairs sp = radix_sort_pairs(keys, (uint64_t*)vals, m, pair_shifts(b), tmp, c.st, b);
  assemble(c, sp.keys, (double*)sp.vals, m, nc, out);
}

// lambda_max(D^-1 L) by eig_iters Lanczos steps in the D inner product.
// Runs on the side stream after the work queued so far on the main stream;
// setup_hierarchy joins the streams before reading the results.
void lanczos(Ctx& c, Level& L, int level, double* out) {
  const lg_setup_opts& o = c.h->opts;
  const hipStream_t st = c.side.s;
  LG_HIP(hipEventRecord(c.side.ready, c.st));
  LG_HIP(hipStreamWaitEvent(st, c.side.ready, 0));
  Arena& tmp = c.side_tmp;
  const int64_t n = L.n;
  double* q = tmp.get<double>(n);
  double* qp = tmp.get<double>(n);
  double* u = tmp.get<double>(n);
  double* lz = tmp.get<double>(LZ_SIZE);
  const int steps = std::min(o.eig_iters, 64);
  hipLaunchKernelGGL(k_lz_init_scalars, dim3(1), dim3(64), 0, st, lz);
  if (n < 2 || steps < 1) {
    hipLaunchKernelGGL(k_lz_eig, dim3(1), dim3(64), 0, st, lz, out);
    if ((int)c.side.level_done.size() <= level) c.side.level_done.resize(level + 1, nullptr);
    LG_HIP(hipEventCreateWithFlags(&c.side.level_done[level], hipEventDisableTiming));
    LG_HIP(hipEventRecord(c.side.level_done[level], st));
    return;
  }
  const int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, ceil_div(n, kBlock)));
  XPartial* part = tmp.get<XPartial>(kRedBlocks);
  XPartial* part2 = tmp.get<XPartial>(kRedBlocks);
  hipLaunchKernelGGL(k_lz_start, dim3(nblk(n)), dim3(kBlock), 0, st, q, qp, n, c.key, level);
  hipLaunchKernelGGL((k_xred<RED_SUM>), dim3(nb), dim3(kBlock), 0, st, (const double*)q,
                     (const double*)nullptr, (const double*)nullptr, n, part);
  hipLaunchKernelGGL(k_xred_final, dim3(1), dim3(kBlock), 0, st, (const XPartial*)part, nb,
                     lz + LZ_SUM, c.flags);
  hipLaunchKernelGGL(k_lz_center, dim3(nblk(n)), dim3(kBlock), 0, st, q, n, lz);
  hipLaunchKernelGGL((k_xred<RED_DDOT>), dim3(nb), dim3(kBlock), 0, st, (const double*)q,
                     (const double*)nullptr, (const double*)L.d, n, part);
  hipLaunchKernelGGL(k_xred_final, dim3(1), dim3(kBlock), 0, st, (const XPartial*)part, nb,
                     lz + LZ_B2, c.flags);
  hipLaunchKernelGGL(k_lz_scale, dim3(nblk(n)), dim3(kBlock), 0, st, q, n, lz);
  for (int j = 0; j < steps; j++) {
    run_rows(L.sched, L.rp, LzXsumOp{L.col, L.w, L.d, q, u, c.flags}, st, "lanczos",
             4.0 * (n + 1) + 12.0 * L.nnz + 24.0 * n);
    hipLaunchKernelGGL((k_xred<RED_DOT>), dim3(nb), dim3(kBlock), 0, st, (const double*)q,
                       (const double*)u, (const double*)nullptr, n, part);
    hipLaunchKernelGGL(k_lz_update_x, dim3(nb), dim3(kBlock), 0, st, u, (const double*)q,
                       (const double*)qp, (const double*)L.d, n, lz, j, (const XPartial*)part, nb,
                       part2, c.flags);
    hipLaunchKernelGGL(k_lz_beta_x, dim3(1), dim3(kBlock), 0, st, (const XPartial*)part2, nb, lz,
                       j, steps, c.flags);
    hipLaunchKernelGGL(k_lz_next, dim3(nblk(n)), dim3(kBlock), 0, st, u, q, qp, n, lz, j);
  }
  hipLaunchKernelGGL(k_lz_eig, dim3(1), dim3(64), 0, st, lz, out);
  LG_LAUNCH_CHECK();
  // the point after which the level may be rewritten (solve order)
  if ((int)c.side.level_done.size() <= level) c.side.level_done.resize(level + 1, nullptr);
  LG_HIP(hipEventCreateWithFlags(&c.side.level_done[level], hipEventDisableTiming));
  LG_HIP(hipEventRecord(c.side.level_done[level], st));
}

void coarsest(Ctx& c, Level& L) {
  lg_hierarchy* h = c.h;
  const int64_t n = L.n;
  if (n > kDenseLimit)
    fail(LG_E_ARG, "coarsening stalled: coarsest level has " + std::to_string(n) +
                       " vertices (dense solve limit " + std::to_string(kDenseLimit) + ")");
  {
    Arena::Mark m = c.tmp.mark();
    int* seen = c.tmp.get<int>(n);
    int* qa = c.tmp.get<int>(n);
    int* qb = c.tmp.get<int>(n);
    // reported with the other flags at the end of setup; a split coarsest
    // level only makes the dense elimination below produce unused values
    hipLaunchKernelGGL(k_coarse_connected, dim3(1), dim3(1024), 0, c.st, L.rp, L.col, (int)n, seen,
                       qa, qb, c.flags);
    LG_LAUNCH_CHECK();
    c.tmp.rewind(m);
  }
  h->Lplus = h->mem.get<double>(n * n);
  double* shift = c.tmp.get<double>(1);
  hipLaunchKernelGGL(k_coarse_shift, dim3(1), dim3(kBlock), 0, c.st, L.d, n, shift);
  hipLaunchKernelGGL(k_dense_lap, dim3((unsigned)n), dim3(kBlock), 0, c.st, L.rp, L.col, L.w, L.d,
                     n, shift, h->Lplus);
  double* colbuf = c.tmp.get<double>(n);
  hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(1024), 0, c.st, h->Lplus, (int)n, colbuf);
  hipLaunchKernelGGL(k_sub_shift, dim3(nblk(n * n)), dim3(kBlock), 0, c.st, h->Lplus, n * n, n,
                     shift);
  LG_LAUNCH_CHECK();
}


// A CSR (nr rows, ne entries; val optional) renumbered in place: the new row
// i holds the old row rperm[i] (rmap is its inverse; both null: rows keep
// their places), entries keep their order within the row, and their indices
// map through emap (null: unchanged).  sched is the old row schedule (for the
// entries' rows); its row lists are rebuilt for the new numbering.
void permute_csr(Ctx& c, Sched& sched, int32_t* ptr, int32_t* idx, double* val, int64_t nr,
                 int64_t ne, const int32_t* rperm, const int32_t* rmap, const int32_t* emap) {
  Arena& tmp = c.tmp;
  Arena::Mark m = tmp.mark();
  if (nr == 0) return;
  int32_t* ptr0 = tmp.get<int32_t>(nr + 1);
  LG_HIP(hipMemcpyAsync(ptr0, ptr, sizeof(int32_t) * (nr + 1), hipMemcpyDeviceToDevice, c.st));
  if (ne > 0) {
    int32_t* idx0 = tmp.get<int32_t>(ne);
    LG_HIP(hipMemcpyAsync(idx0, idx, sizeof(int32_t) * ne, hipMemcpyDeviceToDevice, c.st));
    double* val0 = nullptr;
    if (val) {
      val0 = tmp.get<double>(ne);
      LG_HIP(hipMemcpyAsync(val0, val, sizeof(double) * ne, hipMemcpyDeviceToDevice, c.st));
    }
    if (rperm) {
      int32_t* deg = tmp.get<int32_t>(nr);
      int64_t* p64 = tmp.get<int64_t>(nr + 1);
      hipLaunchKernelGGL(k_perm_degrees, dim3(nblk(nr)), dim3(kBlock), 0, c.st, ptr0, rperm, nr, deg);
      scan_i32_to_i64(deg, p64, nr, tmp, c.st, false);
      hipLaunchKernelGGL(k_i64_to_i32, dim3(nblk(nr + 1)), dim3(kBlock), 0, c.st, p64, nr + 1, ptr);
    }
    // over the old rows (the old schedule still describes ptr0)
    run_rows(sched, ptr0,
             PermEntriesOp{ptr0, idx0, val0, rmap, emap, (const int32_t*)ptr, idx, val}, c.st);
    LG_LAUNCH_CHECK();
  } else if (rperm) {
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk(nr + 1)), dim3(kBlock), 0, c.st, ptr, nr + 1, 0);
  }
  if (rperm) sched_fill(sched, ptr, tmp, c.st);
  tmp.rewind(m);
}

// Levels of at least this many vertices whose degrees are skewed and whose
// mean degree is moderate get the solve order.  Smaller levels are cache
// resident; near-regular ones, such as grids, keep the locality of their own
// numbering; on dense levels every row gathers from most of the vector
// whatever the order.  Among elimination levels only level 0 runs a product
// (one per CG iteration), and only when the solve is at least kReorderMinK
// columns wide does that product gain more than the renumbering pass (one
// gather per stored entry, whatever the width) costs: measured, C4's level 0
// gains about 2 ms per 16-column solve for a 2 ms pass, and R-MAT's level 0
// 0.08 ms per one-column solve for a 0.4 ms pass.
constexpr int64_t kReorderMinRows = (int64_t)1 << 14;
constexpr int64_t kReorderSkew = 8;       // largest degree >= kReorderSkew x mean degree
constexpr int64_t kReorderMaxMean = 128;  // mean degree at most this
constexpr int kReorderMinK = 4;

bool wants_order(const Level& L, int level, int K) {
  if (L.n < kReorderMinRows || L.nnz == 0) return false;
  if (!(L.type == LG_LEVEL_AGG || (L.type == LG_LEVEL_ELIM && level == 0 && K >= kReorderMinK)))
    return false;
  return (int64_t)L.sched.max_deg * L.n >= kReorderSkew * L.nnz && L.nnz <= kReorderMaxMean * L.n;
}

// The solve-time vertex order of every level that wants one: computed in the
// setup's numbering, then the level's matrix, diagonal, transfer maps and
// row schedules are renumbered.  Each row keeps its entries in their order,
// so every row's sum (products, restriction, elimination transfers) is formed
// exactly as in the setup's numbering.
void reorder_levels(Ctx& c) {
  lg_hierarchy* h = c.h;
  Arena& tmp = c.tmp;
  const int nl = (int)h->lev.size();
  for (int l = 0; l < nl; l++) {
    Level& L = h->lev[l];
    if (!wants_order(L, l, h->K)) continue;
    Arena::Mark m = tmp.mark();
    uint64_t* keys = tmp.get<uint64_t>(L.n);
    uint64_t* vals = tmp.get<uint64_t>(L.n);
    hipLaunchKernelGGL(k_order_keys, dim3(nblk(L.n)), dim3(kBlock), 0, c.st, L.rp, L.n,
                       L.sched.hub_deg, keys, vals);
    const SortedPairs sp = radix_sort_pairs(keys, vals, L.n, {0}, tmp, c.st);
    L.perm = h->mem.get<int32_t>(L.n);
    L.iperm = h->mem.get<int32_t>(L.n);
    hipLaunchKernelGGL(k_order_perm, dim3(nblk(L.n)), dim3(kBlock), 0, c.st, (const uint64_t*)sp.vals,
                       L.n, L.perm, L.iperm);
    LG_LAUNCH_CHECK();
    tmp.rewind(m);
  }
  for (int l = 0; l + 1 < nl; l++) {
    Level& L = h->lev[l];
    const Level& C = h->lev[l + 1];
    if (!L.perm && !C.perm) continue;
    const int64_t n = L.n;
    // the level's matrix and diagonal, once its Lanczos steps (which read
    // them on the side stream) are done
    if (L.perm) {
      if (l < (int)c.side.level_done.size() && c.side.level_done[l])
        LG_HIP(hipStreamWaitEvent(c.st, c.side.level_done[l], 0));
      permute_csr(c, L.sched, L.rp, L.col, L.w, n, L.nnz, L.perm, L.iperm, L.iperm);
      Arena::Mark m = tmp.mark();
      double* t = tmp.get<double>(n);
      for (double* v : {L.d, L.dinv}) {
        LG_HIP(hipMemcpyAsync(t, v, sizeof(double) * n, hipMemcpyDeviceToDevice, c.st));
        hipLaunchKernelGGL(k_perm_f64, dim3(nblk(n)), dim3(kBlock), 0, c.st, (const double*)t,
                           (const int32_t*)L.perm, n, v);
      }
      LG_LAUNCH_CHECK();
      tmp.rewind(m);
    }
    Arena::Mark m = tmp.mark();
    int32_t* t = tmp.get<int32_t>(std::max<int64_t>(n, L.nc));
    if (L.type == LG_LEVEL_AGG) {
      // aggregate of each (new) vertex, in the coarse level's new numbering
      LG_HIP(hipMemcpyAsync(t, L.agg, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c.st));
      hipLaunchKernelGGL(k_perm_index, dim3(nblk(n)), dim3(kBlock), 0, c.st, (const int32_t*)t,
                         (const int32_t*)L.perm, (const int32_t*)C.iperm, n, L.agg);
      // members of each coarse vertex (restriction), in their order
      permute_csr(c, L.msched, L.mptr, L.mem, nullptr, L.nc, n, C.perm, C.iperm, L.iperm);
    } else {
      // coarse index of each fine vertex, fine vertex of each coarse one
      LG_HIP(hipMemcpyAsync(t, L.cidx, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c.st));
      hipLaunchKernelGGL(k_perm_index, dim3(nblk(n)), dim3(kBlock), 0, c.st, (const int32_t*)t,
                         (const int32_t*)L.perm, (const int32_t*)C.iperm, n, L.cidx);
      LG_HIP(hipMemcpyAsync(t, L.cvert, sizeof(int32_t) * L.nc, hipMemcpyDeviceToDevice, c.st));
      hipLaunchKernelGGL(k_perm_index, dim3(nblk(L.nc)), dim3(kBlock), 0, c.st, (const int32_t*)t,
                         (const int32_t*)C.perm, (const int32_t*)L.iperm, L.nc, L.cvert);
      // the F part of P^T over coarse rows
      permute_csr(c, L.ptsched, L.ptrp, L.ptf, L.ptc, L.nc, L.nnzP - L.nc, C.perm, C.iperm, L.iperm);
    }
    LG_LAUNCH_CHECK();
    tmp.rewind(m);
  }
}

void make_f32(Ctx& c, Level& L) {
  lg_hierarchy* h = c.h;
  L.wf = h->mem.get<float>(L.nnz);
  L.df = h->mem.get<float>(L.n);
  L.dinvf = h->mem.get<float>(L.n);
  if (L.nnz) hipLaunchKernelGGL(k_to_f32, dim3(nblk(L.nnz)), dim3(kBlock), 0, c.st, L.w, L.wf, L.nnz);
  hipLaunchKernelGGL(k_to_f32, dim3(nblk(L.n)), dim3(kBlock), 0, c.st, L.d, L.df, L.n);
  hipLaunchKernelGGL(k_to_f32, dim3(nblk(L.n)), dim3(kBlock), 0, c.st, L.dinv, L.dinvf, L.n);
  if (L.type == LG_LEVEL_ELIM) {
    const int64_t npt = L.nnzP - L.nc;
    L.ptcf = h->mem.get<float>(npt);
    if (npt)
      hipLaunchKernelGGL(k_to_f32, dim3(nblk(npt)), dim3(kBlock), 0, c.st, L.ptc, L.ptcf, npt);
  }
  LG_LAUNCH_CHECK();
}

}  // namespace

void setup_hierarchy(lg_hierarchy* h, const lg_graph* g, hipStream_t st) {
  const lg_setup_opts& o = h->opts;
  Ctx c;
  c.h = h;
  c.st = st;
  c.key = seed_key(o.seed);
  c.flags = h->mem.get<int>(4);
  if (!h->capture_stream) LG_HIP(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
  c.side.s = h->capture_stream;
  LG_HIP(hipEventCreateWithFlags(&c.side.ready, hipEventDisableTiming));
  LG_HIP(hipEventCreateWithFlags(&c.side.done, hipEventDisableTiming));
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, st, (int32_t*)c.flags, (int64_t)4, 0);
  const int64_t n = g->n, nnz = g->nnz;
  h->lev.emplace_back();
  Level* L0 = &h->lev.back();
  L0->n = n;
  L0->nnz = nnz;
  L0->rp = h->mem.get<int32_t>(n + 1);
  L0->col = h->mem.get<int32_t>(nnz);
  L0->w = h->mem.get<double>(nnz);
  {
    Arena::Mark m = c.tmp.mark();
    int64_t* rp64 = c.tmp.get<int64_t>(n + 1);
    const hipMemcpyKind kind = g->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    LG_HIP(hipMemcpyAsync(rp64, g->row_ptr, sizeof(int64_t) * (n + 1), kind, st));
    if (nnz) {
      LG_HIP(hipMemcpyAsync(L0->col, g->col, sizeof(int32_t) * nnz, kind, st));
      LG_HIP(hipMemcpyAsync(L0->w, g->w, sizeof(double) * nnz, kind, st));
    }
    hipLaunchKernelGGL(k_rowptr_to32, dim3(nblk(n + 1)), dim3(kBlock), 0, st, rp64, L0->rp, n, nnz,
                       c.flags);
    LG_LAUNCH_CHECK();
    check_flags(c);  // row pointers must be sane before any row pass
    c.tmp.rewind(m);
  }
  // level 0's schedule is stable: the CG product's fused dot then sums its
  // terms in the same order on every setup of a graph
  build_sched(L0->sched, L0->rp, n, nnz, h->mem, c.tmp, st, o.merge_path != 0, true);
  check_isolated(*L0);
  if (o.validate && nnz) {
    Arena::Mark m = c.tmp.mark();
    int32_t* rowidx = c.tmp.get<int32_t>(nnz);
    const int64_t nbv = nblk(nnz);
    int32_t* searched = c.tmp.get<int32_t>(nbv);
    run_rows(L0->sched, L0->rp, RowIdxOp{rowidx}, st);
    hipLaunchKernelGGL(k_validate, dim3((unsigned)nbv), dim3(kBlock), 0, st, rowidx, L0->rp, L0->col,
                       L0->w, n, nnz, c.flags, searched);
    hipLaunchKernelGGL(k_validate_pairs, dim3(1), dim3(kPairThreads), 0, st, (const int32_t*)searched,
                       nbv, nnz, c.flags);
    LG_LAUNCH_CHECK();
    c.tmp.rewind(m);  // later work on the stream runs after these kernels
  }
  // The diagonal pass reads the weights along the (already checked) row
  // pointers only, so it runs before the validation flags come back; both
  // come back with the total weight, in one round trip.
  level_diag(c, *L0);
  {
    // total weight guard of the exact sums
    Arena::Mark m = c.tmp.mark();
    double* part = c.tmp.get<double>(kRedBlocks);
    double* tot = c.tmp.get<double>(1);
    reduce_dev<RED_SUM>(L0->d, nullptr, nullptr, n, part, tot, st);
    double total = 0.0;
    int f = 0;
    const DevRead rd[2] = {{&f, c.flags, sizeof(f)}, {&total, tot, sizeof(total)}};
    read_dev_n(rd, 2, st);
    raise_flags(f);
    if (!(total < 0x1p62)) fail(LG_E_RANGE, "total edge weight must be below 2^62");
    c.tmp.rewind(m);
  }

  h->lmax_dev = h->mem.get<double>(kMaxLevelCap);
  int l = 0;
  for (;;) {
    Level* L = &h->lev[l];
    const bool stop_here = (L->n + L->nnz <= o.coarsest_nnz) || (l + 1 >= o.max_levels) ||
                           (l + 2 >= kMaxLevelCap);
    if (stop_here) break;
    Arena::Mark lm = c.tmp.mark();
    // Section 3.4's elimination, repeated on its own result while it still
    // removes more than the minimum fraction (elim_passes > 1)
    bool stop = false;
    for (int pass = 0; o.elim_enable && pass < o.elim_passes; pass++) {
      ElimChoice ch = elim_select(c, *L);
      if (!((double)ch.nf > o.elim_min_fraction * (double)L->n)) {
        c.tmp.rewind(lm);
        break;
      }
      h->lev.emplace_back();
      L = &h->lev[l];
      build_elim(c, *L, ch, h->lev[l + 1]);
      c.tmp.rewind(lm);
      l++;
      L = &h->lev[l];
      if ((L->n + L->nnz <= o.coarsest_nnz) || (l + 1 >= o.max_levels) || (l + 2 >= kMaxLevelCap)) {
        stop = true;
        break;
      }
    }
    if (stop) break;
    // aggregation level
    double* X = o.keep_setup_data ? h->mem.get<double>(4 * L->n) : c.tmp.get<double>(4 * L->n);
    double* S = o.keep_setup_data ? h->mem.get<double>(L->nnz) : c.tmp.get<double>(L->nnz);
    strength(c, *L, l, S, X);
    int32_t *status = nullptr, *votes = nullptr;
    const int64_t nc = aggregate(c, *L, S, &status, &votes);
    if (o.keep_setup_data) {
      L->X = X;
      L->S = S;
      L->status = status;
      L->votes = votes;
    }
    if (nc >= L->n) {  // no progress: this level becomes the coarsest
      L->agg = nullptr;
      c.tmp.rewind(lm);
      break;
    }
    h->lev.emplace_back();
    L = &h->lev[l];
    L->type = LG_LEVEL_AGG;
    L->nc = nc;
    galerkin(c, *L, nc, h->lev[l + 1]);
    lanczos(c, *L, l, h->lmax_dev + l);
    c.tmp.rewind(lm);
    l++;
  }
  h->lev.resize(l + 1);
  h->lev[l].type = LG_LEVEL_COARSEST;
  h->lev[l].nc = 0;
  coarsest(c, h->lev[l]);
  // the solve order rewrites a level after its own Lanczos steps (side stream)
  if (o.reorder) reorder_levels(c);
  if (o.precision == LG_MIXED)
    for (int i = 0; i < l; i++) make_f32(c, h->lev[i]);
  LG_HIP(hipEventRecord(c.side.done, c.side.s));
  LG_HIP(hipStreamWaitEvent(st, c.side.done, 0));
  // After validation the level loop can only raise F_XSUM (an exact sum out of
  // range) and the coarsest level F_SPLIT, neither of which affects an index;
  // they come back here, with the eigenvalue estimates, in one round trip.
  std::vector<double> lm(l + 1, 0.0);
  int f = 0;
  const DevRead rd[2] = {{&f, c.flags, sizeof(f)}, {lm.data(), h->lmax_dev, sizeof(double) * (l + 1)}};
  read_dev_n(rd, 2, st);
  raise_flags(f);
  for (int i = 0; i <= l; i++) h->lev[i].lmax = h->lev[i].type == LG_LEVEL_AGG ? lm[i] : 0.0;
}

}  // namespace lg
