// solve.hip -- the solve phase (Algorithm 1 as a preconditioner for CG, or
// the K-cycle inside flexible CG; Sections 2.3.2, 3.6, 3.7, 4) for k
// right-hand sides at once.  Multi-vectors are n x K row-major with K the
// padded batch width (a power of two up to 32); every kernel streams the
// level's CSR once for all K columns.
//
// Precision: T = double (FP64) or float (the mixed form: hierarchy values,
// smoother and transfers in fp32; the outer Krylov method, its dot products
// and residuals, and the coarsest dense solve stay in fp64).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "impl.h"
#include "ops.h"

namespace lg {

static inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)ceil_div(n, b); }

// ------------------------------------------------------- vector kernels
// Elementwise kernels handle V = 16 / sizeof(T) consecutive entries of an
// n x K multi-vector per thread.  When K is a multiple of V those entries lie
// in one row and move as one 16-byte vector; otherwise (K < V) each entry
// finds its own row.
template <typename T>
struct Vec16 {
  static constexpr int V = 16 / (int)sizeof(T);
  typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
};

template <typename T>
__device__ __forceinline__ typename Vec16<T>::type ld16(const T* p) {
  return *reinterpret_cast<const typename Vec16<T>::type*>(p);
}
template <typename T>
__device__ __forceinline__ void st16(T* p, const typename Vec16<T>::type& v) {
  *reinterpret_cast<typename Vec16<T>::type*>(p) = v;
}

template <typename T, int K>
inline unsigned vec_blocks(int64_t n) {
  return (unsigned)ceil_div(ceil_div(n * K, (int64_t)Vec16<T>::V), (int64_t)kBlock);
}

// x = c0 D^-1 b (one Chebyshev step from a zero guess)
template <typename T, int K>
__global__ void k_cheb_zero(const T* __restrict__ b, const T* __restrict__ dinv,
                            T* __restrict__ x, int64_t n, T c0) {
  constexpr int V = Vec16<T>::V;
  const int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * V;
  if (i0 >= n * K) return;
  if constexpr (K % V == 0) {
    const T di = dinv[i0 / K];
    typename Vec16<T>::type v = ld16(b + i0);
#pragma unroll
    for (int e = 0; e < V; e++) v[e] = (di * v[e]) * c0;
    st16(x + i0, v);
  } else {
    for (int e = 0; e < V && i0 + e < n * K; e++)
      x[i0 + e] = (dinv[(i0 + e) / K] * b[i0 + e]) * c0;
  }
}

// out = x + P xc with P the aggregation's piecewise-constant prolongation
template <typename T, int K>
__global__ void k_agg_prolong(const T* __restrict__ x, const T* __restrict__ xc,
                              const int32_t* __restrict__ agg, T* __restrict__ out, int64_t n) {
  constexpr int V = Vec16<T>::V;
  const int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * V;
  if (i0 >= n * K) return;
  if constexpr (K % V == 0) {
    const int64_t row = i0 / K;
    const int c = (int)(i0 - row * K);
    typename Vec16<T>::type v = ld16(x + i0);
    const typename Vec16<T>::type u = ld16(xc + (int64_t)agg[row] * K + c);
#pragma unroll
    for (int e = 0; e < V; e++) v[e] += u[e];
    st16(out + i0, v);
  } else {
    for (int e = 0; e < V && i0 + e < n * K; e++) {
      const int64_t i = i0 + e, row = i / K;
      out[i] = x[i] + xc[(int64_t)agg[row] * K + (i - row * K)];
    }
  }
}

// x = P_elim x_c + [D_FF^-1 b_F; 0] (Section 3.4, additive two-level form):
// a kept vertex copies its coarse value, an eliminated one averages its
// (kept) neighbours' coarse values and adds its own D^-1 b.
template <typename T, int K>
__global__ void k_elim_prolong(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                               const T* __restrict__ w, const T* __restrict__ dinv,
                               const int32_t* __restrict__ cidx, const T* __restrict__ xc,
                               const T* __restrict__ b, T* __restrict__ x, int64_t n) {
  constexpr int V = Vec16<T>::V;
  const int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * V;
  if (i0 >= n * K) return;
  if constexpr (K % V == 0) {
    const int64_t row = i0 / K;
    const int c = (int)(i0 - row * K);
    const int ci = cidx[row];
    if (ci >= 0) {
      st16(x + i0, ld16(xc + (int64_t)ci * K + c));
      return;
    }
    const T di = dinv[row];
    typename Vec16<T>::type s;
#pragma unroll
    for (int e = 0; e < V; e++) s[e] = T(0);
    for (int q = rp[row]; q < rp[row + 1]; q++) {
      const T f = w[q] * di;
      const typename Vec16<T>::type u = ld16(xc + (int64_t)cidx[col[q]] * K + c);
#pragma unroll
      for (int e = 0; e < V; e++) s[e] += f * u[e];
    }
    const typename Vec16<T>::type bv = ld16(b + i0);
#pragma unroll
    for (int e = 0; e < V; e++) s[e] += bv[e] * di;
    st16(x + i0, s);
  } else {
    for (int e = 0; e < V && i0 + e < n * K; e++) {
      const int64_t i = i0 + e, row = i / K;
      const int c = (int)(i - row * K);
      const int ci = cidx[row];
      if (ci >= 0) {
        x[i] = xc[(int64_t)ci * K + c];
        continue;
      }
      const T di = dinv[row];
      T s = T(0);
      for (int q = rp[row]; q < rp[row + 1]; q++) s += (w[q] * di) * xc[(int64_t)cidx[col[q]] * K + c];
      x[i] = s + b[i] * di;
    }
  }
}

// b_c[I] = sum of r over the members of aggregate I (R r, Section 3.5)
template <typename T, int K>
struct GatherSumOp {
  using Acc = VecAcc<T, K>;
  const int32_t* __restrict__ idx;
  const T* __restrict__ src;
  T* __restrict__ out;
  __device__ Acc identity() const {
    Acc a;
#pragma unroll
    for (int c = 0; c < K; c++) a.v[c] = T(0);
    return a;
  }
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc& a, int64_t, int e) const {
    const T* s = src + (int64_t)idx[e] * K;
#pragma unroll
    for (int c = 0; c < K; c++) a.v[c] += s[c];
  }
  __device__ void combine(Acc& a, const Acc& o) const {
#pragma unroll
    for (int c = 0; c < K; c++) a.v[c] += o.v[c];
  }
  __device__ void finish(int64_t row, const Acc& a, int lane, int G) const {
#pragma unroll
    for (int c = 0; c < K; c++)
      if (c % G == lane) out[row * K + c] = a.v[c];
  }
};

// b_c[a'] = b[a] + sum over eliminated neighbours f of (w_af / d_f) b_f  (P_elim^T b)
template <typename T, int K>
struct PtOp {
  using Acc = VecAcc<T, K>;
  const int32_t* __restrict__ ptf;
  const T* __restrict__ ptc;
  const int32_t* __restrict__ cvert;
  const T* __restrict__ b;
  T* __restrict__ bc;
  __device__ Acc identity() const {
    Acc a;
#pragma unroll
    for (int c = 0; c < K; c++) a.v[c] = T(0);
    return a;
  }
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc& a, int64_t, int e) const {
    const T cf = ptc[e];
    const T* s = b + (int64_t)ptf[e] * K;
#pragma unroll
    for (int c = 0; c < K; c++) a.v[c] += cf * s[c];
  }
  __device__ void combine(Acc& a, const Acc& o) const {
#pragma unroll
    for (int c = 0; c < K; c++) a.v[c] += o.v[c];
  }
  __device__ void finish(int64_t row, const Acc& a, int lane, int G) const {
    const int64_t v = cvert[row];
#pragma unroll
    for (int c = 0; c < K; c++)
      if (c % G == lane) bc[row * K + c] = b[v * K + c] + a.v[c];
  }
};

// Column-split forms of the two restrictions (k * sizeof(T) >= 32 bytes).
template <typename T, int K>
struct GatherSumColOp {
  static constexpr int V = 16 / (int)sizeof(T);
  static constexpr int kL = K / V;
  using Acc = VecAcc<T, V>;
  typedef T vec_t __attribute__((ext_vector_type(16 / sizeof(T))));
  const int32_t* __restrict__ idx;
  const T* __restrict__ src;
  T* __restrict__ out;
  __device__ Acc identity() const {
    Acc a;
#pragma unroll
    for (int v = 0; v < V; v++) a.v[v] = T(0);
    return a;
  }
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc& a, int64_t, int e, int part, bool keep = true) const {
    const vec_t s = *reinterpret_cast<const vec_t*>(src + (int64_t)idx[e] * K + part * V);
#pragma unroll
    for (int v = 0; v < V; v++) a.v[v] += keep ? s[v] : T(0);
  }
  __device__ void combine(Acc& a, const Acc& o) const {
#pragma unroll
    for (int v = 0; v < V; v++) a.v[v] += o.v[v];
  }
  struct Pre {};
  __device__ Pre prefetch(int64_t, int) const { return Pre{}; }
  __device__ void finish(int64_t row, const Acc& a, int part, const Pre& = Pre{}) const {
    vec_t o;
#pragma unroll
    for (int v = 0; v < V; v++) o[v] = a.v[v];
    *reinterpret_cast<vec_t*>(out + row * K + part * V) = o;
  }
};

template <typename T, int K>
struct PtColOp {
  static constexpr int V = 16 / (int)sizeof(T);
  static constexpr int kL = K / V;
  using Acc = VecAcc<T, V>;
  typedef T vec_t __attribute__((ext_vector_type(16 / sizeof(T))));
  const int32_t* __restrict__ ptf;
  const T* __restrict__ ptc;
  const int32_t* __restrict__ cvert;
  const T* __restrict__ b;
  T* __restrict__ bc;
  __device__ Acc identity() const {
    Acc a;
#pragma unroll
    for (int v = 0; v < V; v++) a.v[v] = T(0);
    return a;
  }
  __device__ bool active(int64_t) const { return true; }
  __device__ void accum(Acc& a, int64_t, int e, int part, bool keep = true) const {
    const T cf = keep ? ptc[e] : T(0);
    const vec_t s = *reinterpret_cast<const vec_t*>(b + (int64_t)ptf[e] * K + part * V);
#pragma unroll
    for (int v = 0; v < V; v++) a.v[v] += cf * s[v];
  }
  __device__ void combine(Acc& a, const Acc& o) const {
#pragma unroll
    for (int v = 0; v < V; v++) a.v[v] += o.v[v];
  }
  struct Pre {
    vec_t bv;
  };
  __device__ Pre prefetch(int64_t row, int part) const {
    return Pre{*reinterpret_cast<const vec_t*>(b + (int64_t)cvert[row] * K + part * V)};
  }
  __device__ void finish(int64_t row, const Acc& a, int part) const {
    finish(row, a, part, prefetch(row, part));
  }
  __device__ void finish(int64_t row, const Acc& a, int part, const Pre& q) const {
    const vec_t bv = q.bv;
    vec_t o;
#pragma unroll
    for (int v = 0; v < V; v++) o[v] = bv[v] + a.v[v];
    *reinterpret_cast<vec_t*>(bc + row * K + part * V) = o;
  }
};

// Coarsest level: x = L^+ b with the fp64 dense pseudo-inverse; one wavefront per row.
template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_coarse(const double* __restrict__ Lp,
                                                   const T* __restrict__ b, T* __restrict__ x,
                                                   int64_t n) {
  const int64_t row = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double acc[K];
#pragma unroll
  for (int c = 0; c < K; c++) acc[c] = 0.0;
  for (int64_t j = lane; j < n; j += 64) {
    const double l = Lp[row * n + j];
#pragma unroll
    for (int c = 0; c < K; c++) acc[c] += l * (double)b[j * K + c];
  }
#pragma unroll
  for (int c = 0; c < K; c++) {
    double v = acc[c];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    if (lane == (c & 63)) x[row * K + c] = (T)v;
  }
}

template <typename TI, typename TO>
__global__ void k_convert(const TI* __restrict__ in, TO* __restrict__ out, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < m) out[i] = (TO)in[i];
}

template <typename T>
__global__ void k_copy(T* __restrict__ dst, const T* __restrict__ src, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < m) dst[i] = src[i];
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t m, T v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < m) p[i] = v;
}

// The caller's n x k block into the solve's n x K workspace (zero padded),
// row i of the solve order taking the caller's row perm[i] (perm null: i).
__global__ void k_pad_in(const double* __restrict__ B, int k, double* __restrict__ out, int K,
                         int64_t n, const int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n * K) return;
  const int64_t row = i / K;
  const int c = (int)(i - row * K);
  out[i] = c < k ? B[(perm ? (int64_t)perm[row] : row) * k + c] : 0.0;
}

// Back: the caller's row i from the solve order's row iperm[i].
__global__ void k_pad_out(const double* __restrict__ in, int K, double* __restrict__ X, int k,
                          int64_t n, const int32_t* __restrict__ iperm) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n * k) return;
  const int64_t row = i / k;
  const int c = (int)(i - row * k);
  X[i] = in[(iperm ? (int64_t)iperm[row] : row) * K + c];
}

// Deterministic column reductions.  A pass over an n x K multi-vector runs a
// grid sized to the data (at most kDotBlocks workgroups, fixed for a given
// size); each workgroup streams one contiguous range of whole rounds (kBlock
// 16-byte vectors of V entries each), so slot v of thread t always holds
// column (t V + v) mod K.  Each workgroup folds its slots per column through
// LDS in a fixed order into partial[(block * ND + d) * K + c]; k_dots_final
// then reduces the partials of each (product, column) with a fixed tree.
// (Contiguous ranges stream faster than a grid-wide stride: 5.1 against
// 4.2 TB/s for the CG's residual update.)
constexpr int kDotBlocks = kDotPartials;

struct VecRange {
  int64_t beg, end;
};
__device__ __forceinline__ VecRange block_range(int64_t nvec) {
  const int64_t rounds = (nvec + kBlock - 1) / kBlock;
  const int64_t per = (rounds + gridDim.x - 1) / gridDim.x * kBlock;
  const int64_t beg = min((int64_t)blockIdx.x * per, nvec);
  return {beg, min(beg + per, nvec)};
}

template <int K, int V, int ND>
__device__ __forceinline__ void col_partials(const double (&s)[ND][V], double* __restrict__ partial) {
  __shared__ double sm[ND][kBlock * V];
#pragma unroll
  for (int d = 0; d < ND; d++)
#pragma unroll
    for (int v = 0; v < V; v++) sm[d][threadIdx.x * V + v] = s[d][v];
  __syncthreads();
  if ((int)threadIdx.x < K) {
#pragma unroll
    for (int d = 0; d < ND; d++) {
      double t = 0.0;
      for (int q = threadIdx.x; q < kBlock * V; q += K) t += sm[d][q];
      partial[((int64_t)blockIdx.x * ND + d) * K + threadIdx.x] = t;
    }
  }
}

// ND products a_d . b_d per column, or column sums of a_d where b_d is null.
template <typename T, int K, int ND>
__global__ __launch_bounds__(kBlock) void k_dots(const T* __restrict__ a0, const T* __restrict__ b0,
                                                 const T* __restrict__ a1, const T* __restrict__ b1,
                                                 int64_t m, double* __restrict__ partial) {
  constexpr int V = Vec16<T>::V;
  double s[ND][V];
#pragma unroll
  for (int d = 0; d < ND; d++)
#pragma unroll
    for (int v = 0; v < V; v++) s[d][v] = 0.0;
  const int64_t nvec = m / V;  // whole vectors; the rest (only when K < V) below
  const VecRange rg = block_range(nvec);
  for (int64_t q = rg.beg + threadIdx.x; q < rg.end; q += kBlock) {
    const typename Vec16<T>::type x0 = ld16(a0 + q * V);
    typename Vec16<T>::type y0;
    if (b0) y0 = ld16(b0 + q * V);
#pragma unroll
    for (int v = 0; v < V; v++) s[0][v] += b0 ? (double)x0[v] * (double)y0[v] : (double)x0[v];
    if (ND > 1) {
      const typename Vec16<T>::type x1 = ld16(a1 + q * V);
      const typename Vec16<T>::type y1 = ld16(b1 + q * V);
#pragma unroll
      for (int v = 0; v < V; v++) s[ND - 1][v] += (double)x1[v] * (double)y1[v];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int64_t i = nvec * V; i < m; i++) {
      const int v = (int)(i % V);
      s[0][v] += b0 ? (double)a0[i] * (double)b0[i] : (double)a0[i];
      if (ND > 1) s[ND - 1][v] += (double)a1[i] * (double)b1[i];
    }
  }
  col_partials<K, V, ND>(s, partial);
}

// One workgroup per (product, column): a fixed tree over the block partials.
template <int K, int ND>
__global__ __launch_bounds__(kBlock) void k_dots_final(const double* __restrict__ partial, int nb,
                                                       double* __restrict__ out0,
                                                       double* __restrict__ out1,
                                                       double* __restrict__ out2) {
  const int t = blockIdx.x;
  const int d = t / K, c = t % K;
  __shared__ double sm[kBlock];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) s += partial[((int64_t)b * ND + d) * K + c];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int m = kBlock / 2; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m) sm[threadIdx.x] += sm[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) (d == 0 ? out0 : d == 1 ? out1 : out2)[c] = sm[0];
}

template <int K>
__global__ void k_sub_mean(double* __restrict__ v, const double* __restrict__ sums, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n * K) return;
  v[i] -= sums[i % K] / (double)n;
}

// alpha = num / (p . q) for active columns; a non-positive p . q is a breakdown.
template <int K>
__global__ void k_alpha(double* __restrict__ scal, int flexible) {
  const int c = threadIdx.x;
  if (c >= K) return;
  const double act = scal[S_ACTIVE * K + c];
  const double pq = scal[S_PQ * K + c];
  const double num = flexible ? scal[S_PR * K + c] : scal[S_RZ * K + c];
  double a = 0.0;
  if (act > 0.0) {
    if (pq > 0.0) a = num / pq;
    else {
      scal[S_ACTIVE * K + c] = 0.0;
      scal[S_TR * K + c] = 1.0;  // breakdown
    }
  }
  scal[S_ALPHA * K + c] = a;
}

// r -= alpha q per column, with the column sums of r . r of the new r, and
// rc = r in the cycle's precision when rc is set.  The matching x += alpha p
// is deferred to the next direction update (k_xpby_z), which reads p anyway,
// or to k_update_x where x is needed before then.
template <int K, typename TC>
__global__ __launch_bounds__(kBlock) void k_update_r(double* __restrict__ r,
                                                     const double* __restrict__ q,
                                                     const double* __restrict__ scal, int64_t m,
                                                     TC* __restrict__ rc,
                                                     double* __restrict__ partial) {
  constexpr int V = 2;
  double s[1][V] = {{0.0, 0.0}};
  double a[V];
#pragma unroll
  for (int v = 0; v < V; v++) a[v] = scal[S_ALPHA * K + ((int)threadIdx.x * V + v) % K];
  typedef TC tc2 __attribute__((ext_vector_type(2)));
  const int64_t nvec = m / V;
  const VecRange rg = block_range(nvec);
  // two vectors per trip so that four loads are in flight
  for (int64_t t0 = rg.beg + threadIdx.x; t0 < rg.end; t0 += 2 * kBlock) {
    typename Vec16<double>::type rv[2], qv[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const int64_t t = t0 + h * kBlock < rg.end ? t0 + h * kBlock : t0;
      rv[h] = ld16(r + t * V);
      qv[h] = ld16(q + t * V);
    }
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const int64_t t = t0 + h * kBlock;
      if (t >= rg.end) break;
#pragma unroll
      for (int v = 0; v < V; v++) {
        rv[h][v] -= a[v] * qv[h][v];
        s[0][v] += rv[h][v] * rv[h][v];
      }
      st16(r + t * V, rv[h]);
      if (rc) {
        tc2 o;
        o[0] = (TC)rv[h][0];
        o[1] = (TC)rv[h][1];
        *reinterpret_cast<tc2*>(rc + t * V) = o;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // odd m (K = 1): last entry, column 0
    for (int64_t i = nvec * V; i < m; i++) {
      r[i] -= scal[S_ALPHA * K + (int)(i % K)] * q[i];
      s[0][i % V] += r[i] * r[i];
      if (rc) rc[i] = (TC)r[i];
    }
  }
  col_partials<K, V, 1>(s, partial);
}

// x += alpha p per column: the deferred solution update where x is read
// before the next direction update.
template <int K>
__global__ void k_update_x(double* __restrict__ x, const double* __restrict__ p,
                           const double* __restrict__ scal, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < m) x[i] += scal[S_ALPHA * K + (int)(i % K)] * p[i];
}

// Column sums of z (the cycle's output, precision T), of z . y and of y, with
// y the fp64 residual (CG) or q = L p (flexible CG): enough to project z to
// mean zero and form the projected z . y without storing the projection.
template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_zstats(const T* __restrict__ z,
                                                   const double* __restrict__ y, int64_t m,
                                                   double* __restrict__ partial) {
  constexpr int V = Vec16<T>::V;
  double s[3][V];
#pragma unroll
  for (int d = 0; d < 3; d++)
#pragma unroll
    for (int v = 0; v < V; v++) s[d][v] = 0.0;
  const int64_t nvec = m / V;
  const VecRange rg = block_range(nvec);
  for (int64_t t = rg.beg + threadIdx.x; t < rg.end; t += kBlock) {
    const typename Vec16<T>::type zv = ld16(z + t * V);
#pragma unroll
    for (int u = 0; u < V; u += 2) {
      const typename Vec16<double>::type yv = ld16(y + t * V + u);
#pragma unroll
      for (int e = 0; e < 2; e++) {
        const double zd = (double)zv[u + e];
        s[0][u + e] += zd;
        s[1][u + e] += zd * yv[e];
        s[2][u + e] += yv[e];
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int64_t i = nvec * V; i < m; i++) {
      const int v = (int)(i % V);
      const double zd = (double)z[i];
      s[0][v] += zd;
      s[1][v] += zd * y[i];
      s[2][v] += y[i];
    }
  }
  col_partials<K, V, 3>(s, partial);
}

// From the sums of k_zstats: the mean of z, the projected product
// (z - mean) . y = z . y - mean * sum(y), and beta.  CG: beta = rz_new / rz_old
// (rz_old replaced); flexible CG: beta = -(z . q) / (p . q).  first: the
// initial direction (beta = 0, CG records rz).
template <int K>
__global__ void k_beta_z(double* __restrict__ scal, double inv_n, int flexible, int first) {
  const int c = threadIdx.x;
  if (c >= K) return;
  const double mean = scal[S_ZSUM * K + c] * inv_n;
  const double zy = scal[S_ZY * K + c] - mean * scal[S_YSUM * K + c];
  scal[S_MEAN * K + c] = mean;
  const double act = scal[S_ACTIVE * K + c];
  double b = 0.0;
  if (flexible) {
    const double pq = scal[S_PQ * K + c];
    if (!first && act > 0.0 && pq > 0.0) b = -zy / pq;
  } else if (first) {
    scal[S_RZ * K + c] = zy;
  } else if (act > 0.0) {
    const double rz = scal[S_RZ * K + c];
    b = rz != 0.0 ? zy / rz : 0.0;
    scal[S_RZ * K + c] = zy;
  }
  scal[S_BETA * K + c] = b;
}

// p = (z - mean) + beta p, or p = z - mean where every column restarts
// (all = 1) or the column's restart flag is set.  When x is set, first the
// deferred x += alpha p with the direction being replaced.
template <typename T, int K>
__global__ void k_xpby_z(double* __restrict__ p, const T* __restrict__ z,
                         const double* __restrict__ scal, const double* __restrict__ flag,
                         int all, int64_t m, double* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i0 = t * 2;
  if (i0 >= m) return;
  if (i0 + 1 < m) {
    typename Vec16<double>::type pv;
    if (!all || x) pv = ld16(p + i0);
    if (x) {
      typename Vec16<double>::type xv = ld16(x + i0);
#pragma unroll
      for (int e = 0; e < 2; e++) xv[e] += scal[S_ALPHA * K + (int)((i0 + e) % K)] * pv[e];
      st16(x + i0, xv);
    }
#pragma unroll
    for (int e = 0; e < 2; e++) {
      const int c = (int)((i0 + e) % K);
      const double zp = (double)z[i0 + e] - scal[S_MEAN * K + c];
      const bool fresh = all || (flag && flag[c] > 0.0);
      pv[e] = fresh ? zp : zp + scal[S_BETA * K + c] * pv[e];
    }
    st16(p + i0, pv);
  } else {
    const int c = (int)(i0 % K);
    if (x) x[i0] += scal[S_ALPHA * K + c] * p[i0];
    const double zp = (double)z[i0] - scal[S_MEAN * K + c];
    const bool fresh = all || (flag && flag[c] > 0.0);
    p[i0] = fresh ? zp : zp + scal[S_BETA * K + c] * p[i0];
  }
}

// Slot mode: column `slot` of the n x K multi-vector b takes B[i * ldb].
template <int K>
__global__ void k_load_col(double* __restrict__ b, int slot, const double* __restrict__ B, int ldb,
                           int64_t n, const int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i * K + slot] = B[(perm ? (int64_t)perm[i] : i) * ldb];
}

// v -= its column mean in the flagged columns only.
template <int K>
__global__ void k_sub_mean_flagged(double* __restrict__ v, const double* __restrict__ sums,
                                   const double* __restrict__ flag, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n * K && flag[i % K] > 0.0) v[i] -= sums[i % K] / (double)n;
}

// Slot mode, a refilled column: x = 0 and t = b (the restart then takes r = t).
template <int K>
__global__ void k_refill_cols(double* __restrict__ x, double* __restrict__ t,
                              const double* __restrict__ b, const double* __restrict__ flag,
                              int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < m && flag[i % K] > 0.0) {
    x[i] = 0.0;
    t[i] = b[i];
  }
}

// Slot mode, a finished column: X[i * ldx] = x_i - mean(x) (the same
// arithmetic as the projection at the end of a plain solve).
template <int K>
__global__ void k_store_col(const double* __restrict__ x, int slot, const double* __restrict__ sums,
                            int64_t n, double* __restrict__ X, int ldx,
                            const int32_t* __restrict__ iperm) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) X[i * ldx] = x[(iperm ? (int64_t)iperm[i] : i) * K + slot] - sums[slot] / (double)n;
}

// dst = src in the columns whose flag is set (columns never influence each other)
template <int K>
__global__ void k_copy_flagged(double* __restrict__ dst, const double* __restrict__ src,
                               const double* __restrict__ flag, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < m && flag[i % K] > 0.0) dst[i] = src[i];
}

// ---- inner FCG(2) scalars of the K-cycle: [d1 a1 alpha1 zq d2 a2] x K
template <int K>
__global__ void k_fcg_alpha1(double* __restrict__ ks) {
  const int c = threadIdx.x;
  if (c >= K) return;
  const double d1 = ks[0 * K + c], a1 = ks[1 * K + c];
  ks[2 * K + c] = d1 > 0.0 ? a1 / d1 : 0.0;
}

template <typename T, int K>
__global__ void k_fcg_step1(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p1,
                            const T* __restrict__ q1, const double* __restrict__ ks, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n * K) return;
  const T a = (T)ks[2 * K + (i % K)];
  x[i] = a * p1[i];
  r[i] -= a * q1[i];
}

template <typename T, int K>
__global__ void k_fcg_p2(T* __restrict__ z, const T* __restrict__ p1,
                         const double* __restrict__ ks, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n * K) return;
  const int c = (int)(i % K);
  const double d1 = ks[0 * K + c];
  const T g = (T)(d1 > 0.0 ? ks[3 * K + c] / d1 : 0.0);
  z[i] -= g * p1[i];
}

template <typename T, int K>
__global__ void k_fcg_final(T* __restrict__ x, const T* __restrict__ p2,
                            const double* __restrict__ ks, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n * K) return;
  const int c = (int)(i % K);
  const double d2 = ks[4 * K + c];
  const T a = (T)(d2 > 0.0 ? ks[5 * K + c] / d2 : 0.0);
  x[i] += a * p2[i];
}

// ================================================================ host
template <typename T>
struct Vals {
  const T *w, *d, *dinv, *ptc;
};
template <typename T>
inline Vals<T> vals_of(const Level& L);
template <>
inline Vals<double> vals_of<double>(const Level& L) {
  return {L.w, L.d, L.dinv, L.ptc};
}
template <>
inline Vals<float> vals_of<float>(const Level& L) {
  return {L.wf, L.df, L.dinvf, L.ptcf};
}

// Workgroups of a column-dot launch: about four 16-byte loads per thread,
// at most kDotBlocks.
template <typename T>
inline int dot_blocks(int64_t m) {
  const int64_t vecs = ceil_div(m, 16 / (int64_t)sizeof(T));
  return (int)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, ceil_div(vecs, (int64_t)kBlock)));
}

inline double spmm_bytes(const Level& L, int K, int s, int vecs) {
  return 4.0 * (L.n + 1) + (double)L.nnz * (4 + s) + (double)L.n * s + (double)vecs * K * L.n * s;
}

template <typename T, int K>
struct Engine {
  lg_hierarchy* h;
  hipStream_t st;

  // vecs: n x K vectors streamed (reads and writes); the smoother modes also read D^-1
  template <int MODE>
  void lap(const Level& L, const T* x, T* y, const T* b, T* p, T c1, T c2, T c0, const char* fam,
           int vecs, const int32_t* agg = nullptr) {
    Vals<T> v = vals_of<T>(L);
    double bytes =
        spmm_bytes(L, K, (int)sizeof(T), vecs) + (MODE >= LAP_CHEB ? (double)sizeof(T) * L.n : 0);
    if (MODE == LAP_CHEB_FIRST_CC)  // the coarse vector replaces x, plus the map
      bytes += ((double)L.nc - (double)L.n) * K * sizeof(T) + 4.0 * L.n;
    if constexpr (use_col_split<T, K>()) {
      run_rows_col(L.sched, L.rp,
                   LapColOp<T, K, MODE>{L.col, v.w, v.d, v.dinv, x, y, b, p, c1, c2, c0, agg}, st,
                   fam, bytes);
    } else {
      const LapOp<T, K, MODE> op{L.col, v.w, v.d, v.dinv, x, y, b, p, c1, c2, c0};
      if constexpr (K == 1) {
        if (L.sched.merge) {
          run_merge(L.sched, L.rp, op, st, fam, bytes);
          return;
        }
      }
      run_rows(L.sched, L.rp, op, st, fam, bytes);
    }
  }

  template <int ND>
  void dots(const T* a0, const T* b0, const T* a1, const T* b1, int64_t n, double* out0,
            double* out1) {
    const int64_t m = n * K;
    const int nb = dot_blocks<T>(m);
    hipLaunchKernelGGL((k_dots<T, K, ND>), dim3(nb), dim3(kBlock), 0, st, a0, b0, a1, b1, m, h->red);
    hipLaunchKernelGGL((k_dots_final<K, ND>), dim3(ND * K), dim3(kBlock), 0, st, (const double*)h->red, nb,
                       out0, out1, (double*)nullptr);
  }

  // Algorithm 1 from level l with zero initial guess; returns the buffer holding x.
  T* level(int l, const T* b) {
    Level& L = h->lev[l];
    const int64_t n = L.n;
    T* x = (T*)L.vx;
    if (L.type == LG_LEVEL_COARSEST) {
      ProfScope ps("coarse", st, 8.0 * n * n + 2.0 * K * n * sizeof(T));
      hipLaunchKernelGGL((k_coarse<T, K>), dim3(nblk(n, kBlock / 64)), dim3(kBlock), 0, st, h->Lplus,
                         b, x, n);
      return x;
    }
    Level& C = h->lev[l + 1];
    Vals<T> v = vals_of<T>(L);
    if (L.type == LG_LEVEL_ELIM) {
      T* bc = (T*)C.vb;
      {
        ProfScope ps("restrict", st, 0.0);
        if constexpr (use_col_split<T, K>())
          run_rows_col(L.ptsched, L.ptrp, PtColOp<T, K>{L.ptf, v.ptc, L.cvert, b, bc}, st);
        else
          run_rows(L.ptsched, L.ptrp, PtOp<T, K>{L.ptf, v.ptc, L.cvert, b, bc}, st);
      }
      const T* xc = level(l + 1, bc);  // elimination interpolates exactly: no Krylov step here
      ProfScope ps("prolong", st, 0.0);
      hipLaunchKernelGGL((k_elim_prolong<T, K>), dim3(vec_blocks<T, K>(n)), dim3(kBlock), 0, st, L.rp, L.col,
                         v.w, v.dinv, L.cidx, xc, b, x, n);
      return x;
    }
    // aggregation level
    T* x2 = (T*)L.vx2;
    T* r = (T*)L.vr;
    const lg_setup_opts& o = h->opts;
    const int deg = o.cheb_degree;
    const double lo = o.cheb_lo * L.lmax, hi = o.cheb_hi * L.lmax;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
    const double sigma = theta / delta;
    const bool smooth = deg >= 1 && L.lmax > 0.0;
    T* cur = x;
    T* nxt = x2;
    if (smooth && deg == 1) {
      hipLaunchKernelGGL((k_cheb_zero<T, K>), dim3(vec_blocks<T, K>(n)), dim3(kBlock), 0, st, b,
                         v.dinv, cur, n, (T)(1.0 / theta));
    } else if (smooth) {
      double rho = 1.0 / sigma;
      double rho1 = 1.0 / (2.0 * sigma - rho);
      bool one_pass = false;
      if constexpr (use_col_split<T, K>()) one_pass = !L.cheb0_split;
      if (one_pass) {
        // steps 0 and 1 in one pass; step 0's iterate is stored only if more follow
        lap<LAP_CHEB_ZERO>(L, b, cur, b, deg > 2 ? nxt : nullptr, (T)(rho1 * rho),
                           (T)(2.0 * rho1 / delta), (T)(1.0 / theta), "cheb0", deg > 2 ? 3 : 2);
      } else {
        // store step 0's iterate, then step 1 without a D^-1 gather per entry
        hipLaunchKernelGGL((k_cheb_zero<T, K>), dim3(vec_blocks<T, K>(n)), dim3(kBlock), 0, st, b,
                           v.dinv, nxt, n, (T)(1.0 / theta));
        lap<LAP_CHEB_X1>(L, nxt, cur, b, nullptr, (T)(rho1 * rho), (T)(2.0 * rho1 / delta), T(0),
                         "cheb0", 3);
      }
      rho = rho1;
      for (int s = 2; s < deg; s++) {
        rho1 = 1.0 / (2.0 * sigma - rho);
        lap<LAP_CHEB>(L, cur, nxt, b, nullptr, (T)(rho1 * rho), (T)(2.0 * rho1 / delta), T(0),
                      "cheb", 4);
        std::swap(cur, nxt);
        rho = rho1;
      }
    } else {
      hipLaunchKernelGGL((k_fill<T>), dim3(nblk(n * K)), dim3(kBlock), 0, st, cur, n * K, T(0));
    }
    lap<LAP_RESID>(L, cur, r, b, nullptr, T(0), T(0), T(0), "resid", 3);
    T* bc = (T*)C.vb;
    {
      ProfScope ps("restrict", st, 4.0 * (L.nc + 1) + 4.0 * n + 2.0 * K * n * sizeof(T));
      if constexpr (use_col_split<T, K>())
        run_rows_col(L.msched, L.mptr, GatherSumColOp<T, K>{L.mem, r, bc}, st);
      else
        run_rows(L.msched, L.mptr, GatherSumOp<T, K>{L.mem, r, bc}, st);
    }
    const T* xc = (o.cycle == LG_CYCLE_K && C.type != LG_LEVEL_COARSEST) ? fcg2(l + 1, bc)
                                                                          : level(l + 1, bc);
    bool fused_cc = false;
    if constexpr (use_col_split<T, K>()) fused_cc = smooth;
    if (fused_cc) {
      if constexpr (use_col_split<T, K>()) {
        // x += P x_c in place and the first post-smoothing step in one pass,
        // its residual r - L P x_c gathered from the coarse vector, which is a
        // fraction of the fine iterate's size and stays in cache
        lap<LAP_CHEB_FIRST_CC>(L, xc, cur, r, nxt, T(0), (T)(1.0 / theta), T(0), "cheb1", 4, L.agg);
        std::swap(cur, nxt);
      }
    } else {
      {
        ProfScope ps("prolong", st, 4.0 * n + 3.0 * K * n * sizeof(T));
        hipLaunchKernelGGL((k_agg_prolong<T, K>), dim3(vec_blocks<T, K>(n)), dim3(kBlock), 0, st,
                           cur, xc, L.agg, nxt, n);
        std::swap(cur, nxt);
      }
      // nxt keeps the previous iterate, which each further step overwrites
      if (smooth) {
        lap<LAP_CHEB_FIRST>(L, cur, nxt, b, nullptr, T(0), (T)(1.0 / theta), T(0), "cheb1", 3);
        std::swap(cur, nxt);
      }
    }
    if (smooth) {
      double rho = 1.0 / sigma;
      for (int s = 1; s < deg; s++) {
        const double rho1 = 1.0 / (2.0 * sigma - rho);
        lap<LAP_CHEB>(L, cur, nxt, b, nullptr, (T)(rho1 * rho), (T)(2.0 * rho1 / delta), T(0),
                      "cheb", 4);
        std::swap(cur, nxt);
        rho = rho1;
      }
    }
    return cur;
  }

  // Two flexible-CG iterations on L_l x = b preconditioned by the cycle from
  // level l (the coarse solve of the K-cycle, Section 3.7).
  T* fcg2(int l, const T* b) {
    Level& C = h->lev[l];
    const int64_t n = C.n;
    T* r = (T*)C.kr;
    T* p1 = (T*)C.kp1;
    T* q1 = (T*)C.kq1;
    T* q2 = (T*)C.kz;
    T* x = (T*)C.kx;
    double* ks = C.kscal;
    const unsigned g = nblk(n * K);
    hipLaunchKernelGGL((k_copy<T>), dim3(g), dim3(kBlock), 0, st, r, b, n * K);
    const T* z = level(l, r);
    hipLaunchKernelGGL((k_copy<T>), dim3(g), dim3(kBlock), 0, st, p1, z, n * K);
    lap<LAP_SPMV>(C, p1, q1, nullptr, nullptr, T(0), T(0), T(0), "spmm_inner", 2);
    dots<2>(p1, q1, p1, r, n, ks + 0 * K, ks + 1 * K);
    hipLaunchKernelGGL((k_fcg_alpha1<K>), dim3(1), dim3(64), 0, st, ks);
    hipLaunchKernelGGL((k_fcg_step1<T, K>), dim3(g), dim3(kBlock), 0, st, x, r, p1, q1,
                       (const double*)ks, n);
    T* z2 = level(l, r);
    dots<1>(z2, q1, nullptr, nullptr, n, ks + 3 * K, nullptr);
    hipLaunchKernelGGL((k_fcg_p2<T, K>), dim3(g), dim3(kBlock), 0, st, z2, p1, (const double*)ks, n);
    lap<LAP_SPMV>(C, z2, q2, nullptr, nullptr, T(0), T(0), T(0), "spmm_inner", 2);
    dots<2>(z2, q2, z2, r, n, ks + 4 * K, ks + 5 * K);
    hipLaunchKernelGGL((k_fcg_final<T, K>), dim3(g), dim3(kBlock), 0, st, x, z2, (const double*)ks,
                       n);
    LG_LAUNCH_CHECK();
    return x;
  }

  // One cycle on the fp64 residual r: returns M r in precision T (the
  // finest level's output buffer).  In the mixed form the cycle reads its
  // fp32 copy of r from h->cyc_in, refreshed here unless r_ready says the
  // caller has written it already.
  const T* precond(const double* r, bool r_ready) {
    const int64_t m = h->lev[0].n * K;
    const T* in;
    if (sizeof(T) == sizeof(double)) {
      in = (const T*)r;
    } else {
      if (!r_ready)
        hipLaunchKernelGGL((k_convert<double, T>), dim3(nblk(m)), dim3(kBlock), 0, st, r,
                           (T*)h->cyc_in, m);
      in = (const T*)h->cyc_in;
    }
    return cycle(in);
  }

  // One cycle from the finest level.  After a first eager application on
  // this input buffer, the cycle is captured once (on the hierarchy's own
  // capture stream) and later applications replay it with one launch; every
  // kernel of the cycle reads and writes fixed buffers, so the replay is the
  // same computation.  Kernel timing, or the graphs option off, keeps it eager.
  const T* cycle(const T* in) {
    constexpr int slot = K == 1 ? 0 : K == 2 ? 1 : K == 4 ? 2 : K == 8 ? 3 : K == 16 ? 4 : 5;
    lg_hierarchy::CycleGraph& cg = h->cycle_graph[slot];
    if (!h->opts.graphs || prof_active()) return level(0, in);
    if (cg.exec && cg.in == (const void*)in) {
      LG_HIP(hipGraphLaunch(cg.exec, st));
      return (const T*)cg.out;
    }
    if (cg.exec || cg.uses++ == 0 || h->no_capture) return level(0, in);
    if (!h->capture_stream) LG_HIP(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    LG_HIP(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
    Engine<T, K> cap{h, h->capture_stream};
    T* out = nullptr;
    try {
      out = cap.level(0, in);
    } catch (...) {
      (void)hipStreamEndCapture(h->capture_stream, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    LG_HIP(hipStreamEndCapture(h->capture_stream, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    LG_HIP(e);
    cg.exec = exec;
    cg.in = in;
    cg.out = out;
    LG_HIP(hipGraphLaunch(exec, st));
    return out;
  }
};

// fp64 Laplacian product on level l for K columns (outer Krylov method)
// fp64 Laplacian product on level l for K columns (outer Krylov method):
// y = L x, or y = b - L x when b is set.  TAG 1 marks the lg_spmv entry
// point's own kernel instances.
template <int K, int TAG = 0>
void lap64(lg_hierarchy* h, int l, const double* x, double* y, const double* b, hipStream_t st,
           const char* fam) {
  const Level& L = h->lev[l];
  const double bytes = spmm_bytes(L, K, 8, b ? 3 : 2);
  if constexpr (use_col_split<double, K>()) {
    if (b)
      run_rows_col(L.sched, L.rp,
                   LapColOp<double, K, LAP_RESID, TAG>{L.col, L.w, L.d, L.dinv, x, y, b, nullptr,
                                                       0.0, 0.0, 0.0},
                   st, fam, bytes);
    else
      run_rows_col(L.sched, L.rp,
                   LapColOp<double, K, LAP_SPMV, TAG>{L.col, L.w, L.d, L.dinv, x, y, nullptr,
                                                      nullptr, 0.0, 0.0, 0.0},
                   st, fam, bytes);
  } else {
    auto go = [&](const auto& op) {
      if constexpr (K == 1) {
        if (L.sched.merge) {
          run_merge(L.sched, L.rp, op, st, fam, bytes);
          return;
        }
      }
      run_rows(L.sched, L.rp, op, st, fam, bytes);
    };
    if (b)
      go(LapOp<double, K, LAP_RESID, TAG>{L.col, L.w, L.d, L.dinv, x, y, b, nullptr, 0.0, 0.0, 0.0});
    else
      go(LapOp<double, K, LAP_SPMV, TAG>{L.col, L.w, L.d, L.dinv, x, y, nullptr, nullptr, 0.0, 0.0,
                                         0.0});
  }
}

// q = L_0 p and p . q per column into out (K columns, the column-split
// widths): the product's epilogue forms the terms, each workgroup sums its
// share, and one fixed tree adds the partials.  false: not available (the
// caller takes the separate product and dot).
template <int K>
bool lap64_dot(lg_hierarchy* h, const double* p, double* q, double* out, hipStream_t st) {
  if constexpr (use_col_split<double, K>()) {
    const Level& L = h->lev[0];
    using Op = LapColOp<double, K, LAP_SPMV, 2>;
    if (dot_partials(L.sched, col_resident<Op>(L.sched)) > h->dotp_rows) return false;
    const int64_t nb = run_rows_col(L.sched, L.rp,
                                    Op{L.col, L.w, L.d, L.dinv, p, q, nullptr, nullptr, 0.0, 0.0, 0.0},
                                    st, "spmv", spmm_bytes(L, K, 8, 2), h->dotp);
    hipLaunchKernelGGL((k_dots_final<K, 1>), dim3(K), dim3(kBlock), 0, st, (const double*)h->dotp,
                       (int)(nb + L.sched.nsplit), out, (double*)nullptr, (double*)nullptr);
    LG_LAUNCH_CHECK();
    return true;
  } else {
    (void)h, (void)p, (void)q, (void)out, (void)st;
    return false;
  }
}

// Work of one cycle in finest-residual units, following the same recursion
// as Engine::level / fcg2 (Section 2.3.1: operator nonzeros per application).
static double cycle_work(const lg_hierarchy* h, int l) {
  const Level& L = h->lev[l];
  const double unit = (double)(h->lev[0].n + h->lev[0].nnz);
  const double nnzL = (double)(L.n + L.nnz);
  if (L.type == LG_LEVEL_COARSEST) return (double)L.n * (double)L.n / unit;
  if (L.type == LG_LEVEL_ELIM)
    return (2.0 * L.nnzP + (double)L.nF) / unit + cycle_work(h, l + 1);
  const int deg = h->opts.cheb_degree;
  double w = ((2.0 * deg) * nnzL + 2.0 * L.n) / unit;
  const Level& C = h->lev[l + 1];
  if (h->opts.cycle == LG_CYCLE_K && C.type != LG_LEVEL_COARSEST)
    w += 2.0 * (C.n + C.nnz) / unit + 2.0 * cycle_work(h, l + 1);
  else
    w += cycle_work(h, l + 1);
  return w;
}

// CG preconditioned by the cycle (flexible CG with the K-cycle) on K columns
// at once.  Plain mode: the k columns of B, X filled at the end.  Slot mode
// (feed set, B and X unused): columns enter from the feed and leave to it at
// iteration boundaries, each with its own iteration cap.
template <typename T, int K>
lg_status pcg(lg_hierarchy* h, const double* B, double* X, int k, double rtol, int max_iter,
              hipStream_t st, lg_rhs_info* info, SlotFeed* feed = nullptr) {
  Engine<T, K> eng{h, st};
  const Level& L0 = h->lev[0];
  const int64_t n = L0.n;
  const int64_t m = n * K;
  const unsigned g = nblk(m);
  const unsigned g2 = nblk(ceil_div(m, (int64_t)2));
  const bool flex = h->opts.cycle == LG_CYCLE_K;
  const bool mixed = sizeof(T) != sizeof(double);
  double* sc = h->scal;
  double* hs = h->host_scal;
  auto sl = [&](int slot) { return sc + slot * K; };
  auto read_scal = [&]() {
    read_dev(hs, sc, sizeof(double) * S_COUNT * K, st);
  };
  auto write_slot = [&](int slot, const std::vector<double>& v) {
    for (int c = 0; c < K; c++) hs[slot * K + c] = v[c];
    LG_HIP(hipMemcpyAsync(sc + slot * K, hs + slot * K, sizeof(double) * K, hipMemcpyHostToDevice,
                          st));
  };
  const int nb = dot_blocks<double>(m);
  auto final1 = [&](int slot) {
    hipLaunchKernelGGL((k_dots_final<K, 1>), dim3(K), dim3(kBlock), 0, st, (const double*)h->red, nb,
                       sl(slot), (double*)nullptr, (double*)nullptr);
  };
  auto project64 = [&](double* v) {
    hipLaunchKernelGGL((k_dots<double, K, 1>), dim3(nb), dim3(kBlock), 0, st, v,
                       (const double*)nullptr, (const double*)nullptr, (const double*)nullptr, m,
                       h->red);
    final1(S_TMP);
    hipLaunchKernelGGL((k_sub_mean<K>), dim3(g), dim3(kBlock), 0, st, v, (const double*)sl(S_TMP), n);
  };
  auto dot64 = [&](const double* a, const double* b, int slot) {
    hipLaunchKernelGGL((k_dots<double, K, 1>), dim3(nb), dim3(kBlock), 0, st, a, b,
                       (const double*)nullptr, (const double*)nullptr, m, h->red);
    final1(slot);
  };
  auto dot64x2 = [&](const double* a0, const double* b0, const double* a1, const double* b1,
                     int s0, int s1) {
    hipLaunchKernelGGL((k_dots<double, K, 2>), dim3(nb), dim3(kBlock), 0, st, a0, b0, a1, b1, m,
                       h->red);
    hipLaunchKernelGGL((k_dots_final<K, 2>), dim3(2 * K), dim3(kBlock), 0, st, (const double*)h->red,
                       nb, sl(s0), sl(s1), (double*)nullptr);
  };
  // z = M r, projected to mean zero, enters p = z + beta p without being stored
  const int nbz = dot_blocks<T>(m);
  // The solution update x += alpha p of an iteration is deferred (see
  // k_update_r): pending until the next direction update or a flush.
  bool x_pending = false;
  auto flush_x = [&]() {
    if (!x_pending) return;
    hipLaunchKernelGGL((k_update_x<K>), dim3(g), dim3(kBlock), 0, st, h->px, (const double*)h->pp,
                       (const double*)sc, m);
    x_pending = false;
  };
  auto new_direction = [&](const T* z, bool first, const double* flags) {
    hipLaunchKernelGGL((k_zstats<T, K>), dim3(nbz), dim3(kBlock), 0, st, z,
                       (const double*)(flex && !first ? h->pq : h->pr), m, h->red);
    hipLaunchKernelGGL((k_dots_final<K, 3>), dim3(3 * K), dim3(kBlock), 0, st, (const double*)h->red,
                       nbz, sl(S_ZSUM), sl(S_ZY), sl(S_YSUM));
    hipLaunchKernelGGL((k_beta_z<K>), dim3(1), dim3(64), 0, st, sc, 1.0 / (double)n, flex ? 1 : 0,
                       first ? 1 : 0);
    hipLaunchKernelGGL((k_xpby_z<T, K>), dim3(g2), dim3(kBlock), 0, st, h->pp, z, (const double*)sc,
                       flags, first ? 1 : 0, m, x_pending ? h->px : (double*)nullptr);
    x_pending = false;
  };

  const double cw = cycle_work(h, 0);
  std::vector<double> bn(K, 0.0), relres(K, 0.0), work(K, 0.0), active(K, 0.0), zero(K, 0.0);
  std::vector<int> iters(K, 0);
  std::vector<int> converged(K, 0);
  std::vector<SlotFeed::Col> dst(K);  // slot mode: where each slot's solution goes

  auto fill_flags = [&](const std::vector<SlotFeed::Col>& in) {
    std::vector<double> f(K, 0.0);
    for (const SlotFeed::Col& c : in) f[c.slot] = 1.0;
    return f;
  };
  // slot mode: load the offered columns into free slots (b projected to mean
  // zero, x = 0, t = b); returns the refill flags (all zero if none)
  auto load_cols = [&](const std::vector<int>& free_slots) {
    std::vector<SlotFeed::Col> in;
    if (!free_slots.empty()) feed->refill(free_slots, in);
    std::vector<double> f = fill_flags(in);
    if (in.empty()) return f;
    for (const SlotFeed::Col& c : in) {
      dst[c.slot] = c;
      hipLaunchKernelGGL((k_load_col<K>), dim3(nblk(n)), dim3(kBlock), 0, st, h->pb, c.slot, c.B,
                         c.ldb, n, (const int32_t*)L0.perm);
    }
    write_slot(S_FILL, f);
    hipLaunchKernelGGL((k_dots<double, K, 1>), dim3(nb), dim3(kBlock), 0, st, h->pb,
                       (const double*)nullptr, (const double*)nullptr, (const double*)nullptr, m,
                       h->red);
    final1(S_TMP);
    hipLaunchKernelGGL((k_sub_mean_flagged<K>), dim3(g), dim3(kBlock), 0, st, h->pb,
                       (const double*)sl(S_TMP), (const double*)sl(S_FILL), n);
    dot64(h->pb, h->pb, S_BN);
    hipLaunchKernelGGL((k_refill_cols<K>), dim3(g), dim3(kBlock), 0, st, h->px, h->pt,
                       (const double*)h->pb, (const double*)sl(S_FILL), m);
    read_scal();
    for (const SlotFeed::Col& c : in) {
      const int j = c.slot;
      bn[j] = std::sqrt(hs[S_BN * K + j]);
      iters[j] = 0;
      work[j] = 0.0;
      relres[j] = 0.0;
      converged[j] = 0;
      active[j] = bn[j] > 0.0 ? 1.0 : 0.0;
    }
    return f;
  };
  // slot mode: the finished columns' solutions (projected) to their destinations
  auto store_cols = [&](const std::vector<int>& done) {
    if (done.empty()) return;
    hipLaunchKernelGGL((k_dots<double, K, 1>), dim3(nb), dim3(kBlock), 0, st, h->px,
                       (const double*)nullptr, (const double*)nullptr, (const double*)nullptr, m,
                       h->red);
    final1(S_TMP);
    for (int c : done)
      hipLaunchKernelGGL((k_store_col<K>), dim3(nblk(n)), dim3(kBlock), 0, st, (const double*)h->px,
                         c, (const double*)sl(S_TMP), n, dst[c].X, dst[c].ldx,
                         (const int32_t*)L0.iperm);
    LG_LAUNCH_CHECK();
    LG_HIP(hipStreamSynchronize(st));
    for (int c : done) {
      lg_rhs_info ci{};
      ci.iters = iters[c];
      ci.rel_residual = relres[c];
      ci.work_units = work[c];
      ci.wda = (relres[c] > 0.0 && relres[c] < 1.0) ? -work[c] / std::log10(relres[c]) : 0.0;
      feed->finished(c, ci);
    }
  };
  auto any_active = [&]() {
    for (int c = 0; c < K; c++)
      if (active[c] > 0.0) return true;
    return false;
  };

  hipLaunchKernelGGL(k_fill<double>, dim3(nblk(S_COUNT * K)), dim3(kBlock), 0, st, sc,
                     (int64_t)S_COUNT * K, 0.0);
  if (feed) {  // empty slots hold zero vectors
    hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(kBlock), 0, st, h->pb, m, 0.0);
    hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(kBlock), 0, st, h->px, m, 0.0);
    hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(kBlock), 0, st, h->pt, m, 0.0);
    std::vector<int> all(K);
    for (int c = 0; c < K; c++) all[c] = c;
    load_cols(all);
    // empty slots (zero right-hand side) finish at once
    std::vector<int> done;
    for (int c = 0; c < K; c++)
      if (dst[c].X && active[c] == 0.0) done.push_back(c);
    store_cols(done);
    for (int c : done) dst[c] = SlotFeed::Col{};
    LG_HIP(hipMemcpyAsync(h->pr, h->pt, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
  } else {
    hipLaunchKernelGGL(k_pad_in, dim3(g), dim3(kBlock), 0, st, B, k, h->pb, K, n,
                       (const int32_t*)L0.perm);
    project64(h->pb);
    dot64(h->pb, h->pb, S_BN);
    read_scal();
    for (int c = 0; c < K; c++) {
      bn[c] = std::sqrt(hs[S_BN * K + c]);
      active[c] = (c < k && bn[c] > 0.0) ? 1.0 : 0.0;
      converged[c] = active[c] == 0.0;
    }
    hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(kBlock), 0, st, h->px, m, 0.0);
    LG_HIP(hipMemcpyAsync(h->pr, h->pb, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
  }
  write_slot(S_ACTIVE, active);
  if (any_active()) {
    new_direction(eng.precond(h->pr, false), true, nullptr);
    for (int c = 0; c < K; c++) work[c] += active[c] > 0.0 ? cw : 0.0;
  }
  for (int it = 1; (feed || it <= max_iter) && any_active(); it++) {
    if (flex) {
      lap64<K>(h, 0, h->pp, h->pq, nullptr, st, "spmv");
      dot64x2(h->pp, h->pq, h->pp, h->pr, S_PQ, S_PR);
    } else if (!lap64_dot<K>(h, h->pp, h->pq, sl(S_PQ), st)) {
      lap64<K>(h, 0, h->pp, h->pq, nullptr, st, "spmv");
      dot64(h->pp, h->pq, S_PQ);
    }
    hipLaunchKernelGGL((k_alpha<K>), dim3(1), dim3(64), 0, st, sc, flex ? 1 : 0);
    {
      // reads r, q and writes r (fp64), plus r in the cycle's precision
      ProfScope ps("cg_update", st, 24.0 * m + (mixed ? (double)sizeof(T) * m : 0.0));
      hipLaunchKernelGGL((k_update_r<K, T>), dim3(nb), dim3(kBlock), 0, st, h->pr,
                         (const double*)h->pq, (const double*)sc, m,
                         mixed ? (T*)h->cyc_in : (T*)nullptr, h->red);
      x_pending = true;
    }
    final1(S_RR);
    read_scal();
    std::vector<int> newly, done;
    std::vector<int> capped(K, 0);
    for (int c = 0; c < K; c++) {
      if (active[c] == 0.0) continue;
      iters[c]++;
      work[c] += 1.0;
      if (hs[S_ACTIVE * K + c] == 0.0) {  // breakdown flagged on the device
        active[c] = 0.0;
        if (feed) {  // slot mode: the column finishes with its true residual
          capped[c] = 1;
          newly.push_back(c);
        }
        continue;
      }
      capped[c] = feed && iters[c] >= max_iter;
      if (std::sqrt(hs[S_RR * K + c]) / bn[c] <= rtol || capped[c]) newly.push_back(c);
    }
    bool restart = false;
    std::vector<double> rflag(K, 0.0);
    if (!newly.empty()) {
      flush_x();
      lap64<K>(h, 0, h->px, h->pt, h->pb, st, "resid64");
      dot64(h->pt, h->pt, S_TR);
      read_scal();
      for (int c : newly) {
        work[c] += 1.0;
        const double rel = std::sqrt(hs[S_TR * K + c]) / bn[c];
        if (rel <= rtol || capped[c]) {
          active[c] = 0.0;
          converged[c] = rel <= rtol;
          relres[c] = rel;
          if (feed) done.push_back(c);
        } else {
          restart = true;
          rflag[c] = 1.0;
        }
      }
      write_slot(S_ACTIVE, active);
      write_slot(S_TR, zero);
    }
    if (feed) {  // hand finished columns back, refill their slots
      flush_x();
      std::sort(done.begin(), done.end());
      store_cols(done);
      std::vector<int> free_slots;
      for (int c = 0; c < K; c++)
        if (active[c] == 0.0) free_slots.push_back(c);
      for (int c : done) dst[c] = SlotFeed::Col{};
      std::vector<double> f = load_cols(free_slots);
      bool any_fill = false;
      for (int c = 0; c < K; c++)
        if (f[c] > 0.0 && active[c] > 0.0) {
          rflag[c] = 1.0;
          any_fill = true;
        } else if (f[c] > 0.0) {  // a zero right-hand side: done at once
          store_cols({c});
          dst[c] = SlotFeed::Col{};
        }
      if (any_fill) {
        restart = true;
        write_slot(S_ACTIVE, active);
      }
    }
    if (!any_active()) break;
    if (restart) {  // those columns continue from the true residual with a fresh direction
      write_slot(S_RESTART, rflag);
      hipLaunchKernelGGL((k_copy_flagged<K>), dim3(g), dim3(kBlock), 0, st, h->pr,
                         (const double*)h->pt, (const double*)sl(S_RESTART), m);
    }
    const T* z = eng.precond(h->pr, !restart);
    for (int c = 0; c < K; c++) work[c] += active[c] > 0.0 ? cw : 0.0;
    new_direction(z, false, restart ? (const double*)sl(S_RESTART) : nullptr);
    LG_LAUNCH_CHECK();
  }
  flush_x();
  if (feed) {
    std::vector<int> left;  // only after a breakdown ended the loop early
    for (int c = 0; c < K; c++)
      if (dst[c].X) left.push_back(c);
    if (!left.empty()) {
      lap64<K>(h, 0, h->px, h->pt, h->pb, st, "resid64");
      dot64(h->pt, h->pt, S_TR);
      read_scal();
      for (int c : left) relres[c] = bn[c] > 0.0 ? std::sqrt(hs[S_TR * K + c]) / bn[c] : 0.0;
      store_cols(left);
    }
    return LG_OK;
  }
  lg_status status = LG_OK;
  bool need_true = false;
  for (int c = 0; c < k; c++)
    if (!converged[c]) need_true = true;
  if (need_true) {
    lap64<K>(h, 0, h->px, h->pt, h->pb, st, "resid64");
    dot64(h->pt, h->pt, S_TR);
    read_scal();
    for (int c = 0; c < k; c++)
      if (!converged[c]) {
        relres[c] = bn[c] > 0.0 ? std::sqrt(hs[S_TR * K + c]) / bn[c] : 0.0;
        status = LG_E_NOT_CONVERGED;
      }
  }
  project64(h->px);
  hipLaunchKernelGGL(k_pad_out, dim3(nblk(n * k)), dim3(kBlock), 0, st, (const double*)h->px, K, X,
                     k, n, (const int32_t*)L0.iperm);
  LG_LAUNCH_CHECK();
  LG_HIP(hipStreamSynchronize(st));
  if (info) {
    for (int c = 0; c < k; c++) {
      info[c].iters = iters[c];
      info[c].rel_residual = relres[c];
      info[c].work_units = work[c];
      info[c].wda = (relres[c] > 0.0 && relres[c] < 1.0) ? -work[c] / std::log10(relres[c]) : 0.0;
    }
  }
  return status;
}

template <typename T, int K>
void cycle_once(lg_hierarchy* h, const double* B, double* X, int k, hipStream_t st) {
  Engine<T, K> eng{h, st};
  const int64_t n = h->lev[0].n;
  const Level& L0 = h->lev[0];
  hipLaunchKernelGGL(k_pad_in, dim3(nblk(n * K)), dim3(kBlock), 0, st, B, k, h->pb, K, n,
                     (const int32_t*)L0.perm);
  const T* z = eng.precond(h->pb, false);
  const double* z64 = (const double*)z;
  if (sizeof(T) != sizeof(double)) {
    hipLaunchKernelGGL((k_convert<T, double>), dim3(nblk(n * K)), dim3(kBlock), 0, st, z, h->pz,
                       n * K);
    z64 = h->pz;
  }
  hipLaunchKernelGGL(k_pad_out, dim3(nblk(n * k)), dim3(kBlock), 0, st, z64, K, X, k, n,
                     (const int32_t*)L0.iperm);
  LG_LAUNCH_CHECK();
}

// A call with k columns runs at width next_pow2(k) (at most the workspace's
// h->K): narrow calls stream narrow vectors.
static int width(int k) {
  int K = 1;
  while (K < k) K <<= 1;
  return K;
}

template <typename T>
static lg_status solve_k(lg_hierarchy* h, const double* B, double* X, int k, double rtol,
                         int max_iter, hipStream_t st, lg_rhs_info* info) {
  switch (width(k)) {
    case 1: return pcg<T, 1>(h, B, X, k, rtol, max_iter, st, info);
    case 2: return pcg<T, 2>(h, B, X, k, rtol, max_iter, st, info);
    case 4: return pcg<T, 4>(h, B, X, k, rtol, max_iter, st, info);
    case 8: return pcg<T, 8>(h, B, X, k, rtol, max_iter, st, info);
    case 16: return pcg<T, 16>(h, B, X, k, rtol, max_iter, st, info);
    default: return pcg<T, 32>(h, B, X, k, rtol, max_iter, st, info);
  }
}

template <typename T>
static lg_status slots_k(lg_hierarchy* h, int K, double rtol, int max_iter, hipStream_t st,
                         SlotFeed* feed) {
  switch (K) {
    case 1: return pcg<T, 1>(h, nullptr, nullptr, 0, rtol, max_iter, st, nullptr, feed);
    case 2: return pcg<T, 2>(h, nullptr, nullptr, 0, rtol, max_iter, st, nullptr, feed);
    case 4: return pcg<T, 4>(h, nullptr, nullptr, 0, rtol, max_iter, st, nullptr, feed);
    case 8: return pcg<T, 8>(h, nullptr, nullptr, 0, rtol, max_iter, st, nullptr, feed);
    case 16: return pcg<T, 16>(h, nullptr, nullptr, 0, rtol, max_iter, st, nullptr, feed);
    default: return pcg<T, 32>(h, nullptr, nullptr, 0, rtol, max_iter, st, nullptr, feed);
  }
}

lg_status solve_slots(lg_hierarchy* h, int K, double rtol, int max_iter, hipStream_t st,
                      SlotFeed* feed) {
  if (K < 1 || K > h->K || (K & (K - 1)) || !feed) fail(LG_E_ARG, "solve_slots: bad width");
  if (h->opts.precision == LG_MIXED) return slots_k<float>(h, K, rtol, max_iter, st, feed);
  return slots_k<double>(h, K, rtol, max_iter, st, feed);
}

lg_status solve_dispatch(lg_hierarchy* h, const double* B, double* X, int k, double rtol,
                         int max_iter, hipStream_t st, lg_rhs_info* info) {
  if (h->opts.precision == LG_MIXED) return solve_k<float>(h, B, X, k, rtol, max_iter, st, info);
  return solve_k<double>(h, B, X, k, rtol, max_iter, st, info);
}

template <typename T>
static void cycle_k(lg_hierarchy* h, const double* B, double* X, int k, hipStream_t st) {
  switch (width(k)) {
    case 1: return cycle_once<T, 1>(h, B, X, k, st);
    case 2: return cycle_once<T, 2>(h, B, X, k, st);
    case 4: return cycle_once<T, 4>(h, B, X, k, st);
    case 8: return cycle_once<T, 8>(h, B, X, k, st);
    case 16: return cycle_once<T, 16>(h, B, X, k, st);
    default: return cycle_once<T, 32>(h, B, X, k, st);
  }
}

void cycle_dispatch(lg_hierarchy* h, const double* B, double* X, int k, hipStream_t st) {
  if (h->opts.precision == LG_MIXED) cycle_k<float>(h, B, X, k, st);
  else cycle_k<double>(h, B, X, k, st);
}

void spmv_dispatch(lg_hierarchy* h, int level, const double* X, double* Y, int k, hipStream_t st) {
  if (k < 1 || k > 32 || (k & (k - 1))) fail(LG_E_ARG, "lg_spmv: k must be 1, 2, 4, 8, 16 or 32");
  const Level& L = h->lev[level];
  if (L.perm) {
    // X and Y are in the setup's numbering: the product runs on copies in the
    // level's solve order (the solve workspace when it is large enough)
    const int64_t m = L.n * k;
    Arena::Mark mark = h->mem.mark();
    const bool fits = m <= h->lev[0].n * (int64_t)h->K;
    double* xs = fits ? h->pt : h->mem.get<double>(m);
    double* ys = fits ? h->pz : h->mem.get<double>(m);
    hipLaunchKernelGGL(k_pad_in, dim3(nblk(m)), dim3(kBlock), 0, st, X, k, xs, k, L.n,
                       (const int32_t*)L.perm);
    spmv_ordered(h, level, xs, ys, k, st);
    hipLaunchKernelGGL(k_pad_out, dim3(nblk(m)), dim3(kBlock), 0, st, (const double*)ys, k, Y, k, L.n,
                       (const int32_t*)L.iperm);
    LG_LAUNCH_CHECK();
    if (!fits) LG_HIP(hipStreamSynchronize(st));  // before the arena reuses the copies
    h->mem.rewind(mark);
    return;
  }
  spmv_ordered(h, level, X, Y, k, st);
}

// Y = L_level X with X and Y in the level's stored (solve) order.
void spmv_ordered(lg_hierarchy* h, int level, const double* X, double* Y, int k, hipStream_t st) {
  switch (k) {
    case 1: lap64<1, 1>(h, level, X, Y, nullptr, st, "spmm"); break;
    case 2: lap64<2, 1>(h, level, X, Y, nullptr, st, "spmm"); break;
    case 4: lap64<4, 1>(h, level, X, Y, nullptr, st, "spmm"); break;
    case 8: lap64<8, 1>(h, level, X, Y, nullptr, st, "spmm"); break;
    case 16: lap64<16, 1>(h, level, X, Y, nullptr, st, "spmm"); break;
    case 32: lap64<32, 1>(h, level, X, Y, nullptr, st, "spmm"); break;
    default: fail(LG_E_ARG, "lg_spmv: k must be 1, 2, 4, 8, 16 or 32");
  }
  LG_LAUNCH_CHECK();
}

// ----------------------------------------------------------- autotuner
// Lanes (one-column kernels) or lane groups (column-split kernels) per row of
// each degree class are 2^(c - shift); the best shift depends on the degree
// distribution, the width and the precision.  For every level whose product
// is large enough to matter, the tuner times that level's dominant product
// (the smoother-shaped residual at the cycle's precision on an aggregation
// level, the CG's fp64 product on the finest elimination level) for each
// candidate shift and keeps the fastest.  Choices are cached for the process
// by the level's structure, precision and width, so hierarchies of the same
// graph (and repeated setups) reuse them without timing again.
namespace {
constexpr int64_t kTuneMinNnz = (int64_t)1 << 18;
constexpr int kTuneShifts[] = {0, 1, 2};
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, int> g_tune;
}  // namespace

// Smoothing from a zero guess on a column-split aggregation level: time the
// one-pass form against the stored-iterate form (identical arithmetic) and
// keep the faster.  Cached under the level's key with a trailing -1.
template <typename T, int K>
static void tune_cheb0(Engine<T, K>& eng, Level& L, const std::vector<int64_t>& key, hipEvent_t e0,
                       hipEvent_t e1) {
  if constexpr (use_col_split<T, K>()) {
    const hipStream_t st = eng.st;
    T* b = (T*)L.vb;
    T* x = (T*)L.vx;
    T* x2 = (T*)L.vx2;
    const Vals<T> v = vals_of<T>(L);
    auto run = [&](bool split) {
      if (split) {
        hipLaunchKernelGGL((k_cheb_zero<T, K>), dim3(vec_blocks<T, K>(L.n)), dim3(kBlock), 0, st, b,
                           v.dinv, x2, L.n, T(1));
        eng.template lap<LAP_CHEB_X1>(L, x2, x, b, nullptr, T(0), T(1), T(0), "", 3);
      } else {
        eng.template lap<LAP_CHEB_ZERO>(L, b, x, b, nullptr, T(0), T(1), T(1), "", 2);
      }
    };
    float ms[2] = {0.0f, 0.0f};
    for (int split = 0; split < 2; split++) {
      run(split);  // warm-up
      LG_HIP(hipEventRecord(e0, st));
      for (int r = 0; r < 3; r++) run(split);
      LG_HIP(hipEventRecord(e1, st));
      LG_HIP(hipEventSynchronize(e1));
      LG_HIP(hipEventElapsedTime(&ms[split], e0, e1));
    }
    L.cheb0_split = ms[1] < ms[0];
    std::vector<int64_t> k2 = key;
    k2.push_back(-1);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[k2] = L.cheb0_split ? 1 : 0;
  }
}

template <typename T, int K>
static void autotune_k(lg_hierarchy* h, hipStream_t st) {
  Engine<T, K> eng{h, st};
  hipEvent_t e0, e1;
  LG_HIP(hipEventCreate(&e0));
  LG_HIP(hipEventCreate(&e1));
  const int nl = (int)h->lev.size();
  for (int l = 0; l + 1 < nl; l++) {
    Level& L = h->lev[l];
    const bool agg = L.type == LG_LEVEL_AGG;
    if (L.nnz < kTuneMinNnz || (!agg && l != 0)) continue;
    const bool col = agg ? use_col_split<T, K>() : use_col_split<double, K>();
    if (K == 1 && h->opts.merge_path == 2) continue;  // one-column products forced to the merge path
    int& shift = col ? L.sched.col_shift : L.sched.lane_shift;
    // candidates: the class-binned kernels at shifts 0, 1, 2, and (one column)
    // the merge path (cached as -1)
    const bool try_merge = K == 1 && h->opts.merge_path == 1;
    auto apply = [&](int v) {
      L.sched.merge = v < 0;
      if (v >= 0) shift = v;
    };
    const std::vector<int64_t> key{L.n, L.nnz, L.sched.min_deg, L.sched.max_deg, L.sched.nhub,
                                   L.sched.nsplit, agg ? (int64_t)sizeof(T) : 8, K, col ? 1 : 0,
                                   h->opts.merge_path, L.perm ? 1 : 0, h->opts.col_unroll};
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        apply((int)it->second);
        std::vector<int64_t> k2 = key;
        k2.push_back(-1);
        auto it2 = g_tune.find(k2);
        if (it2 != g_tune.end()) L.cheb0_split = it2->second != 0;
        continue;
      }
    }
    // the level's dominant product: the cycle's residual form, or on an
    // elimination level 0 the CG's product (with its fused p . q when the
    // CG takes that form)
    const bool cg_dot = h->opts.cycle != LG_CYCLE_K;
    auto product = [&]() {
      if (agg)
        eng.template lap<LAP_RESID>(L, (const T*)L.vx, (T*)L.vr, (const T*)L.vb, nullptr, T(0), T(0),
                                    T(0), "", 3);
      else if (!cg_dot || !lap64_dot<K>(h, h->pp, h->pq, h->scal + S_PQ * K, st))
        lap64<K>(h, 0, h->pp, h->pq, nullptr, st, "");
    };
    const int64_t m = L.n * K;
    if (agg) {
      hipLaunchKernelGGL((k_fill<T>), dim3(nblk(m)), dim3(kBlock), 0, st, (T*)L.vx, m, T(0));
      hipLaunchKernelGGL((k_fill<T>), dim3(nblk(m)), dim3(kBlock), 0, st, (T*)L.vb, m, T(0));
    } else {
      hipLaunchKernelGGL((k_fill<double>), dim3(nblk(m)), dim3(kBlock), 0, st, h->pp, m, 0.0);
    }
    std::vector<int> cands(std::begin(kTuneShifts), std::end(kTuneShifts));
    if (try_merge) cands.push_back(-1);
    int best = cands[0];
    float best_ms = 0.0f;
    for (size_t ci = 0; ci < cands.size(); ci++) {
      const int cand = cands[ci];
      apply(cand);
      product();  // warm-up at this candidate
      LG_HIP(hipEventRecord(e0, st));
      for (int r = 0; r < 5; r++) product();
      LG_HIP(hipEventRecord(e1, st));
      LG_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      LG_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ci == 0 || ms < best_ms) {
        best_ms = ms;
        best = cand;
      }
    }
    apply(best);
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      g_tune[key] = best;
    }
    if (agg && col) tune_cheb0(eng, L, key, e0, e1);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

template <typename T>
static void autotune_t(lg_hierarchy* h, hipStream_t st) {
  switch (h->K) {
    case 1: return autotune_k<T, 1>(h, st);
    case 2: return autotune_k<T, 2>(h, st);
    case 4: return autotune_k<T, 4>(h, st);
    case 8: return autotune_k<T, 8>(h, st);
    case 16: return autotune_k<T, 16>(h, st);
    default: return autotune_k<T, 32>(h, st);
  }
}

void autotune(lg_hierarchy* h, hipStream_t st) {
  if (h->opts.precision == LG_MIXED) autotune_t<float>(h, st);
  else autotune_t<double>(h, st);
}

// ----------------------------------------------------------- workspace
void alloc_solve_workspace(lg_hierarchy* h, hipStream_t st) {
  const int K = h->K;
  const size_t s = h->opts.precision == LG_MIXED ? sizeof(float) : sizeof(double);
  const int nl = (int)h->lev.size();
  for (int l = 0; l < nl; l++) {
    Level& L = h->lev[l];
    const size_t v = (size_t)L.n * K * s;
    L.vb = h->mem.alloc(v);
    L.vx = h->mem.alloc(v);
    if (L.type == LG_LEVEL_AGG) {
      L.vx2 = h->mem.alloc(v);
      L.vr = h->mem.alloc(v);
    }
    const bool fcg_target = h->opts.cycle == LG_CYCLE_K && l > 0 &&
                            h->lev[l - 1].type == LG_LEVEL_AGG && L.type != LG_LEVEL_COARSEST;
    if (fcg_target) {
      L.kr = h->mem.alloc(v);
      L.kp1 = h->mem.alloc(v);
      L.kq1 = h->mem.alloc(v);
      L.kz = h->mem.alloc(v);
      L.kx = h->mem.alloc(v);
      L.kscal = h->mem.get<double>(8 * K);
    }
  }
  const int64_t m = h->lev[0].n * K;
  h->pb = h->mem.get<double>(m);
  h->px = h->mem.get<double>(m);
  h->pr = h->mem.get<double>(m);
  h->pz = h->mem.get<double>(m);
  h->pp = h->mem.get<double>(m);
  h->pq = h->mem.get<double>(m);
  h->pt = h->mem.get<double>(m);
  if (h->opts.precision == LG_MIXED) h->cyc_in = h->mem.alloc((size_t)m * s);
  h->scal = h->mem.get<double>(S_COUNT * K);
  h->red = h->mem.get<double>((int64_t)kDotPartials * 3 * K);
  {
    // the fused p . q of the CG product on level 0 (column-split widths)
    int dev = 0, cus = 0;
    LG_HIP(hipGetDevice(&dev));
    LG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    h->dotp_rows = dot_partials(h->lev[0].sched, (int64_t)cus * 16);
    h->dotp = h->mem.get<double>(h->dotp_rows * K);
  }
  LG_HIP(hipHostMalloc((void**)&h->host_scal, sizeof(double) * S_COUNT * K, hipHostMallocDefault));
  (void)st;
}

}  // namespace lg
