// ops.h -- Laplacian products L X = D X - A X over k right-hand sides with
// fused epilogues (residual, Chebyshev step), plus small vector kernels.
#pragma once

#include "common.h"

namespace lg {

template <typename T, int K>
struct VecAcc {
  T v[K];
};

enum {
  LAP_SPMV = 0, LAP_RESID = 1, LAP_CHEB = 2, LAP_CHEB_FIRST = 3, LAP_CHEB_ZERO = 4, LAP_CHEB_X1 = 5,
  LAP_CHEB_FIRST_CC = 6
};

// Row i: s = sum_j w_ij x_j (k columns), (L x)_i = d_i x_i - s.  The Chebyshev
// modes use the three-term recurrence on iterates (Section 3.6 smoother):
//  LAP_SPMV:       y = L x
//  LAP_RESID:      y = b - L x
//  LAP_CHEB:       y = x + c1 (x - y) + c2 dinv (b - L x)   (y holds the previous
//                  iterate on entry and is overwritten in place, row by row)
//  LAP_CHEB_FIRST: y = x + c2 dinv (b - L x)
//  LAP_CHEB_ZERO:  the first two steps from a zero guess in one pass: with
//                  x1 = c0 dinv b (never stored unless p is set, then p = x1),
//                  y = x1 + c1 x1 + c2 dinv (b - L x1); x must point at b.
//  LAP_CHEB_X1:    the second step from a zero guess with x1 stored in x:
//                  y = x + c1 x + c2 dinv (b - L x).  (CHEB_ZERO gathers dinv
//                  with every neighbour, which pays off only for wide rows.)
//  LAP_CHEB_FIRST_CC (column-split form only): the coarse correction and the
//                  first post-smoothing step in one pass.  On entry y holds the
//                  pre-smoothed iterate x, b its residual r = b - L x, and x
//                  points at the coarse solution x_c with agg the aggregate
//                  map; with x' = x + P x_c (written back to y) the step is
//                  p = x' + c2 dinv (r - L P x_c), which equals
//                  x' + c2 dinv (b - L x') in exact arithmetic.  Row i's gathers
//                  read x_c[agg_j], a vector the size of the coarse level.
// TAG only separates kernel instances (lg_spmv's own launches from the
// solver's) so that profiles attribute time per call site.
template <typename T, int K, int MODE, int TAG = 0>
struct LapOp {
  using Acc = VecAcc<T, K>;
  static constexpr int kUnroll = LG_LAP_UNROLL;
  const int32_t* __restrict__ col;
  const T* __restrict__ w;
  const T* __restrict__ d;
  const T* __restrict__ dinv;
  const T* __restrict__ x;
  T* __restrict__ y;
  const T* __restrict__ b;
  T* __restrict__ p;
  T c1, c2, c0;

  __device__ __forceinline__ Acc identity() const {
    Acc a;
#pragma unroll
    for (int c = 0; c < K; c++) a.v[c] = T(0);
    return a;
  }
  __device__ __forceinline__ bool active(int64_t) const { return true; }
  __device__ __forceinline__ void accum(Acc& a, int64_t, int e) const {
    const int j = col[e];
    const T wv = w[e];
    const T* xj = x + (int64_t)j * K;
    if (MODE == LAP_CHEB_ZERO) {
      const T dj = dinv[j];
#pragma unroll
      for (int c = 0; c < K; c++) a.v[c] += wv * ((dj * xj[c]) * c0);
    } else {
#pragma unroll
      for (int c = 0; c < K; c++) a.v[c] += wv * xj[c];
    }
  }
  __device__ __forceinline__ void combine(Acc& a, const Acc& o) const {
#pragma unroll
    for (int c = 0; c < K; c++) a.v[c] += o.v[c];
  }

  // merge-path interface (one column): an entry's term of the row sum, and
  // the epilogue's slope d y_row / d(row sum) for partial sums added late
  using Val = T;
  __device__ __forceinline__ T term(int e) const {
    const int j = col[e];
    return MODE == LAP_CHEB_ZERO ? w[e] * ((dinv[j] * x[j]) * c0) : w[e] * x[j];
  }
  __device__ __forceinline__ T slope(int64_t row) const {
    return MODE == LAP_SPMV ? T(-1) : MODE == LAP_RESID ? T(1) : c2 * dinv[row];
  }
  __device__ __forceinline__ void add_to_row(int64_t row, T s) const { y[row] += slope(row) * s; }

  __device__ __forceinline__ void finish(int64_t row, const Acc& a, int lane, int G) const {
    const T di = d[row];
#pragma unroll
    for (int c = 0; c < K; c++) {
      if (c % G != lane) continue;  // lanes share the k columns of the row
      const int64_t idx = row * K + c;
      const T xi = MODE == LAP_CHEB_ZERO ? (dinv[row] * x[idx]) * c0 : x[idx];
      const T lx = di * xi - a.v[c];
      if (MODE == LAP_SPMV) {
        y[idx] = lx;
      } else if (MODE == LAP_RESID) {
        y[idx] = b[idx] - lx;
      } else {
        const T r = dinv[row] * (b[idx] - lx);
        T pn;
        if (MODE == LAP_CHEB_FIRST) pn = c2 * r;
        else if (MODE == LAP_CHEB) pn = c1 * (xi - y[idx]) + c2 * r;
        else pn = c1 * xi + c2 * r;  // CHEB_ZERO, CHEB_X1
        if (MODE == LAP_CHEB_ZERO && p) p[idx] = xi;
        y[idx] = xi + pn;
      }
    }
  }
};

// Column-split form of LapOp for k * sizeof(T) >= 32 bytes: each of kL lanes
// owns V = 16 / sizeof(T) consecutive columns.
template <typename T, int K, int MODE, int TAG = 0>
struct LapColOp {
  static constexpr int V = 16 / (int)sizeof(T);
  static constexpr int kL = K / V;
  static_assert(kL >= 2 && K % V == 0, "column split needs at least two 16-byte slices");
  using Acc = VecAcc<T, V>;
  typedef T vec_t __attribute__((ext_vector_type(16 / sizeof(T))));
  const int32_t* __restrict__ col;
  const T* __restrict__ w;
  const T* __restrict__ d;
  const T* __restrict__ dinv;
  const T* __restrict__ x;
  T* __restrict__ y;
  const T* __restrict__ b;
  T* __restrict__ p;
  T c1, c2, c0;
  const int32_t* __restrict__ agg = nullptr;  // LAP_CHEB_FIRST_CC: aggregate of each row
  // TAG 2 with LAP_SPMV: the CG's product, whose epilogue also forms p . q
  // (p = x, q = y) per column; see finish_dot and the row kernels' dot_store
  static constexpr bool kDot = MODE == LAP_SPMV && TAG == 2;

  __device__ __forceinline__ Acc identity() const {
    Acc a;
#pragma unroll
    for (int v = 0; v < V; v++) a.v[v] = T(0);
    return a;
  }
  __device__ __forceinline__ bool active(int64_t) const { return true; }
  // keep = false: a padding slot of an unrolled loop (e is a valid index, weight 0)
  __device__ __forceinline__ void accum(Acc& a, int64_t, int e, int part, bool keep = true) const {
    const int j = MODE == LAP_CHEB_FIRST_CC ? agg[col[e]] : col[e];
    const T wv = keep ? w[e] : T(0);
    const vec_t xv = *reinterpret_cast<const vec_t*>(x + (int64_t)j * K + part * V);
    if (MODE == LAP_CHEB_ZERO) {
      const T dj = dinv[j];
#pragma unroll
      for (int v = 0; v < V; v++) a.v[v] += wv * ((dj * xv[v]) * c0);
    } else {
#pragma unroll
      for (int v = 0; v < V; v++) a.v[v] += wv * xv[v];
    }
  }
  __device__ __forceinline__ void combine(Acc& a, const Acc& o) const {
#pragma unroll
    for (int v = 0; v < V; v++) a.v[v] += o.v[v];
  }
  // Row-local operands of finish, loaded before the row's gather so that
  // their latency overlaps it.
  struct Pre {
    T di, dv;
    vec_t xv, bv, yv;
  };
  __device__ __forceinline__ Pre prefetch(int64_t row, int part) const {
    Pre q;
    const int64_t base = row * K + part * V;
    q.di = d[row];
    // CC: xv is the row's own coarse value x_c[agg_row]
    q.xv = *reinterpret_cast<const vec_t*>(
        x + (MODE == LAP_CHEB_FIRST_CC ? (int64_t)agg[row] * K + part * V : base));
    if (MODE != LAP_SPMV) q.bv = MODE == LAP_CHEB_ZERO ? q.xv : *reinterpret_cast<const vec_t*>(b + base);
    if (MODE >= LAP_CHEB) q.dv = dinv[row];
    if (MODE == LAP_CHEB || MODE == LAP_CHEB_FIRST_CC)
      q.yv = *reinterpret_cast<const vec_t*>(y + base);
    return q;
  }
  __device__ __forceinline__ void finish(int64_t row, const Acc& a, int part) const {
    finish(row, a, part, prefetch(row, part));
  }
  // y = L x as LAP_SPMV, and the lane's terms x_row * y_row added to d (kDot)
  __device__ __forceinline__ void finish_dot(int64_t row, const Acc& a, int part, const Pre& q,
                                             double (&d)[V]) const {
    const int64_t base = row * K + part * V;
    vec_t out;
#pragma unroll
    for (int v = 0; v < V; v++) out[v] = q.di * q.xv[v] - a.v[v];
    *reinterpret_cast<vec_t*>(y + base) = out;
#pragma unroll
    for (int v = 0; v < V; v++) d[v] += (double)q.xv[v] * (double)out[v];
  }
  __device__ __forceinline__ void finish(int64_t row, const Acc& a, int part, const Pre& q) const {
    const T di = q.di;
    const int64_t base = row * K + part * V;
    vec_t xv = q.xv;
    if (MODE == LAP_CHEB_ZERO) {
#pragma unroll
      for (int v = 0; v < V; v++) xv[v] = (q.dv * xv[v]) * c0;
    }
    vec_t out;
    if (MODE == LAP_CHEB_FIRST_CC) {
      vec_t xn;
#pragma unroll
      for (int v = 0; v < V; v++) {
        xn[v] = q.yv[v] + xv[v];                            // x' = x + P x_c
        const T r = q.dv * (q.bv[v] - (di * xv[v] - a.v[v]));  // dinv (r - L P x_c)
        out[v] = xn[v] + c2 * r;
      }
      *reinterpret_cast<vec_t*>(y + base) = xn;
      *reinterpret_cast<vec_t*>(p + base) = out;
      return;
    }
    if (MODE == LAP_SPMV) {
#pragma unroll
      for (int v = 0; v < V; v++) out[v] = di * xv[v] - a.v[v];
    } else if (MODE == LAP_RESID) {
#pragma unroll
      for (int v = 0; v < V; v++) out[v] = q.bv[v] - (di * xv[v] - a.v[v]);
    } else {
#pragma unroll
      for (int v = 0; v < V; v++) {
        const T r = q.dv * (q.bv[v] - (di * xv[v] - a.v[v]));
        T pn;
        if (MODE == LAP_CHEB_FIRST) pn = c2 * r;
        else if (MODE == LAP_CHEB) pn = c1 * (xv[v] - q.yv[v]) + c2 * r;
        else pn = c1 * xv[v] + c2 * r;  // CHEB_ZERO, CHEB_X1
        out[v] = xv[v] + pn;
      }
      if (MODE == LAP_CHEB_ZERO && p) *reinterpret_cast<vec_t*>(p + base) = xv;
    }
    *reinterpret_cast<vec_t*>(y + base) = out;
  }
};

template <typename T, int K>
constexpr bool use_col_split() {
  return K * (int)sizeof(T) >= 32;
}

}  // namespace lg
