// ops.h -- Laplacian products L X = D X - A X over k right-hand sides with
// fused epilogues (residual, Chebyshev step), plus small vector kernels.
#pragma once

#include "common.h"

namespace lg {

template <typename T, int K>
struct VecAcc {
  T v[K];
};

enum { LAP_SPMV = 0, LAP_RESID = 1, LAP_CHEB = 2, LAP_CHEB_FIRST = 3 };

// Row i: s = sum_j w_ij x_j (k columns), (L x)_i = d_i x_i - s.
//  LAP_SPMV:       y = L x
//  LAP_RESID:      y = b - L x
//  LAP_CHEB:       r = dinv (b - L x); p = c1 p + c2 r; xo = x + p
//  LAP_CHEB_FIRST: same with p = c2 r (p is not read)
template <typename T, int K, int MODE>
struct LapOp {
  using Acc = VecAcc<T, K>;
  const int32_t* __restrict__ col;
  const T* __restrict__ w;
  const T* __restrict__ d;
  const T* __restrict__ dinv;
  const T* __restrict__ x;
  T* __restrict__ y;
  const T* __restrict__ b;
  T* __restrict__ p;
  T c1, c2;

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
#pragma unroll
    for (int c = 0; c < K; c++) a.v[c] += wv * xj[c];
  }
  __device__ __forceinline__ void combine(Acc& a, const Acc& o) const {
#pragma unroll
    for (int c = 0; c < K; c++) a.v[c] += o.v[c];
  }
  __device__ __forceinline__ void finish(int64_t row, const Acc& a, int lane, int G) const {
    const T di = d[row];
#pragma unroll
    for (int c = 0; c < K; c++) {
      if (c % G != lane) continue;  // lanes share the k columns of the row
      const int64_t idx = row * K + c;
      const T xi = x[idx];
      const T lx = di * xi - a.v[c];
      if (MODE == LAP_SPMV) {
        y[idx] = lx;
      } else if (MODE == LAP_RESID) {
        y[idx] = b[idx] - lx;
      } else {
        const T r = dinv[row] * (b[idx] - lx);
        const T pn = (MODE == LAP_CHEB_FIRST) ? c2 * r : c1 * p[idx] + c2 * r;
        p[idx] = pn;
        y[idx] = xi + pn;
      }
    }
  }
};

// Column-split form of LapOp for k * sizeof(T) >= 32 bytes: each of kL lanes
// owns V = 16 / sizeof(T) consecutive columns.
template <typename T, int K, int MODE>
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
  T c1, c2;

  __device__ __forceinline__ Acc identity() const {
    Acc a;
#pragma unroll
    for (int v = 0; v < V; v++) a.v[v] = T(0);
    return a;
  }
  __device__ __forceinline__ bool active(int64_t) const { return true; }
  __device__ __forceinline__ void accum(Acc& a, int64_t, int e, int part) const {
    const int j = col[e];
    const T wv = w[e];
    const vec_t xv = *reinterpret_cast<const vec_t*>(x + (int64_t)j * K + part * V);
#pragma unroll
    for (int v = 0; v < V; v++) a.v[v] += wv * xv[v];
  }
  __device__ __forceinline__ void combine(Acc& a, const Acc& o) const {
#pragma unroll
    for (int v = 0; v < V; v++) a.v[v] += o.v[v];
  }
  __device__ __forceinline__ void finish(int64_t row, const Acc& a, int part) const {
    const T di = d[row];
    const int64_t base = row * K + part * V;
    const vec_t xv = *reinterpret_cast<const vec_t*>(x + base);
    vec_t out;
    if (MODE == LAP_SPMV) {
#pragma unroll
      for (int v = 0; v < V; v++) out[v] = di * xv[v] - a.v[v];
    } else if (MODE == LAP_RESID) {
      const vec_t bv = *reinterpret_cast<const vec_t*>(b + base);
#pragma unroll
      for (int v = 0; v < V; v++) out[v] = bv[v] - (di * xv[v] - a.v[v]);
    } else {
      const vec_t bv = *reinterpret_cast<const vec_t*>(b + base);
      const T dv = dinv[row];
      vec_t pv;
      if (MODE == LAP_CHEB) pv = *reinterpret_cast<const vec_t*>(p + base);
#pragma unroll
      for (int v = 0; v < V; v++) {
        const T r = dv * (bv[v] - (di * xv[v] - a.v[v]));
        const T pn = (MODE == LAP_CHEB_FIRST) ? c2 * r : c1 * pv[v] + c2 * r;
        pv[v] = pn;
        out[v] = xv[v] + pn;
      }
      *reinterpret_cast<vec_t*>(p + base) = pv;
    }
    *reinterpret_cast<vec_t*>(y + base) = out;
  }
};

template <typename T, int K>
constexpr bool use_col_split() {
  return K * (int)sizeof(T) >= 32;
}

}  // namespace lg
