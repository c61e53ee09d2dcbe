// eigen.hip -- smallest nonzero eigenpairs of L (the Fiedler vector and its
// successors, Section 2.1: spectral partitioning and drawing use them, and
// eigensolvers for them spend most of their time applying L^+).
//
// Block inverse subspace iteration on the mean-zero space: a block of b
// vectors is orthonormalised (Cholesky QR, twice), a Rayleigh-Ritz step on L
// rotates it to Ritz vectors, and the next block solves L Z = Y with the
// multigrid-preconditioned CG of this library (all b columns in one batched
// solve).  Eigenvector i converges like (lambda_i / lambda_{b+1})^iteration.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "impl.h"
#include "ops.h"

namespace lg {
namespace {

inline unsigned blocks_of(int64_t n) { return (unsigned)ceil_div(n, (int64_t)kBlock); }

// Seeded start block: counter-based uniform(-1, 1) values, stream 65.
__global__ void k_eig_start(double* __restrict__ Y, int64_t n, int K, int b, uint64_t key) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n * K) return;
  const int64_t row = i / K;
  const int c = (int)(i - row * K);
  Y[i] = c < b ? counter_uniform(key, 65, c, row) : 0.0;
}

// Per-block partial Gram matrices G = A^T B over rows (K x K, row-major), in
// a fixed order: each thread owns rows t, t + stride, ...; the block folds
// its threads through LDS column by column.
template <int K>
__global__ __launch_bounds__(kBlock) void k_gram(const double* __restrict__ A,
                                                 const double* __restrict__ B, int64_t n,
                                                 double* __restrict__ partial) {
  double acc[K][K];
#pragma unroll
  for (int p = 0; p < K; p++)
#pragma unroll
    for (int q = 0; q < K; q++) acc[p][q] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    double a[K], bb[K];
#pragma unroll
    for (int p = 0; p < K; p++) {
      a[p] = A[i * K + p];
      bb[p] = B[i * K + p];
    }
#pragma unroll
    for (int p = 0; p < K; p++)
#pragma unroll
      for (int q = 0; q < K; q++) acc[p][q] += a[p] * bb[q];
  }
  __shared__ double sm[kBlock];
#pragma unroll
  for (int p = 0; p < K; p++)
#pragma unroll
    for (int q = 0; q < K; q++) {
      sm[threadIdx.x] = acc[p][q];
      __syncthreads();
      for (int m = kBlock / 2; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) sm[threadIdx.x] += sm[threadIdx.x + m];
        __syncthreads();
      }
      if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * K * K + p * K + q] = sm[0];
      __syncthreads();
    }
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_gram_final(const double* __restrict__ partial, int nb,
                                                       double* __restrict__ G) {
  const int e = blockIdx.x;  // one workgroup per entry
  __shared__ double sm[kBlock];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) s += partial[(int64_t)b * K * K + e];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int m = kBlock / 2; m > 0; m >>= 1) {
    if ((int)threadIdx.x < m) sm[threadIdx.x] += sm[threadIdx.x + m];
    __syncthreads();
  }
  if (threadIdx.x == 0) G[e] = sm[0];
}

// Out = In * M row by row (M is K x K, row-major, in device memory).
template <int K>
__global__ void k_rotate(const double* __restrict__ In, const double* __restrict__ M, int64_t n,
                         double* __restrict__ Out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double a[K];
#pragma unroll
  for (int p = 0; p < K; p++) a[p] = In[i * K + p];
#pragma unroll
  for (int q = 0; q < K; q++) {
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < K; p++) s += a[p] * M[p * K + q];
    Out[i * K + q] = s;
  }
}

// R = W - Y diag(theta) (theta in device memory, K entries)
template <int K>
__global__ void k_ritz_resid(const double* __restrict__ W, const double* __restrict__ Y,
                             const double* __restrict__ theta, int64_t n, double* __restrict__ R) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n * K) return;
  R[i] = W[i] - theta[i % K] * Y[i];
}

// ---- small dense algebra on the host (b <= 8)

// Upper Cholesky factor R of the b x b symmetric G (G = R^T R); false if not
// positive definite.
bool cholesky_upper(const std::vector<double>& G, int b, int K, std::vector<double>& R) {
  R.assign((size_t)K * K, 0.0);
  for (int j = 0; j < b; j++) {
    double d = G[j * K + j];
    for (int k = 0; k < j; k++) d -= R[k * K + j] * R[k * K + j];
    if (!(d > 0.0)) return false;
    R[j * K + j] = std::sqrt(d);
    for (int i = j + 1; i < b; i++) {
      double s = G[j * K + i];
      for (int k = 0; k < j; k++) s -= R[k * K + j] * R[k * K + i];
      R[j * K + i] = s / R[j * K + j];
    }
  }
  return true;
}

// Inverse of the upper triangular R (b x b within a K x K array).
std::vector<double> upper_inverse(const std::vector<double>& R, int b, int K) {
  std::vector<double> X((size_t)K * K, 0.0);
  for (int j = 0; j < b; j++) {
    X[j * K + j] = 1.0 / R[j * K + j];
    for (int i = j - 1; i >= 0; i--) {
      double s = 0.0;
      for (int k = i + 1; k <= j; k++) s += R[i * K + k] * X[k * K + j];
      X[i * K + j] = -s / R[i * K + i];
    }
  }
  return X;
}

// Eigen-decomposition of the symmetric b x b H by cyclic Jacobi rotations:
// H = Q diag(theta) Q^T, eigenvalues ascending, columns of Q the vectors.
void jacobi_eigen(std::vector<double> H, int b, int K, std::vector<double>& theta,
                  std::vector<double>& Q) {
  Q.assign((size_t)K * K, 0.0);
  for (int i = 0; i < b; i++) Q[i * K + i] = 1.0;
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < b; p++)
      for (int q = 0; q < b; q++) (p == q ? diag : off) += H[p * K + q] * H[p * K + q];
    if (off <= 1e-32 * diag) break;
    for (int p = 0; p < b; p++)
      for (int q = p + 1; q < b; q++) {
        const double apq = H[p * K + q];
        if (apq == 0.0) continue;
        const double tau = (H[q * K + q] - H[p * K + p]) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < b; k++) {  // H <- J^T H J
          const double hkp = H[k * K + p], hkq = H[k * K + q];
          H[k * K + p] = c * hkp - s * hkq;
          H[k * K + q] = s * hkp + c * hkq;
        }
        for (int k = 0; k < b; k++) {
          const double hpk = H[p * K + k], hqk = H[q * K + k];
          H[p * K + k] = c * hpk - s * hqk;
          H[q * K + k] = s * hpk + c * hqk;
        }
        for (int k = 0; k < b; k++) {
          const double qkp = Q[k * K + p], qkq = Q[k * K + q];
          Q[k * K + p] = c * qkp - s * qkq;
          Q[k * K + q] = s * qkp + c * qkq;
        }
      }
  }
  std::vector<int> ord(b);
  for (int i = 0; i < b; i++) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int c) { return H[a * K + a] < H[c * K + c]; });
  std::vector<double> Qs((size_t)K * K, 0.0);
  theta.assign(b, 0.0);
  for (int j = 0; j < b; j++) {
    theta[j] = H[ord[j] * K + ord[j]];
    for (int i = 0; i < b; i++) Qs[i * K + j] = Q[i * K + ord[j]];
  }
  Q = Qs;
}

template <int K>
struct Eig {
  lg_hierarchy* h;
  hipStream_t st;
  int64_t n;
  int b;  // block width (K)
  double *Y, *W, *Z, *M, *G, *part;
  int nb;

  std::vector<double> gram(const double* A, const double* B) {
    hipLaunchKernelGGL((k_gram<K>), dim3(nb), dim3(kBlock), 0, st, A, B, n, part);
    hipLaunchKernelGGL((k_gram_final<K>), dim3(K * K), dim3(kBlock), 0, st, (const double*)part, nb,
                       G);
    LG_LAUNCH_CHECK();
    std::vector<double> out((size_t)K * K);
    LG_HIP(hipMemcpyAsync(out.data(), G, sizeof(double) * K * K, hipMemcpyDeviceToHost, st));
    LG_HIP(hipStreamSynchronize(st));
    return out;
  }

  // dst = src * Mh (Mh on the host)
  void rotate(const double* src, const std::vector<double>& Mh, double* dst) {
    LG_HIP(hipMemcpyAsync(M, Mh.data(), sizeof(double) * K * K, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL((k_rotate<K>), dim3(blocks_of(n)), dim3(kBlock), 0, st, src, (const double*)M,
                       n, dst);
    LG_LAUNCH_CHECK();
  }

  // Y <- Y R^-1 with Y^T Y = R^T R (twice, for orthonormality to rounding)
  bool orthonormalise() {
    for (int pass = 0; pass < 2; pass++) {
      std::vector<double> R;
      if (!cholesky_upper(gram(Y, Y), b, K, R)) return false;
      rotate(Y, upper_inverse(R, b, K), Z);
      std::swap(Y, Z);
    }
    return true;
  }
};

// Workgroups of the Gram reductions for n rows.
inline int gram_blocks(int64_t n) {
  return (int)std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(n, (int64_t)kBlock * 8)));
}

// Doubles of per-call scratch for a block of K columns on n rows: Y, W, Z
// (n x K), M, G (K x K) and the Gram partials, each rounded up to 256 bytes.
inline int64_t eig_scratch_doubles(int64_t n, int K) {
  auto up = [](int64_t v) { return (v + 31) / 32 * 32; };
  return 3 * up(n * K) + 2 * up((int64_t)K * K) + up((int64_t)gram_blocks(n) * K * K);
}

// scratch == nullptr: the per-call buffers come from the hierarchy's arena
// (which may allocate a chunk); else they are carved from scratch, which
// holds at least eig_scratch_doubles(n, K) doubles.
template <int K>
lg_status eigs_k(lg_hierarchy* h, int nev, double tol, int max_iter, double* X, double* lambda,
                 int* iters, double* resid, hipStream_t st, double* scratch) {
  constexpr int b = K;
  const Level& L0 = h->lev[0];
  Eig<K> e{h, st, L0.n, b};
  const int64_t m = e.n * K;
  e.nb = gram_blocks(e.n);
  Arena::Mark mark = h->mem.mark();
  if (scratch) {
    auto up = [](int64_t v) { return (v + 31) / 32 * 32; };
    double* p = scratch;
    e.Y = p;
    p += up(m);
    e.W = p;
    p += up(m);
    e.Z = p;
    p += up(m);
    e.M = p;
    p += up(K * K);
    e.G = p;
    p += up(K * K);
    e.part = p;
  } else {
    e.Y = h->mem.get<double>(m);
    e.W = h->mem.get<double>(m);
    e.Z = h->mem.get<double>(m);
    e.M = h->mem.get<double>(K * K);
    e.G = h->mem.get<double>(K * K);
    e.part = h->mem.get<double>((int64_t)e.nb * K * K);
  }
  struct Release {
    lg_hierarchy* h;
    Arena::Mark m;
    ~Release() { h->mem.rewind(m); }
  } release{h, mark};
  hipLaunchKernelGGL(k_eig_start, dim3(blocks_of(m)), dim3(kBlock), 0, st, e.Y, e.n, K, b,
                     seed_key(h->opts.seed));
  LG_LAUNCH_CHECK();
  // inner solves to a tenth of the outer tolerance (the solver projects to mean zero)
  std::vector<lg_rhs_info> info(b);
  const double inner = std::max(1e-12, std::min(1e-4, 0.1 * tol));
  auto solve = [&]() {
    const lg_status s = solve_dispatch(h, e.Y, e.Z, b, inner, 2000, st, info.data());
    if (s != LG_OK && s != LG_E_NOT_CONVERGED) fail(s, "lg_eigs: inner solve failed");
    std::swap(e.Y, e.Z);
  };
  solve();
  std::vector<double> theta, Q, res(b, 0.0);
  int it = 0;
  for (;; it++) {
    if (!e.orthonormalise()) fail(LG_E_NOT_CONVERGED, "lg_eigs: the block lost rank");
    spmv_dispatch(h, 0, e.Y, e.W, K, st);
    std::vector<double> H = e.gram(e.Y, e.W);
    for (int p = 0; p < b; p++)  // symmetrise the rounding
      for (int q = p + 1; q < b; q++) H[p * K + q] = H[q * K + p] = 0.5 * (H[p * K + q] + H[q * K + p]);
    jacobi_eigen(H, b, K, theta, Q);
    e.rotate(e.Y, Q, e.Z);
    std::swap(e.Y, e.Z);
    e.rotate(e.W, Q, e.Z);
    std::swap(e.W, e.Z);
    // residuals ||L y_i - theta_i y_i|| of the unit Ritz vectors
    std::vector<double> th(K, 0.0);
    for (int i = 0; i < b; i++) th[i] = theta[i];
    LG_HIP(hipMemcpyAsync(e.M, th.data(), sizeof(double) * K, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL((k_ritz_resid<K>), dim3(blocks_of(m)), dim3(kBlock), 0, st,
                       (const double*)e.W, (const double*)e.Y, (const double*)e.M, e.n, e.Z);
    LG_LAUNCH_CHECK();
    std::vector<double> RR = e.gram(e.Z, e.Z);
    bool done = true;
    for (int i = 0; i < nev; i++) {
      res[i] = std::sqrt(std::max(0.0, RR[i * K + i]));
      if (!(res[i] <= tol * theta[i])) done = false;
    }
    if (done || it >= max_iter) break;
    solve();
  }
  // the first nev Ritz vectors, n x nev row-major
  std::vector<double> Yh((size_t)m);
  LG_HIP(hipMemcpyAsync(Yh.data(), e.Y, sizeof(double) * m, hipMemcpyDeviceToHost, st));
  LG_HIP(hipStreamSynchronize(st));
  std::vector<double> Xh((size_t)e.n * nev);
  for (int64_t i = 0; i < e.n; i++)
    for (int c = 0; c < nev; c++) Xh[i * nev + c] = Yh[i * K + c];
  LG_HIP(hipMemcpyAsync(X, Xh.data(), sizeof(double) * Xh.size(), hipMemcpyHostToDevice, st));
  LG_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < nev; i++) {
    lambda[i] = theta[i];
    if (resid) resid[i] = res[i];
  }
  if (iters) *iters = it;
  for (int i = 0; i < nev; i++)
    if (!(res[i] <= tol * theta[i])) return LG_E_NOT_CONVERGED;
  return LG_OK;
}


// The allocation-free variant's scratch: a file-scope device array, one copy
// per GPU the library runs on, held until the process ends.  Host code uses
// its device address from hipGetSymbolAddress (kept per device), never the
// array's name.  Every lg_eigs_noalloc call on a GPU shares that GPU's copy.
constexpr int64_t kEigScratchBytes = (int64_t)64 << 20;
__device__ __align__(256) double scratch[kEigScratchBytes / 8];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

double* scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) fail(LG_E_ARG, "lg_eigs_noalloc: device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      fail(LG_E_HIP, std::string("lg_eigs_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
    g_scratch[device] = (double*)p;
  }
  return g_scratch[device];
}

int eig_width(lg_hierarchy* h, int nev) {
  int K = 2;
  while (K < nev + 1) K <<= 1;
  if (K > 8 || K > h->opts.max_rhs)
    fail(LG_E_ARG, "lg_eigs: needs nev + 1 <= 8 and a block of next_pow2(nev + 1) <= max_rhs");
  return K;
}

lg_status eigs_run(lg_hierarchy* h, int nev, double tol, int max_iter, double* X, double* lambda,
                   int* iters, double* resid, hipStream_t st, double* scr) {
  switch (eig_width(h, nev)) {
    case 2: return eigs_k<2>(h, nev, tol, max_iter, X, lambda, iters, resid, st, scr);
    case 4: return eigs_k<4>(h, nev, tol, max_iter, X, lambda, iters, resid, st, scr);
    default: return eigs_k<8>(h, nev, tol, max_iter, X, lambda, iters, resid, st, scr);
  }
}

}  // namespace

// Block width: the next power of two above nev (one guard vector at least),
// at most 8 and at most the hierarchy's max_rhs.
lg_status eigs_dispatch(lg_hierarchy* h, int nev, double tol, int max_iter, double* X,
                        double* lambda, int* iters, double* resid, hipStream_t st) {
  return eigs_run(h, nev, tol, max_iter, X, lambda, iters, resid, st, nullptr);
}

// As eigs_dispatch, with the per-call buffers in the static scratch array and
// no cycle graph captured during the call (an existing one is replayed).
lg_status eigs_noalloc_dispatch(lg_hierarchy* h, int nev, double tol, int max_iter, double* X,
                                double* lambda, int* iters, double* resid, hipStream_t st) {
  int dev = -1;
  LG_HIP(hipGetDevice(&dev));
  if (dev != h->device) fail(LG_E_ARG, "lg_eigs_noalloc: the hierarchy lives on another device");
  const int K = eig_width(h, nev);
  const int64_t need = eig_scratch_doubles(h->lev[0].n, K) * 8;
  if (need > kEigScratchBytes)
    fail(LG_E_ARG, "lg_eigs_noalloc: a block of " + std::to_string(K) + " columns on " +
                       std::to_string(h->lev[0].n) + " vertices needs " + std::to_string(need) +
                       " bytes of scratch; the static buffer holds " +
                       std::to_string(kEigScratchBytes));
  double* scr = scratch_on(dev);
  struct NoCapture {
    lg_hierarchy* h;
    ~NoCapture() { h->no_capture = false; }
  } guard{h};
  h->no_capture = true;
  return eigs_run(h, nev, tol, max_iter, X, lambda, iters, resid, st, scr);
}

}  // namespace lg
