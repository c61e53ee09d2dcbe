// common.h -- shared device helpers and the row-scheduled reduction framework
// of liblgmg (gfx950).
//
// Every per-row pass of the method (row sums, the elimination and aggregation
// semiring products of Algorithms 2 and 3, the Jacobi sweeps and affinities of
// Section 3.5, the Laplacian SpMV of the smoother and CG) is expressed as an
// "Op" reduced over the stored entries of each CSR row:
//   - ordinary rows: a group of G lanes (G = power of two <= 64) per row, the
//     lanes stride the row, then a butterfly reduction inside the group;
//   - hub rows (degree > hub_deg): split into HUB_CHUNK-entry chunks, one
//     256-thread workgroup per chunk writes a partial, and a fix-up pass
//     combines each hub's partials in chunk order and runs the epilogue.
// The split keeps a vertex of degree 1e5 from serialising one wavefront.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lgmg.h"

typedef unsigned __int128 u128;
typedef __int128 s128;

namespace lg {

constexpr int kBlock = 256;
constexpr int kHubChunk = 4096;
constexpr uint64_t kGolden = 0x9e3779b97f4a7c15ULL;

// ------------------------------------------------------------------ errors
struct Error {
  lg_status code;
  std::string msg;
};
[[noreturn]] void fail(lg_status code, const std::string& msg);
void set_last_error(const std::string& msg);
const char* last_error_cstr();

#define LG_HIP(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess)                                                                  \
      ::lg::fail(e_ == hipErrorOutOfMemory ? LG_E_NOMEM : LG_E_HIP,                        \
                 std::string(#x) + ": " + hipGetErrorString(e_));                           \
  } while (0)

#define LG_LAUNCH_CHECK() LG_HIP(hipGetLastError())

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ----------------------------------------------------- counter-based RNG
// SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014).
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
// Elimination hash (Section 3.4): i-th SplitMix64 output from state 0.
__host__ __device__ __forceinline__ uint64_t vertex_hash(int64_t i, int mode) {
  return mode == 1 ? (uint64_t)i : mix64((uint64_t)(i + 1) * kGolden);
}
__host__ __device__ __forceinline__ uint64_t seed_key(uint64_t seed) {
  return mix64((seed + 1) * kGolden);
}
// Entry k of vertex i of the random vectors on `level`: uniform on [-1, 1) with
// a 53-bit grid.  Stream k = 64 seeds the Lanczos start vector.
__host__ __device__ __forceinline__ double counter_uniform(uint64_t key, int level, int k,
                                                           int64_t i) {
  uint64_t ctr = key ^ (((uint64_t)level << 56) | ((uint64_t)k << 48) | (uint64_t)i);
  uint64_t u = mix64((ctr + 1) * kGolden) >> 11;
  return 2.0 * ((double)u * 0x1p-53) - 1.0;
}
constexpr int kLanczosStream = 64;

// ------------------------------------------------ exact (order-free) sums
// A sum that feeds a decision is formed on the fixed-point grid 2^-64: each
// fp64 term is rounded to the nearest multiple of 2^-64 (ties to even), the
// 128-bit integers are added (wrapping; associative, hence order free) and the
// total is rounded once to the nearest fp64 (ties to even).
__device__ __forceinline__ u128 xs_term(double v, int& bad) {
  const uint64_t bits = (uint64_t)__double_as_longlong(v);
  const uint64_t mag = bits & 0x7fffffffffffffffULL;
  const int ex = (int)(mag >> 52);
  uint64_t m = mag & 0x000fffffffffffffULL;
  if (ex == 0x7ff) {
    bad = 1;
    return 0;
  }
  int e = ex;
  if (e == 0) {
    if (m == 0) return 0;
    e = 1;
  } else {
    m |= 0x0010000000000000ULL;
  }
  // |v| = m * 2^(e-1075); times 2^64 -> m * 2^(e-1011)
  const int sh = e - 1011;
  u128 r;
  if (sh >= 0) {
    if (sh > 73) {  // |v| * 2^64 >= 2^126
      bad = 1;
      return 0;
    }
    r = (u128)m << sh;
  } else {
    const int rs = -sh;
    if (rs > 54) {
      r = 0;  // below half a unit of 2^-64
    } else {
      uint64_t q = m >> rs;
      const uint64_t rem = m & ((1ULL << rs) - 1);
      const uint64_t half = 1ULL << (rs - 1);
      if (rem > half || (rem == half && (q & 1))) q++;
      r = q;
    }
  }
  return (bits >> 63) ? (u128)0 - r : r;
}

__device__ __forceinline__ double xs_value(u128 s) {
  if (s == 0) return 0.0;
  const bool neg = (s >> 127) != 0;
  const u128 a = neg ? (u128)0 - s : s;
  const uint64_t hi = (uint64_t)(a >> 64), lo = (uint64_t)a;
  const int lead = hi ? 127 - __clzll((long long)hi) : 63 - __clzll((long long)lo);
  uint64_t mant;
  int ex2;
  if (lead <= 52) {
    mant = lo;
    ex2 = 0;
  } else {
    int rs = lead - 52;
    u128 q = a >> rs;
    const u128 rem = a & (((u128)1 << rs) - 1);
    const u128 half = (u128)1 << (rs - 1);
    if (rem > half || (rem == half && (q & 1))) q++;
    if (q >> 53) {
      q >>= 1;
      rs++;
    }
    mant = (uint64_t)q;
    ex2 = rs;
  }
  const double r = ldexp((double)mant, ex2 - 64);
  return neg ? -r : r;
}

// -------------------------------------------------------------- shuffles
template <typename T>
__device__ __forceinline__ T shfl_xor_any(const T& v, int mask) {
  static_assert(sizeof(T) % 4 == 0, "shuffle of a type whose size is not a multiple of 4");
  constexpr int W = sizeof(T) / 4;
  int tmp[W];
  __builtin_memcpy(tmp, &v, sizeof(T));
#pragma unroll
  for (int k = 0; k < W; k++) tmp[k] = __shfl_xor(tmp[k], mask);
  T out;
  __builtin_memcpy(&out, tmp, sizeof(T));
  return out;
}

// ---------------------------------------------------------- row schedule
struct Sched {
  int64_t n = 0, nnz = 0;
  int G = 8;            // lanes per ordinary row
  int hub_deg = 1 << 30;  // rows with more entries are hubs
  int64_t nhub = 0, nchunk = 0;
  int32_t* hub_rows = nullptr;   // [nhub]
  int32_t* hub_cptr = nullptr;   // [nhub + 1] first chunk of each hub
  int32_t* chunk_hub = nullptr;  // [nchunk] hub of each chunk
  void* partial = nullptr;       // [nchunk * kPartialBytes]
};
constexpr int kPartialBytes = 512;

// Ordinary rows: G lanes per row.
template <class Op, int G>
__global__ __launch_bounds__(kBlock) void k_rows(Op op, const int32_t* __restrict__ rp, int64_t n,
                                                 int hub_deg) {
  const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (row >= n) return;
  const int beg = rp[row], end = rp[row + 1];
  if (end - beg > hub_deg) return;
  typename Op::Acc acc = op.identity();
  if (op.active(row)) {
    for (int e = beg + lane; e < end; e += G) op.accum(acc, row, e);
#pragma unroll
    for (int m = G / 2; m > 0; m >>= 1) op.combine(acc, shfl_xor_any(acc, m));
  }
  op.finish(row, acc, lane, G);
}

// Hub rows, phase 1: one workgroup per chunk writes a partial.
template <class Op>
__global__ __launch_bounds__(kBlock) void k_hub_chunks(Op op, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ hub_rows,
                                                       const int32_t* __restrict__ hub_cptr,
                                                       const int32_t* __restrict__ chunk_hub,
                                                       typename Op::Acc* __restrict__ partial) {
  using Acc = typename Op::Acc;
  const int c = blockIdx.x;
  const int h = chunk_hub[c];
  const int64_t row = hub_rows[h];
  const int k = c - hub_cptr[h];
  const int beg = rp[row] + k * kHubChunk;
  const int end = min(rp[row + 1], beg + kHubChunk);
  Acc acc = op.identity();
  if (op.active(row))
    for (int e = beg + (int)threadIdx.x; e < end; e += kBlock) op.accum(acc, row, e);
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) op.combine(acc, shfl_xor_any(acc, m));
  __shared__ Acc red[kBlock / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    Acc t = red[0];
#pragma unroll
    for (int w = 1; w < kBlock / 64; w++) op.combine(t, red[w]);
    partial[c] = t;
  }
}

// Hub rows, phase 2: combine partials in chunk order, run the epilogue.
template <class Op>
__global__ __launch_bounds__(64) void k_hub_fix(Op op, const int32_t* __restrict__ hub_rows,
                                                const int32_t* __restrict__ hub_cptr,
                                                const typename Op::Acc* __restrict__ partial,
                                                int64_t nhub) {
  const int64_t h = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (h >= nhub) return;
  const int64_t row = hub_rows[h];
  typename Op::Acc acc = op.identity();
  for (int c = hub_cptr[h]; c < hub_cptr[h + 1]; c++) op.combine(acc, partial[c]);
  op.finish(row, acc, 0, 1);
}

template <class Op, int G>
inline void launch_rows_g(const Sched& s, const int32_t* rp, const Op& op, hipStream_t st) {
  const int64_t blocks = ceil_div(s.n * G, kBlock);
  hipLaunchKernelGGL((k_rows<Op, G>), dim3((unsigned)blocks), dim3(kBlock), 0, st, op, rp, s.n,
                     s.hub_deg);
}

// Run Op over every row of the CSR described by (s, rp) on stream st.
template <class Op>
void run_rows(const Sched& s, const int32_t* rp, const Op& op, hipStream_t st) {
  static_assert(sizeof(typename Op::Acc) <= kPartialBytes, "accumulator larger than a partial slot");
  if (s.n == 0) return;
  switch (s.G) {
    case 1: launch_rows_g<Op, 1>(s, rp, op, st); break;
    case 2: launch_rows_g<Op, 2>(s, rp, op, st); break;
    case 4: launch_rows_g<Op, 4>(s, rp, op, st); break;
    case 8: launch_rows_g<Op, 8>(s, rp, op, st); break;
    case 16: launch_rows_g<Op, 16>(s, rp, op, st); break;
    case 32: launch_rows_g<Op, 32>(s, rp, op, st); break;
    default: launch_rows_g<Op, 64>(s, rp, op, st); break;
  }
  LG_LAUNCH_CHECK();
  if (s.nhub) {
    auto* part = reinterpret_cast<typename Op::Acc*>(s.partial);
    hipLaunchKernelGGL((k_hub_chunks<Op>), dim3((unsigned)s.nchunk), dim3(kBlock), 0, st, op, rp,
                       s.hub_rows, s.hub_cptr, s.chunk_hub, part);
    hipLaunchKernelGGL((k_hub_fix<Op>), dim3((unsigned)ceil_div(s.nhub, 64)), dim3(64), 0, st, op,
                       s.hub_rows, s.hub_cptr, (const typename Op::Acc*)part, s.nhub);
    LG_LAUNCH_CHECK();
  }
}

// ------------------------------------------------------------- memory
// Bump allocator over large device chunks.  The hierarchy owns one for its
// lifetime; setup uses a second one for temporaries and rewinds it per level.
class Arena {
 public:
  explicit Arena(size_t chunk = (size_t)64 << 20) : chunk_(chunk) {}
  ~Arena() { release(); }
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  void* alloc(size_t bytes);
  template <typename T>
  T* get(int64_t count) {
    return static_cast<T*>(alloc(sizeof(T) * (size_t)(count > 0 ? count : 1)));
  }
  struct Mark {
    size_t chunk, off;
  };
  Mark mark() const { return {cur_, off_}; }
  void rewind(Mark m) {
    cur_ = m.chunk;
    off_ = m.off;
  }
  void release();
  size_t bytes() const { return total_; }

 private:
  struct Chunk {
    char* p;
    size_t size;
  };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0, off_ = 0, total_ = 0, chunk_;
};

// ------------------------------------------------- profiling (HIP events)
struct ProfScope {
  ProfScope(const char* family, hipStream_t st, double bytes);
  ~ProfScope();
  bool on;
  hipStream_t st;
  double bytes;
  hipEvent_t a, b;
};

// ------------------------------------------------------------- helpers
void build_sched(Sched& s, const int32_t* rp, int64_t n, int64_t nnz, Arena& keep, Arena& tmp,
                 hipStream_t st);
// out[i] = sum_{j<i} in[j] for i <= n (out has n+1 entries); returns out[n] on the host
// when want_total (synchronises the stream).
int64_t scan_i64(const int64_t* in, int64_t* out, int64_t n, Arena& tmp, hipStream_t st,
                 bool want_total);
int64_t scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, Arena& tmp, hipStream_t st,
                        bool want_total);
// Stable LSD radix sort of (key, val) pairs over the listed 8-bit digit shifts.
void radix_sort_pairs(uint64_t* keys, uint64_t* vals, int64_t n, const std::vector<int>& shifts,
                      Arena& tmp, hipStream_t st);
std::vector<int> digit_shifts(int bits_lo, int bits_hi);  // digits covering [0,bits_lo) and [32,32+bits_hi)
int bits_for(int64_t max_value);
int64_t read_i64(const int64_t* dev, hipStream_t st);

}  // namespace lg
