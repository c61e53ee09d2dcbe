// common.h -- shared device helpers and the row-scheduled reduction framework
// of liblgmg (gfx950).
//
// Every per-row pass of the method (row sums, the elimination and aggregation
// semiring products of Algorithms 2 and 3, the Jacobi sweeps and affinities of
// Section 3.5, the Laplacian SpMV of the smoother and CG) is expressed as an
// "Op" reduced over the stored entries of each CSR row:
//   - ordinary rows: a group of G lanes (G = power of two <= 64, chosen per row
//     from its degree class) per row, the lanes stride the row, then a
//     butterfly reduction inside the group;
//   - hub rows: one 256-thread workgroup per row in the same launch; rows
//     beyond kSplitDeg entries are split into chunks whose partials a second
//     pass combines in chunk order.
// This keeps a vertex of degree 1e5 from serialising one wavefront.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <string>
#include <type_traits>
#include <vector>

#include "lgmg.h"

typedef unsigned __int128 u128;
typedef __int128 s128;

namespace lg {

constexpr int kBlock = 256;
#ifndef LG_HUB_CHUNK
#define LG_HUB_CHUNK 2048
#endif
#ifndef LG_SPLIT_DEG
#define LG_SPLIT_DEG 4096
#endif
#ifndef LG_HUB_DEG
#define LG_HUB_DEG 1024
#endif
#ifndef LG_PER_LANE
#define LG_PER_LANE 4
#endif
#ifndef LG_LAP_UNROLL
#define LG_LAP_UNROLL 4
#endif
constexpr int kHubChunk = LG_HUB_CHUNK;
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
// 128-bit two's-complement integers are added (wrapping; associative, hence
// order free) and the total is rounded once to the nearest fp64 (ties to even).
//
// A term is added as four 32-bit limbs of its 128-bit integer into four 64-bit
// accumulators, with fp64 arithmetic only and no branches: |v| 2^64 is exact,
// rint rounds it to the grid, and floor and the subtractions that peel the
// limbs off are exact.  A negative term adds the complemented limbs plus one
// (its two's complement mod 2^128), with no carries between limbs until
// xs_limbs_total.  The low two accumulators stay below 2^64 for fewer than
// 2^32 terms, the bound for exactness mod 2^128.  Terms that are not finite or
// have |v| 2^64 >= 2^126 add nothing and set `bad`.
__device__ __forceinline__ void xs_limbs_add(double v, uint64_t (&acc)[4], int& bad) {
  const double a = fabs(v) * 0x1p64;
  const bool ok = a < 0x1p126;  // false for NaN and infinities
  bad |= !ok;
  const double y = ok ? rint(a) : 0.0;
  const double t3 = floor(y * 0x1p-96);
  const double y3 = y - t3 * 0x1p96;
  const double t2 = floor(y3 * 0x1p-64);
  const double y2 = y3 - t2 * 0x1p64;
  const double t1 = floor(y2 * 0x1p-32);
  const double t0 = y2 - t1 * 0x1p32;
  const uint32_t neg = (ok && signbit(v)) ? 0xffffffffu : 0u;
  acc[0] += (uint64_t)(((uint32_t)t0) ^ neg) + (neg & 1u);
  acc[1] += (uint64_t)(((uint32_t)t1) ^ neg);
  acc[2] += (uint64_t)(((uint32_t)t2) ^ neg);
  acc[3] += (uint64_t)(((uint32_t)t3) ^ neg);
}

__device__ __forceinline__ u128 xs_limbs_total(const uint64_t (&acc)[4]) {
  return (u128)acc[0] + ((u128)acc[1] << 32) + ((u128)acc[2] << 64) + ((u128)acc[3] << 96);
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
// Rows are grouped by degree once per matrix (a stable counting sort):
//   class c < 7: degree <= kPerLane * 2^c; one-column kernels give such a row
//                class_lanes(c) = 2^(c-1) lanes (up to 2 kPerLane entries
//                each), column-split kernels 2^(c-1) lane groups;
//   class 7:     kPerLane * 64 < degree <= hub_deg, 64 lanes striding the row;
//   hubs:        hub_deg < degree <= kSplitDeg, one 256-thread workgroup each,
//                dispatched first in the same launch;
//   split rows:  degree > kSplitDeg, kHubChunk-entry chunks, one workgroup
//                each, dispatched first; a second launch combines each row's
//                partials in chunk order and runs the epilogue.
// Every row is reduced by one fixed set of lanes in a fixed order, so
// results do not depend on scheduling.
constexpr int kClasses = 8;
constexpr int kPartialBytes = 512;
// Entries each lane group of a column-split row kernel loads per trip (all
// issued together), 4 or 6.  Fewer in flight per wavefront take fewer
// registers and allow more wavefronts.  Measured in whole solves, products of
// at most 16 columns (fp64 and fp32) ran faster at 4 and those of 32 columns
// at 6, so a schedule's unroll of 0 takes that rule; a group adds its entries
// in the same order at either value.
template <class Op>
constexpr int col_unroll_of() {
  return Op::kL * Op::V <= 16 ? 4 : 6;
}
constexpr int kSplitDeg = LG_SPLIT_DEG;  // rows above this are split into kHubChunk-entry chunks

struct ClassTable {
  int32_t cls_start[kClasses + 1];  // row ranges of each class in perm
  int32_t blk_start[kClasses + 1];  // block ranges of each class (after the hubs)
};

struct Sched {
  int64_t n = 0, nnz = 0;
  int hub_deg = LG_HUB_DEG;
  int min_deg = 0, max_deg = 0;
  int32_t* perm = nullptr;  // non-hub rows grouped by class
  ClassTable ct{};
  int64_t nhub = 0;  // workgroup-per-row hubs
  int32_t* hub_rows = nullptr;
  int64_t nsplit = 0, nchunk = 0;  // split rows
  int32_t* split_rows = nullptr;   // [nsplit]
  int32_t* split_cptr = nullptr;   // [nsplit + 1] first chunk of each split row
  int32_t* chunk_split = nullptr;  // [nchunk] split row of each chunk
  void* partial = nullptr;         // [nchunk * kPartialBytes]
  // lanes (one-column kernels) or lane groups (column-split kernels) of a
  // class-c row: 2^(c - shift), chosen per matrix by the autotuner
  int lane_shift = 1, col_shift = 1;
  int col_unroll = 0;  // column-split kernels: entries per group per trip (0: col_unroll_of)
  // merge-path tiles for one-column Laplacian products (see k_merge_rows):
  // tile_row[t] = rows whose end marker precedes merged item t * kMergeTile
  int64_t ntile = 0;
  int32_t* tile_row = nullptr;   // [ntile + 1]
  int32_t* carry_row = nullptr;  // [ntile] row cut by the tile's end, or -1
  double* carry_val = nullptr;   // [ntile] its partial sum in the tile
  bool merge = false;            // one-column Laplacian products use the merge path
  bool stable = false;           // row lists in increasing row order (not only grouped):
                                 // workgroups then see the same rows on every build
};

// Merge path: the rows' entries and end markers form one list of n + nnz
// items (row r's marker sits at rp[r+1] + r); a workgroup takes kMergeTile
// consecutive items, whatever the degrees.
constexpr int kMergeIPT = 8;
constexpr int64_t kMergeTile = (int64_t)kBlock * kMergeIPT;

// Degree unit of the classes (entries per lane per step of a full-width row).
constexpr int kPerLane = LG_PER_LANE;

// Lanes of a one-column row kernel for class c (see above) at a given shift.
__host__ __device__ constexpr int class_lanes(int c, int shift = 1) {
  return c >= kClasses - 1 ? 64 : (1 << (c > shift ? c - shift : 0));
}

// ------------------------------------------------- profiling (HIP events)
// Times the launches between construction and destruction when family is
// the enabled one.  attached = true: the scope encloses exactly one launch,
// which takes start() and stop() as the events of its own dispatch
// (hipExtLaunchKernelGGL), so the time is the kernel's alone; otherwise the
// events are recorded on the stream around the enclosed work.
bool prof_active();  // true while a kernel family is being timed
bool prof_wants(const char* family);  // that family is being timed

struct ProfScope {
  ProfScope(const char* family, hipStream_t st, double bytes, bool attached = false);
  ~ProfScope();
  hipEvent_t start() const { return on ? a : nullptr; }
  hipEvent_t stop() const { return on ? b : nullptr; }
  bool on;
  bool attached;
  hipStream_t st;
  double bytes;
  hipEvent_t a, b;
};

__host__ __device__ inline int degree_class(int d, int hub_deg) {
  if (d > hub_deg) return kClasses;  // hub or split
  if (d > kPerLane * 64) return kClasses - 1;
  int c = 0;
  while (kPerLane * (1 << c) < d) c++;
  return c;
}

// Whole-row reduction by one workgroup; the epilogue runs on thread 0.
// Entries a lane loads ahead in the row loops: Op::kUnroll if the op sets it
// (ops with wide accumulators trade it for occupancy), else 4.
template <class Op, class = void>
struct op_unroll {
  static constexpr int value = 4;
};
template <class Op>
struct op_unroll<Op, std::void_t<decltype(Op::kUnroll)>> {
  static constexpr int value = Op::kUnroll;
};

// op.accum over the entries e, e + step, ... below end.
template <class Op>
__device__ __forceinline__ void accum_strided(const Op& op, typename Op::Acc& acc, int64_t row,
                                              int e, int end, int step) {
  constexpr int U = op_unroll<Op>::value;
  for (; e + (U - 1) * step < end; e += U * step) {
#pragma unroll
    for (int u = 0; u < U; u++) op.accum(acc, row, e + u * step);
  }
  if constexpr (U > 1)
    for (; e < end; e += step) op.accum(acc, row, e);
}

template <class Op>
__device__ __forceinline__ void block_row(const Op& op, const int32_t* __restrict__ rp,
                                          int64_t row) {
  using Acc = typename Op::Acc;
  Acc acc = op.identity();
  if (op.active(row)) {
    accum_strided(op, acc, row, rp[row] + (int)threadIdx.x, rp[row + 1], kBlock);
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) op.combine(acc, shfl_xor_any(acc, m));
  __shared__ Acc red[kBlock / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    Acc t = red[0];
#pragma unroll
    for (int w = 1; w < kBlock / 64; w++) op.combine(t, red[w]);
    op.finish(row, t, 0, 1);
  }
}

// G lanes per row for the rows perm[pos_begin, pos_end).
template <class Op, int G>
__device__ __forceinline__ void rows_class(const Op& op, const int32_t* __restrict__ rp,
                                           const int32_t* __restrict__ perm, int64_t pos_begin,
                                           int64_t pos_end, int64_t local_block) {
  const int64_t pos = pos_begin + (local_block * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (pos >= pos_end) return;
  const int64_t row = perm[pos];
  typename Op::Acc acc = op.identity();
  if (op.active(row)) {
    accum_strided(op, acc, row, rp[row] + lane, rp[row + 1], G);
#pragma unroll
    for (int m = G / 2; m > 0; m >>= 1) op.combine(acc, shfl_xor_any(acc, m));
  }
  op.finish(row, acc, lane, G);
}

// One chunk of a split row: its partial goes to the chunk's slot; a second
// launch combines each row's partials in chunk order.
template <class Op>
__device__ __forceinline__ void split_chunk(const Op& op, const int32_t* __restrict__ rp,
                                            const int32_t* __restrict__ split_rows,
                                            const int32_t* __restrict__ split_cptr,
                                            const int32_t* __restrict__ chunk_split,
                                            typename Op::Acc* __restrict__ partial, int64_t c) {
  using Acc = typename Op::Acc;
  const int h = chunk_split[c];
  const int64_t row = split_rows[h];
  const int beg = rp[row] + (int)(c - split_cptr[h]) * kHubChunk;
  const int end = min(rp[row + 1], beg + kHubChunk);
  Acc acc = op.identity();
  if (op.active(row)) {
    accum_strided(op, acc, row, beg + (int)threadIdx.x, end, kBlock);
  }
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

// Split rows, phase 2: combine partials in chunk order, run the epilogue.
template <class Op>
__global__ __launch_bounds__(64) void k_split_fix(Op op, const int32_t* __restrict__ split_rows,
                                                  const int32_t* __restrict__ split_cptr,
                                                  const typename Op::Acc* __restrict__ partial,
                                                  int64_t nsplit) {
  const int64_t h = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (h >= nsplit) return;
  const int64_t row = split_rows[h];
  typename Op::Acc acc = op.identity();
  for (int c = split_cptr[h]; c < split_cptr[h + 1]; c++) op.combine(acc, partial[c]);
  op.finish(row, acc, 0, 1);
}

// Ordinary rows run on a persistent grid of workgroups (as many as the chip
// holds at once, see resident_grid) that loop over the logical row blocks:
// short rows make short-lived waves, and re-dispatching them costs more than
// the work they do.  Workgroups are dealt to the 8 XCDs round-robin by index
// and each XCD has its own L2.  The column-split kernels therefore start the
// row region at a multiple of 8 and let XCD x take the x-th contiguous eighth
// of every degree class: neighbouring rows (which share cache lines and, on
// meshes, neighbours) stay in one L2, while each XCD still gets an equal
// share of every class.  The one-column kernels, whose rows are 8 bytes wide,
// keep the plain round-robin order, which measured faster for them.
constexpr int kXcds = 8;

__host__ __device__ inline int64_t round_up8(int64_t v) { return (v + kXcds - 1) / kXcds * kXcds; }

// Calls f(c, q) for the logical blocks q of class c owned by this workgroup.
template <class F>
__device__ __forceinline__ void for_class_blocks(const ClassTable& ct, int64_t b, int64_t slots,
                                                 F&& f) {
  const int64_t x = b % kXcds, s = b / kXcds;
  for (int c = 0; c < kClasses; c++) {
    const int64_t c0 = ct.blk_start[c], nbc = ct.blk_start[c + 1] - c0;
    const int64_t lo = c0 + x * nbc / kXcds, hi = c0 + (x + 1) * nbc / kXcds;
    for (int64_t q = lo + s; q < hi; q += slots) f(c, q - c0);
  }
}

template <class Op>
__global__ __launch_bounds__(kBlock) void k_rows(Op op, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ perm, ClassTable ct,
                                                 int64_t nhub, const int32_t* __restrict__ hub_rows,
                                                 int64_t nchunk, const int32_t* __restrict__ split_rows,
                                                 const int32_t* __restrict__ split_cptr,
                                                 const int32_t* __restrict__ chunk_split,
                                                 typename Op::Acc* __restrict__ partial,
                                                 int shift) {
  int64_t b = blockIdx.x;
  if (b < nchunk) {
    split_chunk(op, rp, split_rows, split_cptr, chunk_split, partial, b);
    return;
  }
  b -= nchunk;
  if (b < nhub) {
    block_row(op, rp, (int64_t)hub_rows[b]);
    return;
  }
  b -= nhub;
  const int64_t pad = round_up8(nchunk + nhub) - nchunk - nhub;
  if (b < pad) return;
  b -= pad;
  const int64_t total = ct.blk_start[kClasses];
  const int64_t stride = (int64_t)gridDim.x - nchunk - nhub - pad;
  for (int64_t q = b; q < total; q += stride) {
    int c = 0;
#pragma unroll
    for (int k = 1; k < kClasses; k++) c += (q >= ct.blk_start[k]) ? 1 : 0;
    const int64_t lb = q - ct.blk_start[c];
    const int64_t p0 = ct.cls_start[c], p1 = ct.cls_start[c + 1];
    switch (class_lanes(c, shift)) {
      case 1: rows_class<Op, 1>(op, rp, perm, p0, p1, lb); break;
      case 2: rows_class<Op, 2>(op, rp, perm, p0, p1, lb); break;
      case 4: rows_class<Op, 4>(op, rp, perm, p0, p1, lb); break;
      case 8: rows_class<Op, 8>(op, rp, perm, p0, p1, lb); break;
      case 16: rows_class<Op, 16>(op, rp, perm, p0, p1, lb); break;
      case 32: rows_class<Op, 32>(op, rp, perm, p0, p1, lb); break;
      default: rows_class<Op, 64>(op, rp, perm, p0, p1, lb); break;
    }
  }
}

// Run Op over every row of the CSR described by (s, rp) on stream st: one launch.
// Workgroups of kBlock threads that the whole chip holds at once for this
// kernel (its occupancy, at most max_per_cu, times the compute units): the
// size of a persistent row grid, so that no workgroup waits for a second
// round.  Computed once per kernel (a kernel takes one max_per_cu).
template <auto Kernel>
inline int64_t resident_grid(int max_per_cu = 1 << 30) {
  static std::atomic<int64_t> cached{0};  // threads that race compute the same value
  int64_t v = cached.load(std::memory_order_relaxed);
  if (v == 0) {
    int per_cu = 0, dev = 0, cus = 0;
    LG_HIP(hipGetDevice(&dev));
    LG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    LG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, Kernel, kBlock, 0));
    v = std::max<int64_t>(1, (int64_t)std::min(per_cu, max_per_cu) * cus);
    cached.store(v, std::memory_order_relaxed);
  }
  return v;
}

// fam/bytes: the kernel-timing family and algorithmic bytes of this product;
// the events enclose the row kernel alone (not the split-row epilogue).
template <class Op>
void run_rows(const Sched& s, const int32_t* rp, const Op& op, hipStream_t st,
              const char* fam = "", double bytes = 0.0) {
  static_assert(sizeof(typename Op::Acc) <= kPartialBytes, "accumulator larger than a partial slot");
  static_assert(sizeof(typename Op::Acc) % 4 == 0, "accumulator size must be a multiple of 4");
  if (s.n == 0) return;
  ClassTable ct = s.ct;
  int64_t total = 0;
  for (int c = 0; c < kClasses; c++) {
    ct.blk_start[c] = (int32_t)total;
    total += ceil_div((int64_t)(s.ct.cls_start[c + 1] - s.ct.cls_start[c]) * class_lanes(c, s.lane_shift),
                      (int64_t)kBlock);
  }
  ct.blk_start[kClasses] = (int32_t)total;
  const int64_t head = round_up8(s.nchunk + s.nhub);
  const int64_t blocks = head + round_up8(std::min<int64_t>(total, resident_grid<k_rows<Op>>()));
  if (blocks == 0) return;
  if (head > 0 && prof_wants("hubs")) {
    // hub and split rows timed as a launch of their own (see run_rows_col)
    {
      ProfScope ps("hubs", st, 0.0, true);
      hipExtLaunchKernelGGL((k_rows<Op>), dim3((unsigned)head), dim3(kBlock), 0, st, ps.start(),
                            ps.stop(), 0, op, rp, (const int32_t*)s.perm, ct, s.nhub,
                            (const int32_t*)s.hub_rows, s.nchunk, (const int32_t*)s.split_rows,
                            (const int32_t*)s.split_cptr, (const int32_t*)s.chunk_split,
                            reinterpret_cast<typename Op::Acc*>(s.partial), s.lane_shift);
    }
    if (blocks > head) {
      ProfScope ps(fam, st, bytes, true);
      hipExtLaunchKernelGGL((k_rows<Op>), dim3((unsigned)(blocks - head)), dim3(kBlock), 0, st,
                            ps.start(), ps.stop(), 0, op, rp, (const int32_t*)s.perm, ct, (int64_t)0,
                            (const int32_t*)s.hub_rows, (int64_t)0, (const int32_t*)s.split_rows,
                            (const int32_t*)s.split_cptr, (const int32_t*)s.chunk_split,
                            reinterpret_cast<typename Op::Acc*>(s.partial), s.lane_shift);
    }
  } else {
    ProfScope ps(fam, st, bytes, true);
    hipExtLaunchKernelGGL((k_rows<Op>), dim3((unsigned)blocks), dim3(kBlock), 0, st, ps.start(),
                          ps.stop(), 0, op, rp, (const int32_t*)s.perm, ct, s.nhub,
                          (const int32_t*)s.hub_rows, s.nchunk, (const int32_t*)s.split_rows,
                          (const int32_t*)s.split_cptr, (const int32_t*)s.chunk_split,
                          reinterpret_cast<typename Op::Acc*>(s.partial), s.lane_shift);
  }
  LG_LAUNCH_CHECK();
  if (s.nsplit) {
    hipLaunchKernelGGL((k_split_fix<Op>), dim3((unsigned)ceil_div(s.nsplit, 64)), dim3(64), 0, st, op,
                       (const int32_t*)s.split_rows, (const int32_t*)s.split_cptr,
                       (const typename Op::Acc*)s.partial, s.nsplit);
    LG_LAUNCH_CHECK();
  }
}

// ----------------------------------------------- column-split row ops
// For k right-hand sides whose row of values spans at least 32 bytes, kL =
// k * sizeof(T) / 16 lanes share each matrix entry and each lane owns one
// 16-byte slice of the k columns (one vector load per entry).  An ordinary row
// is reduced by one such group with no cross-lane sums; a hub row by all the
// groups of a workgroup; a split row by one workgroup per chunk plus a second
// pass.  Op interface: kL, Acc, identity(), active(row),
// accum(acc, row, e, part), combine(a, b), finish(row, acc, part).
//
// Ops with kDot = true also form a dot product per column in the epilogue:
// finish_dot(row, acc, part, pre, d) adds the row's terms for the lane's V
// columns to d[V]; each workgroup sums its lanes' shares in a fixed order
// (dot_store), and split rows keep theirs per row (k_split_fix_col).
template <class Op, class = void>
struct op_dot : std::false_type {};
template <class Op>
struct op_dot<Op, std::void_t<decltype(Op::kDot)>> : std::integral_constant<bool, Op::kDot> {};
template <class Op>
constexpr int dot_width() {
  if constexpr (op_dot<Op>::value) return Op::V;
  else return 1;
}

// Per workgroup: column c = (lane & (kL - 1)) * V + v of the lanes' shares d,
// summed over the workgroup in a fixed order, to out[blockIdx.x * kL * V + c].
template <class Op>
__device__ __forceinline__ void dot_store(const double (&d)[dot_width<Op>()], double* __restrict__ out) {
  if constexpr (op_dot<Op>::value) {
    constexpr int V = Op::V, K = Op::kL * Op::V;
    __shared__ double sm[kBlock * V];
#pragma unroll
    for (int v = 0; v < V; v++) sm[threadIdx.x * V + v] = d[v];
    __syncthreads();
    if ((int)threadIdx.x < K) {
      double t = 0.0;
      for (int q = threadIdx.x; q < kBlock * V; q += K) t += sm[q];
      out[(int64_t)blockIdx.x * K + threadIdx.x] = t;
    }
  }
}

// M groups of kL lanes per row for the rows perm[p0, p1): group g takes entries
// beg + g, beg + g + M, ... (U per trip); the groups' sums are combined by a
// butterfly.
template <class Op, int M, int U>
__device__ __forceinline__ void col_rows(const Op& op, const int32_t* __restrict__ rp,
                                         const int32_t* __restrict__ perm, int64_t p0, int64_t p1,
                                         int64_t lb, double (&dacc)[dot_width<Op>()]) {
  constexpr int L = Op::kL, T = L * M;
  const int64_t pos = p0 + (lb * kBlock + threadIdx.x) / T;
  const int part = threadIdx.x & (L - 1);
  const int grp = (threadIdx.x / L) & (M - 1);
  if (pos >= p1) return;
  const int64_t row = perm[pos];
  typename Op::Pre pre;
  if (grp == 0) pre = op.prefetch(row, part);
  typename Op::Acc acc = op.identity();
  if (op.active(row)) {
    const int end = rp[row + 1];
    // U entries per trip, all loads issued together: slots past the row's end
    // re-read its last entry with weight zero (adding +-0 to a sum that
    // started at +0 leaves its bits unchanged)
    for (int e = rp[row] + grp; e < end; e += U * M) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int eu = e + u * M;
        op.accum(acc, row, eu < end ? eu : end - 1, part, eu < end);
      }
    }
#pragma unroll
    for (int m = T / 2; m >= L; m >>= 1) op.combine(acc, shfl_xor_any(acc, m));
  }
  if (grp == 0) {
    if constexpr (op_dot<Op>::value) op.finish_dot(row, acc, part, pre, dacc);
    else op.finish(row, acc, part, pre);
  }
}

// Entries [beg, end) of `row` by all kBlock / kL groups of the workgroup; the
// per-part totals end up on threads 0 .. kL-1 (returned there, identity elsewhere).
template <class Op>
__device__ __forceinline__ typename Op::Acc col_block_reduce(const Op& op, int64_t row, int beg,
                                                             int end) {
  using Acc = typename Op::Acc;
  constexpr int L = Op::kL, NG = kBlock / L;
  const int grp = threadIdx.x / L, part = threadIdx.x & (L - 1);
  Acc acc = op.identity();
  if (op.active(row)) {
    int e = beg + grp;
    for (; e + 3 * NG < end; e += 4 * NG) {
      op.accum(acc, row, e, part);
      op.accum(acc, row, e + NG, part);
      op.accum(acc, row, e + 2 * NG, part);
      op.accum(acc, row, e + 3 * NG, part);
    }
    for (; e < end; e += NG) op.accum(acc, row, e, part);
  }
#pragma unroll
  for (int m = 32; m >= L; m >>= 1) op.combine(acc, shfl_xor_any(acc, m));
  __shared__ Acc red[kBlock / 64][L];
  if ((threadIdx.x & 63) < L) red[threadIdx.x >> 6][threadIdx.x & 63] = acc;
  __syncthreads();
  Acc t = op.identity();
  if (threadIdx.x < L) {
    t = red[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kBlock / 64; w++) op.combine(t, red[w][threadIdx.x]);
  }
  return t;
}

// dotp (ops with kDot): each workgroup's column sums of the epilogue's dot
// terms, kL * V per workgroup (zero for chunk and padding workgroups).
template <class Op, int U>
__global__ __launch_bounds__(kBlock) void k_rows_col(Op op, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ perm,
                                                     ClassTable ct, int64_t nhub,
                                                     const int32_t* __restrict__ hub_rows,
                                                     int64_t nchunk,
                                                     const int32_t* __restrict__ split_rows,
                                                     const int32_t* __restrict__ split_cptr,
                                                     const int32_t* __restrict__ chunk_split,
                                                     typename Op::Acc* __restrict__ partial,
                                                     int shift, double* __restrict__ dotp) {
  constexpr int L = Op::kL;
  double dacc[dot_width<Op>()] = {};
  int64_t b = blockIdx.x;
  if (b < nchunk) {
    const int h = chunk_split[b];
    const int64_t row = split_rows[h];
    const int beg = rp[row] + (int)(b - split_cptr[h]) * kHubChunk;
    const int end = min(rp[row + 1], beg + kHubChunk);
    const typename Op::Acc t = col_block_reduce(op, row, beg, end);
    if (threadIdx.x < L) partial[b * L + threadIdx.x] = t;
    dot_store<Op>(dacc, dotp);
    return;
  }
  b -= nchunk;
  if (b < nhub) {
    const int64_t row = hub_rows[b];
    const typename Op::Acc t = col_block_reduce(op, row, rp[row], rp[row + 1]);
    if (threadIdx.x < L) {
      if constexpr (op_dot<Op>::value)
        op.finish_dot(row, t, (int)threadIdx.x, op.prefetch(row, (int)threadIdx.x), dacc);
      else
        op.finish(row, t, (int)threadIdx.x);
    }
    dot_store<Op>(dacc, dotp);
    return;
  }
  b -= nhub;
  const int64_t pad = round_up8(nchunk + nhub) - nchunk - nhub;
  if (b < pad) {
    dot_store<Op>(dacc, dotp);
    return;
  }
  b -= pad;
  const int64_t slots = ((int64_t)gridDim.x - nchunk - nhub - pad) / kXcds;
  constexpr int MM = 64 / L;  // most groups a row may span inside one wavefront
  for_class_blocks(ct, b, slots, [&](int c, int64_t lb) {
    const int64_t p0 = ct.cls_start[c], p1 = ct.cls_start[c + 1];
    switch (c >= kClasses - 1 ? 0 : min(class_lanes(c, shift), MM)) {
      case 1: col_rows<Op, 1, U>(op, rp, perm, p0, p1, lb, dacc); break;
      case 2: col_rows<Op, (2 < MM ? 2 : MM), U>(op, rp, perm, p0, p1, lb, dacc); break;
      case 4: col_rows<Op, (4 < MM ? 4 : MM), U>(op, rp, perm, p0, p1, lb, dacc); break;
      case 8: col_rows<Op, (8 < MM ? 8 : MM), U>(op, rp, perm, p0, p1, lb, dacc); break;
      case 16: col_rows<Op, (16 < MM ? 16 : MM), U>(op, rp, perm, p0, p1, lb, dacc); break;
      case 32: col_rows<Op, (32 < MM ? 32 : MM), U>(op, rp, perm, p0, p1, lb, dacc); break;
      default: {  // one workgroup per row (class 7)
        const int64_t row = perm[p0 + lb];
        const typename Op::Acc t = col_block_reduce(op, row, rp[row], rp[row + 1]);
        if (threadIdx.x < L) {
          if constexpr (op_dot<Op>::value)
            op.finish_dot(row, t, (int)threadIdx.x, op.prefetch(row, (int)threadIdx.x), dacc);
          else
            op.finish(row, t, (int)threadIdx.x);
        }
        __syncthreads();  // the next row reuses the reduction buffer
        break;
      }
    }
  });
  dot_store<Op>(dacc, dotp);
}

// dotp (ops with kDot): the dot terms of split row h at dotp[h * kL * V + ...].
template <class Op>
__global__ __launch_bounds__(64) void k_split_fix_col(Op op, const int32_t* __restrict__ split_rows,
                                                      const int32_t* __restrict__ split_cptr,
                                                      const typename Op::Acc* __restrict__ partial,
                                                      int64_t nsplit, double* __restrict__ dotp) {
  constexpr int L = Op::kL;
  const int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (t >= nsplit * L) return;
  const int64_t h = t / L;
  const int part = (int)(t % L);
  typename Op::Acc acc = op.identity();
  for (int c = split_cptr[h]; c < split_cptr[h + 1]; c++) op.combine(acc, partial[(int64_t)c * L + part]);
  const int64_t row = split_rows[h];
  if constexpr (op_dot<Op>::value) {
    double d[Op::V] = {};
    op.finish_dot(row, acc, part, op.prefetch(row, part), d);
#pragma unroll
    for (int v = 0; v < Op::V; v++) dotp[(h * L + part) * Op::V + v] = d[v];
  } else {
    op.finish(row, acc, part);
  }
}

// Persistent grid of a column-split kernel: at most kColMaxPerCu workgroups
// (one wavefront per SIMD each) per compute unit.  With more rows in flight
// the gathers ran slower (measured: the 4M-vertex power-law product at 16
// fp64 columns, occupancy 8 against 7), as they evict x rows that other rows
// reuse.
constexpr int kColMaxPerCu = 7;
template <class Op, int U>
int64_t col_grid() {
  return resident_grid<k_rows_col<Op, U>>(kColMaxPerCu);
}

// Returns the workgroups launched.  dotp (ops with kDot): their dot partials,
// followed by those of the split rows (see dot_partials).
template <class Op, int U>
int64_t run_rows_col_u(const Sched& s, const int32_t* rp, const Op& op, hipStream_t st,
                       const char* fam, double bytes, double* dotp) {
  constexpr int L = Op::kL;
  static_assert(sizeof(typename Op::Acc) * L <= kPartialBytes, "partial slot too small");
  if (s.n == 0) return 0;
  ClassTable ct = s.ct;
  int64_t blk = 0;
  for (int c = 0; c < kClasses; c++) {
    ct.blk_start[c] = (int32_t)blk;
    const int64_t rows = s.ct.cls_start[c + 1] - s.ct.cls_start[c];
    const int64_t M = std::min<int64_t>(class_lanes(c, s.col_shift), 64 / L);
    blk += c == kClasses - 1 ? rows : ceil_div(rows * L * M, kBlock);
  }
  ct.blk_start[kClasses] = (int32_t)blk;
  const int64_t head = round_up8(s.nchunk + s.nhub);
  const int64_t blocks = head + round_up8(std::min<int64_t>(blk, col_grid<Op, U>()));
  if (blocks == 0) return 0;
  if (head > 0 && prof_wants("hubs")) {
    // timing the hub and split rows: their workgroups as a launch of their
    // own (family "hubs"), then the class rows; every row is reduced as in
    // the single launch
    {
      ProfScope ps("hubs", st, 0.0, true);
      hipExtLaunchKernelGGL((k_rows_col<Op, U>), dim3((unsigned)head), dim3(kBlock), 0, st, ps.start(),
                            ps.stop(), 0, op, rp, (const int32_t*)s.perm, ct, s.nhub,
                            (const int32_t*)s.hub_rows, s.nchunk, (const int32_t*)s.split_rows,
                            (const int32_t*)s.split_cptr, (const int32_t*)s.chunk_split,
                            reinterpret_cast<typename Op::Acc*>(s.partial), s.col_shift, dotp);
    }
    if (blocks > head) {
      ProfScope ps(fam, st, bytes, true);
      hipExtLaunchKernelGGL((k_rows_col<Op, U>), dim3((unsigned)(blocks - head)), dim3(kBlock), 0, st,
                            ps.start(), ps.stop(), 0, op, rp, (const int32_t*)s.perm, ct, (int64_t)0,
                            (const int32_t*)s.hub_rows, (int64_t)0, (const int32_t*)s.split_rows,
                            (const int32_t*)s.split_cptr, (const int32_t*)s.chunk_split,
                            reinterpret_cast<typename Op::Acc*>(s.partial), s.col_shift,
                            dotp ? dotp + head * (int64_t)L * dot_width<Op>() : nullptr);
    }
  } else {
    ProfScope ps(fam, st, bytes, true);
    hipExtLaunchKernelGGL((k_rows_col<Op, U>), dim3((unsigned)blocks), dim3(kBlock), 0, st, ps.start(),
                          ps.stop(), 0, op, rp, (const int32_t*)s.perm, ct, s.nhub,
                          (const int32_t*)s.hub_rows, s.nchunk, (const int32_t*)s.split_rows,
                          (const int32_t*)s.split_cptr, (const int32_t*)s.chunk_split,
                          reinterpret_cast<typename Op::Acc*>(s.partial), s.col_shift, dotp);
  }
  LG_LAUNCH_CHECK();
  if (s.nsplit) {
    hipLaunchKernelGGL((k_split_fix_col<Op>), dim3((unsigned)ceil_div(s.nsplit * L, 64)), dim3(64), 0,
                       st, op, (const int32_t*)s.split_rows, (const int32_t*)s.split_cptr,
                       (const typename Op::Acc*)s.partial, s.nsplit,
                       dotp ? dotp + blocks * (int64_t)L * dot_width<Op>() : nullptr);
    LG_LAUNCH_CHECK();
  }
  return blocks;
}

// The column-split product of Op over schedule s, at the schedule's unroll.
template <class Op>
int64_t run_rows_col(const Sched& s, const int32_t* rp, const Op& op, hipStream_t st,
                     const char* fam = "", double bytes = 0.0, double* dotp = nullptr) {
  if ((s.col_unroll ? s.col_unroll : col_unroll_of<Op>()) == 4)
    return run_rows_col_u<Op, 4>(s, rp, op, st, fam, bytes, dotp);
  return run_rows_col_u<Op, 6>(s, rp, op, st, fam, bytes, dotp);
}

// Workgroups of Op's column-split kernel resident on the device at s's unroll.
template <class Op>
int64_t col_resident(const Sched& s) {
  return (s.col_unroll ? s.col_unroll : col_unroll_of<Op>()) == 4 ? col_grid<Op, 4>() : col_grid<Op, 6>();
}

// Dot partials of one run_rows_col launch on schedule s: at most this many
// rows of k columns (workgroups, then split rows).
inline int64_t dot_partials(const Sched& s, int64_t resident) {
  return round_up8(s.nchunk + s.nhub) + round_up8(resident) + s.nsplit;
}

// ------------------------------------------------------------ merge path
// One-column products over a fixed share of the merged list per workgroup
// (Merrill & Garland's merge-based CSR traversal): the tile's products
// w_e x_col(e) are staged in LDS by coalesced loads, each thread walks
// kMergeIPT items and finishes the rows whose entries it saw entirely; rows
// cut between threads get the earlier threads' partial sums from a segmented
// scan; a row cut by the tile's end is finished by its last tile and the
// earlier tiles' partials are added by k_merge_fix, through the epilogue's
// slope (every Laplacian epilogue is affine in the row sum).  All partitions
// and orders are fixed, so results are deterministic.
// Op: Val, term(e), slope(row), finish(row, acc, 0, 1), identity().
template <class Op>
__global__ __launch_bounds__(kBlock) void k_merge_rows(Op op, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ tile_row,
                                                       int64_t n, int64_t nnz,
                                                       int32_t* __restrict__ carry_row,
                                                       double* __restrict__ carry_val) {
  using T = typename Op::Val;
  __shared__ T prod[kMergeTile];
  __shared__ int32_t mpos[kMergeTile];
  __shared__ T sv[2][kBlock];
  __shared__ int32_t sf[2][kBlock];
  const int64_t t = blockIdx.x;
  const int64_t d0 = t * kMergeTile, d1 = min(d0 + kMergeTile, n + nnz);
  const int64_t i0 = tile_row[t], i1 = tile_row[t + 1];
  const int64_t j0 = d0 - i0, j1 = d1 - i1;
  for (int64_t e = j0 + threadIdx.x; e < j1; e += kBlock) prod[e - j0] = op.term((int)e);
  for (int64_t r = i0 + threadIdx.x; r < i1; r += kBlock) mpos[r - i0] = (int32_t)(rp[r + 1] + r - d0);
  __syncthreads();
  // this thread's items [dk, dk1) and its starting row: markers before dk
  const int rel0 = (int)min((int64_t)threadIdx.x * kMergeIPT, d1 - d0);
  const int rel1 = (int)min((int64_t)rel0 + kMergeIPT, d1 - d0);
  int lo = 0, hi = (int)(i1 - i0);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (mpos[mid] < rel0) lo = mid + 1;
    else hi = mid;
  }
  int i = lo;                      // row index within the tile
  int j = rel0 - lo;               // entry index within the tile (items = rows + entries)
  const int first = i;
  T run = T(0), first_sum = T(0);
  bool ended = false;
  typename Op::Acc acc;
  for (int pos = rel0; pos < rel1; pos++) {
    if (i < (int)(i1 - i0) && mpos[i] == pos) {  // row i ends here
      if (!ended) {
        first_sum = run;
        ended = true;
      } else {  // started and ended inside this thread: complete
        acc = op.identity();
        acc.v[0] = run;
        op.finish(i0 + i, acc, 0, 1);
      }
      run = T(0);
      i++;
    } else {
      run += prod[j];
      j++;
    }
  }
  // segmented inclusive scan of the threads' trailing partials, keyed by row
  const int k = threadIdx.x;
  int buf = 0;
  sv[0][k] = run;
  sf[0][k] = i;  // the row the trailing partial belongs to
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    T v = sv[buf][k];
    if (k >= o && sf[buf][k - o] == sf[buf][k]) v += sv[buf][k - o];
    sv[buf ^ 1][k] = v;
    sf[buf ^ 1][k] = sf[buf][k];
    buf ^= 1;
    __syncthreads();
  }
  // rows whose entries began in earlier threads of this tile
  if (ended) {
    const T carry_in = (k > 0 && sf[buf][k - 1] == first) ? sv[buf][k - 1] : T(0);
    acc = op.identity();
    acc.v[0] = first_sum + carry_in;
    op.finish(i0 + first, acc, 0, 1);
  }
  if (k == kBlock - 1) {
    const bool cut = i1 < n;  // row i1 continues into the next tile
    carry_row[t] = cut ? (int32_t)i1 : -1;
    carry_val[t] = cut ? (double)sv[buf][k] : 0.0;
  }
}

// Rows cut by tile ends: add the earlier tiles' partials (in tile order) to
// the row the following tile finished.
template <class Op>
__global__ void k_merge_fix(Op op, const int32_t* __restrict__ carry_row,
                            const double* __restrict__ carry_val, int64_t ntile) {
  using T = typename Op::Val;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= ntile) return;
  const int32_t r = carry_row[t];
  if (r < 0 || (t > 0 && carry_row[t - 1] == r)) return;
  double s = 0.0;
  for (int64_t u = t; u < ntile && carry_row[u] == r; u++) s += carry_val[u];
  op.add_to_row(r, (T)s);
}

template <class Op>
void run_merge(const Sched& s, const int32_t* rp, const Op& op, hipStream_t st,
               const char* fam = "", double bytes = 0.0) {
  if (s.n == 0 || s.ntile == 0) return;
  {
    ProfScope ps(fam, st, bytes, true);
    hipExtLaunchKernelGGL((k_merge_rows<Op>), dim3((unsigned)s.ntile), dim3(kBlock), 0, st,
                          ps.start(), ps.stop(), 0, op, rp, (const int32_t*)s.tile_row, s.n, s.nnz,
                          s.carry_row, s.carry_val);
  }
  LG_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_merge_fix<Op>), dim3((unsigned)ceil_div(s.ntile, (int64_t)kBlock)),
                     dim3(kBlock), 0, st, op, (const int32_t*)s.carry_row,
                     (const double*)s.carry_val, s.ntile);
  LG_LAUNCH_CHECK();
}

// ------------------------------------------------------------- memory
// Bump allocator over large device chunks.  The hierarchy owns one for its
// lifetime; setup uses a second one for temporaries and rewinds it per level.
// Released chunks go to a process-wide cache (bounded) that later arenas on
// the same device draw from before calling hipMalloc.
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
    int dev;
  };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0, off_ = 0, total_ = 0, chunk_;
};

// Setup temporaries live in arenas that are reused across lg_setup calls
// (a pool, so concurrent setups on different threads do not share one).
Arena* acquire_temp_arena();
void release_temp_arena(Arena* a);
struct TempArena {
  TempArena() : a(acquire_temp_arena()) {}
  ~TempArena() { release_temp_arena(a); }
  TempArena(const TempArena&) = delete;
  TempArena& operator=(const TempArena&) = delete;
  Arena* a;
};


// ------------------------------------------------------------- helpers
// Row statistics behind a schedule: max degree, min degree, 8 class counts,
// hubs, split rows, split chunks (and spare slots).
constexpr int kStat = 16;

// Row schedule of the CSR (rp, n rows, nnz entries): statistics, read back,
// layout.  tiles: also the merge-path tiles (level matrices whose one-column
// products may take the merge path).
void build_sched(Sched& s, const int32_t* rp, int64_t n, int64_t nnz, Arena& keep, Arena& tmp,
                 hipStream_t st, bool tiles = false, bool stable = false);
// The two halves, for callers that read the statistics together with other
// values: sched_stats launches the kernels that fill kStat ints (returned, on
// the device, in tmp; n_dev optionally holds the actual row count <= n) and
// sched_layout builds the schedule from those ints once they are on the host.
int* sched_stats(const int32_t* rp, int64_t n, const int64_t* n_dev, Arena& tmp, hipStream_t st);
void sched_layout(Sched& s, const int* t, const int32_t* rp, int64_t n, int64_t nnz, bool tiles,
                  Arena& keep, Arena& tmp, hipStream_t st, bool stable = false);
void sched_fill(Sched& s, const int32_t* rp, Arena& tmp, hipStream_t st);
// out[i] = sum_{j<i} in[j] for i <= n (out has n+1 entries); returns out[n] on the host
// when want_total (synchronises the stream).
int64_t scan_i64(const int64_t* in, int64_t* out, int64_t n, Arena& tmp, hipStream_t st,
                 bool want_total);
int64_t scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, Arena& tmp, hipStream_t st,
                        bool want_total);
// Stable LSD radix sort of (key, val) pairs over the listed 8-bit digit shifts.
// pack > 0: keys are (hi << 32 | lo) with hi, lo < 2^pack and the shifts index
// the packed value (hi << pack | lo) (see pair_shifts).  The sorted pairs are
// left either in the input arrays or in two arrays taken from tmp (which stay
// allocated until the caller rewinds tmp); the result says where.
struct SortedPairs {
  uint64_t* keys;
  uint64_t* vals;
};
SortedPairs radix_sort_pairs(uint64_t* keys, uint64_t* vals, int64_t n,
                             const std::vector<int>& shifts, Arena& tmp, hipStream_t st,
                             int pack = 0);
std::vector<int> pair_shifts(int bits);  // digits of a packed pair of two bits-wide halves
std::vector<int> digit_shifts(int bits_lo, int bits_hi);  // digits covering [0,bits_lo) and [32,32+bits_hi)
int bits_for(int64_t max_value);
int64_t read_i64(const int64_t* dev, hipStream_t st);
void read_dev(void* host, const void* dev, size_t bytes, hipStream_t st);
// Several small device values in one round trip (up to 4 segments of whole,
// 4-byte aligned words; waits for the work queued on st before them).
struct DevRead {
  void* host;
  const void* dev;
  size_t bytes;
};
void read_dev_n(const DevRead* r, int count, hipStream_t st);

}  // namespace lg
