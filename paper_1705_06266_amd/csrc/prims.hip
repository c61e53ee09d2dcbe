// prims.hip -- device primitives shared by the setup passes: exclusive scans,
// a stable LSD radix sort of (key, payload) pairs, the row scheduler, the
// device arena and the HIP-event profiler behind lg_profile_*.
#include <cstring>
#include <atomic>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace lg {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

[[noreturn]] void fail(lg_status code, const std::string& msg) { throw Error{code, msg}; }

// ------------------------------------------------------------------ arena
// Device chunks of released arenas are kept, up to chunk_cache_cap() bytes
// per process (a sixteenth of the device's memory, at least 4 GB), and
// handed to later arenas on the same device: hipMalloc and hipFree of tens of
// megabytes cost tens to hundreds of microseconds each, which a setup that
// follows a release (a serving loop, a benchmark) would otherwise pay every
// time.  A cached chunk serves a request of at least 4/5 of its size.  When
// hipMalloc fails, the device's cached chunks are freed and it is tried once
// more.
namespace {
struct CachedChunk {
  char* p;
  size_t size;
  int dev;
};
std::mutex g_chunk_mu;
std::vector<CachedChunk> g_chunk_cache;
size_t g_chunk_cache_bytes = 0;

size_t chunk_cache_cap() {
  static std::atomic<size_t> cap{0};  // threads that race compute the same value
  size_t v = cap.load(std::memory_order_relaxed);
  if (v == 0) {
    int dev = 0;
    size_t total = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceTotalMem(&total, dev) != hipSuccess) total = 0;
    v = std::max((size_t)4 << 30, total / 16);
    cap.store(v, std::memory_order_relaxed);
  }
  return v;
}

// Frees the cached chunks of device dev (no queued work uses them: a chunk
// enters the cache after a device synchronisation); false if there were none.
bool chunk_flush(int dev) {
  std::lock_guard<std::mutex> g(g_chunk_mu);
  bool any = false;
  for (size_t k = 0; k < g_chunk_cache.size();) {
    if (g_chunk_cache[k].dev == dev) {
      (void)hipFree(g_chunk_cache[k].p);
      g_chunk_cache_bytes -= g_chunk_cache[k].size;
      g_chunk_cache.erase(g_chunk_cache.begin() + k);
      any = true;
    } else {
      k++;
    }
  }
  return any;
}

char* chunk_take(size_t want, int dev, size_t* got) {
  std::lock_guard<std::mutex> g(g_chunk_mu);
  int best = -1;
  for (size_t k = 0; k < g_chunk_cache.size(); k++) {
    const CachedChunk& c = g_chunk_cache[k];
    if (c.dev == dev && c.size >= want && c.size - want <= want / 4 &&
        (best < 0 || c.size < g_chunk_cache[best].size))
      best = (int)k;
  }
  if (best < 0) return nullptr;
  const CachedChunk c = g_chunk_cache[best];
  g_chunk_cache.erase(g_chunk_cache.begin() + best);
  g_chunk_cache_bytes -= c.size;
  *got = c.size;
  return c.p;
}
}  // namespace

void* Arena::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  while (cur_ < chunks_.size()) {
    Chunk& c = chunks_[cur_];
    if (off_ + bytes <= c.size) {
      void* p = c.p + off_;
      off_ += bytes;
      return p;
    }
    cur_++;
    off_ = 0;
  }
  size_t sz = bytes > chunk_ ? bytes : chunk_;
  int dev = 0;
  LG_HIP(hipGetDevice(&dev));
  size_t got = 0;
  char* p = chunk_take(sz, dev, &got);
  if (p) {
    sz = got;
  } else {
    hipError_t e = hipMalloc((void**)&p, sz);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      if (chunk_flush(dev)) e = hipMalloc((void**)&p, sz);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(LG_E_NOMEM, "device allocation of " + std::to_string(sz) + " bytes failed");
    }
  }
  chunks_.push_back({p, sz, dev});
  total_ += sz;
  cur_ = chunks_.size() - 1;
  off_ = bytes;
  return p;
}

void Arena::release() {
  if (chunks_.empty()) return;
  int dev = -1;
  (void)hipGetDevice(&dev);
  // work still queued on the device may use the memory: wait for it, as
  // hipFree would, before another arena can take a chunk
  bool synced = false;
  for (auto& c : chunks_) {
    bool keep = false;
    if (c.dev == dev) {
      std::lock_guard<std::mutex> g(g_chunk_mu);
      keep = g_chunk_cache_bytes + c.size <= chunk_cache_cap();
      if (keep) g_chunk_cache_bytes += c.size;  // reserved; the chunk is added below
    }
    if (!keep) {
      (void)hipFree(c.p);
      continue;
    }
    if (!synced) {
      (void)hipDeviceSynchronize();
      synced = true;
    }
    std::lock_guard<std::mutex> g(g_chunk_mu);
    g_chunk_cache.push_back({c.p, c.size, c.dev});
  }
  chunks_.clear();
  cur_ = off_ = total_ = 0;
}

namespace {
std::mutex g_pool_mu;
std::vector<Arena*> g_pool;
}  // namespace

Arena* acquire_temp_arena() {
  std::lock_guard<std::mutex> g(g_pool_mu);
  if (!g_pool.empty()) {
    Arena* a = g_pool.back();
    g_pool.pop_back();
    a->rewind({0, 0});
    return a;
  }
  return new Arena((size_t)256 << 20);
}

void release_temp_arena(Arena* a) {
  std::lock_guard<std::mutex> g(g_pool_mu);
  a->rewind({0, 0});
  g_pool.push_back(a);
}

// ---------------------------------------------------------------- profiler
namespace {
struct Prof {
  std::mutex mu;
  std::atomic<bool> enabled{false};  // checked without the lock on every launch
  std::vector<std::string> families;  // the enabled families
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<double> pending_bytes;
  std::vector<hipEvent_t> pool;
  int64_t launches = 0;
  double ms = 0.0, bytes = 0.0;
};
Prof& prof() {
  static Prof p;
  return p;
}
hipEvent_t take_event(Prof& p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  LG_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace

bool prof_active() { return prof().enabled.load(std::memory_order_relaxed); }

bool prof_wants(const char* family) {
  Prof& p = prof();
  if (!p.enabled.load(std::memory_order_relaxed)) return false;
  std::lock_guard<std::mutex> g(p.mu);
  return std::find(p.families.begin(), p.families.end(), family) != p.families.end();
}

ProfScope::ProfScope(const char* family, hipStream_t s, double b, bool att)
    : on(false), attached(att), st(s), bytes(b) {
  Prof& p = prof();
  if (!p.enabled.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> g(p.mu);
  if (std::find(p.families.begin(), p.families.end(), family) == p.families.end()) return;
  a = take_event(p);
  this->b = take_event(p);
  if (!attached) LG_HIP(hipEventRecord(a, st));
  on = true;
}

ProfScope::~ProfScope() {
  if (!on) return;
  Prof& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  if (!attached) (void)hipEventRecord(b, st);
  p.pending.push_back({a, b});
  p.pending_bytes.push_back(bytes);
}

}  // namespace lg

extern "C" lg_status lg_profile_enable(const char* family) {
  auto& p = lg::prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.families.clear();
  if (family) {
    std::string f;
    for (const char* c = family;; c++) {
      if (*c == ',' || *c == '\0') {
        if (!f.empty()) p.families.push_back(f);
        f.clear();
        if (*c == '\0') break;
      } else {
        f.push_back(*c);
      }
    }
  }
  p.enabled.store(!p.families.empty());
  p.launches = 0;
  p.ms = p.bytes = 0.0;
  return LG_OK;
}

extern "C" lg_status lg_profile_read(int64_t* launches, double* total_ms, double* total_bytes) {
  auto& p = lg::prof();
  std::lock_guard<std::mutex> g(p.mu);
  for (size_t i = 0; i < p.pending.size(); i++) {
    float ms = 0.f;
    if (hipEventSynchronize(p.pending[i].second) != hipSuccess ||
        hipEventElapsedTime(&ms, p.pending[i].first, p.pending[i].second) != hipSuccess) {
      lg::set_last_error("profiler event query failed");
      return LG_E_HIP;
    }
    p.ms += ms;
    p.bytes += p.pending_bytes[i];
    p.launches++;
    p.pool.push_back(p.pending[i].first);
    p.pool.push_back(p.pending[i].second);
  }
  p.pending.clear();
  p.pending_bytes.clear();
  if (launches) *launches = p.launches;
  if (total_ms) *total_ms = p.ms;
  if (total_bytes) *total_bytes = p.bytes;
  p.launches = 0;
  p.ms = p.bytes = 0.0;
  return LG_OK;
}

extern "C" const char* lg_profile_names(void) {
  return "spmv,lanczos,spmm,resid64,cg_update,cheb0,cheb1,cheb,resid,spmm_inner,restrict,prolong,coarse,"
         "hubs,jacobi_xsum,row_xsum,affinity,vote,elim_select,radix,galerkin_reduce";
}

namespace lg {

// ------------------------------------------------------------------- scan
// Reduce-then-scan over tiles of kScanTile items; each thread owns kScanIPT
// consecutive items, moved with 16-byte vector loads and stores when the
// buffers are 16-byte aligned.  Pass 1 writes tile sums; pass 2 writes
// out[i] = tile offset + in-tile prefix, each workgroup summing the tile sums
// before its own (up to kScanFuse tiles; beyond that the sums are scanned
// recursively first).
constexpr int kScanIPT = 8;
constexpr int kScanTile = kBlock * kScanIPT;

template <typename TI>
__device__ __forceinline__ void scan_load8(const TI* __restrict__ in, int64_t i0, int64_t n,
                                           bool vec, int64_t v[kScanIPT]) {
  if (vec && i0 + kScanIPT <= n) {
    if constexpr (sizeof(TI) == 4) {
      const int4* p = reinterpret_cast<const int4*>(in + i0);
      const int4 a = p[0], b = p[1];
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
      v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
      const longlong2* p = reinterpret_cast<const longlong2*>(in + i0);
#pragma unroll
      for (int k = 0; k < kScanIPT / 2; k++) {
        const longlong2 a = p[k];
        v[2 * k] = a.x;
        v[2 * k + 1] = a.y;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanIPT; k++) v[k] = i0 + k < n ? (int64_t)in[i0 + k] : 0;
  }
}

// Block-wide sum of one value per thread (valid in every thread).
__device__ __forceinline__ int64_t block_sum_i64(int64_t x, int64_t* wsum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if (lane == 0) wsum[w] = x;
  __syncthreads();
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; k++) s += wsum[k];
  return s;
}

template <typename TI>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const TI* __restrict__ in, int64_t n,
                                                        bool vec, int64_t* __restrict__ sums) {
  __shared__ int64_t wsum[kBlock / 64];
  int64_t v[kScanIPT];
  scan_load8(in, (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT, n, vec, v);
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanIPT; k++) s += v[k];
  s = block_sum_i64(s, wsum);
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

// A tile's offset: offs[tile] if offs is set, else the sum of sums[0, tile)
// formed by the workgroup itself if sums is set (at most kScanFuse tiles),
// else 0 (a single tile).  The last tile also writes out[n], the total.
constexpr int kScanFuse = 4 * kBlock;

template <typename TI>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const TI* __restrict__ in,
                                                       int64_t* __restrict__ out, int64_t n,
                                                       bool vec, const int64_t* __restrict__ offs,
                                                       const int64_t* __restrict__ sums) {
  __shared__ int64_t wsum[kBlock / 64];
  __shared__ int64_t wbase[kBlock / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int64_t base = 0;
  if (offs) {
    base = offs[blockIdx.x];
  } else if (sums) {
    int64_t p = 0;
    for (int k = t; k < (int)blockIdx.x; k += kBlock) p += sums[k];
    base = block_sum_i64(p, wbase);
  }
  const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanIPT;
  int64_t v[kScanIPT];
  scan_load8(in, i0, n, vec, v);
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanIPT; k++) s += v[k];
  int64_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int64_t run = base;
  for (int k = 0; k < w; k++) run += wsum[k];
  run += x - s;
  int64_t r[kScanIPT];
#pragma unroll
  for (int k = 0; k < kScanIPT; k++) {
    r[k] = run;
    run += v[k];
  }
  if (vec && i0 + kScanIPT <= n) {
    longlong2* p = reinterpret_cast<longlong2*>(out + i0);
#pragma unroll
    for (int k = 0; k < kScanIPT / 2; k++) p[k] = make_longlong2(r[2 * k], r[2 * k + 1]);
  } else {
#pragma unroll
    for (int k = 0; k < kScanIPT; k++)
      if (i0 + k < n) out[i0 + k] = r[k];
  }
  if (blockIdx.x == gridDim.x - 1 && t == kBlock - 1) out[n] = run;
}

__global__ void k_zero_i64(int64_t* dst) { *dst = 0; }

template <typename TI>
static void scan_core(const TI* in, int64_t* out, int64_t n, Arena& tmp, hipStream_t st) {
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, st, out);
    return;
  }
  const int64_t nb = ceil_div(n, kScanTile);
  const bool vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  const int64_t* offs = nullptr;
  int64_t* sums = nullptr;
  if (nb > 1) {
    sums = tmp.get<int64_t>(nb);
    hipLaunchKernelGGL((k_scan_reduce<TI>), dim3((unsigned)nb), dim3(kBlock), 0, st, in, n, vec,
                       sums);
    LG_LAUNCH_CHECK();
    if (nb > kScanFuse) {
      // too many tiles for each workgroup to sum its predecessors: scan the sums
      int64_t* o = tmp.get<int64_t>(nb + 1);
      scan_core<int64_t>(sums, o, nb, tmp, st);
      offs = o;
      sums = nullptr;
    }
  }
  hipLaunchKernelGGL((k_scan_tiles<TI>), dim3((unsigned)nb), dim3(kBlock), 0, st, in, out, n, vec,
                     offs, sums);
  LG_LAUNCH_CHECK();
}

int64_t read_i64(const int64_t* dev, hipStream_t st) {
  int64_t v = 0;
  read_dev(&v, dev, sizeof(v), st);
  return v;
}

int64_t scan_i64(const int64_t* in, int64_t* out, int64_t n, Arena& tmp, hipStream_t st,
                 bool want_total) {
  Arena::Mark m = tmp.mark();
  scan_core<int64_t>(in, out, n, tmp, st);
  int64_t total = want_total ? read_i64(out + n, st) : -1;
  tmp.rewind(m);
  return total;
}

int64_t scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, Arena& tmp, hipStream_t st,
                        bool want_total) {
  Arena::Mark m = tmp.mark();
  scan_core<int32_t>(in, out, n, tmp, st);
  int64_t total = want_total ? read_i64(out + n, st) : -1;
  tmp.rewind(m);
  return total;
}

// ------------------------------------------------------------- radix sort
constexpr int kRadixIPT = 8;
constexpr int kRadixTile = kBlock * kRadixIPT;
constexpr int kBlockSortMax = 2 * kRadixTile;  // sorted by one workgroup in LDS
constexpr int kBlockSortRounds = kBlockSortMax / kBlock;
constexpr int kMaxDigits = 8;

struct RadixShifts {
  int count;
  int s[kMaxDigits];
};

// Digit of a key.  pack > 0: the key holds a pair (hi << 32 | lo) with
// hi, lo < 2^pack, and digits are taken from the contiguous (hi << pack | lo),
// which sorts in the same order with fewer digits.
__device__ __forceinline__ int radix_digit(uint64_t key, int shift, int pack) {
  if (pack) key = ((key >> 32) << pack) | (key & 0xffffffffULL);
  return (int)((key >> shift) & 255);
}

// Exclusive prefix sum of one int per thread over a kBlock-thread workgroup.
__device__ __forceinline__ int block_excl_scan(int v, int* wtot) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wtot[w] = x;
  __syncthreads();
  int pre = 0;
  for (int k = 0; k < w; k++) pre += wtot[k];
  __syncthreads();
  return pre + x - v;
}

// One round of a stable counting sort: the workgroup's threads hold one item
// each, in index order.  Returns the item's position run[d] + (items of
// earlier waves with digit d) + (earlier lanes of this wave with digit d) and
// advances run[] past the round's items.
__device__ __forceinline__ int radix_round(bool valid, int d, int* run, int (*wc)[256]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int k = 0; k < kBlock / 64; k++) wc[k][t] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ULL : ((~0ULL) >> (64 - lane));
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; b++) {
    const int bit = (d >> b) & 1;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  if (valid && (int)(__ffsll((unsigned long long)peers) - 1) == lane) wc[w][d] = __popcll(peers);
  __syncthreads();
  int pos = 0;
  if (valid) {
    pos = run[d] + __popcll(peers & lt);
    for (int k = 0; k < w; k++) pos += wc[k][d];
  }
  __syncthreads();
  int add = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; k++) add += wc[k][t];
  run[t] += add;
  return pos;
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                       int shift, int pack,
                                                       int32_t* __restrict__ hist, int64_t nb) {
  __shared__ int cnt[256];
  const int t = threadIdx.x;
  cnt[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
  for (int r = 0; r < kRadixIPT; r++) {
    const int64_t i = base + (int64_t)r * kBlock + t;
    if (i < n) atomicAdd(&cnt[radix_digit(keys[i], shift, pack)], 1);
  }
  __syncthreads();
  hist[(int64_t)t * nb + blockIdx.x] = cnt[t];
}

// Stable scatter of one tile.  The tile is first ordered by digit in LDS
// (items ranked in index order), then written out so that consecutive threads
// store consecutive positions of a digit's output range.  offs is the
// exclusive scan of the digit-major histogram (256 * nb + 1 entries).
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint64_t* __restrict__ kin, const uint64_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint64_t* __restrict__ vout, int64_t n, int shift, int pack, const int64_t* __restrict__ offs,
    int64_t nb) {
  __shared__ uint64_t sk[kRadixTile], sv[kRadixTile];
  __shared__ int64_t gbase[256];
  __shared__ int run[256];
  __shared__ int wc[kBlock / 64][256];
  __shared__ int wtot[kBlock / 64];
  const int t = threadIdx.x;
  const int64_t b = blockIdx.x, base = b * kRadixTile;
  const int64_t o0 = offs[(int64_t)t * nb + b];
  const int c = (int)(offs[(int64_t)t * nb + b + 1] - o0);
  const int ex = block_excl_scan(c, wtot);
  run[t] = ex;
  gbase[t] = o0 - ex;
  // radix_round's first barrier publishes run[]
  for (int r = 0; r < kRadixIPT; r++) {
    const int64_t i = base + (int64_t)r * kBlock + t;
    const bool valid = i < n;
    uint64_t key = 0, val = 0;
    int d = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
      d = radix_digit(key, shift, pack);
    }
    const int pos = radix_round(valid, d, run, wc);
    if (valid) {
      sk[pos] = key;
      sv[pos] = val;
    }
  }
  __syncthreads();
  const int cnt = (int)min((int64_t)kRadixTile, n - base);
  for (int j = t; j < cnt; j += kBlock) {
    const uint64_t key = sk[j];
    const int64_t pos = gbase[radix_digit(key, shift, pack)] + j;
    kout[pos] = key;
    vout[pos] = sv[j];
  }
}

// All digit passes of a sort of n <= kBlockSortMax pairs in one workgroup.
__global__ __launch_bounds__(kBlock) void k_radix_block_sort(uint64_t* __restrict__ keys,
                                                             uint64_t* __restrict__ vals, int n,
                                                             RadixShifts sh, int pack) {
  __shared__ uint64_t sk[kBlockSortMax], sv[kBlockSortMax];
  __shared__ int cnt[256], run[256];
  __shared__ int wc[kBlock / 64][256];
  __shared__ int wtot[kBlock / 64];
  const int t = threadIdx.x;
  for (int j = t; j < n; j += kBlock) {
    sk[j] = keys[j];
    sv[j] = vals[j];
  }
  for (int p = 0; p < sh.count; p++) {
    const int shift = sh.s[p];
    cnt[t] = 0;
    __syncthreads();
    for (int j = t; j < n; j += kBlock) atomicAdd(&cnt[radix_digit(sk[j], shift, pack)], 1);
    __syncthreads();
    run[t] = block_excl_scan(cnt[t], wtot);
    uint64_t k[kBlockSortRounds], v[kBlockSortRounds];
#pragma unroll
    for (int r = 0; r < kBlockSortRounds; r++) {
      const int j = r * kBlock + t;
      k[r] = j < n ? sk[j] : 0;
      v[r] = j < n ? sv[j] : 0;
    }
    // radix_round's first barrier orders these reads before the writes below
#pragma unroll
    for (int r = 0; r < kBlockSortRounds; r++) {
      if (r * kBlock >= n) break;  // the same for every thread: only rounds that hold items
      const bool valid = r * kBlock + t < n;
      const int d = valid ? radix_digit(k[r], shift, pack) : 0;
      const int pos = radix_round(valid, d, run, wc);
      if (valid) {
        sk[pos] = k[r];
        sv[pos] = v[r];
      }
    }
    __syncthreads();
  }
  for (int j = t; j < n; j += kBlock) {
    keys[j] = sk[j];
    vals[j] = sv[j];
  }
}

int bits_for(int64_t v) {
  int b = 0;
  while (b < 63 && (v >> b) != 0) b++;
  return b;
}

std::vector<int> digit_shifts(int bits_lo, int bits_hi) {
  std::vector<int> s;
  for (int b = 0; b < bits_lo; b += 8) s.push_back(b);
  for (int b = 0; b < bits_hi; b += 8) s.push_back(32 + b);
  return s;
}

std::vector<int> pair_shifts(int bits) {
  std::vector<int> s;
  for (int b = 0; b < 2 * bits; b += 8) s.push_back(b);
  return s;
}

SortedPairs radix_sort_pairs(uint64_t* keys, uint64_t* vals, int64_t n,
                             const std::vector<int>& shifts, Arena& tmp, hipStream_t st, int pack) {
  if (n <= 1 || shifts.empty()) return {keys, vals};
  ProfScope prof_scope("radix", st, (double)n * 32.0 * shifts.size());
  if (n <= kBlockSortMax && (int)shifts.size() <= kMaxDigits) {
    RadixShifts sh{};
    sh.count = (int)shifts.size();
    for (int k = 0; k < sh.count; k++) sh.s[k] = shifts[k];
    hipLaunchKernelGGL(k_radix_block_sort, dim3(1), dim3(kBlock), 0, st, keys, vals, (int)n, sh,
                       pack);
    LG_LAUNCH_CHECK();
    return {keys, vals};
  }
  // the second pair of arrays may hold the result: allocated before the mark
  uint64_t* k2 = tmp.get<uint64_t>(n);
  uint64_t* v2 = tmp.get<uint64_t>(n);
  Arena::Mark m = tmp.mark();
  const int64_t nb = ceil_div(n, kRadixTile);
  int32_t* hist = tmp.get<int32_t>(256 * nb);
  int64_t* offs = tmp.get<int64_t>(256 * nb + 1);
  uint64_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
  for (int sh : shifts) {
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kBlock), 0, st, ka, n, sh, pack, hist,
                       nb);
    Arena::Mark m2 = tmp.mark();
    scan_core<int32_t>(hist, offs, 256 * nb, tmp, st);
    tmp.rewind(m2);
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kBlock), 0, st, ka, va, kb, vb, n,
                       sh, pack, offs, nb);
    LG_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  tmp.rewind(m);
  return {ka, va};
}

// ------------------------------------------------------------ row schedule
enum { ST_MAX = 0, ST_MIN = 1, ST_CLS = 2, ST_HUB = 10, ST_SPLIT = 11, ST_CHUNK = 12 };

constexpr int kStatRows = 16;  // rows per thread in k_sched_stats

// n_dev (optional): the actual row count on the device, at most n.
__global__ __launch_bounds__(kBlock) void k_sched_stats(const int32_t* __restrict__ rp, int64_t n,
                                                        const int64_t* __restrict__ n_dev,
                                                        int rows, int hub_deg,
                                                        int* __restrict__ partial) {
  if (n_dev) n = min(n, *n_dev);
  int v[kStat];
#pragma unroll
  for (int k = 0; k < kStat; k++) v[k] = 0;
  v[ST_MIN] = 0x7fffffff;
  for (int q = 0; q < rows; q++) {
    const int64_t i = ((int64_t)blockIdx.x * rows + q) * kBlock + threadIdx.x;
    if (i >= n) break;
    const int d = rp[i + 1] - rp[i];
    const int c = degree_class(d, hub_deg);
    v[ST_MAX] = max(v[ST_MAX], d);
    v[ST_MIN] = min(v[ST_MIN], d);
    if (c < kClasses) v[ST_CLS + c]++;
    else if (d > kSplitDeg) {
      v[ST_SPLIT]++;
      v[ST_CHUNK] += (d + kHubChunk - 1) / kHubChunk;
    } else {
      v[ST_HUB]++;
    }
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    v[ST_MAX] = max(v[ST_MAX], __shfl_xor(v[ST_MAX], m));
    v[ST_MIN] = min(v[ST_MIN], __shfl_xor(v[ST_MIN], m));
#pragma unroll
    for (int k = 2; k < kStat; k++) v[k] += __shfl_xor(v[k], m);
  }
  __shared__ int sm[kBlock / 64][kStat];
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < kStat; k++) sm[threadIdx.x >> 6][k] = v[k];
  __syncthreads();
  if (threadIdx.x < kStat) {
    const int k = threadIdx.x;
    int r = sm[0][k];
    for (int w = 1; w < kBlock / 64; w++)
      r = k == ST_MAX ? max(r, sm[w][k]) : k == ST_MIN ? min(r, sm[w][k]) : r + sm[w][k];
    partial[(int64_t)blockIdx.x * kStat + k] = r;
  }
}

// One wavefront per statistic, fixed lane order.
__global__ __launch_bounds__(kStat * 64) void k_sched_final(const int* __restrict__ partial,
                                                            int64_t nb, int* __restrict__ out) {
  const int k = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int r = k == ST_MIN ? 0x7fffffff : 0;
  for (int64_t b = lane; b < nb; b += 64) {
    const int v = partial[b * kStat + k];
    r = k == ST_MAX ? max(r, v) : k == ST_MIN ? min(r, v) : r + v;
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const int o = __shfl_xor(r, m);
    r = k == ST_MAX ? max(r, o) : k == ST_MIN ? min(r, o) : r + o;
  }
  if (lane == 0) out[k] = r;
}

// Rows grouped by degree class, in one kernel.  A workgroup takes ipt * kBlock
// consecutive rows (ipt grows with n so that the class reservations stay
// few): it counts its rows of each class, reserves its share of each class
// with one atomic per class (ctr[2 + c]), then places its rows in row order,
// a round of kBlock rows at a time; hubs and split rows are
// appended to their lists (ctr[0], ctr[1]; split rows with their chunk
// counts).  ctr is zero on entry.  Where a workgroup's share lands varies
// between runs; a row's result does not depend on its place in the schedule.
constexpr int kPermMaxIPT = 16;

// Rounds of kBlock rows per workgroup: one below about 2^17 rows, at most
// kPermMaxIPT (about 512 workgroups, 8 reservations each, before that cap).
inline int perm_ipt(int64_t n) {
  return (int)std::min<int64_t>(kPermMaxIPT, std::max<int64_t>(1, ceil_div(n, (int64_t)kBlock * 512)));
}

__global__ __launch_bounds__(kBlock) void k_class_perm(
    const int32_t* __restrict__ rp, int64_t n, int ipt, int hub_deg, ClassTable ct,
    int* __restrict__ ctr, int32_t* __restrict__ perm, int32_t* __restrict__ hub_rows,
    int32_t* __restrict__ split_rows, int32_t* __restrict__ split_nch) {
  __shared__ int wcnt[kBlock / 64][kClasses];
  __shared__ int run[kClasses];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t b0 = (int64_t)blockIdx.x * ipt * kBlock;
  // pass 1: this workgroup's class counts; hubs and split rows go to their lists
  int cnt[kClasses];
#pragma unroll
  for (int k = 0; k < kClasses; k++) cnt[k] = 0;
  for (int r = 0; r < ipt; r++) {
    const int64_t i = b0 + (int64_t)r * kBlock + t;
    if (i >= n) break;
    const int d = rp[i + 1] - rp[i];
    const int c = degree_class(d, hub_deg);
    if (c < kClasses) {
#pragma unroll
      for (int k = 0; k < kClasses; k++) cnt[k] += (c == k);
    } else if (d > kSplitDeg) {
      const int k = atomicAdd(&ctr[1], 1);
      split_rows[k] = (int32_t)i;
      split_nch[k] = (d + kHubChunk - 1) / kHubChunk;
    } else {
      hub_rows[atomicAdd(&ctr[0], 1)] = (int32_t)i;
    }
  }
#pragma unroll
  for (int k = 0; k < kClasses; k++) {
    int v = cnt[k];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    if (lane == 0) wcnt[w][k] = v;
  }
  __syncthreads();
  if (t < kClasses) {
    int tot = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; k++) tot += wcnt[k][t];
    run[t] = tot ? atomicAdd(&ctr[2 + t], tot) : 0;
  }
  // pass 2: place the class rows in row order
  const uint64_t lt = (lane == 0) ? 0ULL : ((~0ULL) >> (64 - lane));
  for (int r = 0; r < ipt; r++) {
    if (b0 + (int64_t)r * kBlock >= n) break;  // the same for every thread
    const int64_t i = b0 + (int64_t)r * kBlock + t;
    int c = -1;
    if (i < n) {
      c = degree_class(rp[i + 1] - rp[i], hub_deg);
      if (c >= kClasses) c = -1;
    }
    __syncthreads();  // run[] is current, the previous round's wcnt is read
    int rank = 0;
#pragma unroll
    for (int k = 0; k < kClasses; k++) {
      const uint64_t m = __ballot(c == k);
      if (c == k) rank = __popcll(m & lt);
      if (lane == 0) wcnt[w][k] = __popcll(m);
    }
    __syncthreads();
    if (c >= 0) {
      int pos = run[c] + rank;
      for (int k = 0; k < w; k++) pos += wcnt[k][c];
      perm[ct.cls_start[c] + pos] = (int32_t)i;
    }
    __syncthreads();
    if (t < kClasses) {
      int add = 0;
#pragma unroll
      for (int k = 0; k < kBlock / 64; k++) add += wcnt[k][t];
      run[t] += add;
    }
  }
}

__global__ void k_split_chunk_owner(const int32_t* __restrict__ nch, const int64_t* __restrict__ start,
                                    int64_t nsplit, int32_t* __restrict__ cptr,
                                    int32_t* __restrict__ chunk_split) {
  const int64_t h = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (h > nsplit) return;
  cptr[h] = (int32_t)start[h];
  if (h == nsplit) return;
  for (int k = 0; k < nch[h]; k++) chunk_split[start[h] + k] = (int32_t)h;
}

__global__ void k_zero_i32n(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Small device values the host needs (sizes, flags, convergence scalars) are
// read through a mailbox: a one-workgroup kernel copies them into
// fine-grained (coherent) pinned host memory, makes them visible system-wide
// and then writes a sequence number there, which the host polls.  This skips
// the copy-engine round trip and the stream-synchronisation wake-up.  Each
// host thread owns one mailbox (kept until the process ends).
constexpr int kMailHeader = 16;     // 32-bit words before the data
constexpr size_t kMailBytes = 65536;  // largest read

constexpr int kMailSegs = 4;
struct MailSegs {
  const uint32_t* src[kMailSegs];
  int words[kMailSegs];
  int count;
};

// Copies the segments back to back into the mailbox, then publishes seq.
__global__ void k_mail(MailSegs segs, uint32_t* __restrict__ box, uint32_t seq) {
  int at = kMailHeader;
  for (int k = 0; k < segs.count; k++) {
    for (int i = threadIdx.x; i < segs.words[k]; i += blockDim.x) box[at + i] = segs.src[k][i];
    at += segs.words[k];
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(box, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void read_dev_n(const DevRead* r, int count, hipStream_t st) {
  if (count < 1 || count > kMailSegs) fail(LG_E_ARG, "read_dev_n: 1 to 4 segments");
  MailSegs segs{};
  segs.count = count;
  size_t total = 0;
  for (int k = 0; k < count; k++) {
    if ((r[k].bytes & 3) || (reinterpret_cast<uintptr_t>(r[k].dev) & 3))
      fail(LG_E_ARG, "read_dev_n: segments must be 4-byte aligned whole words");
    segs.src[k] = static_cast<const uint32_t*>(r[k].dev);
    segs.words[k] = (int)(r[k].bytes / 4);
    total += r[k].bytes;
  }
  if (total > kMailBytes) fail(LG_E_ARG, "read_dev_n: too large");
  static thread_local uint32_t* box = nullptr;
  static thread_local uint32_t* box_dev = nullptr;
  static thread_local uint32_t seq = 0;
  if (!box) {
    LG_HIP(hipHostMalloc((void**)&box, kMailHeader * 4 + kMailBytes,
                         hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable));
    LG_HIP(hipHostGetDevicePointer((void**)&box_dev, box, 0));
    __atomic_store_n(box, 0u, __ATOMIC_RELAXED);
  }
  if (++seq == 0) seq = 1;  // 0 is the initial value
  hipLaunchKernelGGL(k_mail, dim3(1), dim3(kBlock), 0, st, segs, box_dev, seq);
  LG_LAUNCH_CHECK();
  for (uint64_t spin = 1; __atomic_load_n(box, __ATOMIC_ACQUIRE) != seq; spin++) {
    if (spin % 1024) continue;
    const hipError_t e = hipStreamQuery(st);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(LG_E_HIP, std::string("HIP error: ") + hipGetErrorString(e));
    }
    if (__atomic_load_n(box, __ATOMIC_ACQUIRE) != seq)
      fail(LG_E_HIP, "device read: the stream finished without publishing the value");
  }
  const char* data = reinterpret_cast<const char*>(box + kMailHeader);
  for (int k = 0; k < count; k++) {
    memcpy(r[k].host, data, r[k].bytes);
    data += r[k].bytes;
  }
}

void read_dev(void* host, const void* dev, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  if (bytes > kMailBytes) fail(LG_E_ARG, "read_dev: too large");
  if ((bytes & 3) || (reinterpret_cast<uintptr_t>(dev) & 3)) {
    static thread_local char* pinned = nullptr;
    if (!pinned) LG_HIP(hipHostMalloc((void**)&pinned, kMailBytes, hipHostMallocDefault));
    LG_HIP(hipMemcpyAsync(pinned, dev, bytes, hipMemcpyDeviceToHost, st));
    LG_HIP(hipStreamSynchronize(st));
    memcpy(host, pinned, bytes);
    return;
  }
  const DevRead r{host, dev, bytes};
  read_dev_n(&r, 1, st);
}

// tile_row[t] = rows whose end marker (at rp[r+1] + r) precedes merged item
// min(t * kMergeTile, n + nnz), by binary search (the positions increase).
__global__ void k_merge_split(const int32_t* __restrict__ rp, int64_t n, int64_t nnz,
                              int64_t ntile, int32_t* __restrict__ tile_row) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t > ntile) return;
  const int64_t d = min(t * kMergeTile, n + nnz);
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)rp[mid + 1] + mid < d) lo = mid + 1;
    else hi = mid;
  }
  tile_row[t] = (int32_t)lo;
}

int* sched_stats(const int32_t* rp, int64_t n, const int64_t* n_dev, Arena& tmp, hipStream_t st) {
  // rows per thread: one up to about 2^18 rows, then up to kStatRows
  const int rows =
      (int)std::min<int64_t>(kStatRows, std::max<int64_t>(1, ceil_div(n, (int64_t)kBlock * 1024)));
  const int64_t nbs = std::max<int64_t>(1, ceil_div(n, (int64_t)kBlock * rows));
  int* part = tmp.get<int>(kStat * nbs);
  hipLaunchKernelGGL(k_sched_stats, dim3((unsigned)nbs), dim3(kBlock), 0, st, rp, n, n_dev, rows,
                     (int)LG_HUB_DEG, part);
  if (nbs == 1) {  // one workgroup's statistics are the totals
    LG_LAUNCH_CHECK();
    return part;
  }
  int* tot = tmp.get<int>(kStat);
  hipLaunchKernelGGL(k_sched_final, dim3(1), dim3(kStat * 64), 0, st, (const int*)part, nbs, tot);
  LG_LAUNCH_CHECK();
  return tot;
}

// Stable row lists: key 0 split rows, 1 hub rows, 2 + c class c; a stable
// sort then lays them out as [split | hub | class 0 | ... | class 7], each in
// increasing row order.
__global__ void k_sched_keys(const int32_t* __restrict__ rp, int64_t n, int hub_deg,
                             uint64_t* __restrict__ keys, uint64_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int d = rp[i + 1] - rp[i];
  const int c = degree_class(d, hub_deg);
  keys[i] = c >= kClasses ? (d > kSplitDeg ? 0u : 1u) : (uint64_t)(2 + c);
  vals[i] = (uint64_t)i;
}

__global__ void k_sched_lists(const int32_t* __restrict__ rp, const uint64_t* __restrict__ sorted,
                              int64_t n, int64_t nsplit, int64_t nhub, int32_t* __restrict__ split_rows,
                              int32_t* __restrict__ split_nch, int32_t* __restrict__ hub_rows,
                              int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t r = (int32_t)sorted[i];
  if (i < nsplit) {
    split_rows[i] = r;
    split_nch[i] = (rp[r + 1] - rp[r] + kHubChunk - 1) / kHubChunk;
  } else if (i < nsplit + nhub) {
    hub_rows[i - nsplit] = r;
  } else {
    perm[i - nsplit - nhub] = r;
  }
}

void build_sched(Sched& s, const int32_t* rp, int64_t n, int64_t nnz, Arena& keep, Arena& tmp,
                 hipStream_t st, bool tiles, bool stable) {
  int t[kStat] = {};
  Arena::Mark m = tmp.mark();
  if (n > 0) read_dev(t, sched_stats(rp, n, nullptr, tmp, st), sizeof(t), st);
  sched_layout(s, t, rp, n, nnz, tiles, keep, tmp, st, stable);
  tmp.rewind(m);
}

void sched_layout(Sched& s, const int* t, const int32_t* rp, int64_t n, int64_t nnz, bool tiles,
                  Arena& keep, Arena& tmp, hipStream_t st, bool stable) {
  s = Sched();
  s.n = n;
  s.nnz = nnz;
  s.stable = stable;
  if (n == 0) return;
  s.hub_deg = LG_HUB_DEG;
  Arena::Mark m = tmp.mark();
  const int64_t nb = ceil_div(n, kBlock);
  s.max_deg = t[ST_MAX];
  s.min_deg = t[ST_MIN];
  s.nhub = t[ST_HUB];
  s.nsplit = t[ST_SPLIT];
  s.nchunk = t[ST_CHUNK];
  int64_t pos = 0, blk = 0;
  for (int c = 0; c < kClasses; c++) {
    s.ct.cls_start[c] = (int32_t)pos;
    s.ct.blk_start[c] = (int32_t)blk;
    const int G = class_lanes(c, s.lane_shift);
    pos += t[ST_CLS + c];
    blk += ceil_div((int64_t)t[ST_CLS + c] * G, kBlock);
  }
  s.ct.cls_start[kClasses] = (int32_t)pos;
  s.ct.blk_start[kClasses] = (int32_t)blk;
  s.perm = keep.get<int32_t>(pos);
  s.hub_rows = s.nhub ? keep.get<int32_t>(s.nhub) : nullptr;
  s.split_rows = s.nsplit ? keep.get<int32_t>(s.nsplit) : nullptr;
  if (s.nsplit) {
    s.split_cptr = keep.get<int32_t>(s.nsplit + 1);
    s.chunk_split = keep.get<int32_t>(s.nchunk);
    s.partial = keep.alloc((size_t)s.nchunk * kPartialBytes);
  }
  if (tiles) {  // merge-path tiles
    s.ntile = ceil_div(n + nnz, kMergeTile);
    s.tile_row = keep.get<int32_t>(s.ntile + 1);
    s.carry_row = keep.get<int32_t>(s.ntile);
    s.carry_val = keep.get<double>(s.ntile);
  }
  sched_fill(s, rp, tmp, st);
  tmp.rewind(m);
}

// The row lists of a laid-out schedule from rp: rows grouped by class, hubs
// and split rows listed (one pass, k_class_perm), the split rows' chunk
// owners and the merge-path tiles.  Rerun after the rows are renumbered with
// their degrees kept.
void sched_fill(Sched& s, const int32_t* rp, Arena& tmp, hipStream_t st) {
  if (s.n == 0) return;
  Arena::Mark m = tmp.mark();
  int32_t* nch = s.nsplit ? tmp.get<int32_t>(s.nsplit) : nullptr;
  if (s.stable) {
    // one stable radix pass over the group keys: split rows, hubs, classes
    uint64_t* keys = tmp.get<uint64_t>(s.n);
    uint64_t* vals = tmp.get<uint64_t>(s.n);
    hipLaunchKernelGGL(k_sched_keys, dim3((unsigned)ceil_div(s.n, (int64_t)kBlock)), dim3(kBlock), 0,
                       st, rp, s.n, s.hub_deg, keys, vals);
    const SortedPairs sp = radix_sort_pairs(keys, vals, s.n, {0}, tmp, st);
    hipLaunchKernelGGL(k_sched_lists, dim3((unsigned)ceil_div(s.n, (int64_t)kBlock)), dim3(kBlock), 0,
                       st, rp, (const uint64_t*)sp.vals, s.n, s.nsplit, s.nhub, s.split_rows, nch,
                       s.hub_rows, s.perm);
  } else {
    int* ctr = tmp.get<int>(kClasses + 2);
    hipLaunchKernelGGL(k_zero_i32n, dim3(1), dim3(kBlock), 0, st, (int32_t*)ctr,
                       (int64_t)(kClasses + 2));
    const int ipt = perm_ipt(s.n);
    hipLaunchKernelGGL(k_class_perm, dim3((unsigned)ceil_div(s.n, (int64_t)ipt * kBlock)),
                       dim3(kBlock), 0, st, rp, s.n, ipt, s.hub_deg, s.ct, ctr, s.perm, s.hub_rows,
                       s.split_rows, nch);
  }
  LG_LAUNCH_CHECK();
  if (s.nsplit) {
    int64_t* start = tmp.get<int64_t>(s.nsplit + 1);
    scan_i32_to_i64(nch, start, s.nsplit, tmp, st, false);
    hipLaunchKernelGGL(k_split_chunk_owner, dim3((unsigned)ceil_div(s.nsplit + 1, kBlock)),
                       dim3(kBlock), 0, st, (const int32_t*)nch, (const int64_t*)start, s.nsplit,
                       s.split_cptr, s.chunk_split);
    LG_LAUNCH_CHECK();
  }
  if (s.tile_row) {
    hipLaunchKernelGGL(k_merge_split, dim3((unsigned)ceil_div(s.ntile + 1, kBlock)), dim3(kBlock), 0,
                       st, rp, s.n, s.nnz, s.ntile, s.tile_row);
    LG_LAUNCH_CHECK();
  }
  tmp.rewind(m);
}

}  // namespace lg
