// prims.hip -- device primitives shared by the setup passes: exclusive scans,
// a stable LSD radix sort of (key, payload) pairs, the row scheduler, the
// device arena and the HIP-event profiler behind lg_profile_*.
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
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(LG_E_NOMEM, "device allocation of " + std::to_string(sz) + " bytes failed");
  }
  chunks_.push_back({(char*)p, sz});
  total_ += sz;
  cur_ = chunks_.size() - 1;
  off_ = bytes;
  return p;
}

void Arena::release() {
  for (auto& c : chunks_) (void)hipFree(c.p);
  chunks_.clear();
  cur_ = off_ = total_ = 0;
}

// ---------------------------------------------------------------- profiler
namespace {
struct Prof {
  std::mutex mu;
  std::string family;
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

ProfScope::ProfScope(const char* family, hipStream_t s, double b) : on(false), st(s), bytes(b) {
  Prof& p = prof();
  if (p.family.empty() || p.family != family) return;
  std::lock_guard<std::mutex> g(p.mu);
  a = take_event(p);
  this->b = take_event(p);
  LG_HIP(hipEventRecord(a, st));
  on = true;
}

ProfScope::~ProfScope() {
  if (!on) return;
  Prof& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  (void)hipEventRecord(b, st);
  p.pending.push_back({a, b});
  p.pending_bytes.push_back(bytes);
}

}  // namespace lg

extern "C" lg_status lg_profile_enable(const char* family) {
  auto& p = lg::prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.family = family ? family : "";
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
  return "spmm,cheb,resid,restrict,prolong,coarse,pcg_vec,jacobi_xsum,affinity,vote,"
         "elim_select,radix,galerkin_reduce";
}

namespace lg {

// ------------------------------------------------------------------- scan
constexpr int kScanIPT = 8;
constexpr int kScanTile = kBlock * kScanIPT;

template <typename TI>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const TI* __restrict__ in,
                                                       int64_t* __restrict__ out,
                                                       int64_t* __restrict__ sums, int64_t n) {
  __shared__ int64_t wsum[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int64_t v[kScanIPT];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanIPT; k++) {
    const int64_t i = base + (int64_t)t * kScanIPT + k;
    v[k] = i < n ? (int64_t)in[i] : 0;
    s += v[k];
  }
  int64_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int64_t wpre = 0;
  for (int k = 0; k < w; k++) wpre += wsum[k];
  int64_t run = wpre + x - s;
#pragma unroll
  for (int k = 0; k < kScanIPT; k++) {
    const int64_t i = base + (int64_t)t * kScanIPT + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (t == kBlock - 1) sums[blockIdx.x] = wpre + x;
}

__global__ void k_scan_add(int64_t* __restrict__ out, const int64_t* __restrict__ offs, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] += offs[i / kScanTile];
}

__global__ void k_copy_i64(int64_t* dst, const int64_t* src) { *dst = *src; }
__global__ void k_zero_i64(int64_t* dst) { *dst = 0; }

template <typename TI>
static void scan_core(const TI* in, int64_t* out, int64_t n, Arena& tmp, hipStream_t st) {
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, st, out);
    return;
  }
  const int64_t nb = ceil_div(n, kScanTile);
  int64_t* sums = tmp.get<int64_t>(nb);
  hipLaunchKernelGGL((k_scan_tiles<TI>), dim3((unsigned)nb), dim3(kBlock), 0, st, in, out, sums, n);
  if (nb == 1) {
    hipLaunchKernelGGL(k_copy_i64, dim3(1), dim3(1), 0, st, out + n, sums);
  } else {
    int64_t* offs = tmp.get<int64_t>(nb + 1);
    scan_core<int64_t>(sums, offs, nb, tmp, st);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, st, out,
                       offs, n);
    hipLaunchKernelGGL(k_copy_i64, dim3(1), dim3(1), 0, st, out + n, offs + nb);
  }
  LG_LAUNCH_CHECK();
}

int64_t read_i64(const int64_t* dev, hipStream_t st) {
  static thread_local int64_t* pinned = nullptr;
  if (!pinned) LG_HIP(hipHostMalloc((void**)&pinned, sizeof(int64_t), hipHostMallocDefault));
  LG_HIP(hipMemcpyAsync(pinned, dev, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  LG_HIP(hipStreamSynchronize(st));
  return *pinned;
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
constexpr int kRadixIPT = 16;
constexpr int kRadixTile = kBlock * kRadixIPT;

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                       int shift, int32_t* __restrict__ hist,
                                                       int64_t nb) {
  __shared__ int cnt[256];
  const int t = threadIdx.x;
  cnt[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
  for (int r = 0; r < kRadixIPT; r++) {
    const int64_t i = base + (int64_t)r * kBlock + t;
    if (i < n) atomicAdd(&cnt[(int)((keys[i] >> shift) & 255)], 1);
  }
  __syncthreads();
  hist[(int64_t)t * nb + blockIdx.x] = cnt[t];
}

// Stable scatter: items are visited in (round, thread) order, which is their
// index order inside the tile; equal digits keep that order.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint64_t* __restrict__ kin, const uint64_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint64_t* __restrict__ vout, int64_t n, int shift, const int64_t* __restrict__ offs, int64_t nb) {
  __shared__ int64_t run[256];
  __shared__ int wc[kBlock / 64][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  run[t] = offs[(int64_t)t * nb + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  const uint64_t lt = (lane == 0) ? 0ULL : ((~0ULL) >> (64 - lane));
  for (int r = 0; r < kRadixIPT; r++) {
#pragma unroll
    for (int k = 0; k < kBlock / 64; k++) wc[k][t] = 0;
    __syncthreads();
    const int64_t i = base + (int64_t)r * kBlock + t;
    const bool valid = i < n;
    uint64_t key = 0, val = 0;
    int d = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
      d = (int)((key >> shift) & 255);
    }
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const int bit = (d >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & lt);
    if (valid && (int)(__ffsll((unsigned long long)peers) - 1) == lane) wc[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int64_t pos = run[d] + rank;
      for (int k = 0; k < w; k++) pos += wc[k][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; k++) add += wc[k][t];
    run[t] += add;
    __syncthreads();
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

void radix_sort_pairs(uint64_t* keys, uint64_t* vals, int64_t n, const std::vector<int>& shifts,
                      Arena& tmp, hipStream_t st) {
  if (n <= 1 || shifts.empty()) return;
  ProfScope prof_scope("radix", st, (double)n * 32.0 * shifts.size());
  Arena::Mark m = tmp.mark();
  const int64_t nb = ceil_div(n, kRadixTile);
  uint64_t* k2 = tmp.get<uint64_t>(n);
  uint64_t* v2 = tmp.get<uint64_t>(n);
  int32_t* hist = tmp.get<int32_t>(256 * nb);
  int64_t* offs = tmp.get<int64_t>(256 * nb + 1);
  uint64_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
  for (int sh : shifts) {
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kBlock), 0, st, ka, n, sh, hist, nb);
    Arena::Mark m2 = tmp.mark();
    scan_core<int32_t>(hist, offs, 256 * nb, tmp, st);
    tmp.rewind(m2);
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kBlock), 0, st, ka, va, kb, vb, n,
                       sh, offs, nb);
    LG_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    LG_HIP(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, st));
    LG_HIP(hipMemcpyAsync(vals, va, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, st));
  }
  tmp.rewind(m);
}

// ------------------------------------------------------------ row schedule
__global__ void k_max_degree(const int32_t* __restrict__ rp, int64_t n, int* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int d = (i < n) ? rp[i + 1] - rp[i] : 0;
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) d = max(d, __shfl_xor(d, m));
  if ((threadIdx.x & 63) == 0) atomicMax(out, d);
}

__global__ void k_hub_flags(const int32_t* __restrict__ rp, int64_t n, int hub_deg,
                            int32_t* __restrict__ flag, int32_t* __restrict__ nch) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int d = rp[i + 1] - rp[i];
  const bool h = d > hub_deg;
  flag[i] = h;
  nch[i] = h ? (d + kHubChunk - 1) / kHubChunk : 0;
}

__global__ void k_hub_lists(const int32_t* __restrict__ flag, const int32_t* __restrict__ nch,
                            const int64_t* __restrict__ hidx, const int64_t* __restrict__ cstart,
                            int64_t n, int32_t* __restrict__ hub_rows, int32_t* __restrict__ hub_cptr,
                            int32_t* __restrict__ chunk_hub) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || !flag[i]) return;
  const int64_t h = hidx[i];
  hub_rows[h] = (int32_t)i;
  hub_cptr[h] = (int32_t)cstart[i];
  for (int k = 0; k < nch[i]; k++) chunk_hub[cstart[i] + k] = (int32_t)h;
}

__global__ void k_set_i32(int32_t* p, int32_t v) { *p = v; }
__global__ void k_zero_i32n(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0;
}

void build_sched(Sched& s, const int32_t* rp, int64_t n, int64_t nnz, Arena& keep, Arena& tmp,
                 hipStream_t st) {
  s = Sched();
  s.n = n;
  s.nnz = nnz;
  if (n == 0) return;
  const double avg = (double)nnz / (double)n;
  int G = 4;
  while (G < 64 && G < avg) G <<= 1;
  s.G = G;
  s.hub_deg = 32 * G > 256 ? 32 * G : 256;
  Arena::Mark m = tmp.mark();
  int32_t* mx = tmp.get<int32_t>(2);
  hipLaunchKernelGGL(k_zero_i32n, dim3(1), dim3(kBlock), 0, st, mx, (int64_t)2);
  hipLaunchKernelGGL(k_max_degree, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, st, rp, n,
                     (int*)mx);
  LG_LAUNCH_CHECK();
  int64_t both = read_i64((const int64_t*)mx, st);
  const int maxdeg = (int)(both & 0xffffffff);
  if (maxdeg <= s.hub_deg) {
    tmp.rewind(m);
    return;
  }
  int32_t* flag = tmp.get<int32_t>(n);
  int32_t* nch = tmp.get<int32_t>(n);
  int64_t* hidx = tmp.get<int64_t>(n + 1);
  int64_t* cstart = tmp.get<int64_t>(n + 1);
  hipLaunchKernelGGL(k_hub_flags, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, st, rp, n,
                     s.hub_deg, flag, nch);
  s.nhub = scan_i32_to_i64(flag, hidx, n, tmp, st, true);
  s.nchunk = scan_i32_to_i64(nch, cstart, n, tmp, st, true);
  s.hub_rows = keep.get<int32_t>(s.nhub);
  s.hub_cptr = keep.get<int32_t>(s.nhub + 1);
  s.chunk_hub = keep.get<int32_t>(s.nchunk);
  s.partial = keep.alloc((size_t)s.nchunk * kPartialBytes);
  hipLaunchKernelGGL(k_hub_lists, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, st, flag,
                     nch, hidx, cstart, n, s.hub_rows, s.hub_cptr, s.chunk_hub);
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, st, s.hub_cptr + s.nhub, (int32_t)s.nchunk);
  LG_LAUNCH_CHECK();
  tmp.rewind(m);
}

}  // namespace lg
