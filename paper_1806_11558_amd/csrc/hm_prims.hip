// Device-wide primitives: exclusive scan and a stable LSD radix sort.
//
// The level-wise tree construction and traversal of Sec. 3.1 ("Block cluster
// tree traversal") compute output offsets by parallel scans; the Morton
// clustering ("Spatial data structure") needs a parallel sort.  Both are
// written here for wave64: the sort ranks keys inside a wavefront with
// ballots (no atomics on the ranking path), so it is stable and
// deterministic.
#include <map>
#include <mutex>

#include "hm_internal.h"

namespace hm {

// ------------------------------------------------------------------ memory
// All device memory of the library comes from one stream-ordered pool per
// device, created on first use.  Freed memory stays cached in the pool (its
// release threshold is unlimited), so a rebuild reuses it instead of going
// back to the driver: allocations of recently freed device memory wait for
// the driver to clear it, which cost seconds for tens of GB.  trim_pool()
// (hm_release_memory) hands the cache back.
namespace {
constexpr uint64_t kPoolKeep = ~uint64_t(0);
std::mutex g_pool_mu;
hipMemPool_t g_pool[64] = {};
}  // namespace

hipMemPool_t lib_pool() {
  int dev = 0;
  HM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error{HM_ERR_HIP, "device index out of range"};
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (!g_pool[dev]) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    HM_HIP(hipMemPoolCreate(&pool, &props));
    uint64_t keep = kPoolKeep;
    HM_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
    g_pool[dev] = pool;
  }
  return g_pool[dev];
}

void trim_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (g_pool[dev]) (void)hipMemPoolTrimTo(g_pool[dev], 0);
  (void)hipGetLastError();
}

// Blocks of freed handles, per device, by size.  A later build that asks for
// a block of about the same size (at most 1/8 larger) takes it back, so that
// rebuilding a problem reuses its storage instead of fresh driver memory.
namespace {
std::mutex g_cache_mu;
std::multimap<size_t, void*> g_cache[64];
}  // namespace

void* cache_take(size_t bytes, size_t* got) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto& c = g_cache[dev];
  auto it = c.lower_bound(bytes);
  if (it == c.end() || it->first > bytes + bytes / 8) return nullptr;
  void* p = it->second;
  *got = it->first;
  c.erase(it);
  return p;
}

void cache_put(void* p, size_t bytes) {
  int dev = 0;
  if (!p || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache[dev].emplace(bytes, p);
}

void cache_release() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto& e : g_cache[dev]) (void)hipFreeAsync(e.second, nullptr);
  g_cache[dev].clear();
  (void)hipStreamSynchronize(nullptr);
}

void* dalloc(size_t bytes, hipStream_t s) {
  void* p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMallocFromPoolAsync(&p, bytes, lib_pool(), s);
  if (e != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    throw Error{HM_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
  }
  return p;
}

void dfree(void* p, hipStream_t s) {
  if (p) (void)hipFreeAsync(p, s);
}

int64_t d2h_i64(const int64_t* d, hipStream_t s) {
  int64_t v = 0;
  HM_HIP(hipMemcpyAsync(&v, d, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HM_HIP(hipStreamSynchronize(s));
  return v;
}

// ------------------------------------------------------------------ scan
namespace {
constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;   // 1024

__device__ inline int64_t wave_incl_scan(int64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ inline int64_t block_excl_scan(int64_t v, int64_t* out, int64_t* lds_w) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t inc = wave_incl_scan(v);
  if (lane == 63) lds_w[wave] = inc;
  __syncthreads();
  int64_t wpre = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    int64_t x = lds_w[w];
    if (w < wave) wpre += x;
    total += x;
  }
  *out = wpre + inc - v;
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const int64_t* in, int64_t n,
                                                            int64_t* sums) {
  __shared__ int64_t lds_w[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t v = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    int64_t i = base + (int64_t)threadIdx.x * kScanPer + k;
    if (i < n) v += in[i];
  }
  int64_t ex;
  int64_t total = block_excl_scan(v, &ex, lds_w);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// out[i] = offs[tile] + the exclusive prefix of in within the tile; the
// thread of element n - 1 also writes the grand total when total is given.
__global__ __launch_bounds__(kScanThreads) void k_tile_apply(const int64_t* in, int64_t* out,
                                                             int64_t n, const int64_t* offs,
                                                             int64_t* total) {
  __shared__ int64_t lds_w[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t loc[kScanPer];
  int64_t v = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    int64_t i = base + (int64_t)threadIdx.x * kScanPer + k;
    loc[k] = (i < n) ? in[i] : 0;
    v += loc[k];
  }
  int64_t ex;
  block_excl_scan(v, &ex, lds_w);
  int64_t run = ex + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    int64_t i = base + (int64_t)threadIdx.x * kScanPer + k;
    if (i < n) out[i] = run;
    if (total && i == n - 1) *total = run + loc[k];
    run += loc[k];
  }
}
}  // namespace

void scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* d_total, hipStream_t s) {
  if (n <= 0) {
    if (d_total) HM_HIP(hipMemsetAsync(d_total, 0, sizeof(int64_t), s));
    return;
  }
  const int64_t tiles = ceil_div(n, kScanTile);
  if (tiles == 1) {
    k_tile_apply<<<1, kScanThreads, 0, s>>>(in, out, n, nullptr, d_total);
    HM_LAUNCH_CHECK();
  } else {
    int64_t* sums = dalloc_t<int64_t>(tiles, s);
    int64_t* offs = dalloc_t<int64_t>(tiles, s);
    k_tile_sums<<<(unsigned)tiles, kScanThreads, 0, s>>>(in, n, sums);
    HM_LAUNCH_CHECK();
    scan_excl_i64(sums, offs, tiles, nullptr, s);
    k_tile_apply<<<(unsigned)tiles, kScanThreads, 0, s>>>(in, out, n, offs, d_total);
    HM_LAUNCH_CHECK();
    dfree(sums, s);
    dfree(offs, s);
  }
}

// ------------------------------------------------------------------ radix sort
namespace {
constexpr int kRadixThreads = 256;
constexpr int kRadixWaves = kRadixThreads / 64;
constexpr int kRadixPer = 4;                             // sub-rounds per tile
constexpr int kRadixTile = kRadixThreads * kRadixPer;    // 1024 keys
constexpr int kBins = 256;

__device__ inline uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Histogram of one digit per tile, stored digit-major: hist[d * tiles + tile].
__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const uint64_t* keys, int64_t n,
                                                              int shift, int64_t tiles,
                                                              int64_t* hist) {
  __shared__ int cnt[kBins];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  for (int k = 0; k < kRadixPer; ++k) {
    int64_t i = base + (int64_t)k * kRadixThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(int)((keys[i] >> shift) & 0xFF)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: keys of a tile are visited in index order, ranked inside
// each wavefront by ballot matching, then across wavefronts via LDS.
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(
    const uint64_t* kin, const int32_t* vin, uint64_t* kout, int32_t* vout, int64_t n, int shift,
    int64_t tiles, const int64_t* offs) {
  __shared__ int wcnt[kRadixWaves][kBins];
  __shared__ int run[kBins];
  const int wave = threadIdx.x >> 6;
  run[threadIdx.x] = 0;
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  for (int k = 0; k < kRadixPer; ++k) {
#pragma unroll
    for (int w = 0; w < kRadixWaves; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = base + (int64_t)k * kRadixThreads + threadIdx.x;
    const bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0;
    int32_t val = valid ? vin[i] : 0;
    const int d = (int)((key >> shift) & 0xFF);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int rank = (int)lanes_below(peers);
    const int npeers = __popcll(peers);
    if (valid && rank == npeers - 1) wcnt[wave][d] = npeers;   // last peer writes the count
    __syncthreads();
    {
      // thread t owns digit t: turn per-wave counts into exclusive offsets
      const int t = threadIdx.x;
      int acc = run[t];
#pragma unroll
      for (int w = 0; w < kRadixWaves; ++w) {
        int c = wcnt[w][t];
        wcnt[w][t] = acc;
        acc += c;
      }
      run[t] = acc;
    }
    __syncthreads();
    if (valid) {
      int64_t pos = offs[(int64_t)d * tiles + blockIdx.x] + wcnt[wave][d] + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
  }
}
}  // namespace

void radix_sort_u64_i32(uint64_t* keys, int32_t* vals, int64_t n, int bits, hipStream_t s) {
  if (n <= 1 || bits <= 0) return;
  const int passes = (bits + 7) / 8;
  const int64_t tiles = ceil_div(n, kRadixTile);
  uint64_t* k2 = dalloc_t<uint64_t>(n, s);
  int32_t* v2 = dalloc_t<int32_t>(n, s);
  int64_t* hist = dalloc_t<int64_t>(tiles * kBins, s);
  int64_t* offs = dalloc_t<int64_t>(tiles * kBins, s);
  uint64_t *ka = keys, *kb = k2;
  int32_t *va = vals, *vb = v2;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    k_radix_hist<<<(unsigned)tiles, kRadixThreads, 0, s>>>(ka, n, shift, tiles, hist);
    HM_LAUNCH_CHECK();
    scan_excl_i64(hist, offs, tiles * kBins, nullptr, s);
    k_radix_scatter<<<(unsigned)tiles, kRadixThreads, 0, s>>>(ka, va, kb, vb, n, shift, tiles,
                                                              offs);
    HM_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    HM_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    HM_HIP(hipMemcpyAsync(vals, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
  dfree(k2, s);
  dfree(v2, s);
  dfree(hist, s);
  dfree(offs, s);
}

}  // namespace hm
