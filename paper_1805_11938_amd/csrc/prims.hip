// Device primitives used by the format conversions: exclusive scans, a
// stable LSD radix sort of (key, value) pairs, reductions and fills.
#include <cstdarg>
#include <cstdlib>
#include <map>
#include <mutex>
#include <unordered_map>

#include "common.h"

namespace spmv {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;
thread_local RunTiming* g_timing = nullptr;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

spmv_status_t fail(spmv_status_t st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

const char* last_error_cstr() { return g_err.c_str(); }

// --------------------------------------------------------------- memory
// Device arrays come from hipMalloc, and freed ones are kept for reuse per
// device: hipMalloc and hipFree each cost tens of microseconds and hipFree
// waits for the device, while a format conversion allocates and frees a
// dozen arrays.  A request takes the smallest kept block of its device that
// holds it and wastes at most a quarter of it; blocks are rounded up to
// 256 B below 1 MiB and to 2 MiB above.  At most SPMV_CACHE_BYTES (read
// once; default 16 GiB, 0 keeps nothing) are kept, largest released first;
// a failed hipMalloc releases every kept block of the device and tries once
// more.  dfree waits for the device before keeping a block, as hipFree
// would, so no kernel still reads it when it is handed out again.
static std::mutex g_mem_mu;
static int64_t g_live = 0;    // bytes handed out (as requested)
static int64_t g_cached = 0;  // bytes of kept free blocks
struct LiveBlock {
  size_t req, cap;
  int dev;
};
static std::unordered_map<void*, LiveBlock> g_blocks;
static std::multimap<std::pair<int, size_t>, void*> g_free;  // (device, block bytes) -> block

static int64_t mem_cap() {
  static int64_t cap = [] {
    const char* e = getenv("SPMV_MEM_CAP_BYTES");
    return e ? (int64_t)strtoll(e, nullptr, 10) : (int64_t)0;
  }();
  return cap;
}

static int64_t cache_cap() {
  static int64_t cap = [] {
    const char* e = getenv("SPMV_CACHE_BYTES");
    return e ? (int64_t)strtoll(e, nullptr, 10) : (int64_t)16 << 30;
  }();
  return cap;
}

int64_t default_max_bytes() {
  static int64_t v = [] {
    const char* e = getenv("SPMV_MAX_BYTES");
    return e ? (int64_t)strtoll(e, nullptr, 10) : (int64_t)64 << 30;
  }();
  return v;
}

static size_t block_bytes(size_t b) {
  if (b <= ((size_t)1 << 20)) return (b + 255) / 256 * 256;
  const size_t m = (size_t)2 << 20;
  return (b + m - 1) / m * m;
}

// releases kept blocks of device dev (all devices when dev < 0) until at
// most keep bytes stay kept; largest first.  Caller holds g_mem_mu.
static int64_t release_locked(int dev, int64_t keep) {
  int64_t freed = 0;
  for (auto it = g_free.end(); it != g_free.begin() && g_cached > keep;) {
    --it;
    if (dev >= 0 && it->first.first != dev) continue;
    (void)hipFree(it->second);
    g_cached -= (int64_t)it->first.second;
    freed += (int64_t)it->first.second;
    it = g_free.erase(it);
  }
  return freed;
}

spmv_status_t dmalloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;  // never hand out null for an empty array
  int dev = 0;
  (void)hipGetDevice(&dev);
  const size_t want = block_bytes(bytes);
  std::lock_guard<std::mutex> g(g_mem_mu);
  const int64_t cap = mem_cap();
  if (cap > 0 && g_live + (int64_t)bytes > cap)
    return fail(SPMV_ERR_OOM, "SPMV_MEM_CAP_BYTES=%lld exceeded (live %lld + %zu)", (long long)cap,
                (long long)g_live, bytes);
  auto it = g_free.lower_bound(std::make_pair(dev, want));
  if (it != g_free.end() && it->first.first == dev && it->first.second <= want + want / 4) {
    *p = it->second;
    g_cached -= (int64_t)it->first.second;
    g_blocks[*p] = LiveBlock{bytes, it->first.second, dev};
    g_free.erase(it);
    g_live += (int64_t)bytes;
    return SPMV_OK;
  }
  hipError_t e = hipMalloc(p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release_locked(dev, 0);
    e = hipMalloc(p, want);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(SPMV_ERR_OOM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
  }
  g_blocks[*p] = LiveBlock{bytes, want, dev};
  g_live += (int64_t)bytes;
  return SPMV_OK;
}

void dfree(void* p) {
  if (!p) return;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> g(g_mem_mu);
  auto it = g_blocks.find(p);
  if (it == g_blocks.end()) return;  // not ours
  const LiveBlock b = it->second;
  g_blocks.erase(it);
  g_live -= (int64_t)b.req;
  if (cache_cap() <= 0 || (int64_t)b.cap > cache_cap()) {
    (void)hipFree(p);
    return;
  }
  if (b.dev != dev) (void)hipSetDevice(b.dev);
  (void)hipDeviceSynchronize();  // the block's last use has finished
  if (b.dev != dev) (void)hipSetDevice(dev);
  g_free.emplace(std::make_pair(b.dev, b.cap), p);
  g_cached += (int64_t)b.cap;
  if (g_cached > cache_cap()) release_locked(-1, cache_cap());
}

int64_t mem_in_use() {
  std::lock_guard<std::mutex> g(g_mem_mu);
  return g_live;
}

int64_t mem_release() {
  std::lock_guard<std::mutex> g(g_mem_mu);
  return release_locked(-1, 0);
}

int64_t resident_blocks(int per_cu) {
  static int cus[64] = {0};
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) dev = 0;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev] = n;
  }
  return (int64_t)cus[dev] * per_cu;
}

spmv_status_t copy_to_host(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return SPMV_OK;
  SPMV_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

// ----------------------------------------------------------------- fills
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static inline unsigned grid_for(int64_t n, int per_block = BS, int64_t cap = 1 << 20) {
  int64_t g = cdiv(n, per_block);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

spmv_status_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return SPMV_OK;
  k_fill_i32<<<grid_for(n), BS, 0, s>>>(p, v, n);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

// ------------------------------------------------------------ max length
__global__ void k_max_i32(const int32_t* a, int64_t n, int lens_from_ptr, int32_t* out) {
  __shared__ int32_t red[BS / WAVE];
  int32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = lens_from_ptr ? a[i + 1] - a[i] : a[i];
    m = v > m ? v : m;
  }
  for (int o = 32; o > 0; o >>= 1) {
    int32_t w = __shfl_xor(m, o, 64);
    m = w > m ? w : m;
  }
  if (__lane_id() == 0) red[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t r = red[0];
    for (int w = 1; w < BS / WAVE; ++w) r = red[w] > r ? red[w] : r;
    atomicMax(out, r);
  }
}

spmv_status_t device_max_i32(const int32_t* a, int64_t n, int lens_from_ptr, int32_t* out_host, hipStream_t s) {
  *out_host = 0;
  if (n <= 0) return SPMV_OK;
  DTmp d;
  SPMV_TRY(d.alloc(sizeof(int32_t)));
  SPMV_HIP(hipMemsetAsync(d.p, 0, sizeof(int32_t), s));
  k_max_i32<<<grid_for(n, BS, 1024), BS, 0, s>>>(a, n, lens_from_ptr, d.as<int32_t>());
  SPMV_LAUNCH_CHECK();
  return copy_to_host(out_host, d.p, sizeof(int32_t), s);
}

// ------------------------------------------------------------------ scan
// Tile = 256 threads x 8 items.  Pass 1 reduces tiles, the tile sums are
// scanned (recursively), pass 2 scans each tile and adds its offset.
constexpr int SCAN_IT = 8;
constexpr int SCAN_TILE = BS * SCAN_IT;

template <typename Tin>
__global__ void k_scan_reduce(const Tin* in, int64_t n, int64_t* part) {
  __shared__ int64_t red[BS / WAVE];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_IT; ++j) {
    int64_t i = base + j * BS + threadIdx.x;
    if (i < n) s += (int64_t)in[i];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (__lane_id() == 0) red[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Block-wide exclusive scan of one int64 per thread (256 threads).
__device__ int64_t block_excl_scan(int64_t v, int64_t* sh /* >= 4 */, int64_t* total) {
  const int lane = __lane_id(), w = threadIdx.x / WAVE;
  int64_t inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    int64_t u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  int64_t off = 0, tot = 0;
  for (int i = 0; i < BS / WAVE; ++i) {
    if (i < w) off += sh[i];
    tot += sh[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

template <typename Tin, typename Tout>
__global__ void k_scan_down(const Tin* in, int64_t n, const int64_t* part_off, Tout* out) {
  __shared__ int64_t stage[SCAN_TILE];
  __shared__ int64_t sh[BS / WAVE];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
  for (int j = 0; j < SCAN_IT; ++j) {
    int64_t i = base + j * BS + threadIdx.x;
    stage[j * BS + threadIdx.x] = i < n ? (int64_t)in[i] : 0;
  }
  __syncthreads();
  int64_t loc[SCAN_IT], s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_IT; ++j) {
    loc[j] = s;
    s += stage[threadIdx.x * SCAN_IT + j];
  }
  int64_t tot;
  int64_t off = block_excl_scan(s, sh, &tot) + part_off[blockIdx.x];
#pragma unroll
  for (int j = 0; j < SCAN_IT; ++j) stage[threadIdx.x * SCAN_IT + j] = off + loc[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < SCAN_IT; ++j) {
    int64_t i = base + j * BS + threadIdx.x;
    if (i < n) out[i] = (Tout)stage[j * BS + threadIdx.x];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = (Tout)(part_off[blockIdx.x] + tot);
}

template <typename Tin, typename Tout>
static spmv_status_t scan_impl(const Tin* in, Tout* out, int64_t n, hipStream_t s) {
  if (n <= 0) {
    SPMV_HIP(hipMemsetAsync(out, 0, sizeof(Tout), s));
    return SPMV_OK;
  }
  int64_t nb = cdiv(n, SCAN_TILE);
  DTmp part, part_off;
  SPMV_TRY(part.alloc(sizeof(int64_t) * nb));
  SPMV_TRY(part_off.alloc(sizeof(int64_t) * (nb + 1)));
  if (nb == 1) {
    SPMV_HIP(hipMemsetAsync(part_off.p, 0, sizeof(int64_t), s));  // one tile: offset 0
  } else {
    k_scan_reduce<Tin><<<(unsigned)nb, BS, 0, s>>>(in, n, part.as<int64_t>());
    SPMV_LAUNCH_CHECK();
    SPMV_TRY((scan_impl<int64_t, int64_t>(part.as<int64_t>(), part_off.as<int64_t>(), nb, s)));
  }
  k_scan_down<Tin, Tout><<<(unsigned)nb, BS, 0, s>>>(in, n, part_off.as<int64_t>(), out);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

spmv_status_t scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, hipStream_t s) {
  return scan_impl<int32_t, int64_t>(in, out, n, s);
}
spmv_status_t scan_i64_to_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  return scan_impl<int64_t, int64_t>(in, out, n, s);
}
spmv_status_t scan_i32_to_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
  return scan_impl<int32_t, int32_t>(in, out, n, s);
}

// ------------------------------------------------------------ radix sort
// Stable LSD radix sort, 8 bits per pass.  A tile is 8 rounds of 256 keys
// in input order; the scatter ranks each key among equal digits of earlier
// rounds (running counters), earlier waves (per-wave counts) and earlier
// lanes (ballot match), so equal digits keep their input order.
constexpr int RS_ROUNDS = 8;
constexpr int RS_TILE = BS * RS_ROUNDS;

__global__ void k_rs_hist(const uint64_t* keys, int64_t n, int shift, int32_t* counts, int64_t nb) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    int64_t i = base + r * BS + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_rs_scatter(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout, int64_t n,
                             int shift, const int32_t* offsets, int64_t nb) {
  __shared__ int32_t base_d[256];
  __shared__ int32_t wcnt[BS / WAVE][256];
  const int t = threadIdx.x, w = t / WAVE;
  base_d[t] = offsets[(int64_t)t * nb + blockIdx.x];
#pragma unroll
  for (int q = 0; q < BS / WAVE; ++q) wcnt[q][t] = 0;
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  const int64_t tile0 = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = tile0 + r * BS + t;
    const bool valid = i < n;
    uint64_t k = 0;
    uint32_t v = 0;
    if (valid) {
      k = kin[i];
      v = vin[i];
    }
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const int rank = __popcll(peers & lt);
    if (valid && (peers & lt) == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int off = base_d[d] + rank;
      for (int q = 0; q < w; ++q) off += wcnt[q][d];
      kout[off] = k;
      vout[off] = v;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int q = 0; q < BS / WAVE; ++q) {
      add += wcnt[q][t];
      wcnt[q][t] = 0;
    }
    base_d[t] += add;
    __syncthreads();
  }
}

spmv_status_t radix_sort_pairs(uint64_t** keys, uint32_t** vals, uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                               int key_bits, hipStream_t s) {
  if (n <= 1 || key_bits <= 0) return SPMV_OK;
  if (n >= ((int64_t)1 << 31)) return fail(SPMV_ERR_TOO_LARGE, "radix sort limited to < 2^31 keys");
  const int64_t nb = cdiv(n, RS_TILE);
  DTmp counts, offs;
  SPMV_TRY(counts.alloc(sizeof(int32_t) * 256 * nb));
  SPMV_TRY(offs.alloc(sizeof(int32_t) * (256 * nb + 1)));
  uint64_t *ka = *keys, *kb = keys_alt;
  uint32_t *va = *vals, *vb = vals_alt;
  for (int shift = 0; shift < key_bits; shift += 8) {
    k_rs_hist<<<(unsigned)nb, BS, 0, s>>>(ka, n, shift, counts.as<int32_t>(), nb);
    SPMV_LAUNCH_CHECK();
    SPMV_TRY(scan_i32_to_i32(counts.as<int32_t>(), offs.as<int32_t>(), 256 * nb, s));
    k_rs_scatter<<<(unsigned)nb, BS, 0, s>>>(ka, va, kb, vb, n, shift, offs.as<int32_t>(), nb);
    SPMV_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  *keys = ka;
  *vals = va;
  return SPMV_OK;
}

// ------------------------------------------------------ structure hash
// Order-independent 64-bit fingerprint of a CSR structure (ptr and col):
// the sum mod 2^64 of SplitMix64 finalisers of (position, value) pairs.
// Used to key the autotuner's cache; values do not affect performance and
// are not hashed.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(BS) void k_struct_hash(int64_t M, int64_t nnz, const int32_t* ptr, const int32_t* col,
                                                    unsigned long long* part) {
  __shared__ unsigned long long sh[BS / WAVE];
  unsigned long long h = 0;
  const int64_t n = M + 1 + nnz;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t v = i <= M ? (uint64_t)(uint32_t)ptr[i] : (uint64_t)(uint32_t)col[i - M - 1];
    h += mix64((uint64_t)i * 0x9E3779B97F4A7C15ull ^ (v << 1) ^ (i <= M ? 1ull : 0ull));
  }
  for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
  if (__lane_id() == 0) sh[threadIdx.x / WAVE] = h;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

spmv_status_t structure_hash(const spmv_mat_s* A, uint64_t* out, hipStream_t s) {
  constexpr int G = 512;
  DTmp part;
  SPMV_TRY(part.alloc(sizeof(unsigned long long) * G));
  k_struct_hash<<<G, BS, 0, s>>>(A->M, A->nnz, A->ptr, A->col, part.as<unsigned long long>());
  SPMV_LAUNCH_CHECK();
  unsigned long long h[G];
  SPMV_TRY(copy_to_host(h, part.p, sizeof(h), s));
  uint64_t t = 0;
  for (int i = 0; i < G; ++i) t += h[i];
  *out = t;
  return SPMV_OK;
}

}  // namespace spmv
