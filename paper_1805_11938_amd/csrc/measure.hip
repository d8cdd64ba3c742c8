// Measurement (the timing protocol of Sec. V-B, "Generating Training
// Data": repeat until the 95% confidence interval is within the requested
// relative width), the cache scrub and a copy-bandwidth probe.
#include <cmath>
#include <mutex>

#include "common.h"

namespace spmv {

// ------------------------------------------------------------ cache scrub
// MI355X has 4 MB of L2 per XCD and a 256 MB memory-side Infinity Cache; a
// read pass over a buffer well above both evicts the matrix between timed
// launches.  The pass only reads, so the caches are left holding clean lines:
// a timed launch that evicts them pays no write-back that a real sequence of
// SpMVs would not pay.  (The buffer is zero; the sum is never 1, so the
// conditional store keeps the loads alive without ever writing.)
static std::mutex g_scrub_mu;
static float* g_scrub = nullptr;
static int64_t g_scrub_bytes = 0;

__global__ void k_scrub(const float4* __restrict__ p, int64_t n, float* __restrict__ sink) {
  float acc = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float4 v = p[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  if (acc == 1.0f) sink[0] = acc;
}

spmv_status_t scrub(int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return SPMV_OK;
  bytes = (bytes + 15) / 16 * 16;
  const float* buf = nullptr;
  float* sink = nullptr;
  {
    std::lock_guard<std::mutex> g(g_scrub_mu);
    if (bytes > g_scrub_bytes) {
      if (g_scrub) dfree(g_scrub);
      g_scrub = nullptr;
      g_scrub_bytes = 0;
      void* p = nullptr;
      SPMV_TRY(dmalloc(&p, (size_t)bytes + 16));  // + a sink word past the buffer
      SPMV_HIP(hipMemsetAsync(p, 0, (size_t)bytes + 16, s));
      g_scrub = (float*)p;
      g_scrub_bytes = bytes;
    }
    buf = g_scrub;
    sink = g_scrub + g_scrub_bytes / 4;
  }
  const int64_t n = bytes / 16;
  k_scrub<<<(unsigned)std::min<int64_t>(cdiv(n, BS), 8192), BS, 0, s>>>((const float4*)buf, n, sink);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

// ------------------------------------------------------------ copy probe
typedef double d2 __attribute__((ext_vector_type(2)));
__global__ void k_copy(const d2* __restrict__ a, d2* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = __builtin_nontemporal_load(a + i);
}

// Student t quantile t_{0.975, df}
static double t975(int df) {
  static const double tab[] = {0,      12.706, 4.303, 3.182, 2.776, 2.571, 2.447, 2.365, 2.306, 2.262, 2.228,
                               2.201,  2.179,  2.160, 2.145, 2.131, 2.120, 2.110, 2.101, 2.093, 2.086, 2.080,
                               2.074,  2.069,  2.064, 2.060, 2.056, 2.052, 2.048, 2.045, 2.042};
  if (df <= 0) return 1e9;
  if (df <= 30) return tab[df];
  if (df <= 60) return 2.000;
  if (df <= 120) return 1.980;
  return 1.960;
}

struct Stats {
  double median, mean, half, n, min;
};

static Stats summarize(std::vector<float>& t) {
  Stats st{0, 0, 0, (double)t.size(), 0};
  if (t.empty()) return st;
  std::vector<float> c(t);
  std::sort(c.begin(), c.end());
  const size_t n = c.size();
  st.median = n % 2 ? c[n / 2] : 0.5 * ((double)c[n / 2 - 1] + c[n / 2]);
  st.min = c[0];
  double m = 0;
  for (float v : c) m += v;
  m /= n;
  double var = 0;
  for (float v : c) var += (v - m) * (v - m);
  var = n > 1 ? var / (n - 1) : 0;
  st.mean = m;
  st.half = t975((int)n - 1) * std::sqrt(var / n);
  return st;
}

template <class Launch>
static spmv_status_t timed(Launch&& launch, int warmup, int min_reps, int max_reps, double rel_ci, int64_t scrub_bytes,
                           hipStream_t s, double out[5]) {
  if (min_reps < 1) min_reps = 1;
  if (max_reps < min_reps) max_reps = min_reps;
  for (int i = 0; i < warmup; ++i) SPMV_TRY(launch());
  hipEvent_t e0, e1;
  SPMV_HIP(hipEventCreate(&e0));
  SPMV_HIP(hipEventCreate(&e1));
  std::vector<float> ts;
  spmv_status_t st = SPMV_OK;
  for (int r = 0; r < max_reps; ++r) {
    if (scrub_bytes > 0 && (st = scrub(scrub_bytes, s)) != SPMV_OK) break;
    if (hipEventRecord(e0, s) != hipSuccess) { st = fail(SPMV_ERR_HIP, "hipEventRecord"); break; }
    if ((st = launch()) != SPMV_OK) break;
    if (hipEventRecord(e1, s) != hipSuccess) { st = fail(SPMV_ERR_HIP, "hipEventRecord"); break; }
    if (hipEventSynchronize(e1) != hipSuccess) { st = fail(SPMV_ERR_HIP, "hipEventSynchronize"); break; }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ts.push_back(ms);
    if ((int)ts.size() >= min_reps) {
      Stats q = summarize(ts);
      if (q.mean > 0 && 2.0 * q.half / q.mean < rel_ci) break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != SPMV_OK) return st;
  Stats q = summarize(ts);
  out[0] = q.median;
  out[1] = q.mean;
  out[2] = q.half;
  out[3] = q.n;
  out[4] = q.min;
  return SPMV_OK;
}

spmv_status_t time_run(spmv_mat_s* A, const void* x, void* y, int warmup, int min_reps, int max_reps, double rel_ci,
                       int64_t scrub_bytes, hipStream_t s, double out[5]) {
  return timed([&] { return dispatch_run(A, x, y, s); }, warmup, min_reps, max_reps, rel_ci, scrub_bytes, s, out);
}

// ------------------------------------------------------------ gather probe
// A perfectly balanced SpMV without any locality in x: row i sums GP_J
// products v * x[c] whose columns are uniform over [0, nx) (SplitMix64 of
// the slot index and a seed), stored slot-major so the column and value
// loads are coalesced, with every load of a row in flight at once.  Its time
// is the floor for gathering that many entries from an x of nx values: the
// roofline of launches bound by scattered gathers rather than by HBM bytes.
constexpr int GP_J = 16;

__global__ void k_gp_fill(int64_t total, uint64_t nx, uint64_t seed, int32_t* __restrict__ col) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)t * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    col[t] = (int32_t)(z % nx);
  }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_gather_probe(int64_t rows, const int32_t* __restrict__ col,
                                                     const T* __restrict__ val, const T* __restrict__ x,
                                                     T* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= rows) return;
  int32_t c[GP_J];
  T v[GP_J], xv[GP_J];
#pragma unroll
  for (int j = 0; j < GP_J; ++j) c[j] = ldnt(col + (int64_t)j * rows + i);
#pragma unroll
  for (int j = 0; j < GP_J; ++j) v[j] = ldnt(val + (int64_t)j * rows + i);
  issue_fence();
#pragma unroll
  for (int j = 0; j < GP_J; ++j) xv[j] = x[c[j]];
  issue_fence();
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < GP_J; ++j) s += (double)v[j] * (double)xv[j];
  y[i] = (T)s;
}

}  // namespace spmv

using namespace spmv;

extern "C" {

spmv_status_t spmv_time(spmv_fmt_t fmt, spmv_mat_t A, const void* x, void* y, int warmup, int min_reps, int max_reps,
                        double rel_ci, int64_t scrub_bytes, spmv_stream_t s, double out[5]) {
  if (!A || !out) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if (fmt != A->fmt) return fail(SPMV_ERR_INVALID_ARG, "format mismatch");
  if (A->M && (!y || (A->N && !x))) return fail(SPMV_ERR_INVALID_ARG, "null x or y");
  return time_run(A, x, y, warmup, min_reps, max_reps, rel_ci, scrub_bytes, hs(s), out);
}

spmv_status_t spmv_scrub(int64_t scrub_bytes, spmv_stream_t s) { return scrub(scrub_bytes, hs(s)); }

spmv_status_t spmv_copy_probe(int64_t bytes, int reps, spmv_stream_t s, double* gbps) {
  if (bytes <= 0 || !gbps) return fail(SPMV_ERR_INVALID_ARG, "bytes/gbps");
  bytes = (bytes + 15) / 16 * 16;
  DTmp a, b;
  SPMV_TRY(a.alloc((size_t)bytes));
  SPMV_TRY(b.alloc((size_t)bytes));
  hipStream_t st = hs(s);
  SPMV_HIP(hipMemsetAsync(a.p, 0, (size_t)bytes, st));
  const int64_t n = bytes / 16;
  const unsigned g = (unsigned)std::min<int64_t>(cdiv(n, BS), 1 << 16);
  double out[5];
  SPMV_TRY(timed(
      [&]() -> spmv_status_t {
        k_copy<<<g, BS, 0, st>>>(a.as<d2>(), b.as<d2>(), n);
        SPMV_LAUNCH_CHECK();
        return SPMV_OK;
      },
      3, reps, reps, 0.0, 0, st, out));
  *gbps = 2.0 * (double)bytes / (out[0] * 1e-3) / 1e9;
  return SPMV_OK;
}

spmv_status_t spmv_gather_probe(int64_t nx, int64_t rows, spmv_dtype_t dt, int reps, int64_t scrub_bytes,
                                spmv_stream_t s, double* ms) {
  if (nx < 1 || nx >= ((int64_t)1 << 31) || rows < 1 || rows > ((int64_t)1 << 27) || !ms || reps < 1)
    return fail(SPMV_ERR_INVALID_ARG, "gather probe: need 1 <= nx < 2^31, 1 <= rows <= 2^27, reps >= 1, ms");
  if (dt != SPMV_F64 && dt != SPMV_F32) return fail(SPMV_ERR_INVALID_ARG, "dtype %d", (int)dt);
  const int64_t sv = value_size(dt), total = rows * GP_J;
  DTmp x, c, v, y;
  SPMV_TRY(x.alloc((size_t)(nx * sv)));
  SPMV_TRY(c.alloc((size_t)(total * 4)));
  SPMV_TRY(v.alloc((size_t)(total * sv)));
  SPMV_TRY(y.alloc((size_t)(rows * sv)));
  hipStream_t st = hs(s);
  SPMV_HIP(hipMemsetAsync(x.p, 0, (size_t)(nx * sv), st));
  SPMV_HIP(hipMemsetAsync(v.p, 0, (size_t)(total * sv), st));
  k_gp_fill<<<(unsigned)std::min<int64_t>(cdiv(total, BS), 8192), BS, 0, st>>>(total, (uint64_t)nx, 0x5EEDull,
                                                                              c.as<int32_t>());
  SPMV_LAUNCH_CHECK();
  const unsigned g = (unsigned)cdiv(rows, BS);
  double out[5];
  SPMV_TRY(timed(
      [&]() -> spmv_status_t {
        if (dt == SPMV_F64)
          k_gather_probe<double><<<g, BS, 0, st>>>(rows, c.as<int32_t>(), v.as<double>(), x.as<double>(), y.as<double>());
        else
          k_gather_probe<float><<<g, BS, 0, st>>>(rows, c.as<int32_t>(), v.as<float>(), x.as<float>(), y.as<float>());
        SPMV_LAUNCH_CHECK();
        return SPMV_OK;
      },
      2, reps, reps, 0.0, scrub_bytes, st, out));
  *ms = out[0];
  return SPMV_OK;
}

}  // extern "C"
