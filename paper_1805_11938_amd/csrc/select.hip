// Format selection (Sec. V): static matrix features (Table IV plus nnz,
// ELL padding ratio, bandwidth and the Gini index of row lengths), feature
// scaling with the training set's minimum and maximum (Sec. V-B, "Feature
// Scaling"), and a multilayer-perceptron classifier (one of the alternative
// models of Sec. V-D): 12 -> 64 -> 64 -> 5, ReLU, softmax cross-entropy,
// trained with Adam by the kernels below.
//
// Features are exact integer reductions on the device (row-length moments
// in int64, Gini from a histogram of row lengths), finished in FP64.  The
// MLP runs in FP32 with fixed summation orders (no atomics), so training
// is reproducible run to run.
#include <cmath>
#include <cstring>
#include <mutex>

#include "common.h"

namespace spmv {

// =============================================================== features
struct FeatAcc {
  int32_t minlen, maxlen, band, pad;
  unsigned long long sum, sumsq, gini;  // gini: two's complement int64 accumulated mod 2^64
};

__global__ void k_feat_init(FeatAcc* a) {
  a->minlen = INT32_MAX;
  a->maxlen = 0;
  a->band = 0;
  a->pad = 0;
  a->sum = a->sumsq = a->gini = 0;
}

// Per-block partials (no contended atomics): minimum, maximum and the
// bandwidth of the block's rows, their length sum and sum of squares.
struct FeatPart {
  int32_t minlen, maxlen, band, pad;
  unsigned long long sum, sumsq;
};

__global__ __launch_bounds__(BS) void k_feat_rows(int64_t M, const int32_t* ptr, const int32_t* col, FeatPart* part) {
  __shared__ int32_t smin[BS / WAVE], smax[BS / WAVE], sband[BS / WAVE];
  __shared__ unsigned long long ssum[BS / WAVE], ssq[BS / WAVE];
  int32_t mn = INT32_MAX, mx = 0, band = 0;
  unsigned long long sum = 0, sq = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = ptr[i], b = ptr[i + 1], len = b - a;
    mn = len < mn ? len : mn;
    mx = len > mx ? len : mx;
    sum += (unsigned long long)len;
    sq += (unsigned long long)len * (unsigned long long)len;
    if (len > 0) {  // columns are sorted: the extremes are the first and last
      const int64_t d0 = i - (int64_t)col[a], d1 = (int64_t)col[b - 1] - i;
      const int64_t d = d0 > d1 ? d0 : d1;
      band = d > band ? (int32_t)d : band;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64), c = __shfl_xor(band, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
    band = c > band ? c : band;
    sum += __shfl_xor(sum, o, 64);
    sq += __shfl_xor(sq, o, 64);
  }
  const int w = threadIdx.x / WAVE;
  if (__lane_id() == 0) {
    smin[w] = mn;
    smax[w] = mx;
    sband[w] = band;
    ssum[w] = sum;
    ssq[w] = sq;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < BS / WAVE; ++q) {
      mn = smin[q] < mn ? smin[q] : mn;
      mx = smax[q] > mx ? smax[q] : mx;
      band = sband[q] > band ? sband[q] : band;
      sum += ssum[q];
      sq += ssq[q];
    }
    FeatPart p;
    p.minlen = mn;
    p.maxlen = mx;
    p.band = band;
    p.pad = 0;
    p.sum = sum;
    p.sumsq = sq;
    part[blockIdx.x] = p;
  }
}

// One workgroup folds the per-block partials into the accumulator.
__global__ __launch_bounds__(BS) void k_feat_fold(int nparts, const FeatPart* part, FeatAcc* acc) {
  __shared__ int32_t smin[BS / WAVE], smax[BS / WAVE], sband[BS / WAVE];
  __shared__ unsigned long long ssum[BS / WAVE], ssq[BS / WAVE];
  int32_t mn = INT32_MAX, mx = 0, band = 0;
  unsigned long long sum = 0, sq = 0;
  for (int i = threadIdx.x; i < nparts; i += BS) {
    const FeatPart p = part[i];
    mn = p.minlen < mn ? p.minlen : mn;
    mx = p.maxlen > mx ? p.maxlen : mx;
    band = p.band > band ? p.band : band;
    sum += p.sum;
    sq += p.sumsq;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64), c = __shfl_xor(band, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
    band = c > band ? c : band;
    sum += __shfl_xor(sum, o, 64);
    sq += __shfl_xor(sq, o, 64);
  }
  const int w = threadIdx.x / WAVE;
  if (__lane_id() == 0) {
    smin[w] = mn;
    smax[w] = mx;
    sband[w] = band;
    ssum[w] = sum;
    ssq[w] = sq;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < BS / WAVE; ++q) {
      mn = smin[q] < mn ? smin[q] : mn;
      mx = smax[q] > mx ? smax[q] : mx;
      band = sband[q] > band ? sband[q] : band;
      sum += ssum[q];
      sq += ssq[q];
    }
    acc->minlen = mn;
    acc->maxlen = mx;
    acc->band = band;
    acc->pad = 0;
    acc->sum = sum;
    acc->sumsq = sq;
    acc->gini = 0;
  }
}

// Row-length histogram.  Regular matrices put most rows in a handful of
// bins, so each block counts lengths below HB in LDS and adds its non-zero
// bins to the global histogram once; only longer rows go to global atomics.
constexpr int HB = 4096;

__global__ __launch_bounds__(BS) void k_feat_hist(int64_t M, int64_t nv, const int32_t* ptr, int32_t* hist) {
  __shared__ int32_t sh[HB];
  for (int b = threadIdx.x; b < HB; b += BS) sh[b] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t len = ptr[i + 1] - ptr[i];
    if (len < HB)
      atomicAdd(&sh[len], 1);
    else
      atomicAdd(&hist[len], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < HB && b < nv; b += BS)
    if (sh[b]) atomicAdd(&hist[b], sh[b]);
}

// Gini numerator: rows of length v fill sorted positions a_v+1 .. a_v+c_v
// (1-based), contributing v * sum (2i - M - 1) = v * c_v * (2 a_v + c_v - M).
__global__ void k_feat_gini(int64_t nv, int64_t M, const int32_t* hist, const int64_t* below, FeatAcc* acc) {
  __shared__ unsigned long long s[BS / WAVE];
  unsigned long long g = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = hist[v];
    if (c) g += (unsigned long long)(v * c * (2 * below[v] + c - M));
  }
  for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o, 64);
  if (__lane_id() == 0) s[threadIdx.x / WAVE] = g;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&acc->gini, s[0] + s[1] + s[2] + s[3]);
}

__global__ void k_feat_final(int64_t M, int64_t N, int64_t nnz, const FeatAcc* acc, double* f) {
  const double Md = (double)M, nz = (double)nnz;
  const int64_t mn = M > 0 ? acc->minlen : 0, mx = acc->maxlen;
  const unsigned long long S = acc->sum, Q = acc->sumsq;
  // population variance (M*Q - S^2) / M^2 with the numerator in 128 bits
  const unsigned long long p1lo = (unsigned long long)M * Q, p1hi = __umul64hi((unsigned long long)M, Q);
  const unsigned long long p2lo = S * S, p2hi = __umul64hi(S, S);
  const unsigned long long lo = p1lo - p2lo, hi = p1hi - p2hi - (p1lo < p2lo ? 1ull : 0ull);
  const double num = (double)hi * 18446744073709551616.0 + (double)lo;
  const double mean = M > 0 ? (double)S / Md : 0.0;
  const double sd = M > 0 ? sqrt(num / (Md * Md)) : 0.0;
  f[0] = Md;
  f[1] = (double)N;
  f[2] = nz;
  f[3] = (M > 0 && N > 0) ? nz / (Md * (double)N) : 0.0;
  f[4] = (double)mn;
  f[5] = (double)mx;
  f[6] = mean;
  f[7] = sd;
  f[8] = mean > 0.0 ? sd / mean : 0.0;
  f[9] = nnz > 0 ? Md * (double)mx / nz : 0.0;
  f[10] = (double)acc->band;
  f[11] = nnz > 0 ? (double)(long long)acc->gini / (Md * nz) : 0.0;
}

// Exclusive scan of the histogram by one workgroup (nv is at most the
// longest row + 1, so this is short), carrying the running total in int64.
__global__ __launch_bounds__(BS) void k_feat_below(int64_t nv, const int32_t* hist, int64_t* below) {
  __shared__ int64_t wsum[BS / WAVE];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = __lane_id(), w = threadIdx.x / WAVE;
  for (int64_t c0 = 0; c0 < nv; c0 += BS) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < nv ? hist[i] : 0;
    int64_t inc = v;  // inclusive scan inside the wave
    for (int o = 1; o < WAVE; o <<= 1) {
      const int64_t u = __shfl_up(inc, o, 64);
      if (lane >= o) inc += u;
    }
    if (lane == WAVE - 1) wsum[w] = inc;
    __syncthreads();
    int64_t before = carry;
    for (int q = 0; q < w; ++q) before += wsum[q];
    if (i < nv) below[i] = before + inc - v;
    __syncthreads();
    if (threadIdx.x == BS - 1) carry = before + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) below[nv] = carry;
}

// Feature workspace: kept for the life of the process (grow-only) and used
// under a lock, so a features call allocates nothing after the first.
static std::mutex g_feat_mu;
static void* g_feat_ws = nullptr;
static size_t g_feat_bytes = 0;

spmv_status_t features(spmv_mat_s* A, double* out_host, hipStream_t s) {
  if (A->fmt != SPMV_FMT_CSR || !A->sub.empty())
    return fail(SPMV_ERR_INVALID_ARG, "features need a CSR handle without column bands");
  const int64_t M = A->M;
  std::lock_guard<std::mutex> lock(g_feat_mu);
  auto reserve = [&](size_t bytes) -> spmv_status_t {
    if (bytes <= g_feat_bytes) return SPMV_OK;
    if (g_feat_ws) {
      SPMV_HIP(hipDeviceSynchronize());
      dfree(g_feat_ws);
      g_feat_ws = nullptr;
      g_feat_bytes = 0;
    }
    SPMV_TRY(dmalloc(&g_feat_ws, bytes));
    g_feat_bytes = bytes;
    return SPMV_OK;
  };
  constexpr int MAXG = 2048;                                // feature blocks
  constexpr size_t SMALL = 256 + MAXG * sizeof(FeatPart);  // FeatAcc, 12 doubles, per-block partials
  SPMV_TRY(reserve(SMALL + 4096));
  FeatAcc* acc = (FeatAcc*)g_feat_ws;
  double* fo = (double*)((char*)g_feat_ws + 128);
  FeatPart* parts = (FeatPart*)((char*)g_feat_ws + 256);
  k_feat_init<<<1, 1, 0, s>>>(acc);
  SPMV_LAUNCH_CHECK();
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(M, BS), MAXG));
  if (M) {
    k_feat_rows<<<g, BS, 0, s>>>(M, A->ptr, A->col, parts);
    SPMV_LAUNCH_CHECK();
    k_feat_fold<<<1, BS, 0, s>>>((int)g, parts, acc);
    SPMV_LAUNCH_CHECK();
    FeatAcc h;
    SPMV_TRY(copy_to_host(&h, acc, sizeof(FeatAcc), s));
    const int64_t nv = (int64_t)h.maxlen + 1;
    const size_t hb = ((size_t)nv * sizeof(int32_t) + 255) / 256 * 256;
    SPMV_TRY(reserve(SMALL + hb + sizeof(int64_t) * (nv + 1)));
    acc = (FeatAcc*)g_feat_ws;
    fo = (double*)((char*)g_feat_ws + 128);
    int32_t* hist = (int32_t*)((char*)g_feat_ws + SMALL);
    int64_t* below = (int64_t*)((char*)g_feat_ws + SMALL + hb);
    SPMV_HIP(hipMemcpyAsync(acc, &h, sizeof(FeatAcc), hipMemcpyHostToDevice, s));  // the buffer may have moved
    SPMV_HIP(hipMemsetAsync(hist, 0, sizeof(int32_t) * nv, s));
    k_feat_hist<<<(unsigned)std::min<int64_t>(g, 512), BS, 0, s>>>(M, nv, A->ptr, hist);
    SPMV_LAUNCH_CHECK();
    if (nv <= 65536) {  // short: one workgroup, no temporaries
      k_feat_below<<<1, BS, 0, s>>>(nv, hist, below);
      SPMV_LAUNCH_CHECK();
    } else {
      SPMV_TRY(scan_i32_to_i64(hist, below, nv, s));
    }
    const unsigned gv = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(nv, BS), 2048));
    k_feat_gini<<<gv, BS, 0, s>>>(nv, M, hist, below, acc);
    SPMV_LAUNCH_CHECK();
  }
  k_feat_final<<<1, 1, 0, s>>>(M, A->N, A->nnz, acc, fo);
  SPMV_LAUNCH_CHECK();
  return copy_to_host(out_host, fo, 12 * sizeof(double), s);
}

// ==================================================================== MLP
constexpr int NIN = 12, NH = 64, NOUT = 5;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NIN * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NOUT, NPARAM = OFF_B3 + NOUT;
static_assert(NPARAM == SPMV_MLP_NPARAM, "parameter layout");

// Forward of one sample by one wave (lane j = hidden unit j).  Hidden
// activations are exchanged with shuffles; every sum runs in index order.
struct Fwd {
  float a1, h1, a2, h2, z;  // z valid on lanes 0..4
};

__device__ __forceinline__ Fwd mlp_fwd_wave(const float* __restrict__ P, const float* __restrict__ xrow) {
  const int j = __lane_id();
  Fwd r;
  float a = P[OFF_B1 + j];
#pragma unroll
  for (int i = 0; i < NIN; ++i) a = fmaf(xrow[i], P[OFF_W1 + i * NH + j], a);
  r.a1 = a;
  r.h1 = fmaxf(a, 0.0f);
  a = P[OFF_B2 + j];
#pragma unroll 8
  for (int i = 0; i < NH; ++i) a = fmaf(__shfl(r.h1, i, 64), P[OFF_W2 + i * NH + j], a);
  r.a2 = a;
  r.h2 = fmaxf(a, 0.0f);
  const int c = j < NOUT ? j : 0;
  a = P[OFF_B3 + c];
#pragma unroll 8
  for (int i = 0; i < NH; ++i) a = fmaf(__shfl(r.h2, i, 64), P[OFF_W3 + i * NOUT + c], a);
  r.z = a;
  return r;
}

__global__ __launch_bounds__(BS) void k_mlp_forward(const float* __restrict__ P, const float* __restrict__ X, int32_t B,
                                                    float* __restrict__ Z, float* __restrict__ A1,
                                                    float* __restrict__ A2) {
  const int64_t nw = (int64_t)gridDim.x * (BS / WAVE);
  const int j = __lane_id();
  for (int64_t b = (int64_t)blockIdx.x * (BS / WAVE) + threadIdx.x / WAVE; b < B; b += nw) {
    const Fwd r = mlp_fwd_wave(P, X + b * NIN);
    if (j < NOUT) Z[b * NOUT + j] = r.z;
    if (A1) A1[b * NH + j] = r.a1;
    if (A2) A2[b * NH + j] = r.a2;
  }
}

// Backward deltas of one sample per wave; the mean over the batch is folded
// into dz = (softmax(z) - onehot(label)) / B.
__global__ __launch_bounds__(BS) void k_mlp_delta(const float* __restrict__ P, const float* __restrict__ X,
                                                  const int32_t* __restrict__ labels, int32_t B,
                                                  float* __restrict__ H1, float* __restrict__ H2,
                                                  float* __restrict__ DZ, float* __restrict__ DA1,
                                                  float* __restrict__ DA2, float* __restrict__ loss) {
  const int64_t nw = (int64_t)gridDim.x * (BS / WAVE);
  const int j = __lane_id();
  for (int64_t b = (int64_t)blockIdx.x * (BS / WAVE) + threadIdx.x / WAVE; b < B; b += nw) {
    const Fwd r = mlp_fwd_wave(P, X + b * NIN);
    float zc[NOUT];
#pragma unroll
    for (int c = 0; c < NOUT; ++c) zc[c] = __shfl(r.z, c, 64);
    float m = zc[0];
#pragma unroll
    for (int c = 1; c < NOUT; ++c) m = fmaxf(m, zc[c]);
    float se = 0.0f;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) se += expf(zc[c] - m);
    const int y = min(max(labels[b], 0), NOUT - 1);  // labels outside 0..4 are clamped
    const float invB = 1.0f / (float)B;
    float dz = 0.0f;
    if (j < NOUT) dz = (expf(zc[j] - m) / se - (j == y ? 1.0f : 0.0f)) * invB;
    float dh2 = 0.0f;
#pragma unroll
    for (int c = 0; c < NOUT; ++c) dh2 = fmaf(__shfl(dz, c, 64), P[OFF_W3 + j * NOUT + c], dh2);
    const float da2 = r.a2 > 0.0f ? dh2 : 0.0f;
    float dh1 = 0.0f;
#pragma unroll 8
    for (int q = 0; q < NH; ++q) dh1 = fmaf(__shfl(da2, q, 64), P[OFF_W2 + j * NH + q], dh1);
    const float da1 = r.a1 > 0.0f ? dh1 : 0.0f;
    H1[b * NH + j] = r.h1;
    H2[b * NH + j] = r.h2;
    DA1[b * NH + j] = da1;
    DA2[b * NH + j] = da2;
    if (j < NOUT) DZ[b * NOUT + j] = dz;
    if (j == 0) loss[b] = (m + logf(se)) - zc[y];
  }
}

// One thread per parameter: the gradient is a sum over the batch in order.
__global__ void k_mlp_wgrad(const float* __restrict__ X, const float* __restrict__ H1, const float* __restrict__ H2,
                            const float* __restrict__ DZ, const float* __restrict__ DA1,
                            const float* __restrict__ DA2, int32_t B, float* __restrict__ G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float* in = nullptr;
  const float* d = nullptr;
  int nin = 0, nd = 0, i = 0, jj = 0;
  bool bias = false;
  if (p < OFF_B1) { in = X; nin = NIN; d = DA1; nd = NH; i = p / NH; jj = p % NH; }
  else if (p < OFF_W2) { d = DA1; nd = NH; jj = p - OFF_B1; bias = true; }
  else if (p < OFF_B2) { in = H1; nin = NH; d = DA2; nd = NH; i = (p - OFF_W2) / NH; jj = (p - OFF_W2) % NH; }
  else if (p < OFF_W3) { d = DA2; nd = NH; jj = p - OFF_B2; bias = true; }
  else if (p < OFF_B3) { in = H2; nin = NH; d = DZ; nd = NOUT; i = (p - OFF_W3) / NOUT; jj = (p - OFF_W3) % NOUT; }
  else { d = DZ; nd = NOUT; jj = p - OFF_B3; bias = true; }
  float g = 0.0f;
  for (int b = 0; b < B; ++b) g = bias ? g + d[b * nd + jj] : fmaf(in[b * nin + i], d[b * nd + jj], g);
  G[p] = g;
}

__global__ void k_mean(const float* __restrict__ v, int32_t n, float* __restrict__ out, float* __restrict__ acc,
                       float weight) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.0f;
  for (int i = 0; i < n; ++i) s += v[i];
  s /= (float)n;
  if (out) *out = s;
  if (acc) *acc += s * weight;
}

__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ m, float* __restrict__ v,
                       int32_t t, float lr, float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float bc1 = 1.0f - powf(b1, (float)t), bc2 = 1.0f - powf(b2, (float)t);
  const float g = G[p];
  const float mi = b1 * m[p] + (1.0f - b1) * g;
  const float vi = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mi;
  v[p] = vi;
  P[p] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// log transform + min-max scaling (FP64), stored as FP32
__device__ __forceinline__ double feat_transform(int k, double v) {
  if (k == 3) return log2(v > 5.421010862427522e-20 ? v : 5.421010862427522e-20);  // 2^-64 floor
  if (k == 8 || k == 11) return v;
  return log2(1.0 + v);
}

__global__ void k_scale(const double* __restrict__ F, int32_t n, const double* __restrict__ lo,
                        const double* __restrict__ hi, float* __restrict__ X) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * NIN) return;
  const int k = (int)(q % NIN);
  const double t = feat_transform(k, F[q]);
  const double span = hi[k] - lo[k];
  X[q] = span > 0.0 ? (float)((t - lo[k]) / span) : 0.0f;
}

// per-feature minimum and maximum of the transformed features (one thread
// per feature, rows in order)
__global__ void k_feat_range(const double* __restrict__ F, int32_t n, double* __restrict__ lo,
                             double* __restrict__ hi) {
  const int k = threadIdx.x;
  if (k >= NIN) return;
  double a = 1e308, b = -1e308;
  for (int32_t i = 0; i < n; ++i) {
    const double t = feat_transform(k, F[(int64_t)i * NIN + k]);
    a = t < a ? t : a;
    b = t > b ? t : b;
  }
  lo[k] = a;
  hi[k] = b;
}

// single-sample inference: scale, forward, argmax (ties -> lower index)
__global__ void k_select(const float* __restrict__ P, const double* __restrict__ F, const double* __restrict__ lo,
                         const double* __restrict__ hi, int32_t* __restrict__ best, float* __restrict__ scores) {
  __shared__ float xs[NIN];
  const int j = __lane_id();
  if (j < NIN) {
    const double t = feat_transform(j, F[j]);
    const double span = hi[j] - lo[j];
    xs[j] = span > 0.0 ? (float)((t - lo[j]) / span) : 0.0f;
  }
  __syncthreads();
  const Fwd r = mlp_fwd_wave(P, xs);
  float zc[NOUT];
#pragma unroll
  for (int c = 0; c < NOUT; ++c) zc[c] = __shfl(r.z, c, 64);
  if (j < NOUT) scores[j] = r.z;
  if (j == 0) {
    int bi = 0;
    for (int c = 1; c < NOUT; ++c)
      if (zc[c] > zc[bi]) bi = c;
    *best = bi;
  }
}

__global__ void k_gather_batch(const float* __restrict__ X, const int32_t* __restrict__ labels,
                               const int32_t* __restrict__ order, int32_t nb, float* __restrict__ Xb,
                               int32_t* __restrict__ yb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nb * NIN) return;
  const int r = q / NIN, k = q % NIN;
  const int32_t src = order[r];
  Xb[q] = X[(int64_t)src * NIN + k];
  if (k == 0) yb[r] = labels[src];
}

// Scratch of the backward pass: activations, deltas and per-sample losses.
struct BwdPtrs {
  float *h1, *h2, *dz, *da1, *da2, *loss;
};

struct BwdBuf {
  DTmp h1, h2, dz, da1, da2, loss;
  spmv_status_t alloc(int32_t B) {
    SPMV_TRY(h1.alloc(sizeof(float) * B * NH));
    SPMV_TRY(h2.alloc(sizeof(float) * B * NH));
    SPMV_TRY(dz.alloc(sizeof(float) * B * NOUT));
    SPMV_TRY(da1.alloc(sizeof(float) * B * NH));
    SPMV_TRY(da2.alloc(sizeof(float) * B * NH));
    SPMV_TRY(loss.alloc(sizeof(float) * B));
    return SPMV_OK;
  }
  BwdPtrs ptrs() const {
    return {h1.as<float>(), h2.as<float>(), dz.as<float>(), da1.as<float>(), da2.as<float>(), loss.as<float>()};
  }
};

// The backward scratch of spmv_mlp_backward_noalloc: the six buffers of
// BwdBuf for SPMV_NOALLOC_MAX_BATCH samples, at fixed offsets, in one array
// that the code object carries (each GPU holds its own copy for the life of
// the process).  Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch).
constexpr int64_t NA_B = SPMV_NOALLOC_MAX_BATCH;
constexpr int64_t NA_H1 = 0, NA_H2 = NA_H1 + NA_B * NH, NA_DZ = NA_H2 + NA_B * NH, NA_DA1 = NA_DZ + NA_B * NOUT,
                  NA_DA2 = NA_DA1 + NA_B * NH, NA_LOSS = NA_DA2 + NA_B * NH, NA_FLOATS = NA_LOSS + NA_B;
static __device__ __align__(256) float scratch[NA_FLOATS];

static std::mutex g_na_mu;
static float* g_na_ptr[64] = {nullptr};  // per device: the device address of scratch

static spmv_status_t noalloc_scratch(BwdPtrs* out) {
  int dev = -1;
  SPMV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(SPMV_ERR_UNSUPPORTED, "device %d (at most 64 devices)", dev);
  std::lock_guard<std::mutex> g(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(SPMV_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    }
    g_na_ptr[dev] = (float*)p;
  }
  float* b = g_na_ptr[dev];
  *out = {b + NA_H1, b + NA_H2, b + NA_DZ, b + NA_DA1, b + NA_DA2, b + NA_LOSS};
  return SPMV_OK;
}

static unsigned waves_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 4), 4096)); }

static spmv_status_t backward(const float* P, const float* X, const int32_t* labels, int32_t B, float* G,
                              float* loss_out, float* loss_acc, float weight, const BwdPtrs& w, hipStream_t s) {
  k_mlp_delta<<<waves_grid(B), BS, 0, s>>>(P, X, labels, B, w.h1, w.h2, w.dz, w.da1, w.da2, w.loss);
  SPMV_LAUNCH_CHECK();
  k_mlp_wgrad<<<(unsigned)cdiv(NPARAM, BS), BS, 0, s>>>(X, w.h1, w.h2, w.dz, w.da1, w.da2, B, G);
  SPMV_LAUNCH_CHECK();
  if (loss_out || loss_acc) {
    k_mean<<<1, 1, 0, s>>>(w.loss, B, loss_out, loss_acc, weight);
    SPMV_LAUNCH_CHECK();
  }
  return SPMV_OK;
}

}  // namespace spmv

using namespace spmv;

// ================================================================ C-ABI
extern "C" {

spmv_status_t spmv_features(spmv_mat_t A, double out[12], spmv_stream_t s) {
  if (!A || !out) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  return features(A, out, hs(s));
}

spmv_status_t spmv_mlp_forward(const float* params, const float* X, int32_t B, float* Z, float* A1, float* A2,
                               spmv_stream_t s) {
  if (!params || !X || !Z || B < 0) return fail(SPMV_ERR_INVALID_ARG, "forward arguments");
  if (B == 0) return SPMV_OK;
  k_mlp_forward<<<waves_grid(B), BS, 0, hs(s)>>>(params, X, B, Z, A1, A2);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

spmv_status_t spmv_mlp_backward(const float* params, const float* X, const int32_t* labels, int32_t B, float* grads,
                                float* loss, spmv_stream_t s) {
  if (!params || !X || !labels || !grads || B <= 0) return fail(SPMV_ERR_INVALID_ARG, "backward arguments");
  BwdBuf w;
  SPMV_TRY(w.alloc(B));
  SPMV_TRY(backward(params, X, labels, B, grads, loss, nullptr, 0.0f, w.ptrs(), hs(s)));
  SPMV_HIP(hipStreamSynchronize(hs(s)));
  return SPMV_OK;
}

spmv_status_t spmv_mlp_backward_noalloc(const float* params, const float* X, const int32_t* labels, int32_t B,
                                        float* grads, float* loss, spmv_stream_t s) {
  if (!params || !X || !labels || !grads || B <= 0) return fail(SPMV_ERR_INVALID_ARG, "backward arguments");
  if (B > SPMV_NOALLOC_MAX_BATCH)
    return fail(SPMV_ERR_TOO_LARGE, "batch of %d samples (the allocation-free backward takes at most %d)", (int)B,
                SPMV_NOALLOC_MAX_BATCH);
  BwdPtrs w;
  SPMV_TRY(noalloc_scratch(&w));
  // every scratch element the kernels read is written first by this call's
  // k_mlp_delta, so nothing needs clearing
  return backward(params, X, labels, B, grads, loss, nullptr, 0.0f, w, hs(s));
}

spmv_status_t spmv_mlp_adam(float* params, const float* grads, float* m, float* v, int32_t t, float lr, float beta1,
                            float beta2, float eps, spmv_stream_t s) {
  if (!params || !grads || !m || !v || t < 1) return fail(SPMV_ERR_INVALID_ARG, "adam arguments");
  k_adam<<<(unsigned)cdiv(NPARAM, BS), BS, 0, hs(s)>>>(params, grads, m, v, t, lr, beta1, beta2, eps);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

spmv_status_t spmv_scale_features(const double* F, int32_t n, const double fmin[12], const double fmax[12], float* X,
                                  spmv_stream_t s) {
  if (!F || !X || !fmin || !fmax || n < 0) return fail(SPMV_ERR_INVALID_ARG, "scale arguments");
  if (n == 0) return SPMV_OK;
  DTmp lo, hi;
  SPMV_TRY(lo.alloc(12 * sizeof(double)));
  SPMV_TRY(hi.alloc(12 * sizeof(double)));
  SPMV_HIP(hipMemcpyAsync(lo.p, fmin, 12 * sizeof(double), hipMemcpyHostToDevice, hs(s)));
  SPMV_HIP(hipMemcpyAsync(hi.p, fmax, 12 * sizeof(double), hipMemcpyHostToDevice, hs(s)));
  k_scale<<<(unsigned)cdiv((int64_t)n * NIN, BS), BS, 0, hs(s)>>>(F, n, lo.as<double>(), hi.as<double>(), X);
  SPMV_LAUNCH_CHECK();
  SPMV_HIP(hipStreamSynchronize(hs(s)));
  return SPMV_OK;
}

spmv_status_t spmv_feature_range(const double* F, int32_t n, double fmin[12], double fmax[12], spmv_stream_t s) {
  if (!F || n <= 0 || !fmin || !fmax) return fail(SPMV_ERR_INVALID_ARG, "feature range arguments");
  DTmp r;
  SPMV_TRY(r.alloc(24 * sizeof(double)));
  k_feat_range<<<1, WAVE, 0, hs(s)>>>(F, n, r.as<double>(), r.as<double>() + 12);
  SPMV_LAUNCH_CHECK();
  double h[24];
  SPMV_TRY(copy_to_host(h, r.p, sizeof(h), hs(s)));
  memcpy(fmin, h, 12 * sizeof(double));
  memcpy(fmax, h + 12, 12 * sizeof(double));
  return SPMV_OK;
}

spmv_status_t spmv_mlp_train(float* params, const float* X, const int32_t* labels, int32_t n, const int32_t* order,
                             int32_t epochs, int32_t batch, float lr, spmv_stream_t s, float* loss_out) {
  if (!params || !X || !labels || !order || n <= 0 || epochs < 0 || batch <= 0)
    return fail(SPMV_ERR_INVALID_ARG, "train arguments");
  hipStream_t st = hs(s);
  BwdBuf w;
  DTmp G, m, v, Xb, yb, eloss;
  SPMV_TRY(w.alloc(batch));
  SPMV_TRY(G.alloc(sizeof(float) * NPARAM));
  SPMV_TRY(m.alloc(sizeof(float) * NPARAM));
  SPMV_TRY(v.alloc(sizeof(float) * NPARAM));
  SPMV_TRY(Xb.alloc(sizeof(float) * batch * NIN));
  SPMV_TRY(yb.alloc(sizeof(int32_t) * batch));
  SPMV_TRY(eloss.alloc(sizeof(float) * std::max(epochs, 1)));
  SPMV_HIP(hipMemsetAsync(m.p, 0, sizeof(float) * NPARAM, st));
  SPMV_HIP(hipMemsetAsync(v.p, 0, sizeof(float) * NPARAM, st));
  SPMV_HIP(hipMemsetAsync(eloss.p, 0, sizeof(float) * std::max(epochs, 1), st));
  int32_t t = 0;
  for (int32_t e = 0; e < epochs; ++e) {
    for (int32_t b0 = 0; b0 < n; b0 += batch) {
      const int32_t nb = std::min(batch, n - b0);
      k_gather_batch<<<(unsigned)cdiv(nb * NIN, BS), BS, 0, st>>>(X, labels, order + (int64_t)e * n + b0, nb,
                                                                   Xb.as<float>(), yb.as<int32_t>());
      SPMV_LAUNCH_CHECK();
      SPMV_TRY(backward(params, Xb.as<float>(), yb.as<int32_t>(), nb, G.as<float>(), nullptr,
                        eloss.as<float>() + e, (float)nb / (float)n, w.ptrs(), st));
      ++t;
      k_adam<<<(unsigned)cdiv(NPARAM, BS), BS, 0, st>>>(params, G.as<float>(), m.as<float>(), v.as<float>(), t, lr,
                                                          0.9f, 0.999f, 1e-8f);
      SPMV_LAUNCH_CHECK();
    }
  }
  if (loss_out && epochs > 0) SPMV_TRY(copy_to_host(loss_out, eloss.p, sizeof(float) * epochs, st));
  SPMV_HIP(hipStreamSynchronize(st));
  return SPMV_OK;
}

// --------------------------------------------------------------- models
struct ModelFile {
  char magic[8];
  uint32_t version, nparam, nfeat, transform;
  char arch[32];
  double fmin[12], fmax[12];
};

static std::mutex g_sel_mu;

spmv_status_t spmv_model_create(const float* params, const double fmin[12], const double fmax[12], spmv_model_t* out) {
  if (!params || !fmin || !fmax || !out) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  spmv_model_s* m = new spmv_model_s();
  memcpy(m->h_params, params, sizeof(float) * NPARAM);
  memcpy(m->fmin, fmin, sizeof(m->fmin));
  memcpy(m->fmax, fmax, sizeof(m->fmax));
  void* p = nullptr;
  spmv_status_t st = dmalloc(&p, sizeof(float) * NPARAM);
  if (st != SPMV_OK) {
    delete m;
    return st;
  }
  m->d_params = (float*)p;
  if (hipMemcpy(m->d_params, params, sizeof(float) * NPARAM, hipMemcpyHostToDevice) != hipSuccess) {
    dfree(p);
    delete m;
    return fail(SPMV_ERR_HIP, "model upload failed");
  }
  *out = m;
  return SPMV_OK;
}

spmv_status_t spmv_model_save(spmv_model_t m, const char* path) {
  if (!m || !path) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  ModelFile h;
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, "SPMVMLP", 8);
  h.version = 1;
  h.nparam = NPARAM;
  h.nfeat = NIN;
  h.transform = 1;
  strncpy(h.arch, "gfx950", sizeof(h.arch) - 1);
  memcpy(h.fmin, m->fmin, sizeof(h.fmin));
  memcpy(h.fmax, m->fmax, sizeof(h.fmax));
  FILE* f = fopen(path, "wb");
  if (!f) return fail(SPMV_ERR_MODEL, "cannot write %s", path);
  const bool ok = fwrite(&h, sizeof(h), 1, f) == 1 && fwrite(m->h_params, sizeof(float), NPARAM, f) == (size_t)NPARAM;
  fclose(f);
  return ok ? SPMV_OK : fail(SPMV_ERR_MODEL, "short write to %s", path);
}

spmv_status_t spmv_model_load(const char* path, spmv_model_t* out) {
  if (!path || !out) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  FILE* f = fopen(path, "rb");
  if (!f) return fail(SPMV_ERR_MODEL, "cannot open %s", path);
  ModelFile h;
  std::vector<float> buf(NPARAM);
  const bool ok = fread(&h, sizeof(h), 1, f) == 1 && fread(buf.data(), sizeof(float), NPARAM, f) == (size_t)NPARAM;
  fclose(f);
  if (!ok || memcmp(h.magic, "SPMVMLP", 8) != 0 || h.version != 1 || h.nparam != (uint32_t)NPARAM ||
      h.nfeat != (uint32_t)NIN || h.transform != 1)
    return fail(SPMV_ERR_MODEL, "%s is not a version-1 selector model", path);
  return spmv_model_create(buf.data(), h.fmin, h.fmax, out);
}

spmv_status_t spmv_model_params(spmv_model_t m, float* params_out, double fmin[12], double fmax[12]) {
  if (!m) return fail(SPMV_ERR_INVALID_ARG, "null model");
  if (params_out) memcpy(params_out, m->h_params, sizeof(float) * NPARAM);
  if (fmin) memcpy(fmin, m->fmin, sizeof(m->fmin));
  if (fmax) memcpy(fmax, m->fmax, sizeof(m->fmax));
  return SPMV_OK;
}

void spmv_model_free(spmv_model_t m) {
  if (!m) return;
  dfree(m->d_params);
  delete m;
}

spmv_status_t spmv_select(spmv_model_t m, const double features[12], spmv_fmt_t* best, float scores[5]) {
  if (!m || !features || !best) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> g(g_sel_mu);
  DTmp buf;  // features(12) fmin(12) fmax(12) doubles, then best + scores
  SPMV_TRY(buf.alloc(36 * sizeof(double) + 8 * sizeof(float)));
  double* d = buf.as<double>();
  double host[36];
  memcpy(host, features, 12 * sizeof(double));
  memcpy(host + 12, m->fmin, 12 * sizeof(double));
  memcpy(host + 24, m->fmax, 12 * sizeof(double));
  SPMV_HIP(hipMemcpy(d, host, sizeof(host), hipMemcpyHostToDevice));
  int32_t* dbest = (int32_t*)(d + 36);
  float* dsc = (float*)(d + 36) + 2;
  k_select<<<1, WAVE, 0, 0>>>(m->d_params, d, d + 12, d + 24, dbest, dsc);
  SPMV_LAUNCH_CHECK();
  float out[7];
  SPMV_HIP(hipMemcpy(out, d + 36, sizeof(out), hipMemcpyDeviceToHost));
  int32_t b;
  memcpy(&b, out, sizeof(b));
  *best = (spmv_fmt_t)b;
  if (scores) memcpy(scores, out + 2, 5 * sizeof(float));
  return SPMV_OK;
}

}  // extern "C"
