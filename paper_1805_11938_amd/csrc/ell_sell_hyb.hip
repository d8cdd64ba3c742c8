// ELL, SELL-C-sigma and HYB (Sec. II-B; Table I): device conversions from
// CSR, their inverses, and the SpMV kernels.
//
// ELL: M x K, K = longest row, column-major (slot (i,k) at k*M + i) so a
//   wave's 64 rows read 64 consecutive slots per k; padding (-1, +0.0) is
//   skipped by predicate and never reads x.  One thread per row.
// SELL-C-sigma: strips of C rows, each its own ELL of width w_c, column-
//   major inside the strip (slot (p,k) at cs[c] + k*C + p); rows sorted by
//   descending length, stably, inside windows of sigma rows (perm maps a
//   stored position to its row; y is written through it).  One thread per
//   stored position.
// HYB: ELL(K) + COO tail.  K from the one-third rule unless given.  The ELL
//   kernel writes y, then the COO pass adds the tail: one wave per tile of
//   1,024 consecutive entries, a segmented scan in registers, no barrier;
//   rows that cross tiles are finished by an ordered fix-up pass, without
//   atomics.
#include "common.h"

namespace spmv {

static unsigned grid_rows(int64_t n) {
  int64_t g = cdiv(n, BS);
  if (g < 1) g = 1;
  if (g > (1 << 20)) g = 1 << 20;
  return (unsigned)g;
}

static int bits_for(uint64_t v) {
  int b = 0;
  while (b < 64 && (v >> b)) ++b;
  return b;
}

// ================================================================== ELL
template <typename T>
__global__ void k_csr_to_ell(int64_t M, int64_t K, const int32_t* ptr, const int32_t* col, const T* val, int32_t* ecol,
                             T* eval) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = ptr[i], len = ptr[i + 1] - a;
    for (int64_t k = 0; k < K; ++k) {
      const int64_t q = k * M + i;
      if (k < len) {
        ecol[q] = col[a + k];
        eval[q] = val[a + k];
      } else {
        ecol[q] = -1;
        eval[q] = (T)0;
      }
    }
  }
}

// entries of row i kept in the ELL part: the first min(len, K)
__global__ void k_ell_count(int64_t M, int64_t K, const int32_t* ecol, int32_t* len) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t k = 0;
    while (k < K && ecol[k * M + i] >= 0) ++k;
    len[i] = (int32_t)k;
  }
}

// copies the ell_len[i] (<= K) ELL entries of row i to ptr[i] onward
template <typename T>
__global__ void k_ell_to_csr(int64_t M, const int32_t* ecol, const T* eval, const int32_t* ell_len, const int32_t* ptr,
                             int32_t* col, T* val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = ptr[i], len = ell_len[i];
    for (int64_t k = 0; k < len; ++k) {
      col[a + k] = ecol[k * M + i];
      val[a + k] = eval[k * M + i];
    }
  }
}

// Eight slots per step: all 16 loads of a step are issued before the x
// gathers, so each wave keeps many requests in flight.
template <typename T>
__global__ __launch_bounds__(BS) void k_ell(int64_t M, int64_t K, const int32_t* __restrict__ ecol,
                                            const T* __restrict__ eval, const T* __restrict__ x, T* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < M; i += (int64_t)gridDim.x * BS) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t k = 0;
  for (; k + 7 < K; k += 8) {
    int32_t c[8];
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = ldnt32(ecol + (k + u) * M, (uint32_t)i);  // uniform column base
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ldnt32(eval + (k + u) * M, (uint32_t)i);
    issue_fence();
    T xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) xv[u] = ld32(x, (uint32_t)(c[u] >= 0 ? c[u] : 0));  // branch-free gathers
    issue_fence();
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u & 3] += c[u] >= 0 ? (double)v[u] * (double)xv[u] : 0.0;
  }
  for (; k < K; ++k) {
    const int32_t c = ldnt(ecol + k * M + i);
    const T v = ldnt(eval + k * M + i);
    const T xv = x[c >= 0 ? c : 0];
    s[0] += c >= 0 ? (double)v * (double)xv : 0.0;
  }
  y[i] = (T)((s[0] + s[1]) + (s[2] + s[3]));
  }
}

// Two adjacent rows per lane (M even): the column and value slots of a row
// pair are loaded as one 8-byte and one 16-byte vector, halving the number of
// load instructions per byte.
template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
  typedef double __attribute__((ext_vector_type(2))) type;
};
template <>
struct Vec2<float> {
  typedef float __attribute__((ext_vector_type(2))) type;
};
typedef int32_t __attribute__((ext_vector_type(2))) i32x2;

template <typename T>
__global__ __launch_bounds__(BS) void k_ell2(int64_t M, int64_t K, const int32_t* __restrict__ ecol,
                                             const T* __restrict__ eval, const T* __restrict__ x,
                                             T* __restrict__ y) {
  typedef typename Vec2<T>::type T2;
  const int64_t M2 = M >> 1;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < M2; i += (int64_t)gridDim.x * BS) {
    double s0[2] = {0.0, 0.0}, s1[2] = {0.0, 0.0};
    int64_t k = 0;
    for (; k + 3 < K; k += 4) {
      i32x2 c[4];
      T2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) c[u] = ldnt32((const i32x2*)(ecol + (k + u) * M), (uint32_t)i);
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = ldnt32((const T2*)(eval + (k + u) * M), (uint32_t)i);
      issue_fence();
      T xa[4], xb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xa[u] = ld32(x, (uint32_t)(c[u].x >= 0 ? c[u].x : 0));
        xb[u] = ld32(x, (uint32_t)(c[u].y >= 0 ? c[u].y : 0));
      }
      issue_fence();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        s0[u & 1] += c[u].x >= 0 ? (double)v[u].x * (double)xa[u] : 0.0;
        s1[u & 1] += c[u].y >= 0 ? (double)v[u].y * (double)xb[u] : 0.0;
      }
    }
    for (; k < K; ++k) {
      const i32x2 c = ldnt32((const i32x2*)(ecol + k * M), (uint32_t)i);
      const T2 v = ldnt32((const T2*)(eval + k * M), (uint32_t)i);
      const T xa = ld32(x, (uint32_t)(c.x >= 0 ? c.x : 0)), xb = ld32(x, (uint32_t)(c.y >= 0 ? c.y : 0));
      s0[0] += c.x >= 0 ? (double)v.x * (double)xa : 0.0;
      s1[0] += c.y >= 0 ? (double)v.y * (double)xb : 0.0;
    }
    T2 out;
    out.x = (T)(s0[0] + s0[1]);
    out.y = (T)(s1[0] + s1[1]);
    *(T2*)(y + 2 * i) = out;
  }
}

// Narrow ELL (K <= 32): one row per lane with every slot's column and value
// load in flight at once, then every gather, then the sum -- two memory
// round trips per row in total.  The kernel is instantiated for each K, so
// no slot is loaded twice or masked.  With XCD, blocks are remapped so that
// each XCD takes a contiguous range of rows (the x window of neighbouring
// rows stays in one L2).
template <typename T, int KC, bool XCD>
__global__ __launch_bounds__(WAVE) void k_ell_kc(int64_t M, const int32_t* __restrict__ ecol,
                                                 const T* __restrict__ eval, const T* __restrict__ x,
                                                 T* __restrict__ y) {
  const int64_t i = (int64_t)(XCD ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x) * WAVE + threadIdx.x;
  if (i >= M) return;
  int32_t c[KC];
  T v[KC], xv[KC];
#pragma unroll
  for (int u = 0; u < KC; ++u) c[u] = ldnt32(ecol + (int64_t)u * M, (uint32_t)i);
#pragma unroll
  for (int u = 0; u < KC; ++u) v[u] = ldnt32(eval + (int64_t)u * M, (uint32_t)i);
  issue_fence();
#pragma unroll
  for (int u = 0; u < KC; ++u) xv[u] = ld32(x, (uint32_t)(c[u] >= 0 ? c[u] : 0));
  issue_fence();
  double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < KC; ++u) s[u & 3] += c[u] >= 0 ? (double)v[u] * (double)xv[u] : 0.0;
  y[i] = (T)((s[0] + s[1]) + (s[2] + s[3]));
}

// Narrow ELL, four waves per 64 rows: wave h takes the slots [h*q, min(K,
// (h+1)*q)), q = ceil(K/4); the four sums are added in wave order in LDS.
template <typename T, int KC>
__global__ __launch_bounds__(4 * WAVE) void k_ell_kc4(int64_t M, const int32_t* __restrict__ ecol,
                                                     const T* __restrict__ eval, const T* __restrict__ x,
                                                     T* __restrict__ y, int xcd) {
  constexpr int KQ = (KC + 3) / 4;
  __shared__ double part[4][WAVE];
  const int h = (int)__builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
  const int p = (int)(threadIdx.x & (WAVE - 1));
  const int64_t i = (int64_t)(xcd ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x) * WAVE + p;
  const int k0 = h * KQ;
  constexpr int NLAST = KC - 3 * KQ;  // slots of the last wave (may be < KQ, or <= 0)
  const int n = h < 3 ? (KQ < KC - k0 ? KQ : KC - k0) : NLAST;
  double sa[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < M && n > 0) {
    int32_t c[KQ];
    T v[KQ], xv[KQ];
#pragma unroll
    for (int u = 0; u < KQ; ++u) c[u] = u < n ? ldnt32(ecol + (int64_t)(k0 + u) * M, (uint32_t)i) : -1;
#pragma unroll
    for (int u = 0; u < KQ; ++u) v[u] = u < n ? ldnt32(eval + (int64_t)(k0 + u) * M, (uint32_t)i) : (T)0;
    issue_fence();
#pragma unroll
    for (int u = 0; u < KQ; ++u) xv[u] = ld32(x, (uint32_t)(c[u] >= 0 ? c[u] : 0));
    issue_fence();
#pragma unroll
    for (int u = 0; u < KQ; ++u) sa[u & 3] += c[u] >= 0 ? (double)v[u] * (double)xv[u] : 0.0;
  }
  part[h][p] = (sa[0] + sa[1]) + (sa[2] + sa[3]);
  __syncthreads();
  if (h == 0 && i < M) y[i] = (T)(((part[0][p] + part[1][p]) + part[2][p]) + part[3][p]);
}

template <typename T>
static void launch_ell_kc4(int64_t M, int32_t k, const int32_t* ecol, const void* eval, const void* x, void* y,
                           unsigned g, int xcd, hipStream_t s) {
  const T* ev = (const T*)eval;
  const T* xv = (const T*)x;
  T* yv = (T*)y;
  switch (k) {
    case 1: launch(k_ell_kc4<T, 1>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 2: launch(k_ell_kc4<T, 2>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 3: launch(k_ell_kc4<T, 3>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 4: launch(k_ell_kc4<T, 4>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 5: launch(k_ell_kc4<T, 5>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 6: launch(k_ell_kc4<T, 6>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 7: launch(k_ell_kc4<T, 7>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 8: launch(k_ell_kc4<T, 8>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 9: launch(k_ell_kc4<T, 9>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 10: launch(k_ell_kc4<T, 10>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 11: launch(k_ell_kc4<T, 11>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 12: launch(k_ell_kc4<T, 12>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 13: launch(k_ell_kc4<T, 13>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 14: launch(k_ell_kc4<T, 14>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 15: launch(k_ell_kc4<T, 15>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 16: launch(k_ell_kc4<T, 16>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 17: launch(k_ell_kc4<T, 17>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 18: launch(k_ell_kc4<T, 18>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 19: launch(k_ell_kc4<T, 19>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 20: launch(k_ell_kc4<T, 20>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 21: launch(k_ell_kc4<T, 21>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 22: launch(k_ell_kc4<T, 22>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 23: launch(k_ell_kc4<T, 23>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 24: launch(k_ell_kc4<T, 24>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 25: launch(k_ell_kc4<T, 25>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 26: launch(k_ell_kc4<T, 26>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 27: launch(k_ell_kc4<T, 27>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 28: launch(k_ell_kc4<T, 28>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 29: launch(k_ell_kc4<T, 29>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 30: launch(k_ell_kc4<T, 30>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 31: launch(k_ell_kc4<T, 31>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    case 32: launch(k_ell_kc4<T, 32>, g, 4 * WAVE, s, M, ecol, ev, xv, yv, xcd); break;
    default: break;
  }
}

template <typename T, bool XCD>
static void launch_ell_kc(int64_t M, int32_t k, const int32_t* ecol, const void* eval, const void* x, void* y,
                          unsigned g, hipStream_t s) {
  switch (k) {
    case 1: launch(k_ell_kc<T, 1, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 2: launch(k_ell_kc<T, 2, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 3: launch(k_ell_kc<T, 3, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 4: launch(k_ell_kc<T, 4, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 5: launch(k_ell_kc<T, 5, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 6: launch(k_ell_kc<T, 6, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 7: launch(k_ell_kc<T, 7, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 8: launch(k_ell_kc<T, 8, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 9: launch(k_ell_kc<T, 9, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 10: launch(k_ell_kc<T, 10, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 11: launch(k_ell_kc<T, 11, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 12: launch(k_ell_kc<T, 12, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 13: launch(k_ell_kc<T, 13, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 14: launch(k_ell_kc<T, 14, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 15: launch(k_ell_kc<T, 15, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 16: launch(k_ell_kc<T, 16, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 17: launch(k_ell_kc<T, 17, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 18: launch(k_ell_kc<T, 18, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 19: launch(k_ell_kc<T, 19, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 20: launch(k_ell_kc<T, 20, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 21: launch(k_ell_kc<T, 21, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 22: launch(k_ell_kc<T, 22, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 23: launch(k_ell_kc<T, 23, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 24: launch(k_ell_kc<T, 24, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 25: launch(k_ell_kc<T, 25, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 26: launch(k_ell_kc<T, 26, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 27: launch(k_ell_kc<T, 27, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 28: launch(k_ell_kc<T, 28, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 29: launch(k_ell_kc<T, 29, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 30: launch(k_ell_kc<T, 30, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 31: launch(k_ell_kc<T, 31, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    case 32: launch(k_ell_kc<T, 32, XCD>, g, WAVE, s, M, ecol, (const T*)eval, (const T*)x, (T*)y); break;
    default: break;
  }
}

template <typename T>
static spmv_status_t launch_ell(int64_t M, int64_t K, const int32_t* ecol, const void* eval, const void* x, void* y,
                                bool xcd, bool split4, hipStream_t s) {
  if (M == 0) return SPMV_OK;
  if (K >= 1 && K <= 32) {
    const unsigned g = (unsigned)cdiv(M, WAVE);  // one workgroup per 64 rows
    const int32_t k = (int32_t)K;
    if (split4)
      launch_ell_kc4<T>(M, k, ecol, eval, x, y, g, xcd ? 1 : 0, s);
    else if (xcd)
      launch_ell_kc<T, true>(M, k, ecol, eval, x, y, g, s);
    else
      launch_ell_kc<T, false>(M, k, ecol, eval, x, y, g, s);
    SPMV_LAUNCH_CHECK();
    return SPMV_OK;
  }
  if ((M & 1) == 0 && ((uintptr_t)y & (2 * sizeof(T) - 1)) == 0) {
    const unsigned g2 = (unsigned)std::min<int64_t>(cdiv(M / 2, BS), resident_blocks(8));
    launch(k_ell2<T>, g2, BS, s, M, K, ecol, (const T*)eval, (const T*)x, (T*)y);
    SPMV_LAUNCH_CHECK();
    return SPMV_OK;
  }
  const unsigned g = (unsigned)std::min<int64_t>(cdiv(M, BS), resident_blocks(8));  // persistent grid
  launch(k_ell<T>, g, BS, s, M, K, ecol, (const T*)eval, (const T*)x, (T*)y);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

spmv_status_t run_ell(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  const bool xcd = !(A->params.flags & SPMV_FLAG_LINEAR);
  const bool split4 = (A->params.flags & SPMV_FLAG_SPLIT4) != 0;
  if (A->dt == SPMV_F64) return launch_ell<double>(A->M, A->K, A->ecol, A->eval, x, y, xcd, split4, s);
  return launch_ell<float>(A->M, A->K, A->ecol, A->eval, x, y, xcd, split4, s);
}

static spmv_status_t check_cap(const spmv_mat_s* A, int64_t bytes, const char* what) {
  const int64_t cap = A->params.max_bytes > 0 ? A->params.max_bytes : default_max_bytes();
  if (bytes > cap)
    return fail(SPMV_ERR_TOO_LARGE, "%s needs %lld bytes, above the cap of %lld", what, (long long)bytes,
                (long long)cap);
  return SPMV_OK;
}

static spmv_status_t build_ell_part(spmv_mat_s* src, spmv_mat_s* A, int64_t K, hipStream_t s) {
  const int64_t M = src->M;
  A->K = K;
  SPMV_TRY(mat_alloc(A, (void**)&A->ecol, sizeof(int32_t) * M * K));
  SPMV_TRY(mat_alloc(A, &A->eval, (size_t)A->sv * M * K));
  if (M && K) {
    if (A->dt == SPMV_F64)
      k_csr_to_ell<double><<<grid_rows(M), BS, 0, s>>>(M, K, src->ptr, src->col, (const double*)src->val, A->ecol,
                                                       (double*)A->eval);
    else
      k_csr_to_ell<float><<<grid_rows(M), BS, 0, s>>>(M, K, src->ptr, src->col, (const float*)src->val, A->ecol,
                                                      (float*)A->eval);
    SPMV_LAUNCH_CHECK();
  }
  return SPMV_OK;
}

spmv_status_t convert_ell(spmv_mat_s* src, spmv_mat_s* A, hipStream_t s) {
  int32_t K = 0;
  SPMV_TRY(device_max_i32(src->ptr, src->M, 1, &K, s));
  const int64_t slots = src->M * (int64_t)K;
  SPMV_TRY(check_cap(A, slots * (4 + A->sv), "ELL"));
  SPMV_TRY(build_ell_part(src, A, K, s));
  A->pad_slots = slots - src->nnz;
  A->bytes_fmt = slots * (4 + A->sv) + A->N * A->sv + A->M * A->sv;
  return SPMV_OK;
}

// ============================================================ SELL-C-sigma
__global__ void k_sell_keys(int64_t M, const int32_t* ptr, int64_t sigma, int64_t maxlen, uint64_t* key,
                            uint32_t* idx) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t len = ptr[i + 1] - ptr[i];
    key[i] = (uint64_t)(i / sigma) * (uint64_t)(maxlen + 1) + (uint64_t)(maxlen - len);
    idx[i] = (uint32_t)i;
  }
}

__global__ void k_sell_perm(int64_t M, int64_t Mpad, const uint32_t* sorted, int32_t* perm) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < Mpad; p += (int64_t)gridDim.x * blockDim.x)
    perm[p] = p < M ? (int32_t)sorted[p] : -1;
}

__global__ void k_sell_width(int64_t M, int64_t nch, int C, const int32_t* ptr, const int32_t* perm, int64_t* cw) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += (int64_t)gridDim.x * blockDim.x) {
    int64_t w = 0;
    for (int p = 0; p < C; ++p) {
      const int64_t pos = c * C + p;
      const int64_t r = perm ? perm[pos] : (pos < M ? pos : -1);
      if (r >= 0) {
        const int64_t len = ptr[r + 1] - ptr[r];
        w = len > w ? len : w;
      }
    }
    cw[c] = w * C;
  }
}

// A wave fills at most SELL_FILL slots of a chunk; a chunk holding very long
// rows (C x width beyond that) gets extra waves for the rest, one per
// SELL_FILL slots, so no single wave copies millions of slots.
constexpr int64_t SELL_FILL = 16384;

// One wave per unit: slots [q0, q0 + SELL_FILL) of one chunk, written
// slot-major (coalesced) by all lanes together after the chunk's rows are
// looked up once.  units == nullptr: unit u is chunk u from slot 0.
template <typename T>
__global__ __launch_bounds__(WAVE) void k_csr_to_sell(int64_t M, int64_t nunits, int C, const int32_t* ptr,
                                                      const int32_t* col, const T* val, const int32_t* perm,
                                                      const int64_t* cs, const int64_t* units, int32_t* scol,
                                                      T* sval) {
  __shared__ int64_t ra[WAVE], rl[WAVE];
  for (int64_t u = blockIdx.x; u < nunits; u += gridDim.x) {
    const int64_t c = units ? units[2 * u] : u;
    const int64_t q0 = units ? units[2 * u + 1] : 0;
    const int t = threadIdx.x;
    if (t < C) {
      const int64_t pos = c * C + t;
      const int64_t r = perm ? perm[pos] : (pos < M ? pos : -1);
      ra[t] = r >= 0 ? ptr[r] : 0;
      rl[t] = r >= 0 ? ptr[r + 1] - ra[t] : 0;
    }
    __syncthreads();
    const int64_t base = cs[c], n = cs[c + 1] - base;
    const int64_t q1 = n < q0 + SELL_FILL ? n : q0 + SELL_FILL;
    for (int64_t q = q0 + t; q < q1; q += WAVE) {
      const int64_t k = q / C, p = q % C;
      if (k < rl[p]) {
        scol[base + q] = col[ra[p] + k];
        sval[base + q] = val[ra[p] + k];
      } else {
        scol[base + q] = -1;
        sval[base + q] = (T)0;
      }
    }
    __syncthreads();
  }
}

__global__ void k_sell_count(int64_t M, int64_t Mpad, int C, const int32_t* perm, const int64_t* cs,
                             const int32_t* scol, int32_t* len) {
  for (int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pos < Mpad;
       pos += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = perm ? perm[pos] : (pos < M ? pos : -1);
    if (r < 0) continue;
    const int64_t c = pos / C, p = pos % C, base = cs[c], w = (cs[c + 1] - base) / C;
    int64_t k = 0;
    while (k < w && scol[base + k * C + p] >= 0) ++k;
    len[r] = (int32_t)k;
  }
}

template <typename T>
__global__ void k_sell_to_csr(int64_t M, int64_t Mpad, int C, const int32_t* perm, const int64_t* cs,
                              const int32_t* scol, const T* sval, const int32_t* ptr, int32_t* col, T* val) {
  for (int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pos < Mpad;
       pos += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = perm ? perm[pos] : (pos < M ? pos : -1);
    if (r < 0) continue;
    const int64_t c = pos / C, p = pos % C, base = cs[c];
    const int64_t a = ptr[r], len = ptr[r + 1] - a;
    for (int64_t k = 0; k < len; ++k) {
      col[a + k] = scol[base + k * C + p];
      val[a + k] = sval[base + k * C + p];
    }
  }
}

// A work item is a slice of at most SELL_KT columns of one chunk, run by C
// lanes (one per stored row).  Chunks of one slice write y directly; wider
// chunks write per-slice partial sums.  For a chunk of at most SELL_FUSE
// slices the item that finishes last (counted with an atomic) adds them in a
// fixed order and writes y; longer chunks (rows of more than 8,192 entries)
// leave that to k_sell_fix, a workgroup per chunk.  The items run in
// k_sell_mixed, beside the narrow chunks.
constexpr int SELL_KT = 64;
constexpr int SELL_FUSE = 128;
constexpr int SELL_KC_MAX = 32;  // widest chunk the one-pass narrow kernel takes

// The slots of one stored row, KW places (KW >= w): every slot's column and
// value load in flight at once, then every gather, then the sum.  Places
// w..KW-1 reload slot w-1 (same address) and are masked.
template <typename T, int LOGC, int KW>
__device__ __forceinline__ void sell_slots(const int32_t* __restrict__ cc, const T* __restrict__ vv,
                                           const T* __restrict__ x, int w, double* sa) {
  constexpr int C = 1 << LOGC;
  int32_t cg[KW];
  T vg[KW], xg[KW];
#pragma unroll
  for (int u = 0; u < KW; ++u) cg[u] = ldnt32(cc, (uint32_t)((u < w ? u : w - 1) * C));
#pragma unroll
  for (int u = 0; u < KW; ++u) vg[u] = ldnt32(vv, (uint32_t)((u < w ? u : w - 1) * C));
  issue_fence();
#pragma unroll
  for (int u = 0; u < KW; ++u) xg[u] = ld32(x, (uint32_t)(cg[u] >= 0 ? cg[u] : 0));
  issue_fence();
#pragma unroll
  for (int u = 0; u < KW; ++u) sa[u & 3] += (u < w && cg[u] >= 0) ? (double)vg[u] * (double)xg[u] : 0.0;
}

// sell_slots for a column band after the first: the old y of the lane's row
// (r < 0: none) is loaded beside the gathers, not after the sum.
template <typename T, int LOGC, int KW>
__device__ __forceinline__ double sell_slots_y(const int32_t* __restrict__ cc, const T* __restrict__ vv,
                                               const T* __restrict__ x, int w, double* sa,
                                               const T* __restrict__ y, int64_t r) {
  constexpr int C = 1 << LOGC;
  int32_t cg[KW];
  T vg[KW], xg[KW];
#pragma unroll
  for (int u = 0; u < KW; ++u) cg[u] = ldnt32(cc, (uint32_t)((u < w ? u : w - 1) * C));
#pragma unroll
  for (int u = 0; u < KW; ++u) vg[u] = ldnt32(vv, (uint32_t)((u < w ? u : w - 1) * C));
  issue_fence();
  const T yo = y[r >= 0 ? r : 0];
#pragma unroll
  for (int u = 0; u < KW; ++u) xg[u] = ld32(x, (uint32_t)(cg[u] >= 0 ? cg[u] : 0));
  issue_fence();
#pragma unroll
  for (int u = 0; u < KW; ++u) sa[u & 3] += (u < w && cg[u] >= 0) ? (double)vg[u] * (double)xg[u] : 0.0;
  return (double)yo;
}

// Narrow SELL (chunks [c0, nchunks), each at most KC wide): one lane per
// stored row, one pass over the chunks (no persistent loop).  A chunk runs
// in the smallest of 4, 8, 16 and KC places that holds its width (with
// C = 64 the width is the same for the whole wave, so this is a uniform
// branch): chunks much narrower than KC issue no redundant loads.
template <typename T, int LOGC, bool PERM, int KC>
__global__ __launch_bounds__(WAVE) void k_sell_kc(int64_t M, int64_t c0, int64_t nchunks, const int64_t* __restrict__ cs,
                                                  const int32_t* __restrict__ perm, const int32_t* __restrict__ scol,
                                                  const T* __restrict__ sval, const T* __restrict__ x,
                                                  T* __restrict__ y, int remap, int add) {
  constexpr int C = 1 << LOGC;
  // one wave per workgroup (the finest unit the dispatcher balances).  With
  // remap each XCD takes a contiguous range of chunks (neighbouring rows
  // share x in its L2); without it chunks go round-robin over the XCDs, which
  // balances a chunk list sorted by width over long windows.
  const int64_t gid = (int64_t)(remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x) * WAVE + threadIdx.x;
  // C = 64: one chunk per wave, so its offsets are scalar loads
  const int64_t c = c0 + (LOGC == 6 ? (int64_t)__builtin_amdgcn_readfirstlane((int32_t)(gid >> 6)) : gid >> LOGC);
  if (c >= nchunks) return;
  const int p = (int)(gid & (C - 1));
  const int64_t base = cs[c];
  const int w = (int)((cs[c + 1] - base) >> LOGC);
  double sa[4] = {0.0, 0.0, 0.0, 0.0};
  if (w > 0) {
    const int32_t* cc = scol + base + p;
    const T* vv = sval + base + p;
    if (KC > 16 && w > 16) sell_slots<T, LOGC, KC>(cc, vv, x, w, sa);
    else if (KC > 8 && w > 8) sell_slots<T, LOGC, (KC < 16 ? KC : 16)>(cc, vv, x, w, sa);
    else if (KC > 4 && w > 4) sell_slots<T, LOGC, (KC < 8 ? KC : 8)>(cc, vv, x, w, sa);
    else sell_slots<T, LOGC, (KC < 4 ? KC : 4)>(cc, vv, x, w, sa);
  }
  const int64_t pos = c * C + p;
  const int64_t r = PERM ? (int64_t)perm[pos] : (pos < M ? pos : -1);
  if (r >= 0) put_y(y, r, (sa[0] + sa[1]) + (sa[2] + sa[3]), add);
}

// Narrow SELL with C = 64, NW (4 or 6) waves per chunk: wave h takes the
// slots [h*q, min(w, (h+1)*q)) of each stored row, q = ceil(w/NW), with every
// one of its loads in flight; the NW sums are added in wave order through
// LDS.  Against one wave per chunk this holds a fraction of the registers
// per wave (more waves per SIMD) and of the dependent round trip per wave,
// so the chunk streams keep more bytes in flight.  Stencil rows of 27 slots,
// FP64: 65.5 us with one wave, 61.3 with four (7 slots each), 60.0 with six
// (5 each), 61.7 with eight; in FP32 six waves lose (41.6 against 34.9 us),
// so both are autotuner candidates.
template <typename T, bool PERM, int KC, int NW>
__global__ __launch_bounds__(NW * WAVE) void k_sell_kcw(int64_t M, int64_t c0, int64_t nchunks,
                                                      const int64_t* __restrict__ cs, const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ scol, const T* __restrict__ sval,
                                                      const T* __restrict__ x, T* __restrict__ y, int remap,
                                                      int add) {
  constexpr int KQ = (KC + NW - 1) / NW;
  __shared__ double part[NW][WAVE];
  const int h = (int)__builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
  const int p = (int)(threadIdx.x & (WAVE - 1));
  const int64_t c = c0 + (int64_t)(remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x);
  if (c >= nchunks) return;  // uniform over the workgroup
  const int64_t base = cs[c];
  const int w = (int)((cs[c + 1] - base) >> 6);
  const int q = (w + NW - 1) / NW;
  const int k0 = h * q;
  const int n = w - k0 < q ? w - k0 : q;  // this wave's slots (may be <= 0)
  double sa[4] = {0.0, 0.0, 0.0, 0.0};
  if (n > 0) {
    const int32_t* cc = scol + base + (int64_t)k0 * WAVE + p;
    const T* vv = sval + base + (int64_t)k0 * WAVE + p;
    if (KQ > 4 && n > 4) sell_slots<T, 6, KQ>(cc, vv, x, n, sa);
    else if (KQ > 2 && n > 2) sell_slots<T, 6, (KQ < 4 ? KQ : 4)>(cc, vv, x, n, sa);
    else sell_slots<T, 6, (KQ < 2 ? KQ : 2)>(cc, vv, x, n, sa);
  }
  part[h][p] = (sa[0] + sa[1]) + (sa[2] + sa[3]);
  __syncthreads();
  if (h == 0) {
    double t = part[0][p];
#pragma unroll
    for (int i = 1; i < NW; ++i) t += part[i][p];
    const int64_t pos = c * WAVE + p;
    const int64_t r = PERM ? (int64_t)perm[pos] : (pos < M ? pos : -1);
    if (r >= 0) put_y(y, r, t, add);
  }
}

// The slice item of a split chunk (at most SELL_FUSE slices) that finishes
// last.  Each item stores its partial sums with agent-scope atomic stores
// (written through to where every XCD reads them), waits until they are
// done, then counts itself; the item that brings the count to nsl reads the
// chunk's nsl partial sums of its row with agent-scope atomic loads and adds
// them in a fixed order (eight running sums over the slices, combined
// pairwise), writes y and clears the count for the next run.  (Fences
// would write back and invalidate a whole XCD's L2 for every item.)  Lanes
// of one item are C consecutive lanes.
template <typename T, int LOGC, bool PERM>
__device__ __forceinline__ void sell_fix_last(int64_t M, int64_t first, int64_t it, int64_t nsl, int64_t c, int p,
                                              double s, double* part, const int32_t* __restrict__ perm,
                                              int32_t* cnt, T* __restrict__ y, int add) {
  constexpr int C = 1 << LOGC;
  __hip_atomic_store(part + it * C + p, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_s_waitcnt(0);  // the store has completed before the item is counted
  int last = 0;
  if (p == 0) last = __hip_atomic_fetch_add(cnt + first, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (int)nsl - 1;
  last = __shfl(last, (int)(threadIdx.x & ~(unsigned)(C - 1)));
  if (!last) return;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t j = 0; j < nsl; j += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = j + u < nsl ? __hip_atomic_load(part + (first + j + u) * C + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                         : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u];
  }
  const double sum = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  const int64_t pos = c * C + p;
  const int64_t r = PERM ? (int64_t)perm[pos] : (pos < M ? pos : -1);
  if (r >= 0) put_y(y, r, sum, add);
  if (p == 0) cnt[first] = 0;
}

// SELL with wide chunks, one launch: the first nwg_wide workgroups (one wave
// each) take the column slices of the chunks before kc_first (64 slots of one
// chunk per item, C lanes per item), the rest the narrow chunks [c0, nchunks)
// as k_sell_kc does.  The slices start first and keep up to 32 slots of a
// stored row in flight, so their long dependent chains overlap the narrow
// chunks instead of following them.  nwg_wide is a multiple of 8, so the
// narrow part's XCD-aware order holds.
template <typename T, int LOGC, bool PERM, int KC>
__global__ __launch_bounds__(WAVE) void k_sell_mixed(int64_t M, int64_t nitems, const int2* __restrict__ items,
                                                     int64_t nwg_wide, int64_t c0, int64_t nchunks,
                                                     const int64_t* __restrict__ cs, const int32_t* __restrict__ perm,
                                                     const int32_t* __restrict__ scol, const T* __restrict__ sval,
                                                     const T* __restrict__ x, T* __restrict__ y,
                                                     double* part, int32_t* cnt, int remap, int add) {
  constexpr int C = 1 << LOGC;
  double sa[4] = {0.0, 0.0, 0.0, 0.0};
  if ((int64_t)blockIdx.x < nwg_wide) {
    const int64_t gid = (int64_t)blockIdx.x * WAVE + threadIdx.x;
    const int64_t it = gid >> LOGC;
    if (it >= nitems) return;
    const int p = (int)(gid & (C - 1));
    const int2 im = items[it];
    const int64_t c = im.x, k0 = im.y;
    const int64_t base = cs[c];
    const int64_t w = (cs[c + 1] - base) >> LOGC;
    // 0..64 slots of this slice (0: a chunk of empty rows, e.g. a column band
    // that misses them, has one item and nothing to load)
    const int n = (int)((w < k0 + SELL_KT ? w : k0 + SELL_KT) - k0);
    const int32_t* cc = scol + base + k0 * C + p;
    const T* vv = sval + base + k0 * C + p;
    if (n <= 0) {
    } else if (n > 32) {
      sell_slots<T, LOGC, 32>(cc, vv, x, 32, sa);
      sell_slots<T, LOGC, 32>(cc + 32 * C, vv + 32 * C, x, n - 32, sa);
    } else if (n > 16) {
      sell_slots<T, LOGC, 32>(cc, vv, x, n, sa);
    } else if (n > 8) {
      sell_slots<T, LOGC, 16>(cc, vv, x, n, sa);
    } else {
      sell_slots<T, LOGC, 8>(cc, vv, x, n, sa);
    }
    const double s = (sa[0] + sa[1]) + (sa[2] + sa[3]);
    if (w <= SELL_KT) {
      const int64_t pos = c * C + p;
      const int64_t r = PERM ? (int64_t)perm[pos] : (pos < M ? pos : -1);
      if (r >= 0) put_y(y, r, s, add);
    } else {
      const int64_t nsl = (w + SELL_KT - 1) / SELL_KT;
      if (nsl <= SELL_FUSE) sell_fix_last<T, LOGC, PERM>(M, it - k0 / SELL_KT, it, nsl, c, p, s, part, perm, cnt, y, add);
      else part[it * C + p] = s;
    }
    return;
  }
  const uint32_t nb = gridDim.x - (uint32_t)nwg_wide, b = blockIdx.x - (uint32_t)nwg_wide;
  const int64_t gid = (int64_t)(remap ? xcd_block(b, nb) : b) * WAVE + threadIdx.x;
  const int64_t c = c0 + (LOGC == 6 ? (int64_t)__builtin_amdgcn_readfirstlane((int32_t)(gid >> 6)) : gid >> LOGC);
  if (c >= nchunks) return;
  const int p = (int)(gid & (C - 1));
  const int64_t pos = c * C + p;
  const int64_t r = PERM ? (int64_t)perm[pos] : (pos < M ? pos : -1);
  const int64_t base = cs[c];
  const int w = (int)((cs[c + 1] - base) >> LOGC);
  if (add) {  // a band after the first: the old y loaded beside the gathers
    double yo = 0.0;
    if (w > 0) {
      const int32_t* cc = scol + base + p;
      const T* vv = sval + base + p;
      if (KC > 16 && w > 16) yo = sell_slots_y<T, LOGC, KC>(cc, vv, x, w, sa, y, r);
      else if (KC > 8 && w > 8) yo = sell_slots_y<T, LOGC, (KC < 16 ? KC : 16)>(cc, vv, x, w, sa, y, r);
      else if (KC > 4 && w > 4) yo = sell_slots_y<T, LOGC, (KC < 8 ? KC : 8)>(cc, vv, x, w, sa, y, r);
      else yo = sell_slots_y<T, LOGC, (KC < 4 ? KC : 4)>(cc, vv, x, w, sa, y, r);
    } else if (r >= 0) {
      yo = (double)y[r];
    }
    if (r >= 0) y[r] = (T)(yo + ((sa[0] + sa[1]) + (sa[2] + sa[3])));
    return;
  }
  if (w > 0) {
    const int32_t* cc = scol + base + p;
    const T* vv = sval + base + p;
    if (KC > 16 && w > 16) sell_slots<T, LOGC, KC>(cc, vv, x, w, sa);
    else if (KC > 8 && w > 8) sell_slots<T, LOGC, (KC < 16 ? KC : 16)>(cc, vv, x, w, sa);
    else if (KC > 4 && w > 4) sell_slots<T, LOGC, (KC < 8 ? KC : 8)>(cc, vv, x, w, sa);
    else sell_slots<T, LOGC, (KC < 4 ? KC : 4)>(cc, vv, x, w, sa);
  }
  if (r >= 0) put_y(y, r, (sa[0] + sa[1]) + (sa[2] + sa[3]), add);
}

// One workgroup per wide chunk, BS / C threads per stored row: thread j of
// row p sums slices j, j + BS/C, ... (eight loads in flight, eight running
// sums), then thread 0 of the row adds the rows' BS/C sums in order and
// writes y.  The longest chunks (tens of slices on Zipf rows) then take a
// few rounds of loads instead of one per eight slices.
template <typename T, bool PERM>
__global__ __launch_bounds__(BS) void k_sell_fix(int64_t M, int64_t nwide, int C, const int4* __restrict__ wide,
                                                 const int32_t* __restrict__ perm, const double* __restrict__ part,
                                                 T* __restrict__ y, int add) {
  __shared__ double red[BS];
  const int64_t wi = blockIdx.x;
  if (wi >= nwide) return;
  const int t = threadIdx.x, S = BS / C, p = t % C, j = t / C;
  const int4 wd = wide[wi];  // chunk, first item, item count
  const double* q = part + (int64_t)wd.y * C + p;
  // the row and, adding, its old y: loaded before the partial sums
  const int64_t pos = (int64_t)wd.x * C + p;
  const int64_t r = j == 0 ? (PERM ? (int64_t)perm[pos] : (pos < M ? pos : -1)) : -1;
  const double yo = add && r >= 0 ? (double)y[r] : 0.0;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = j; i < wd.z; i += 8 * S) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = i + u * S;
      v[u] = k < wd.z ? q[(int64_t)k * C] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u];
  }
  red[t] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  __syncthreads();
  if (j == 0) {
    double sum = red[p];
    for (int jj = 1; jj < S; ++jj) sum += red[jj * C + p];
    if (r >= 0) y[r] = add ? (T)(yo + sum) : (T)sum;
  }
}

template <typename T, int LOGC, int KC>
static void launch_sell_mixed(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  const int64_t nwide = cdiv(cdiv(A->nitems << LOGC, WAVE), 8) * 8;
  const int64_t nnarrow = cdiv((A->nchunks - A->kc_first) << LOGC, WAVE);
  const int remap = (int64_t)A->sigma * 8 <= A->M;
  const unsigned g = (unsigned)(nwide + nnarrow);
  if (A->perm)
    launch(k_sell_mixed<T, LOGC, true, KC>, g, WAVE, s, A->M, A->nitems, A->items, nwide, A->kc_first, A->nchunks,
           A->cs, A->perm, A->scol, (const T*)A->sval, (const T*)x, (T*)y, A->part, A->wcnt, remap, A->acc);
  else
    launch(k_sell_mixed<T, LOGC, false, KC>, g, WAVE, s, A->M, A->nitems, A->items, nwide, A->kc_first, A->nchunks,
           A->cs, A->perm, A->scol, (const T*)A->sval, (const T*)x, (T*)y, A->part, A->wcnt, remap, A->acc);
}

template <typename T, int LOGC, int KC>
static void launch_sell_kc(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  if (A->kc_first > 0) {  // wide chunks too: one launch for both (the slices' fix-up follows)
    launch_sell_mixed<T, LOGC, KC>(A, x, y, s);
    return;
  }
  const unsigned g = (unsigned)cdiv((A->nchunks - A->kc_first) << LOGC, WAVE);
  // contiguous ranges per XCD only while a sort window is small next to an
  // XCD's share of the rows (chunk widths then do not trend across the list)
  const int remap = (int64_t)A->sigma * 8 <= A->M;
  if (LOGC == 6 && (A->params.flags & SPMV_FLAG_SPLIT6)) {  // g = one workgroup per chunk
    if (A->perm)
      launch(k_sell_kcw<T, true, KC, 6>, g, 6 * WAVE, s, A->M, A->kc_first, A->nchunks, A->cs, A->perm, A->scol,
             (const T*)A->sval, (const T*)x, (T*)y, remap, A->acc);
    else
      launch(k_sell_kcw<T, false, KC, 6>, g, 6 * WAVE, s, A->M, A->kc_first, A->nchunks, A->cs, A->perm, A->scol,
             (const T*)A->sval, (const T*)x, (T*)y, remap, A->acc);
    return;
  }
  if (LOGC == 6 && (A->params.flags & SPMV_FLAG_SPLIT4)) {
    if (A->perm)
      launch(k_sell_kcw<T, true, KC, 4>, g, 4 * WAVE, s, A->M, A->kc_first, A->nchunks, A->cs, A->perm, A->scol,
             (const T*)A->sval, (const T*)x, (T*)y, remap, A->acc);
    else
      launch(k_sell_kcw<T, false, KC, 4>, g, 4 * WAVE, s, A->M, A->kc_first, A->nchunks, A->cs, A->perm, A->scol,
             (const T*)A->sval, (const T*)x, (T*)y, remap, A->acc);
    return;
  }
  if (A->perm)
    launch(k_sell_kc<T, LOGC, true, KC>, g, WAVE, s, A->M, A->kc_first, A->nchunks, A->cs, A->perm, A->scol,
           (const T*)A->sval, (const T*)x, (T*)y, remap, A->acc);
  else
    launch(k_sell_kc<T, LOGC, false, KC>, g, WAVE, s, A->M, A->kc_first, A->nchunks, A->cs, A->perm, A->scol,
           (const T*)A->sval, (const T*)x, (T*)y, remap, A->acc);
}

// Chunks [kc_first, nchunks) (at most SELL_KC_MAX wide) go through the one-pass
// narrow kernel; the chunks before them (with a global sort: the longest
// rows) through the column-slice items.  Both write disjoint rows of y.
template <typename T, int LOGC>
static void launch_sell_c(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  if (A->kc_first < A->nchunks || A->kc_first > 0) {
    if (LOGC == 6) {  // one chunk per wave: instantiated for the exact widest chunk
      switch (A->kc_w) {
      case 1: launch_sell_kc<T, 6, 1>(A, x, y, s); break;
      case 2: launch_sell_kc<T, 6, 2>(A, x, y, s); break;
      case 3: launch_sell_kc<T, 6, 3>(A, x, y, s); break;
      case 4: launch_sell_kc<T, 6, 4>(A, x, y, s); break;
      case 5: launch_sell_kc<T, 6, 5>(A, x, y, s); break;
      case 6: launch_sell_kc<T, 6, 6>(A, x, y, s); break;
      case 7: launch_sell_kc<T, 6, 7>(A, x, y, s); break;
      case 8: launch_sell_kc<T, 6, 8>(A, x, y, s); break;
      case 9: launch_sell_kc<T, 6, 9>(A, x, y, s); break;
      case 10: launch_sell_kc<T, 6, 10>(A, x, y, s); break;
      case 11: launch_sell_kc<T, 6, 11>(A, x, y, s); break;
      case 12: launch_sell_kc<T, 6, 12>(A, x, y, s); break;
      case 13: launch_sell_kc<T, 6, 13>(A, x, y, s); break;
      case 14: launch_sell_kc<T, 6, 14>(A, x, y, s); break;
      case 15: launch_sell_kc<T, 6, 15>(A, x, y, s); break;
      case 16: launch_sell_kc<T, 6, 16>(A, x, y, s); break;
      case 17: launch_sell_kc<T, 6, 17>(A, x, y, s); break;
      case 18: launch_sell_kc<T, 6, 18>(A, x, y, s); break;
      case 19: launch_sell_kc<T, 6, 19>(A, x, y, s); break;
      case 20: launch_sell_kc<T, 6, 20>(A, x, y, s); break;
      case 21: launch_sell_kc<T, 6, 21>(A, x, y, s); break;
      case 22: launch_sell_kc<T, 6, 22>(A, x, y, s); break;
      case 23: launch_sell_kc<T, 6, 23>(A, x, y, s); break;
      case 24: launch_sell_kc<T, 6, 24>(A, x, y, s); break;
      case 25: launch_sell_kc<T, 6, 25>(A, x, y, s); break;
      case 26: launch_sell_kc<T, 6, 26>(A, x, y, s); break;
      case 27: launch_sell_kc<T, 6, 27>(A, x, y, s); break;
      case 28: launch_sell_kc<T, 6, 28>(A, x, y, s); break;
      case 29: launch_sell_kc<T, 6, 29>(A, x, y, s); break;
      case 30: launch_sell_kc<T, 6, 30>(A, x, y, s); break;
      case 31: launch_sell_kc<T, 6, 31>(A, x, y, s); break;
      case 32: launch_sell_kc<T, 6, 32>(A, x, y, s); break;
        default: launch_sell_kc<T, 6, 32>(A, x, y, s); break;  // maxw == 0: nothing to load
      }
    } else if (A->kc_w <= 16) {
      launch_sell_kc<T, LOGC, 16>(A, x, y, s);
    } else {
      launch_sell_kc<T, LOGC, 32>(A, x, y, s);
    }
  }
  if (A->kc_first == 0) return;
  if (A->nwide > 0) {
    const unsigned gf = (unsigned)A->nwide;  // one workgroup per wide chunk
    if (A->perm)
      launch(k_sell_fix<T, true>, gf, BS, s, A->M, A->nwide, 1 << LOGC, A->wide, A->perm, A->part, (T*)y, A->acc);
    else
      launch(k_sell_fix<T, false>, gf, BS, s, A->M, A->nwide, 1 << LOGC, A->wide, A->perm, A->part, (T*)y, A->acc);
  }
}

template <typename T>
static spmv_status_t run_sell_t(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  if (A->M == 0) return SPMV_OK;
  switch (A->C) {
    case 1: launch_sell_c<T, 0>(A, x, y, s); break;
    case 2: launch_sell_c<T, 1>(A, x, y, s); break;
    case 4: launch_sell_c<T, 2>(A, x, y, s); break;
    case 8: launch_sell_c<T, 3>(A, x, y, s); break;
    case 16: launch_sell_c<T, 4>(A, x, y, s); break;
    case 32: launch_sell_c<T, 5>(A, x, y, s); break;
    case 64: launch_sell_c<T, 6>(A, x, y, s); break;
    default: return fail(SPMV_ERR_UNSUPPORTED, "SELL chunk C=%d (need a power of two <= 64)", A->C);
  }
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

spmv_status_t run_sell(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  if (A->dt == SPMV_F64) return run_sell_t<double>(A, x, y, s);
  return run_sell_t<float>(A, x, y, s);
}

// out[0] = 1 + the last chunk wider than SELL_KC_MAX (0 if none)
__global__ void k_sell_lastwide(int64_t nch, int C, const int64_t* cs, int32_t* out) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += (int64_t)gridDim.x * blockDim.x)
    if ((cs[c + 1] - cs[c]) / C > SELL_KC_MAX) atomicMax(out, (int32_t)(c + 1));
}

// out[1] = the widest chunk from out[0] on
__global__ void k_sell_tailw(int64_t nch, int C, const int64_t* cs, int32_t* out) {
  const int64_t c0 = out[0];
  for (int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += (int64_t)gridDim.x * blockDim.x)
    atomicMax(out + 1, (int32_t)((cs[c + 1] - cs[c]) / C));
}

// slices per chunk, and the item / wide-chunk lists
__global__ void k_sell_nslices(int64_t nch, int C, const int64_t* cs, int32_t* ns, int32_t* wideflag) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = (cs[c + 1] - cs[c]) / C;
    const int64_t n = w <= SELL_KT ? 1 : (w + SELL_KT - 1) / SELL_KT;
    ns[c] = (int32_t)n;
    wideflag[c] = n > SELL_FUSE;  // the chunks k_sell_fix finishes
  }
}

__global__ void k_sell_items(int64_t nch, const int32_t* ns, const int32_t* ibase, const int32_t* wideflag,
                             const int32_t* wpos, int2* items, int4* wide) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t b = ibase[c], n = ns[c];
    for (int32_t i = 0; i < n; ++i) items[b + i] = make_int2((int)c, i * SELL_KT);
    if (wideflag[c]) wide[wpos[c]] = make_int4((int)c, b, n, 0);
  }
}

static spmv_status_t sell_fill(spmv_mat_s* src, spmv_mat_s* A, int64_t nunits, const int64_t* units, hipStream_t s) {
  const unsigned gc = (unsigned)std::min<int64_t>(nunits, (int64_t)1 << 20);
  if (A->dt == SPMV_F64)
    k_csr_to_sell<double><<<gc, WAVE, 0, s>>>(src->M, nunits, A->C, src->ptr, src->col, (const double*)src->val,
                                              A->perm, A->cs, units, A->scol, (double*)A->sval);
  else
    k_csr_to_sell<float><<<gc, WAVE, 0, s>>>(src->M, nunits, A->C, src->ptr, src->col, (const float*)src->val,
                                             A->perm, A->cs, units, A->scol, (float*)A->sval);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

spmv_status_t convert_sell(spmv_mat_s* src, spmv_mat_s* A, hipStream_t s) {
  const int64_t M = src->M;
  const int C = A->params.sell_C;
  const int64_t sigma = A->params.sell_sigma;
  if (C < 1 || C > 64 || (C & (C - 1))) return fail(SPMV_ERR_UNSUPPORTED, "SELL C=%d (need a power of two <= 64)", C);
  if (sigma < 1) return fail(SPMV_ERR_INVALID_ARG, "SELL sigma=%lld", (long long)sigma);
  A->C = C;
  A->sigma = (int32_t)sigma;
  A->nchunks = cdiv(M, C);
  A->Mpad = A->nchunks * C;
  const unsigned g = grid_rows(std::max<int64_t>(M, A->Mpad));
  int32_t maxlen = 0;
  if (M > 0) SPMV_TRY(device_max_i32(src->ptr, M, 1, &maxlen, s));
  A->sell_maxw = maxlen;
  if (sigma > 1 && M > 0) {
    DTmp k1, k2, v1, v2;
    SPMV_TRY(k1.alloc(sizeof(uint64_t) * M));
    SPMV_TRY(k2.alloc(sizeof(uint64_t) * M));
    SPMV_TRY(v1.alloc(sizeof(uint32_t) * M));
    SPMV_TRY(v2.alloc(sizeof(uint32_t) * M));
    uint64_t* keys = k1.as<uint64_t>();
    uint32_t* idx = v1.as<uint32_t>();
    k_sell_keys<<<g, BS, 0, s>>>(M, src->ptr, sigma, maxlen, keys, idx);
    SPMV_LAUNCH_CHECK();
    const uint64_t nwin = (uint64_t)cdiv(M, sigma);
    SPMV_TRY(radix_sort_pairs(&keys, &idx, k2.as<uint64_t>(), v2.as<uint32_t>(), M,
                              bits_for(nwin * (uint64_t)(maxlen + 1) - 1), s));
    SPMV_TRY(mat_alloc(A, (void**)&A->perm, sizeof(int32_t) * A->Mpad));
    k_sell_perm<<<g, BS, 0, s>>>(M, A->Mpad, idx, A->perm);
    SPMV_LAUNCH_CHECK();
    SPMV_HIP(hipStreamSynchronize(s));  // k1/k2/v1/v2 are freed on return
  }
  DTmp cw;
  SPMV_TRY(cw.alloc(sizeof(int64_t) * std::max<int64_t>(A->nchunks, 1)));
  SPMV_TRY(mat_alloc(A, (void**)&A->cs, sizeof(int64_t) * (A->nchunks + 1)));
  if (A->nchunks) {
    k_sell_width<<<grid_rows(A->nchunks), BS, 0, s>>>(M, A->nchunks, C, src->ptr, A->perm, cw.as<int64_t>());
    SPMV_LAUNCH_CHECK();
  }
  SPMV_TRY(scan_i64_to_i64(cw.as<int64_t>(), A->cs, A->nchunks, s));
  SPMV_TRY(copy_to_host(&A->nslots, A->cs + A->nchunks, sizeof(int64_t), s));
  SPMV_TRY(check_cap(A, A->nslots * (4 + A->sv), "SELL"));
  SPMV_TRY(mat_alloc(A, (void**)&A->scol, sizeof(int32_t) * A->nslots));
  SPMV_TRY(mat_alloc(A, &A->sval, (size_t)A->sv * A->nslots));
  if (A->Mpad) {
    SPMV_TRY(sell_fill(src, A, A->nchunks, nullptr, s));
    if ((int64_t)maxlen * C > SELL_FILL) {  // the slots of long chunks beyond the first SELL_FILL
      std::vector<int64_t> hcs(A->nchunks + 1), units;
      SPMV_TRY(copy_to_host(hcs.data(), A->cs, sizeof(int64_t) * (A->nchunks + 1), s));
      for (int64_t c = 0; c < A->nchunks; ++c)
        for (int64_t q0 = SELL_FILL; q0 < hcs[c + 1] - hcs[c]; q0 += SELL_FILL) {
          units.push_back(c);
          units.push_back(q0);
        }
      if (!units.empty()) {
        DTmp du;
        SPMV_TRY(du.alloc(sizeof(int64_t) * units.size()));
        SPMV_HIP(hipMemcpyAsync(du.p, units.data(), sizeof(int64_t) * units.size(), hipMemcpyHostToDevice, s));
        SPMV_TRY(sell_fill(src, A, (int64_t)units.size() / 2, du.as<int64_t>(), s));
        SPMV_HIP(hipStreamSynchronize(s));  // du and the host list are freed on return
      }
    }
  }
  // the narrow tail of the chunk list (one-pass kernel): not with C < 8 or
  // when the slice kernel is forced
  A->kc_first = A->nchunks;
  A->kc_w = 0;
  if (C >= 8 && !(A->params.flags & SPMV_FLAG_SELL_SLICES) && A->nchunks > 0) {
    DTmp kw;
    SPMV_TRY(kw.alloc(2 * sizeof(int32_t)));
    SPMV_HIP(hipMemsetAsync(kw.p, 0, 2 * sizeof(int32_t), s));
    k_sell_lastwide<<<grid_rows(A->nchunks), BS, 0, s>>>(A->nchunks, C, A->cs, kw.as<int32_t>());
    SPMV_LAUNCH_CHECK();
    k_sell_tailw<<<grid_rows(A->nchunks), BS, 0, s>>>(A->nchunks, C, A->cs, kw.as<int32_t>());
    SPMV_LAUNCH_CHECK();
    int32_t h[2] = {0, 0};
    SPMV_TRY(copy_to_host(h, kw.p, sizeof(h), s));
    A->kc_first = h[0];
    A->kc_w = h[1];
  }
  // work items: column slices of at most SELL_KT per chunk, for the chunks
  // before kc_first
  {
    const int64_t nch = A->kc_first;
    DTmp ns, wf, ib, wp;
    SPMV_TRY(ns.alloc(sizeof(int32_t) * std::max<int64_t>(nch, 1)));
    SPMV_TRY(wf.alloc(sizeof(int32_t) * std::max<int64_t>(nch, 1)));
    SPMV_TRY(ib.alloc(sizeof(int32_t) * (nch + 1)));
    SPMV_TRY(wp.alloc(sizeof(int32_t) * (nch + 1)));
    if (nch) {
      k_sell_nslices<<<grid_rows(nch), BS, 0, s>>>(nch, C, A->cs, ns.as<int32_t>(), wf.as<int32_t>());
      SPMV_LAUNCH_CHECK();
    }
    SPMV_TRY(scan_i32_to_i32(ns.as<int32_t>(), ib.as<int32_t>(), nch, s));
    SPMV_TRY(scan_i32_to_i32(wf.as<int32_t>(), wp.as<int32_t>(), nch, s));
    int32_t tot[1] = {0}, nw[1] = {0};
    SPMV_TRY(copy_to_host(tot, ib.as<int32_t>() + nch, sizeof(int32_t), s));
    SPMV_TRY(copy_to_host(nw, wp.as<int32_t>() + nch, sizeof(int32_t), s));
    A->nitems = tot[0];
    A->nwide = nw[0];
    SPMV_TRY(mat_alloc(A, (void**)&A->items, sizeof(int2) * std::max<int64_t>(A->nitems, 1)));
    SPMV_TRY(mat_alloc(A, (void**)&A->wide, sizeof(int4) * std::max<int64_t>(A->nwide, 1)));
    if (A->nitems > nch) {  // some chunk has several slices: partial sums and slice counts
      SPMV_TRY(mat_alloc(A, (void**)&A->part, sizeof(double) * A->nitems * C));
      SPMV_TRY(mat_alloc(A, (void**)&A->wcnt, sizeof(int32_t) * A->nitems));
      SPMV_HIP(hipMemsetAsync(A->wcnt, 0, sizeof(int32_t) * A->nitems, s));
    }
    if (nch) {
      k_sell_items<<<grid_rows(nch), BS, 0, s>>>(nch, ns.as<int32_t>(), ib.as<int32_t>(), wf.as<int32_t>(),
                                                 wp.as<int32_t>(), A->items, A->wide);
      SPMV_LAUNCH_CHECK();
    }
    SPMV_HIP(hipStreamSynchronize(s));
  }
  A->pad_slots = A->nslots - src->nnz;
  A->bytes_fmt = A->nslots * (4 + A->sv) + (A->nchunks + 1) * 8 + (A->perm ? A->Mpad * 4 : 0) + A->nitems * 8 +
                 A->N * A->sv + A->M * A->sv;
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

// ================================================================== HYB

__global__ void k_hyb_keys(int64_t M, const int32_t* ptr, int64_t maxlen, uint64_t* key, uint32_t* idx) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    key[i] = (uint64_t)(maxlen - (ptr[i + 1] - ptr[i]));
    idx[i] = (uint32_t)i;
  }
}

__global__ void k_hyb_tail_count(int64_t M, int64_t K, const int32_t* ptr, int32_t* tcnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t len = ptr[i + 1] - ptr[i];
    tcnt[i] = (int32_t)(len > K ? len - K : 0);
  }
}

// one wave per row copies the row's entries beyond K into the COO arrays
template <typename T>
__global__ void k_hyb_fill_coo(int64_t M, int64_t K, const int32_t* ptr, const int32_t* col, const T* val,
                               const int64_t* off, int32_t* crow, int32_t* ccol, T* cval) {
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
  for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; i < M; i += nw) {
    const int64_t a = ptr[i] + K, e = ptr[i + 1], o = off[i] - a;
    for (int64_t k = a + __lane_id(); k < e; k += WAVE) {
      crow[o + k] = (int32_t)i;
      ccol[o + k] = col[k];
      cval[o + k] = val[k];
    }
  }
}

// COO pass by wave tiles (wave_tile_reduce): a wave takes TILE_E
// consecutive tail entries with all loads and gathers in flight and no
// barrier; the tail's rows are added to the y the ELL kernel wrote.
template <typename T>
__global__ __launch_bounds__(BS) void k_coo_tiles(int64_t ncoo, int64_t ntiles, const int32_t* __restrict__ crow,
                                                  const int32_t* __restrict__ ccol, const T* __restrict__ cval,
                                                  const T* __restrict__ x, T* __restrict__ y,
                                                  double* __restrict__ head_part, double* __restrict__ tail_part,
                                                  int32_t* __restrict__ tail_row, int32_t* __restrict__ tinfo) {
  const int64_t t = (int64_t)blockIdx.x * (BS / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  if (t >= ntiles) return;
  const int l = __lane_id();
  const int64_t e0 = t * TILE_E;
  const int nv = (int)(ncoo - e0 < TILE_E ? ncoo - e0 : TILE_E);  // valid entries, >= 1
  int32_t cc[TILE_S], rr[TILE_S];
  T vv[TILE_S];
#pragma unroll
  for (int s = 0; s < TILE_S; ++s) {
    const int k = s * WAVE + l;
    const uint32_t kk = (uint32_t)(k < nv ? k : nv - 1);
    cc[s] = ldnt32(ccol + e0, kk);
    vv[s] = ldnt32(cval + e0, kk);
    rr[s] = ld32(crow + e0, kk);
  }
  const int32_t rprev = t > 0 ? crow[e0 - 1] : -1;                                          // row before the tile
  const int32_t rnext = nv == TILE_E && e0 + TILE_E < ncoo ? crow[e0 + TILE_E] : -2;  // row after it
  issue_fence();
#pragma unroll
  for (int s = 0; s < TILE_S; ++s)
    if (s * WAVE + l >= nv) rr[s] = TILE_NONE;
  wave_tile_reduce<T, true>(t, nv, rr, cc, vv, rprev, rnext, x, y, head_part, tail_part, tail_row, tinfo);
}

// One COO pass over entries [e0, e0 + n) with tile scratch from tile tb on:
// the tiles add their rows onto y, then the fix-up adds the rows that cross
// tiles.  Passes on one stream run in order, so the column bands of a banded
// tail add onto y one after another, in band order.
template <typename T>
static spmv_status_t coo_pass(spmv_mat_s* A, int64_t e0, int64_t n, int64_t tb, const void* x, void* y,
                              hipStream_t s) {
  const int64_t nt = cdiv(n, TILE_E);
  launch(k_coo_tiles<T>, (unsigned)cdiv(nt, BS / WAVE), BS, s, n, nt, A->crow + e0, A->ccol + e0,
         (const T*)A->cval + e0, (const T*)x, (T*)y, A->coo_head + tb, A->coo_tail + tb, A->coo_trow + tb,
         A->coo_tinfo + tb);
  SPMV_LAUNCH_CHECK();
  if (nt > 1) {
    launch(k_tile_fix<T, true>, (unsigned)std::min<int64_t>(cdiv(nt, BS), 4096), BS, s, nt,
           (const double*)A->coo_head + tb, (const double*)A->coo_tail + tb, (const int32_t*)A->coo_trow + tb,
           (const int32_t*)A->coo_tinfo + tb, (T*)y);
    SPMV_LAUNCH_CHECK();
  }
  return SPMV_OK;
}

template <typename T>
static spmv_status_t run_hyb_t(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  if (A->M == 0) return SPMV_OK;
  SPMV_TRY(launch_ell<T>(A->M, A->K, A->ecol, A->eval, x, y, !(A->params.flags & SPMV_FLAG_LINEAR),
                         (A->params.flags & SPMV_FLAG_SPLIT4) != 0, s));
  if (A->ncoo == 0) return SPMV_OK;
  if (A->coo_boff.empty()) return coo_pass<T>(A, 0, A->ncoo, 0, x, y, s);
  int64_t tb = 0;
  for (size_t b = 0; b + 1 < A->coo_boff.size(); ++b) {
    const int64_t e0 = A->coo_boff[b], n = A->coo_boff[b + 1] - e0;
    if (n == 0) continue;
    SPMV_TRY(coo_pass<T>(A, e0, n, tb, x, y, s));
    tb += cdiv(n, TILE_E);
  }
  return SPMV_OK;
}

spmv_status_t run_hyb(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  if (A->dt == SPMV_F64) return run_hyb_t<double>(A, x, y, s);
  return run_hyb_t<float>(A, x, y, s);
}

// K = the ceil(M/3)-th largest row length: the largest k with at least
// ceil(M/3) rows of length >= k.
static spmv_status_t hyb_rule_k(spmv_mat_s* src, int64_t* K, hipStream_t s) {
  const int64_t M = src->M;
  *K = 0;
  if (M == 0) return SPMV_OK;
  int32_t maxlen = 0;
  SPMV_TRY(device_max_i32(src->ptr, M, 1, &maxlen, s));
  DTmp k1, k2, v1, v2;
  SPMV_TRY(k1.alloc(sizeof(uint64_t) * M));
  SPMV_TRY(k2.alloc(sizeof(uint64_t) * M));
  SPMV_TRY(v1.alloc(sizeof(uint32_t) * M));
  SPMV_TRY(v2.alloc(sizeof(uint32_t) * M));
  uint64_t* keys = k1.as<uint64_t>();
  uint32_t* idx = v1.as<uint32_t>();
  k_hyb_keys<<<grid_rows(M), BS, 0, s>>>(M, src->ptr, maxlen, keys, idx);
  SPMV_LAUNCH_CHECK();
  SPMV_TRY(radix_sort_pairs(&keys, &idx, k2.as<uint64_t>(), v2.as<uint32_t>(), M, bits_for((uint64_t)maxlen), s));
  const int64_t need = (M + 2) / 3;
  uint64_t kk = 0;
  SPMV_TRY(copy_to_host(&kk, keys + (need - 1), sizeof(uint64_t), s));
  *K = (int64_t)maxlen - (int64_t)kk;
  return SPMV_OK;
}

__global__ void k_coo_band_keys(int64_t n, const int32_t* ccol, int64_t bw, uint64_t* key, uint32_t* idx) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    key[i] = (uint64_t)(ccol[i] / bw);
    idx[i] = (uint32_t)i;
  }
}

template <typename T>
__global__ void k_coo_gather(int64_t n, const uint32_t* idx, const int32_t* r0, const int32_t* c0, const T* v0,
                             int32_t* r1, int32_t* c1, T* v1) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t j = idx[i];
    r1[i] = r0[j];
    c1[i] = c0[j];
    v1[i] = v0[j];
  }
}

// first index whose (ascending) key is >= b, for b = 0..nb
__global__ void k_key_bounds(int64_t n, const uint64_t* key, int nb, int64_t* bound) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nb) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (key[mid] < (uint64_t)b) lo = mid + 1;
    else hi = mid;
  }
  bound[b] = lo;
}

// Reorder a row-major COO tail (r, c, v) into A's arrays by column band,
// stably, so each band stays in row-major order; record the band offsets.
static spmv_status_t coo_order_by_band(spmv_mat_s* A, int nb, const int32_t* r, const int32_t* c, const void* v,
                                       hipStream_t s) {
  const int64_t n = A->ncoo;
  const int64_t bw = std::max<int64_t>(1, cdiv(A->N, nb));
  A->band_w = bw;
  if (n >= ((int64_t)1 << 32)) return fail(SPMV_ERR_TOO_LARGE, "%lld COO entries", (long long)n);
  DTmp k1, k2, v1, v2, bd;
  SPMV_TRY(k1.alloc(sizeof(uint64_t) * n));
  SPMV_TRY(k2.alloc(sizeof(uint64_t) * n));
  SPMV_TRY(v1.alloc(sizeof(uint32_t) * n));
  SPMV_TRY(v2.alloc(sizeof(uint32_t) * n));
  SPMV_TRY(bd.alloc(sizeof(int64_t) * (nb + 1)));
  uint64_t* key = k1.as<uint64_t>();
  uint32_t* idx = v1.as<uint32_t>();
  k_coo_band_keys<<<grid_rows(n), BS, 0, s>>>(n, c, bw, key, idx);
  SPMV_LAUNCH_CHECK();
  SPMV_TRY(radix_sort_pairs(&key, &idx, k2.as<uint64_t>(), v2.as<uint32_t>(), n, bits_for((uint64_t)(nb - 1)), s));
  if (A->dt == SPMV_F64)
    k_coo_gather<double><<<grid_rows(n), BS, 0, s>>>(n, idx, r, c, (const double*)v, A->crow, A->ccol,
                                                     (double*)A->cval);
  else
    k_coo_gather<float><<<grid_rows(n), BS, 0, s>>>(n, idx, r, c, (const float*)v, A->crow, A->ccol,
                                                    (float*)A->cval);
  SPMV_LAUNCH_CHECK();
  k_key_bounds<<<1, 128, 0, s>>>(n, key, nb, bd.as<int64_t>());
  SPMV_LAUNCH_CHECK();
  A->coo_boff.assign(nb + 1, 0);
  SPMV_TRY(copy_to_host(A->coo_boff.data(), bd.p, sizeof(int64_t) * (nb + 1), s));
  return SPMV_OK;
}

spmv_status_t convert_hyb(spmv_mat_s* src, spmv_mat_s* A, hipStream_t s) {
  const int64_t M = src->M;
  const int nb = A->params.bands;
  if (nb > 64) return fail(SPMV_ERR_UNSUPPORTED, "%d column bands (at most 64)", nb);
  int64_t K = A->params.hyb_K;
  if (K < 0) SPMV_TRY(hyb_rule_k(src, &K, s));
  A->params.hyb_K = (int32_t)K;
  SPMV_TRY(check_cap(A, M * K * (4 + A->sv), "HYB-ELL"));
  SPMV_TRY(build_ell_part(src, A, K, s));
  DTmp tc, off;
  SPMV_TRY(tc.alloc(sizeof(int32_t) * std::max<int64_t>(M, 1)));
  SPMV_TRY(off.alloc(sizeof(int64_t) * (M + 1)));
  if (M) {
    k_hyb_tail_count<<<grid_rows(M), BS, 0, s>>>(M, K, src->ptr, tc.as<int32_t>());
    SPMV_LAUNCH_CHECK();
  }
  SPMV_TRY(scan_i32_to_i64(tc.as<int32_t>(), off.as<int64_t>(), M, s));
  SPMV_TRY(copy_to_host(&A->ncoo, off.as<int64_t>() + M, sizeof(int64_t), s));
  SPMV_TRY(mat_alloc(A, (void**)&A->crow, sizeof(int32_t) * A->ncoo));
  SPMV_TRY(mat_alloc(A, (void**)&A->ccol, sizeof(int32_t) * A->ncoo));
  SPMV_TRY(mat_alloc(A, &A->cval, (size_t)A->sv * A->ncoo));
  const bool banded = nb > 1 && A->ncoo > 0;
  if (A->ncoo) {
    // row-major tail, written straight into the handle or, when banded,
    // into temporaries that are then reordered by column band
    DTmp tr, tcol, tv;
    int32_t* crow = A->crow;
    int32_t* ccol = A->ccol;
    void* cval = A->cval;
    if (banded) {
      SPMV_TRY(tr.alloc(sizeof(int32_t) * A->ncoo));
      SPMV_TRY(tcol.alloc(sizeof(int32_t) * A->ncoo));
      SPMV_TRY(tv.alloc((size_t)A->sv * A->ncoo));
      crow = tr.as<int32_t>();
      ccol = tcol.as<int32_t>();
      cval = tv.p;
    }
    const unsigned gw = (unsigned)std::min<int64_t>(cdiv(M, BS / WAVE), 1 << 20);
    if (A->dt == SPMV_F64)
      k_hyb_fill_coo<double><<<gw, BS, 0, s>>>(M, K, src->ptr, src->col, (const double*)src->val, off.as<int64_t>(),
                                               crow, ccol, (double*)cval);
    else
      k_hyb_fill_coo<float><<<gw, BS, 0, s>>>(M, K, src->ptr, src->col, (const float*)src->val, off.as<int64_t>(),
                                              crow, ccol, (float*)cval);
    SPMV_LAUNCH_CHECK();
    if (banded) SPMV_TRY(coo_order_by_band(A, nb, crow, ccol, cval, s));
  }
  {  // per-tile scratch of the COO pass (each band's tiles start afresh)
    const int64_t nt = std::max<int64_t>(cdiv(A->ncoo, TILE_E) + (banded ? nb : 0), 1);
    SPMV_TRY(mat_alloc(A, (void**)&A->coo_head, sizeof(double) * nt));
    SPMV_TRY(mat_alloc(A, (void**)&A->coo_tail, sizeof(double) * nt));
    SPMV_TRY(mat_alloc(A, (void**)&A->coo_trow, sizeof(int32_t) * nt));
    SPMV_TRY(mat_alloc(A, (void**)&A->coo_tinfo, sizeof(int32_t) * nt));
  }
  A->pad_slots = M * K - (src->nnz - A->ncoo);
  // ELL slots, COO (row, col, val), x once, y written once and the tail rows re-read
  A->bytes_fmt = M * K * (4 + A->sv) + A->ncoo * (8 + A->sv) + A->N * A->sv + A->M * A->sv;
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

// ============================================================ inverses
template <typename T>
static spmv_status_t to_csr_t(spmv_mat_s* A, int32_t* ptr, int32_t* col, T* val, hipStream_t s);

__global__ void k_hyb_len(int64_t M, const int32_t* ell_len, const int32_t* tail_cnt, int32_t* len) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x)
    len[i] = ell_len[i] + tail_cnt[i];
}

__global__ void k_coo_row_keys(int64_t n, const int32_t* crow, uint64_t* key, uint32_t* idx) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    key[i] = (uint64_t)crow[i];
    idx[i] = (uint32_t)i;
  }
}

__global__ void k_coo_rowcount(int64_t n, const int32_t* crow, int32_t* cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[crow[i]], 1);
}

// COO tail of row r goes after its ELL entries: position ptr[r] + ell_len[r] + (k - first tail entry of r)
template <typename T>
__global__ void k_coo_to_csr(int64_t n, const int32_t* crow, const int32_t* ccol, const T* cval, const int32_t* ptr,
                             const int32_t* ell_len, const int64_t* toff, int32_t* col, T* val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = crow[i];
    const int64_t d = (int64_t)ptr[r] + ell_len[r] + (i - toff[r]);
    col[d] = ccol[i];
    val[d] = cval[i];
  }
}

template <typename T>
static spmv_status_t to_csr_t(spmv_mat_s* A, int32_t* ptr, int32_t* col, T* val, hipStream_t s) {
  const int64_t M = A->M;
  const unsigned g = grid_rows(std::max<int64_t>(M, A->Mpad));
  DTmp len;
  SPMV_TRY(len.alloc(sizeof(int32_t) * std::max<int64_t>(M, 1)));
  if (A->fmt == SPMV_FMT_ELL || A->fmt == SPMV_FMT_HYB) {
    if (M) {
      k_ell_count<<<g, BS, 0, s>>>(M, A->K, A->ecol, len.as<int32_t>());
      SPMV_LAUNCH_CHECK();
    }
    if (A->fmt == SPMV_FMT_ELL || A->ncoo == 0) {
      SPMV_TRY(scan_i32_to_i32(len.as<int32_t>(), ptr, M, s));
      if (M) {
        k_ell_to_csr<T><<<g, BS, 0, s>>>(M, A->ecol, (const T*)A->eval, len.as<int32_t>(), ptr, col, val);
        SPMV_LAUNCH_CHECK();
      }
      return SPMV_OK;
    }
    // a banded tail goes back to row-major order first: a stable sort by
    // row keeps each row's bands in band order, i.e. its columns ascending
    const int32_t* crow = A->crow;
    const int32_t* ccol = A->ccol;
    const T* cval = (const T*)A->cval;
    DTmp k1, k2, v1, v2, sr, sc, svv;
    if (!A->coo_boff.empty()) {
      const int64_t n = A->ncoo;
      SPMV_TRY(k1.alloc(sizeof(uint64_t) * n));
      SPMV_TRY(k2.alloc(sizeof(uint64_t) * n));
      SPMV_TRY(v1.alloc(sizeof(uint32_t) * n));
      SPMV_TRY(v2.alloc(sizeof(uint32_t) * n));
      SPMV_TRY(sr.alloc(sizeof(int32_t) * n));
      SPMV_TRY(sc.alloc(sizeof(int32_t) * n));
      SPMV_TRY(svv.alloc(sizeof(T) * n));
      uint64_t* key = k1.as<uint64_t>();
      uint32_t* idx = v1.as<uint32_t>();
      k_coo_row_keys<<<grid_rows(n), BS, 0, s>>>(n, A->crow, key, idx);
      SPMV_LAUNCH_CHECK();
      SPMV_TRY(radix_sort_pairs(&key, &idx, k2.as<uint64_t>(), v2.as<uint32_t>(), n, bits_for((uint64_t)(M - 1)), s));
      k_coo_gather<T><<<grid_rows(n), BS, 0, s>>>(n, idx, A->crow, A->ccol, (const T*)A->cval, sr.as<int32_t>(),
                                                  sc.as<int32_t>(), svv.as<T>());
      SPMV_LAUNCH_CHECK();
      crow = sr.as<int32_t>();
      ccol = sc.as<int32_t>();
      cval = svv.as<T>();
    }
    DTmp cnt, tot, toff;
    SPMV_TRY(cnt.alloc(sizeof(int32_t) * M));
    SPMV_TRY(tot.alloc(sizeof(int32_t) * M));
    SPMV_TRY(toff.alloc(sizeof(int64_t) * (M + 1)));
    SPMV_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * M, s));
    const unsigned gc = grid_rows(A->ncoo);
    k_coo_rowcount<<<gc, BS, 0, s>>>(A->ncoo, crow, cnt.as<int32_t>());
    SPMV_LAUNCH_CHECK();
    SPMV_TRY(scan_i32_to_i64(cnt.as<int32_t>(), toff.as<int64_t>(), M, s));  // first COO entry of each row
    k_hyb_len<<<g, BS, 0, s>>>(M, len.as<int32_t>(), cnt.as<int32_t>(), tot.as<int32_t>());
    SPMV_LAUNCH_CHECK();
    SPMV_TRY(scan_i32_to_i32(tot.as<int32_t>(), ptr, M, s));
    k_ell_to_csr<T><<<g, BS, 0, s>>>(M, A->ecol, (const T*)A->eval, len.as<int32_t>(), ptr, col, val);
    SPMV_LAUNCH_CHECK();
    k_coo_to_csr<T><<<gc, BS, 0, s>>>(A->ncoo, crow, ccol, cval, ptr, len.as<int32_t>(), toff.as<int64_t>(), col,
                                      val);
    SPMV_LAUNCH_CHECK();
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
  }
  // SELL
  if (A->Mpad) {
    k_sell_count<<<g, BS, 0, s>>>(M, A->Mpad, A->C, A->perm, A->cs, A->scol, len.as<int32_t>());
    SPMV_LAUNCH_CHECK();
  }
  SPMV_TRY(scan_i32_to_i32(len.as<int32_t>(), ptr, M, s));
  if (A->Mpad) {
    k_sell_to_csr<T><<<g, BS, 0, s>>>(M, A->Mpad, A->C, A->perm, A->cs, A->scol, (const T*)A->sval, ptr, col, val);
    SPMV_LAUNCH_CHECK();
  }
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

spmv_status_t ell_sell_hyb_to_csr(spmv_mat_s* A, int32_t* ptr, int32_t* col, void* val, hipStream_t s) {
  if (A->dt == SPMV_F64) return to_csr_t<double>(A, ptr, col, (double*)val, s);
  return to_csr_t<float>(A, ptr, col, (float*)val, s);
}

}  // namespace spmv
