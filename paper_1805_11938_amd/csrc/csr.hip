// CSR (Sec. II-B, CSR paragraph): handle creation from CSR or raw COO,
// structural validation, and the CSR SpMV kernels.
//
// Main kernel ("row blocks"): rows are grouped so that block b owns the
// rows r with r + ptr[r] in [b*W, (b+1)*W) -- a split of the merged
// (rows + nonzeros) sequence into equal pieces, so a block sees at most W
// rows-plus-nonzeros except for one trailing long row.  A block streams the
// nonzeros of its rows with coalesced, non-temporal loads, forms the
// products val*x[col] in LDS (FP64), then reduces each row with a group of
// V lanes (V chosen from the block's mean row length) and wave shuffles.
// Every row is reduced by exactly one block: no atomics, no second pass,
// deterministic.  Blocks whose rows exceed the LDS capacity (a long row)
// reduce rows straight from global memory, a wave per row, or the whole
// block per row for rows of LONG or more nonzeros.
//
// Alternative kernel ("vector-V"): V lanes per row over a flat row grid,
// the rows-per-wavefront knob of the autotuner (64/V rows per wave).
#include <cstring>

#include "common.h"

namespace spmv {

constexpr int CSR_W = 2048;    // rows + nonzeros per row block
constexpr int CSR_CAP = 2560;  // nonzeros a block can stage in LDS
constexpr int CSR_IT = CSR_CAP / BS;
constexpr int CSR_LONG = 1024; // rows at least this long are reduced by a whole block
constexpr int WU_ROWS = 512;   // rows + nonzeros per wave unit (see k_csr_waves)
constexpr int LONG_ROW = 1024; // rows longer than this are cut into segments for several waves
constexpr int SEG = 512;       // nonzeros per long-row segment

static_assert(CSR_CAP % BS == 0, "CAP must be a multiple of the block size");

// ------------------------------------------------------------ validation
__global__ void k_csr_validate(int64_t M, int64_t N, int64_t nnz, const int32_t* ptr, const int32_t* col, int check_cols,
                               int* err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = ptr[i], b = ptr[i + 1];
    if (i == 0 && a != 0) atomicOr(err, 1);
    if (i == M - 1 && b != nnz) atomicOr(err, 2);
    if (a < 0 || b < a || b > nnz) {
      atomicOr(err, 4);
      continue;
    }
    if (!check_cols) continue;
    int32_t prev = -1;
    for (int64_t k = a; k < b; ++k) {
      const int32_t c = col[k];
      if (c < 0 || c >= N) {
        atomicOr(err, 8);
        break;
      }
      if (c <= prev) {
        atomicOr(err, 16);
        break;
      }
      prev = c;
    }
  }
}

static spmv_status_t validate_csr(spmv_mat_s* A, int check_cols, hipStream_t s) {
  if (A->M == 0) return A->nnz == 0 ? SPMV_OK : fail(SPMV_ERR_BAD_STRUCTURE, "M = 0 with nnz = %lld", (long long)A->nnz);
  DTmp e;
  SPMV_TRY(e.alloc(sizeof(int)));
  SPMV_HIP(hipMemsetAsync(e.p, 0, sizeof(int), s));
  int64_t g = cdiv(A->M, BS);
  if (g > 65536) g = 65536;
  k_csr_validate<<<(unsigned)g, BS, 0, s>>>(A->M, A->N, A->nnz, A->ptr, A->col, check_cols, e.as<int>());
  SPMV_LAUNCH_CHECK();
  int h = 0;
  SPMV_TRY(copy_to_host(&h, e.p, sizeof(int), s));
  if (h) return fail(SPMV_ERR_BAD_STRUCTURE, "malformed CSR (code %d: 1 ptr[0]!=0, 2 ptr[M]!=nnz, 4 ptr not monotone/in range, 8 col out of range, 16 col not strictly increasing)", h);
  return SPMV_OK;
}

// ------------------------------------------------------------ row blocks
__global__ void k_csr_blocks(const int32_t* ptr, int64_t M, int64_t nblk, int64_t width, int32_t* blk_row) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= nblk; b += (int64_t)gridDim.x * blockDim.x) {
    if (b == nblk) {
      blk_row[b] = (int32_t)M;
      continue;
    }
    const int64_t target = b * width;
    int64_t lo = 0, hi = M;  // first r in [0, M) with r + ptr[r] >= target, else M
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (mid + ptr[mid] >= target) hi = mid;
      else lo = mid + 1;
    }
    blk_row[b] = (int32_t)lo;
  }
}

static spmv_status_t build_partition(spmv_mat_s* A, int64_t width, int64_t* n, int32_t** rows, hipStream_t s) {
  *n = cdiv(A->M + A->nnz, width);
  if (*n < 1) *n = 1;
  SPMV_TRY(mat_alloc(A, (void**)rows, sizeof(int32_t) * (*n + 1)));
  int64_t g = cdiv(*n + 1, BS);
  if (g > 65536) g = 65536;
  k_csr_blocks<<<(unsigned)g, BS, 0, s>>>(A->ptr, A->M, *n, width, *rows);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

// Row partitions of a CSR handle: workgroup-sized blocks (batched launch)
// and wave-sized units (the default kernel).
__global__ void k_long_count(int64_t M, const int32_t* ptr, int32_t* nseg, int32_t* islong) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t len = ptr[r + 1] - ptr[r];
    nseg[r] = len > LONG_ROW ? (int32_t)((len + SEG - 1) / SEG) : 0;
    islong[r] = len > LONG_ROW;
  }
}

__global__ void k_long_fill(int64_t M, const int32_t* ptr, const int32_t* nseg, const int32_t* sbase,
                            const int32_t* lpos, int2* segs, int4* longs) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t n = nseg[r];
    if (!n) continue;
    for (int32_t j = 0; j < n; ++j) segs[sbase[r] + j] = make_int2((int)r, ptr[r] + j * SEG);
    longs[lpos[r]] = make_int4((int)r, sbase[r], n, 0);
  }
}

spmv_status_t csr_build_blocks(spmv_mat_s* A, hipStream_t s) {
  SPMV_TRY(build_partition(A, CSR_W, &A->nblk, &A->blk_row, s));
  SPMV_TRY(build_partition(A, WU_ROWS, &A->nunits, &A->unit_row, s));
  const int64_t M = A->M;
  A->nseg = A->nlong = 0;
  int32_t mx = 0;
  SPMV_TRY(device_max_i32(A->ptr, M, 1, &mx, s));  // the longest row (0 when M = 0)
  A->maxlen = mx;
  if (M == 0) return SPMV_OK;
  DTmp ns, il, sb, lp;
  SPMV_TRY(ns.alloc(sizeof(int32_t) * M));
  SPMV_TRY(il.alloc(sizeof(int32_t) * M));
  SPMV_TRY(sb.alloc(sizeof(int32_t) * (M + 1)));
  SPMV_TRY(lp.alloc(sizeof(int32_t) * (M + 1)));
  const unsigned g = (unsigned)std::min<int64_t>(cdiv(M, BS), 65536);
  k_long_count<<<g, BS, 0, s>>>(M, A->ptr, ns.as<int32_t>(), il.as<int32_t>());
  SPMV_LAUNCH_CHECK();
  SPMV_TRY(scan_i32_to_i32(ns.as<int32_t>(), sb.as<int32_t>(), M, s));
  SPMV_TRY(scan_i32_to_i32(il.as<int32_t>(), lp.as<int32_t>(), M, s));
  int32_t h[2] = {0, 0};
  SPMV_TRY(copy_to_host(&h[0], sb.as<int32_t>() + M, sizeof(int32_t), s));
  SPMV_TRY(copy_to_host(&h[1], lp.as<int32_t>() + M, sizeof(int32_t), s));
  A->nseg = h[0];
  A->nlong = h[1];
  if (A->nlong == 0) return SPMV_OK;
  SPMV_TRY(mat_alloc(A, (void**)&A->segs, sizeof(int2) * A->nseg));
  SPMV_TRY(mat_alloc(A, (void**)&A->longs, sizeof(int4) * A->nlong));
  SPMV_TRY(mat_alloc(A, (void**)&A->seg_part, sizeof(double) * A->nseg));
  k_long_fill<<<g, BS, 0, s>>>(M, A->ptr, ns.as<int32_t>(), sb.as<int32_t>(), lp.as<int32_t>(), A->segs, A->longs);
  SPMV_LAUNCH_CHECK();
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

// ------------------------------------------------------------ kernels
// Lanes per row for the LDS reduction: enough lanes that the block's rows
// are covered in one pass, but no more than the mean row length needs.
__device__ __forceinline__ int lanes_for(int64_t nz, int64_t rows) {
  int V = 1;
  while (V < 64 && V * 2 * rows <= BS) V *= 2;
  const int64_t avg = rows > 0 ? nz / rows : 0;
  while (V > 1 && V > avg) V >>= 1;
  return V;
}

constexpr int CSR_RCAP = 512;  // row pointers a block stages in LDS

// Rows [r0, r1) whose entries [k0, k1) fit the LDS staging (k1 - k0 <=
// CSR_CAP): all loads in flight, products in LDS, each row reduced by V lanes.
template <typename T, typename TY>
__device__ __forceinline__ void csr_rows_staged(int64_t r0, int64_t r1, int64_t k0, int64_t k1,
                                                const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                const T* __restrict__ val, const T* __restrict__ x,
                                                TY* __restrict__ y, double* prod, int32_t* sptr, int add) {
  const int t = threadIdx.x;
  const int64_t E = k1 - k0, nr = r1 - r0;
  const bool staged = nr <= CSR_RCAP;
  if (staged)
    for (int64_t i = t; i <= nr; i += BS) sptr[i] = ptr[r0 + i] - (int32_t)k0;
  if (E > 0) {  // clamped, branch-free loads and gathers keep every request in flight
    int32_t c[CSR_IT];
    T v[CSR_IT], xv[CSR_IT];
    const int32_t* cb = col + k0;  // block-uniform bases, 32-bit lane offsets
    const T* vb = val + k0;
#pragma unroll
    for (int j = 0; j < CSR_IT; ++j) {
      const uint32_t k = (uint32_t)(t + j * BS), kk = k < (uint32_t)E ? k : (uint32_t)E - 1;
      c[j] = ldnt32(cb, kk);
      v[j] = ldnt32(vb, kk);
    }
    issue_fence();
#pragma unroll
    for (int j = 0; j < CSR_IT; ++j) xv[j] = ld32(x, (uint32_t)c[j]);
    issue_fence();
#pragma unroll
    for (int j = 0; j < CSR_IT; ++j) {
      const int64_t k = t + j * BS;
      if (k < E) prod[k] = (double)v[j] * (double)xv[j];
    }
  }
  __syncthreads();
  const int V = lanes_for(E, nr);
  const int g = t / V, lane = t % V, ng = BS / V;
  for (int64_t r = g; r < nr; r += ng) {
    const int a = staged ? sptr[r] : ptr[r0 + r] - (int32_t)k0;
    const int e = staged ? sptr[r + 1] : ptr[r0 + r + 1] - (int32_t)k0;
    double s = 0.0;
    for (int k = a + lane; k < e; k += V) s += prod[k];
    s = group_sum_rt(s, V);
    if (lane == 0) put_y(y, r0 + r, s, add);
  }
  __syncthreads();  // prod / sptr may be reused by the caller's next block
}

// One row block (all threads of the workgroup call this with the same rows).
// TY is the type y is written in (T, or double for partial sums).  A block
// whose entries overflow the LDS staging ends in a long row (the split puts
// at most W rows-plus-nonzeros before it): the rows before that overflow go
// through the staged path, the rest are summed from global memory -- a wave
// per row below CSR_LONG, the whole block above.
template <typename T, typename TY = T>
__device__ __forceinline__ void csr_rows_block(int64_t r0, int64_t r1, int64_t k0, int64_t k1,
                                               const int32_t* __restrict__ ptr,
                                               const int32_t* __restrict__ col, const T* __restrict__ val,
                                               const T* __restrict__ x, TY* __restrict__ y, double* prod,
                                               int32_t* sptr, int add = 0) {
  if (r0 >= r1) return;
  if (k1 - k0 <= CSR_CAP) {
    csr_rows_staged<T, TY>(r0, r1, k0, k1, ptr, col, val, x, y, prod, sptr, add);
    return;
  }
  int64_t lo = r0 + 1, hi = r1;  // first r with ptr[r] - k0 > CSR_CAP (ptr[r1] qualifies)
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (ptr[mid] - k0 > CSR_CAP) hi = mid;
    else lo = mid + 1;
  }
  const int64_t rl = lo - 1;  // rows [r0, rl) fit the staging
  if (rl > r0) csr_rows_staged<T, TY>(r0, rl, k0, ptr[rl], ptr, col, val, x, y, prod, sptr, add);
  const int t = threadIdx.x;
  const int w = t / WAVE, lane = __lane_id();
  for (int64_t r = rl + w; r < r1; r += BS / WAVE) {
    const int64_t a = ptr[r], e = ptr[r + 1];
    if (e - a >= CSR_LONG) continue;
    double s = group_sum<64>(row_dot(col, val, x, a, e, lane, WAVE));
    if (lane == 0) put_y(y, r, s, add);
  }
  for (int64_t r = rl; r < r1; ++r) {
    const int64_t a = ptr[r], e = ptr[r + 1];
    if (e - a < CSR_LONG) continue;
    const double s = block_sum(row_dot(col, val, x, a, e, t, BS), prod);
    if (t == 0) put_y(y, r, s, add);
  }
  __syncthreads();
}

template <typename T, bool XCD>
__global__ __launch_bounds__(BS) void k_csr_rows(int64_t nblk, const int32_t* __restrict__ blk_row,
                                                 const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                 const T* __restrict__ val, const T* __restrict__ x, T* __restrict__ y,
                                                 int add) {
  __shared__ double prod[CSR_CAP];
  __shared__ int32_t sptr[CSR_RCAP + 1];
  const uint32_t b = XCD ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  if (b >= nblk) return;
  const int64_t r0 = blk_row[b], r1 = blk_row[b + 1];
  csr_rows_block<T>(r0, r1, ptr[r0], ptr[r1], ptr, col, val, x, y, prod, sptr, add);
}

// ------------------------------------------------------- column bands
// The columns are split into NBANDS equal bands and each band is stored as a
// CSR of all M rows.  Workgroup g works on band g mod 8 -- the XCD the
// hardware dispatches it to -- so each XCD's L2 caches only its eighth of x,
// which matters when x is larger than one L2 and the columns are scattered.
// Every row of every band is written (0 for a row with no entries there) to
// an FP64 partial-sum vector; k_csr_band_sum adds the bands in order.
constexpr int NBANDS = 8;

struct BandSet {
  const int32_t* ptr[NBANDS];
  const int32_t* col[NBANDS];
  const void* val[NBANDS];
  const int32_t* blk[NBANDS];
  int64_t nblk[NBANDS];
};

template <typename T>
__global__ __launch_bounds__(BS) void k_csr_bands(BandSet b, int64_t M, const T* __restrict__ x,
                                                  double* __restrict__ part) {
  __shared__ double prod[CSR_CAP];
  __shared__ int32_t sptr[CSR_RCAP + 1];
  const int band = blockIdx.x % NBANDS;
  const int64_t j = blockIdx.x / NBANDS;
  if (j >= b.nblk[band]) return;
  const int32_t* ptr = b.ptr[band];
  const int64_t r0 = b.blk[band][j], r1 = b.blk[band][j + 1];
  csr_rows_block<T, double>(r0, r1, ptr[r0], ptr[r1], ptr, b.col[band], (const T*)b.val[band], x,
                            part + band * M, prod, sptr);
}

template <typename T>
__global__ void k_csr_band_sum(int64_t M, const double* __restrict__ part, T* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < NBANDS; ++b) s += part[b * M + i];
    y[i] = (T)s;
  }
}

// entries of each row in each of nb bands (columns are sorted: binary searches)
__global__ void k_band_count(int64_t M, const int32_t* ptr, const int32_t* col, int64_t bw, int nb, int32_t* cnt) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = ptr[r], e = ptr[r + 1];
    int64_t prev = a;
    for (int b = 0; b < nb; ++b) {
      int64_t lo = prev, hi = e;  // first entry with col >= (b+1)*bw
      const int64_t lim = (b + 1) * bw;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < lim) lo = mid + 1;
        else hi = mid;
      }
      cnt[b * M + r] = (int32_t)(lo - prev);
      prev = lo;
    }
  }
}

// one wave per row: the row's entries of each band go to that band's place,
// the lanes copying consecutive entries (a row of 10^5 entries is not left
// to one thread)
template <typename T>
__global__ void k_band_scatter(int64_t M, int nb, const int32_t* ptr, const int32_t* col, const T* val,
                               const int32_t* cnt, const int32_t* bptr, const int64_t* boff, int32_t* bcol, T* bval) {
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
  const int lane = __lane_id();
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; r < M; r += nw) {
    int64_t k = ptr[r];
    for (int b = 0; b < nb; ++b) {
      const int64_t dst = boff[b] + bptr[b * (M + 1) + r];
      const int32_t n = cnt[b * M + r];
      for (int32_t q = lane; q < n; q += WAVE) {
        bcol[dst + q] = col[k + q];
        bval[dst + q] = val[k + q];
      }
      k += n;
    }
  }
}

spmv_status_t csr_split_bands(const spmv_mat_s* src, int nb, int64_t bw, int32_t* bptr, int32_t* bcol, void* bval,
                              std::vector<int64_t>& off, hipStream_t s) {
  const int64_t M = src->M;
  DTmp cnt, doff;
  SPMV_TRY(cnt.alloc(sizeof(int32_t) * nb * std::max<int64_t>(M, 1)));
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(M, BS), 65536));
  if (M) {
    k_band_count<<<g, BS, 0, s>>>(M, src->ptr, src->col, bw, nb, cnt.as<int32_t>());
    SPMV_LAUNCH_CHECK();
  }
  off.assign(nb + 1, 0);
  for (int b = 0; b < nb; ++b) {
    SPMV_TRY(scan_i32_to_i32(cnt.as<int32_t>() + b * M, bptr + b * (M + 1), M, s));
    int32_t n = 0;
    SPMV_TRY(copy_to_host(&n, bptr + b * (M + 1) + M, sizeof(int32_t), s));
    off[b + 1] = off[b] + n;
  }
  SPMV_TRY(doff.alloc(sizeof(int64_t) * (nb + 1)));
  SPMV_HIP(hipMemcpyAsync(doff.p, off.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, s));
  if (M) {
    const unsigned gw = (unsigned)std::min<int64_t>(cdiv(M, BS / WAVE), 1 << 20);
    if (src->dt == SPMV_F64)
      k_band_scatter<double><<<gw, BS, 0, s>>>(M, nb, src->ptr, src->col, (const double*)src->val, cnt.as<int32_t>(),
                                               bptr, doff.as<int64_t>(), bcol, (double*)bval);
    else
      k_band_scatter<float><<<gw, BS, 0, s>>>(M, nb, src->ptr, src->col, (const float*)src->val, cnt.as<int32_t>(),
                                              bptr, doff.as<int64_t>(), bcol, (float*)bval);
    SPMV_LAUNCH_CHECK();
  }
  SPMV_HIP(hipStreamSynchronize(s));  // cnt and doff are freed on return
  return SPMV_OK;
}

spmv_status_t csr_build_bands(spmv_mat_s* A, hipStream_t s) {
  const int64_t M = A->M;
  A->nbands = NBANDS;
  A->band_w = std::max<int64_t>(1, cdiv(A->N, NBANDS));
  SPMV_TRY(mat_alloc(A, (void**)&A->bptr, sizeof(int32_t) * NBANDS * (M + 1)));
  SPMV_TRY(mat_alloc(A, (void**)&A->bcol, sizeof(int32_t) * A->nnz));
  SPMV_TRY(mat_alloc(A, &A->bval, (size_t)A->sv * A->nnz));
  SPMV_TRY(csr_split_bands(A, NBANDS, A->band_w, A->bptr, A->bcol, A->bval, A->band_off, s));
  // row blocks of each band (the same merged rows + nonzeros split)
  A->band_nblk.assign(NBANDS, 0);
  A->band_blk0.assign(NBANDS + 1, 0);
  for (int b = 0; b < NBANDS; ++b) {
    A->band_nblk[b] = std::max<int64_t>(1, cdiv(M + (A->band_off[b + 1] - A->band_off[b]), CSR_W));
    A->band_blk0[b + 1] = A->band_blk0[b] + A->band_nblk[b] + 1;
  }
  SPMV_TRY(mat_alloc(A, (void**)&A->bblk, sizeof(int32_t) * A->band_blk0[NBANDS]));
  for (int b = 0; b < NBANDS; ++b) {
    const int64_t n = A->band_nblk[b];
    k_csr_blocks<<<(unsigned)std::min<int64_t>(cdiv(n + 1, BS), 65536), BS, 0, s>>>(A->bptr + b * (M + 1), M, n,
                                                                                   CSR_W, A->bblk + A->band_blk0[b]);
    SPMV_LAUNCH_CHECK();
  }
  SPMV_TRY(mat_alloc(A, (void**)&A->bpart, sizeof(double) * NBANDS * std::max<int64_t>(M, 1)));
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

template <typename T>
static spmv_status_t run_csr_bands(spmv_mat_s* A, const T* x, T* y, hipStream_t s) {
  BandSet b;
  int64_t maxb = 0;
  for (int i = 0; i < NBANDS; ++i) {
    b.ptr[i] = A->bptr + i * (A->M + 1);
    b.col[i] = A->bcol + A->band_off[i];
    b.val[i] = (const char*)A->bval + (size_t)A->sv * A->band_off[i];
    b.blk[i] = A->bblk + A->band_blk0[i];
    b.nblk[i] = A->band_nblk[i];
    maxb = std::max(maxb, A->band_nblk[i]);
  }
  launch(k_csr_bands<T>, (unsigned)(maxb * NBANDS), BS, s, b, A->M, x, A->bpart);
  SPMV_LAUNCH_CHECK();
  launch(k_csr_band_sum<T>, (unsigned)std::min<int64_t>(cdiv(A->M, BS), 65536), BS, s, A->M,
         (const double*)A->bpart, y);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

// ------------------------------------------------------------ wave units
// Default CSR kernel: the same merged (rows + nonzeros) split, in units of
// WU for one wave each.  Waves never wait on each other (no workgroup
// barrier), so the load, gather and reduce phases of the 4 x 8 resident
// waves per SIMD overlap freely.  Each wave stages its unit's row pointers
// and products in its own LDS slice; rows longer than the slice are summed
// straight from global memory by the whole wave.
constexpr int WU = WU_ROWS;         // rows + nonzeros per wave unit
constexpr int WCAP = 512;           // products a wave stages in LDS
constexpr int WIT = WCAP / WAVE;
constexpr int WRCAP = WU;           // row pointers a wave stages in LDS (a unit never has more rows)

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ int wave_lanes_for(int64_t nz, int64_t rows) {
  int V = 1;
  while (V < 64 && V * 2 * rows <= WAVE) V *= 2;
  const int64_t avg = rows > 0 ? nz / rows : 0;
  while (V > 1 && V > avg) V >>= 1;
  return V;
}

template <typename T>
__device__ __forceinline__ void csr_rows_wave(int64_t r0, int64_t r1, const int32_t* __restrict__ ptr,
                                              const int32_t* __restrict__ col, const T* __restrict__ val,
                                              const T* __restrict__ x, T* __restrict__ y, double* prod,
                                              int32_t* sptr) {
  if (r0 >= r1) return;
  const int lane = __lane_id();
  const int64_t k0 = __builtin_amdgcn_readfirstlane(ptr[r0]), k1 = __builtin_amdgcn_readfirstlane(ptr[r1]);
  const int64_t E = k1 - k0, nr = r1 - r0;
  if (E <= WCAP && nr <= WRCAP) {
    for (int64_t i = lane; i <= nr; i += WAVE) sptr[i] = ptr[r0 + i] - (int32_t)k0;
    if (E > 0) {
      int32_t c[WIT];
      T v[WIT], xv[WIT];
      const int32_t* cb = col + k0;  // wave-uniform bases, 32-bit lane offsets
      const T* vb = val + k0;
      const uint32_t Em1 = (uint32_t)E - 1;
#pragma unroll
      for (int j = 0; j < WIT; ++j) {
        const uint32_t k = (uint32_t)(lane + j * WAVE), kk = k < (uint32_t)E ? k : Em1;
        c[j] = ldnt32(cb, kk);
        v[j] = ldnt32(vb, kk);
      }
      issue_fence();
#pragma unroll
      for (int j = 0; j < WIT; ++j) xv[j] = ld32(x, (uint32_t)c[j]);
      issue_fence();
#pragma unroll
      for (int j = 0; j < WIT; ++j) {
        const int64_t k = lane + j * WAVE;
        if (k < E) prod[k] = (double)v[j] * (double)xv[j];
      }
    }
    wave_lds_sync();
    const int V = wave_lanes_for(E, nr);
    const int g = lane / V, gl = lane % V, ng = WAVE / V;
    for (int64_t r = g; r < nr; r += ng) {
      const int a = sptr[r], e = sptr[r + 1];
      double s0 = 0.0, s1 = 0.0;
      int k = a + gl;
      for (; k + V < e; k += 2 * V) {
        s0 += prod[k];
        s1 += prod[k + V];
      }
      if (k < e) s0 += prod[k];
      const double sum = group_sum_rt(s0 + s1, V);
      if (gl == 0) y[r0 + r] = (T)sum;
    }
    wave_lds_sync();  // the slice is reused by the wave's next unit
    return;
  }
  for (int64_t r = r0; r < r1; ++r) {
    const int64_t a = ptr[r], e = ptr[r + 1];
    if (e - a > LONG_ROW) continue;  // summed by the segment waves
    const double sum = group_sum<64>(row_dot(col, val, x, a, e, lane, WAVE));
    if (lane == 0) y[r] = (T)sum;
  }
}

// Waves u < nunits take wave units; waves nunits + j take segment j of a
// long row (SEG nonzeros, partial sum to part[j]).
template <typename T>
__global__ __launch_bounds__(BS) void k_csr_waves(int64_t nunits, const int32_t* __restrict__ unit_row, int64_t nseg,
                                                  const int2* __restrict__ segs, double* __restrict__ part,
                                                  const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                  const T* __restrict__ val, const T* __restrict__ x,
                                                  T* __restrict__ y) {
  __shared__ double prod[BS / WAVE][WCAP];
  __shared__ int32_t sptr[BS / WAVE][WRCAP + 1];
  // the wave index is uniform: keep it (and everything derived) in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int64_t nw = (int64_t)gridDim.x * (BS / WAVE);
  for (int64_t u = (int64_t)xcd_block(blockIdx.x, gridDim.x) * (BS / WAVE) + w; u < nunits + nseg; u += nw) {
    if (u < nunits) {
      const int32_t r0 = __builtin_amdgcn_readfirstlane(unit_row[u]);
      const int32_t r1 = __builtin_amdgcn_readfirstlane(unit_row[u + 1]);
      csr_rows_wave<T>(r0, r1, ptr, col, val, x, y, prod[w], sptr[w]);
    } else {
      const int2 sg = segs[u - nunits];  // (row, first nonzero)
      const int64_t e = ptr[sg.x + 1];
      const int64_t kb = sg.y, ke = kb + SEG < e ? kb + SEG : e;
      const double sum = group_sum<64>(row_dot(col, val, x, kb, ke, __lane_id(), WAVE));
      if (__lane_id() == 0) part[u - nunits] = sum;
    }
  }
}

// one wave per long row: its segment partials summed in order
template <typename T>
__global__ __launch_bounds__(BS) void k_csr_long_fix(int64_t nlong, const int4* __restrict__ longs,
                                                     const double* __restrict__ part, T* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * (BS / WAVE) + threadIdx.x / WAVE;
  if (i >= nlong) return;
  const int4 L = longs[i];  // row, first segment, segment count
  double s = 0.0;
  for (int j = __lane_id(); j < L.z; j += WAVE) s += part[L.y + j];
  s = group_sum<64>(s);
  if (__lane_id() == 0) y[L.x] = (T)s;
}

template <typename T, int V>
__global__ __launch_bounds__(BS) void k_csr_vector(int64_t M, const int32_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ col, const T* __restrict__ val,
                                                   const T* __restrict__ x, T* __restrict__ y, int add) {
  const int64_t r = (int64_t)blockIdx.x * (BS / V) + threadIdx.x / V;
  const int lane = threadIdx.x % V;
  if (r >= M) return;  // uniform across the V-lane group
  const double s = group_sum<V>(row_dot(col, val, x, ptr[r], ptr[r + 1], lane, V));
  if (lane == 0) put_y(y, r, s, add);
}

// ------------------------------------------------------------ wave tiles
// SPMV_FLAG_CSR_TILES: a wave takes TILE_E consecutive nonzeros (the same
// reduction as HYB's COO pass, wave_tile_reduce), with no barrier and every
// load in flight.  CSR stores no row per entry, so the wave marks where the
// rows starting in its tile begin (a per-wave LDS table: row id at its first
// entry's place, -1 elsewhere) and a running maximum over the places gives
// every entry its row (rows increase along the tile).  Empty rows starting
// in the tile are written as 0.  Per tile, conversion stores tstart (first
// row whose first entry is at or after the tile's first entry; M past the
// end) and tcont (row holding the tile's first entry).
__global__ void k_csr_tile_rows(int64_t M, int64_t nnz, int64_t ntiles, const int32_t* __restrict__ ptr,
                                int32_t* __restrict__ tstart, int32_t* __restrict__ tcont) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= ntiles; t += (int64_t)gridDim.x * blockDim.x) {
    if (t == ntiles) {
      tstart[t] = (int32_t)M;
      tcont[t] = (int32_t)M;
      continue;
    }
    const int64_t e0 = t * TILE_E;
    int64_t lo = 0, hi = M;  // first r with ptr[r] >= e0
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ptr[mid] >= e0) hi = mid;
      else lo = mid + 1;
    }
    tstart[t] = (int32_t)lo;
    lo = 0, hi = M;  // first r with ptr[r] > e0; the row holding entry e0 is the one before
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ptr[mid] > e0) hi = mid;
      else lo = mid + 1;
    }
    tcont[t] = (int32_t)(lo - 1);
  }
}

// One tile t of a CSR (entries [t*TILE_E, ...) of col / val) by one wave:
// rows marked in the wave's LDS table rw, then the segmented reduction.
template <typename T, bool ADD = false>
__device__ __forceinline__ void csr_tile(int64_t t, int64_t nnz, int64_t ntiles, const int32_t* __restrict__ ptr,
                                         const int32_t* __restrict__ col, const T* __restrict__ val,
                                         const int32_t* __restrict__ tstart, const int32_t* __restrict__ tcont,
                                         const T* __restrict__ x, T* __restrict__ y, double* __restrict__ head_part,
                                         double* __restrict__ tail_part, int32_t* __restrict__ tail_row,
                                         int32_t* __restrict__ tinfo, int32_t* rw) {
  const int l = __lane_id();
  const int64_t e0 = t * TILE_E;
  const int nv = (int)(nnz - e0 < TILE_E ? nnz - e0 : TILE_E);  // entries in the tile, >= 1
#pragma unroll
  for (int s = 0; s < TILE_S; ++s) rw[s * WAVE + l] = -1;
  const int32_t r0 = tstart[t], r1 = tstart[t + 1], rc = tcont[t];
  const int32_t rprev = ptr[rc] < e0 ? rc : -1;  // the row holding the first entry began earlier
  const int32_t rn = tcont[t + 1];
  const int32_t rnext = t + 1 < ntiles && ptr[rn] < e0 + TILE_E ? rn : -2;  // the last row continues after
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  for (int64_t r = r0 + l; r < r1; r += WAVE) {  // rows starting in the tile
    const int32_t a = ptr[r], b = ptr[r + 1];
    if (b > a) rw[a - e0] = (int32_t)r;
    else if (!ADD) y[r] = (T)0;  // an empty row (adding nothing onto y when ADD)
  }
  int32_t cc[TILE_S], rr[TILE_S];
  T vv[TILE_S];
#pragma unroll
  for (int s = 0; s < TILE_S; ++s) {
    const int k = s * WAVE + l;
    const uint32_t kk = (uint32_t)(k < nv ? k : nv - 1);
    cc[s] = ldnt32(col + e0, kk);
    vv[s] = ldnt32(val + e0, kk);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  int32_t run = rc;  // row of the entries before the first mark
#pragma unroll
  for (int s = 0; s < TILE_S; ++s) {
    int32_t v = max_scan64(rw[s * WAVE + l]);  // inclusive running maximum over the slice
    v = run > v ? run : v;
    run = __builtin_amdgcn_readlane(v, WAVE - 1);
    rr[s] = s * WAVE + l < nv ? v : TILE_NONE;
  }
  issue_fence();
  wave_tile_reduce<T, ADD>(t, nv, rr, cc, vv, rprev, rnext, x, y, head_part, tail_part, tail_row, tinfo);
}

template <typename T, bool ADD>
__global__ __launch_bounds__(BS) void k_csr_tiles(int64_t nnz, int64_t ntiles, const int32_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col, const T* __restrict__ val,
                                                  const int32_t* __restrict__ tstart, const int32_t* __restrict__ tcont,
                                                  const T* __restrict__ x, T* __restrict__ y,
                                                  double* __restrict__ head_part, double* __restrict__ tail_part,
                                                  int32_t* __restrict__ tail_row, int32_t* __restrict__ tinfo) {
  __shared__ int32_t rid[BS / WAVE][TILE_E];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int64_t t = (int64_t)blockIdx.x * (BS / WAVE) + w;
  if (t >= ntiles) return;
  csr_tile<T, ADD>(t, nnz, ntiles, ptr, col, val, tstart, tcont, x, y, head_part, tail_part, tail_row, tinfo, rid[w]);
}

spmv_status_t csr_build_tiles(spmv_mat_s* A, hipStream_t s) {
  A->ntiles_csr = cdiv(A->nnz, TILE_E);
  if (A->ntiles_csr == 0) return SPMV_OK;  // no entries: the row-block kernel writes the zeros
  const int64_t nt = A->ntiles_csr;
  SPMV_TRY(mat_alloc(A, (void**)&A->ct_start, sizeof(int32_t) * (nt + 1)));
  SPMV_TRY(mat_alloc(A, (void**)&A->ct_cont, sizeof(int32_t) * (nt + 1)));
  SPMV_TRY(mat_alloc(A, (void**)&A->ct_head, sizeof(double) * nt));
  SPMV_TRY(mat_alloc(A, (void**)&A->ct_tail, sizeof(double) * nt));
  SPMV_TRY(mat_alloc(A, (void**)&A->ct_trow, sizeof(int32_t) * nt));
  SPMV_TRY(mat_alloc(A, (void**)&A->ct_info, sizeof(int32_t) * nt));
  k_csr_tile_rows<<<(unsigned)std::min<int64_t>(cdiv(nt + 1, BS), 65536), BS, 0, s>>>(A->M, A->nnz, nt, A->ptr,
                                                                                     A->ct_start, A->ct_cont);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

template <typename T>
static spmv_status_t run_csr_t(spmv_mat_s* A, const T* x, T* y, hipStream_t s) {
  if (A->M == 0) return SPMV_OK;
  const int V = A->params.csr_lanes_per_row;
  const int32_t* ptr = A->ptr;
  const T* val = (const T*)A->val;
  if (V == 0 && A->nbands > 0) return run_csr_bands<T>(A, x, y, s);
  if (V == 0 && A->ntiles_csr > 0) {
    const int64_t nt = A->ntiles_csr;
    const unsigned g = (unsigned)cdiv(nt, BS / WAVE), gf = (unsigned)std::min<int64_t>(cdiv(nt, BS), 4096);
    if (A->acc)
      launch(k_csr_tiles<T, true>, g, BS, s, A->nnz, nt, ptr, A->col, val, A->ct_start, A->ct_cont, x, y, A->ct_head,
             A->ct_tail, A->ct_trow, A->ct_info);
    else
      launch(k_csr_tiles<T, false>, g, BS, s, A->nnz, nt, ptr, A->col, val, A->ct_start, A->ct_cont, x, y, A->ct_head,
             A->ct_tail, A->ct_trow, A->ct_info);
    SPMV_LAUNCH_CHECK();
    if (nt > 1) {
      if (A->acc)
        launch(k_tile_fix<T, true>, gf, BS, s, nt, (const double*)A->ct_head, (const double*)A->ct_tail,
               (const int32_t*)A->ct_trow, (const int32_t*)A->ct_info, y);
      else
        launch(k_tile_fix<T, false>, gf, BS, s, nt, (const double*)A->ct_head, (const double*)A->ct_tail,
               (const int32_t*)A->ct_trow, (const int32_t*)A->ct_info, y);
    }
    SPMV_LAUNCH_CHECK();
    return SPMV_OK;
  }
  if (V == 0) {
    if (!(A->params.flags & SPMV_FLAG_CSR_WAVES)) {
      if (A->params.flags & SPMV_FLAG_LINEAR)
        launch(k_csr_rows<T, false>, (unsigned)A->nblk, BS, s, A->nblk, A->blk_row, ptr, A->col, val, x, y, A->acc);
      else
        launch(k_csr_rows<T, true>, (unsigned)A->nblk, BS, s, A->nblk, A->blk_row, ptr, A->col, val, x, y, A->acc);
    } else
    {
      const unsigned g = (unsigned)std::min<int64_t>(cdiv(A->nunits + A->nseg, BS / WAVE), resident_blocks(8));
      launch(k_csr_waves<T>, g, BS, s, 
          A->nunits, A->unit_row, A->nseg, A->segs, A->seg_part, ptr, A->col, val, x, y);
      if (A->nlong > 0) {
        SPMV_LAUNCH_CHECK();
        launch(k_csr_long_fix<T>, (unsigned)cdiv(A->nlong, BS / WAVE), BS, s, A->nlong, A->longs, A->seg_part, y);
      }
    }
  } else {
    const unsigned g = (unsigned)cdiv(A->M, BS / V);
    switch (V) {
      case 1: launch(k_csr_vector<T, 1>, g, BS, s, A->M, ptr, A->col, val, x, y, A->acc); break;
      case 2: launch(k_csr_vector<T, 2>, g, BS, s, A->M, ptr, A->col, val, x, y, A->acc); break;
      case 4: launch(k_csr_vector<T, 4>, g, BS, s, A->M, ptr, A->col, val, x, y, A->acc); break;
      case 8: launch(k_csr_vector<T, 8>, g, BS, s, A->M, ptr, A->col, val, x, y, A->acc); break;
      case 16: launch(k_csr_vector<T, 16>, g, BS, s, A->M, ptr, A->col, val, x, y, A->acc); break;
      case 32: launch(k_csr_vector<T, 32>, g, BS, s, A->M, ptr, A->col, val, x, y, A->acc); break;
      case 64: launch(k_csr_vector<T, 64>, g, BS, s, A->M, ptr, A->col, val, x, y, A->acc); break;
      default: return fail(SPMV_ERR_UNSUPPORTED, "csr_lanes_per_row must be 0 or a power of two <= 64 (got %d)", V);
    }
  }
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

spmv_status_t run_csr(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  if (A->dt == SPMV_F64) return run_csr_t<double>(A, (const double*)x, (double*)y, s);
  return run_csr_t<float>(A, (const float*)x, (float*)y, s);
}

// ----------------------------------------------------------------- SpMM
// Y = A X for k right-hand sides (row-major, k <= 64).  A workgroup takes a
// block of rows; the block's col/val are staged in LDS once and reused by
// all k columns.  A lane owns VEC consecutive columns of one row: the
// k/VEC lanes of a row read its k values of X per nonzero as k/VEC loads of
// VEC values (16 bytes when VEC > 1) and write k consecutive values of Y.
// VEC > 1 needs k, ldx and ldy multiples of VEC and 16-byte aligned X and
// Y; otherwise VEC = 1.
//
// Blocks: when every row is short enough (rb rows of the longest row, plus
// the 3 entries staging may start below a block's first one, fit the LDS
// staging), blocks of rb = max(G, 64) rows, G = BS / (k/VEC) rows in
// flight per workgroup, so every pass over the rows keeps all lanes busy;
// otherwise the row blocks of the SpMV kernel (rows + nonzeros <= CSR_W).
constexpr int SPMM_CAP = 2048;  // entries a block stages in LDS
// Nonzeros of a row in flight per lane group: 9 (three steps for a 27-point
// stencil row), but 6 for FP32 in 16-byte lanes, where 9 takes the kernel
// from 74 to 112 VGPRs and a third of its waves.
template <typename T, int VEC>
constexpr int spmm_nb() {
  return sizeof(T) == 4 && VEC == 4 ? 6 : 9;
}

template <typename T, int VEC>
struct alignas(sizeof(T) * VEC) VecN {
  T v[VEC];
};

// Y is written once and not read again by the kernel: streaming stores keep
// it from displacing gathered rows of X in the L2.
template <typename T, int VEC>
__device__ __forceinline__ void spmm_store(T* p, const VecN<T, VEC>& o) {
  if constexpr (VEC * sizeof(T) == 16) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    f4 w;
    __builtin_memcpy(&w, &o, 16);
    __builtin_nontemporal_store(w, (f4*)p);
  } else {
    static_assert(VEC == 1, "16-byte lanes or single values");
    __builtin_nontemporal_store(o.v[0], p);
  }
}

// Entries [s0, s0 + E) of col and val (s0 a multiple of 4, E <= SPMM_CAP)
// into LDS with 16-byte loads, all in flight before the LDS stores; the
// vector that would reach past the last entry of the matrix is loaded entry
// by entry.  col and val are 16-byte aligned (device allocations).
template <typename T>
__device__ __forceinline__ void spmm_stage(const int32_t* __restrict__ col, const T* __restrict__ val, int64_t s0,
                                           int64_t E, int64_t nnz, int32_t* scol, T* sval, int t) {
  typedef int i4 __attribute__((ext_vector_type(4)));
  constexpr int VPV = 16 / sizeof(T);          // values per 16-byte vector
  constexpr int NC = SPMM_CAP / 4 / BS;        // column vectors per thread
  constexpr int NV = SPMM_CAP / VPV / BS;      // value vectors per thread
  i4 cv[NC], vv[NV];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int64_t e0 = 4 * (int64_t)(t + j * BS);
    if (e0 < E) {
      if (s0 + e0 + 4 <= nnz) {
        cv[j] = __builtin_nontemporal_load((const i4*)(col + s0 + e0));
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) cv[j][i] = col[s0 + e0 + i < nnz ? s0 + e0 + i : nnz - 1];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int64_t e0 = (int64_t)VPV * (t + j * BS);
    if (e0 < E) {
      if (s0 + e0 + VPV <= nnz) {
        vv[j] = __builtin_nontemporal_load((const i4*)(val + s0 + e0));
      } else {
        T w[VPV];
#pragma unroll
        for (int i = 0; i < VPV; ++i) w[i] = val[s0 + e0 + i < nnz ? s0 + e0 + i : nnz - 1];
        __builtin_memcpy(&vv[j], w, 16);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int e0 = 4 * (t + j * BS);
    if (e0 < E) *(i4*)(scol + e0) = cv[j];
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int e0 = VPV * (t + j * BS);
    if (e0 < E) *(i4*)(sval + e0) = vv[j];
  }
}

template <typename T, int VEC>
__global__ __launch_bounds__(BS) void k_csr_spmm(int64_t nblk, const int32_t* __restrict__ blk_row, int rb,
                                                 int64_t M, const int32_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ col, const T* __restrict__ val,
                                                 const T* __restrict__ X, int64_t ldx, T* __restrict__ Y,
                                                 int64_t ldy, int k, int64_t nnz) {
  typedef VecN<T, VEC> V;
  constexpr int NB = spmm_nb<T, VEC>();
  // staged entries; the long-row path's partial sums reuse the same bytes
  static_assert(SPMM_CAP * (4 + sizeof(T)) >= BS * VEC * sizeof(double), "LDS reuse");
  __shared__ __align__(16) char lds[SPMM_CAP * (4 + sizeof(T))];
  __shared__ int32_t sptr[BS + 1];  // row pointers of a block of at most BS rows (fixed-size blocks)
  int32_t* scol = (int32_t*)lds;
  T* sval = (T*)(lds + SPMM_CAP * 4);
  double* red = (double*)lds;
  const int t = threadIdx.x;
  const int kv = k / VEC;  // lanes per row
  const int G = BS / kv;
  const int g = t / kv, c = (t % kv) * VEC;
  // one workgroup per row block, each XCD a contiguous range of blocks
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= nblk) return;
  const int64_t r0 = rb ? b * rb : blk_row[b];
  const int64_t r1 = rb ? (r0 + rb < M ? r0 + rb : M) : blk_row[b + 1];
  if (r0 >= r1) return;
  // the block's entries are staged from the 4-entry boundary at or below
  // its first one, so every staging load moves 16 bytes
  const int64_t k1 = ptr[r1], s0 = ptr[r0] & ~(int64_t)3, E = k1 - s0;
  if (E <= SPMM_CAP) {
    // fixed-size blocks (rb <= BS rows) read their row pointers from LDS
    if (rb)
      for (int i = t; i <= r1 - r0; i += BS) sptr[i] = ptr[r0 + i] - (int32_t)s0;
    if (k1 > s0) spmm_stage<T>(col, val, s0, E, nnz, scol, sval, t);
    __syncthreads();
    if (g < G)
      for (int64_t r = r0 + g; r < r1; r += G) {
        const int a = rb ? sptr[r - r0] : ptr[r] - (int32_t)s0;
        const int e = rb ? sptr[r - r0 + 1] : ptr[r + 1] - (int32_t)s0;
        double s2[2][VEC];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int v = 0; v < VEC; ++v) s2[i][v] = 0.0;
        // NB nonzeros at a time, all their gathers of X rows in flight
        int q = a;
        for (; q + NB <= e; q += NB) {
          T vq[NB];
          V xq[NB];
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            vq[u] = sval[q + u];
            xq[u] = *(const V*)(X + (int64_t)scol[q + u] * ldx + c);
          }
#pragma unroll
          for (int u = 0; u < NB; ++u)
#pragma unroll
            for (int v = 0; v < VEC; ++v) s2[u & 1][v] += (double)vq[u] * (double)xq[u].v[v];
        }
        // the last n < NB nonzeros: a gather no lane of the wave needs
        // is not issued (every vector-memory instruction costs address and
        // data cycles whatever it moves)
        if (q < e) {
          const int n = e - q;
          T vq[NB - 1];
          V xq[NB - 1];
#pragma unroll
          for (int u = 0; u < NB - 1; ++u) {
            vq[u] = (T)0;
#pragma unroll
            for (int v = 0; v < VEC; ++v) xq[u].v[v] = (T)0;
            if (u < n) {
              vq[u] = sval[q + u];
              xq[u] = *(const V*)(X + (int64_t)scol[q + u] * ldx + c);
            }
          }
#pragma unroll
          for (int u = 0; u < NB - 1; ++u)
#pragma unroll
            for (int v = 0; v < VEC; ++v) s2[u & 1][v] += (double)vq[u] * (double)xq[u].v[v];
        }
        V out;
#pragma unroll
        for (int v = 0; v < VEC; ++v) out.v[v] = (T)(s2[0][v] + s2[1][v]);
        spmm_store<T, VEC>(Y + r * ldy + c, out);
      }
  } else {
    // rows one at a time: G groups stride over the row's nonzeros, then an
    // ordered sum of the groups' partials in LDS
    for (int64_t r = r0; r < r1; ++r) {
      const int64_t a = ptr[r], e = ptr[r + 1];
      double sv[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) sv[v] = 0.0;
      if (g < G)
        for (int64_t q = a + g; q < e; q += G) {
          const double w = (double)ldnt(val + q);
          const V xv = *(const V*)(X + (int64_t)ldnt(col + q) * ldx + c);
#pragma unroll
          for (int v = 0; v < VEC; ++v) sv[v] += w * (double)xv.v[v];
        }
#pragma unroll
      for (int v = 0; v < VEC; ++v) red[t * VEC + v] = sv[v];
      __syncthreads();
      if (g == 0) {
        V out;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          double tot = 0.0;
          for (int gg = 0; gg < G; ++gg) tot += red[(gg * kv + t % kv) * VEC + v];
          out.v[v] = (T)tot;
        }
        spmm_store<T, VEC>(Y + r * ldy + c, out);
      }
      __syncthreads();
    }
  }
}

template <typename T, int VEC>
static void launch_spmm(spmv_mat_s* A, const void* X, int64_t ldx, void* Y, int64_t ldy, int k, hipStream_t s) {
  const int64_t G = BS / (k / VEC);
  const int64_t rb = std::max<int64_t>(G, 64);  // at most BS: the kernel's LDS row pointers
  // (+3: staging starts at the 4-entry boundary below a block's first entry)
  if (A->maxlen >= 0 && rb * std::max<int64_t>(A->maxlen, 1) + 3 <= SPMM_CAP) {
    const int64_t nb = cdiv(A->M, rb);  // blocks of rb rows
    launch(k_csr_spmm<T, VEC>, (unsigned)nb, BS, s, nb, (const int32_t*)nullptr, (int)rb, A->M, A->ptr, A->col,
           (const T*)A->val, (const T*)X, ldx, (T*)Y, ldy, k, A->nnz);
  } else {  // the SpMV kernel's row blocks
    launch(k_csr_spmm<T, VEC>, (unsigned)A->nblk, BS, s, A->nblk, (const int32_t*)A->blk_row, 0, A->M, A->ptr,
           A->col, (const T*)A->val, (const T*)X, ldx, (T*)Y, ldy, k, A->nnz);
  }
}

spmv_status_t run_spmm(spmv_mat_s* A, const void* X, int64_t ldx, void* Y, int64_t ldy, int k, hipStream_t s) {
  if (A->fmt != SPMV_FMT_CSR || !A->sub.empty()) return fail(SPMV_ERR_UNSUPPORTED, "spmm runs on CSR handles without column bands");
  if (k < 1 || k > 64 || ldx < k || ldy < k) return fail(SPMV_ERR_INVALID_ARG, "spmm needs 1 <= k <= 64, ld >= k");
  if (A->M == 0) return SPMV_OK;
  if (((uintptr_t)A->col & 15) || ((uintptr_t)A->val & 15))
    return fail(SPMV_ERR_UNSUPPORTED, "spmm stages col and val with 16-byte loads: arrays must be 16-byte aligned");
  // 16-byte lanes (2 FP64 or 4 FP32 columns) where k, the leading
  // dimensions and the alignment of X and Y allow, else one value per lane.
  // (32-byte lanes, two loads each, measured slower on the stencil.)
  const int vec = 16 / A->sv;
  const bool wide = k % vec == 0 && ldx % vec == 0 && ldy % vec == 0 && ((uintptr_t)X & 15) == 0 &&
                    ((uintptr_t)Y & 15) == 0;
  if (A->dt == SPMV_F64) {
    if (wide) launch_spmm<double, 2>(A, X, ldx, Y, ldy, k, s);
    else launch_spmm<double, 1>(A, X, ldx, Y, ldy, k, s);
  } else {
    if (wide) launch_spmm<float, 4>(A, X, ldx, Y, ldy, k, s);
    else launch_spmm<float, 1>(A, X, ldx, Y, ldy, k, s);
  }
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

// ------------------------------------------------------- batched launch
// A work item is one row block of one matrix; items are numbered across
// the batch in matrix order, so the list is balanced by rows-plus-nonzeros.
// The item table, built once when the batch is created, holds each item's
// matrix arrays, row range and nonzero range, so a workgroup issues its
// column and value loads right after reading one record (no search over
// the matrices, no dependent row-pointer loads).  A SELL-C-sigma matrix
// contributes items of 256 / C chunks (one stored row per thread).
struct BatchItem {
  const void* p0;  // CSR: ptr; SELL: cs (chunk slot offsets); CSR wave tiles: its BatchTiles record
  const int32_t* col;
  const void* val;
  const int32_t* perm;  // SELL with sigma > 1: stored row -> row (else null)
  // kind 0: CSR rows [r0, r1), entries [k0, k1); 1: SELL chunks [r0, r1);
  // 2: CSR wave tiles [r0, r1), at most one per wave of the workgroup
  int32_t kind, m, r0, r1, k0, k1, logc, M;
};

// A CSR handle built with wave tiles (SPMV_FLAG_CSR_TILES): its arrays and
// tile tables, and its index m in the batch (for the fix-up pass).
struct BatchTiles {
  const int32_t* ptr;
  const int32_t* col;
  const void* val;
  const int32_t* tstart;
  const int32_t* tcont;
  double* head;
  double* tail;
  int32_t* trow;
  int32_t* info;
  int64_t nnz, ntiles;
  int32_t m, pad;
};

__global__ void k_batch_items(int64_t nblk, const int32_t* __restrict__ blk_row, const int32_t* __restrict__ ptr,
                              const int32_t* col, const void* val, int32_t m, BatchItem* __restrict__ out) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nblk; b += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r0 = blk_row[b], r1 = blk_row[b + 1];
    BatchItem it;
    it.p0 = ptr;
    it.col = col;
    it.val = val;
    it.perm = nullptr;
    it.kind = 0;
    it.m = m;
    it.r0 = r0;
    it.r1 = r1;
    it.k0 = ptr[r0];
    it.k1 = ptr[r1];
    it.logc = 0;
    it.M = 0;
    out[b] = it;
  }
}

__global__ void k_batch_sell_items(int64_t nitems, int64_t nchunks, int logc, int64_t M, const int64_t* cs,
                                   const int32_t* perm, const int32_t* col, const void* val, int32_t m,
                                   BatchItem* __restrict__ out) {
  const int64_t per = BS >> logc;  // chunks per item
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nitems; b += (int64_t)gridDim.x * blockDim.x) {
    BatchItem it;
    it.p0 = cs;
    it.col = col;
    it.val = val;
    it.perm = perm;
    it.kind = 1;
    it.m = m;
    it.r0 = (int32_t)(b * per);
    it.r1 = (int32_t)std::min<int64_t>(nchunks, (b + 1) * per);
    it.k0 = 0;
    it.k1 = 0;
    it.logc = logc;
    it.M = (int32_t)M;
    out[b] = it;
  }
}

// One SELL item: thread t takes stored row t & (C-1) of chunk r0 + (t >> log C)
// and sums its slots 8 at a time (all loads of a group of 8 in flight;
// padding slots hold column -1 and add nothing).
template <typename T>
__device__ __forceinline__ void sell_item(const BatchItem& it, const T* __restrict__ x, T* __restrict__ y) {
  const int t = threadIdx.x;
  const int64_t c = it.r0 + (t >> it.logc);
  if (c >= it.r1) return;
  const int p = t & ((1 << it.logc) - 1);
  const int64_t* cs = (const int64_t*)it.p0;
  const int64_t base = cs[c];
  const int C = 1 << it.logc;
  const int w = (int)((cs[c + 1] - base) >> it.logc);
  const int32_t* cc = it.col + base + p;
  const T* vv = (const T*)it.val + base + p;
  double sa[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < w; k0 += 8) {
    const int n = w - k0 < 8 ? w - k0 : 8;
    int32_t cg[8];
    T vg[8], xg[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) cg[u] = ldnt(cc + (int64_t)(k0 + (u < n ? u : n - 1)) * C);
#pragma unroll
    for (int u = 0; u < 8; ++u) vg[u] = ldnt(vv + (int64_t)(k0 + (u < n ? u : n - 1)) * C);
    issue_fence();
#pragma unroll
    for (int u = 0; u < 8; ++u) xg[u] = x[cg[u] >= 0 ? cg[u] : 0];
    issue_fence();
#pragma unroll
    for (int u = 0; u < 8; ++u) sa[u & 3] += (u < n && cg[u] >= 0) ? (double)vg[u] * (double)xg[u] : 0.0;
  }
  const int64_t pos = c * C + p;
  const int64_t r = it.perm ? (int64_t)it.perm[pos] : (pos < it.M ? pos : -1);
  if (r >= 0) y[r] = (T)((sa[0] + sa[1]) + (sa[2] + sa[3]));
}

template <typename T>
__global__ __launch_bounds__(BS) void k_csr_batched(int64_t nitems, const BatchItem* __restrict__ items,
                                                    const void* const* __restrict__ xs, void* const* __restrict__ ys) {
  __shared__ double prod[CSR_CAP];
  __shared__ int32_t sptr[CSR_RCAP + 1];
  // one workgroup per item, in dispatch order: the hardware hands each next
  // workgroup to an XCD with room, which balances matrices of unequal cost
  // (a fixed contiguous range per XCD left the XCDs that drew the
  // scattered-column matrices last: 2.89 against 2.56 ms on 512 matrices).
  // Only a few matrices are in flight at once, so their x stays in every L2.
  const int64_t i = blockIdx.x;
  if (i >= nitems) return;
  const BatchItem it = items[i];
  if (it.kind == 1) {  // uniform over the workgroup
    sell_item<T>(it, (const T*)xs[it.m], (T*)ys[it.m]);
    return;
  }
  if (it.kind == 2) {  // one wave per tile; the row tables alias the staging area
    static_assert(sizeof(prod) >= sizeof(int32_t) * (BS / WAVE) * TILE_E, "tile row tables exceed the LDS area");
    const BatchTiles* d = (const BatchTiles*)it.p0;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int64_t t = (int64_t)it.r0 + w;
    if (t >= it.r1) return;
    csr_tile<T>(t, d->nnz, d->ntiles, d->ptr, d->col, (const T*)d->val, d->tstart, d->tcont, (const T*)xs[it.m],
                (T*)ys[it.m], d->head, d->tail, d->trow, d->info, reinterpret_cast<int32_t*>(prod) + w * TILE_E);
    return;
  }
  csr_rows_block<T>(it.r0, it.r1, it.k0, it.k1, (const int32_t*)it.p0, it.col, (const T*)it.val,
                    (const T*)xs[it.m], (T*)ys[it.m], prod, sptr);
}

// The wave-tile matrices' crossing rows, after the batched launch: one
// workgroup per matrix, each tile whose last row continues sums that row's
// partials in tile order (as k_tile_fix does for one matrix).
template <typename T>
__global__ __launch_bounds__(BS) void k_batch_tile_fix(const BatchTiles* __restrict__ d, void* const* __restrict__ ys) {
  const BatchTiles b = d[blockIdx.x];
  T* y = (T*)ys[b.m];
  for (int64_t t = threadIdx.x; t < b.ntiles; t += BS) {
    if (b.info[t] != TILE_TAIL) continue;
    double tot = b.tail[t];
    for (int64_t u = t + 1;; ++u) {
      tot += b.head[u];
      if (b.info[u] != TILE_SPAN) break;
    }
    y[b.trow[t]] = (T)tot;
  }
}

// Items of matrix A (index m of the batch): CSR row blocks, CSR wave tiles
// (handles built with them) or SELL chunk groups.
int64_t batch_item_count(const spmv_mat_s* A) {
  if (A->fmt == SPMV_FMT_SELL) return cdiv(A->nchunks, BS / A->C);
  if (A->ntiles_csr > 0) return cdiv(A->ntiles_csr, BS / WAVE);
  return A->nblk;
}

size_t batch_tiles_size() { return sizeof(BatchTiles); }

// The tile record of matrix A (host) and its items (written to the device at
// items, referring to the record at dev_rec).
spmv_status_t batch_tile_items(const spmv_mat_s* A, int32_t m, void* host_rec, const void* dev_rec, void* items,
                               hipStream_t s) {
  BatchTiles b;
  b.ptr = A->ptr;
  b.col = A->col;
  b.val = A->val;
  b.tstart = A->ct_start;
  b.tcont = A->ct_cont;
  b.head = A->ct_head;
  b.tail = A->ct_tail;
  b.trow = A->ct_trow;
  b.info = A->ct_info;
  b.nnz = A->nnz;
  b.ntiles = A->ntiles_csr;
  b.m = m;
  b.pad = 0;
  memcpy(host_rec, &b, sizeof(b));
  const int64_t n = batch_item_count(A);
  std::vector<BatchItem> v((size_t)n);
  for (int64_t j = 0; j < n; ++j) {
    BatchItem& it = v[(size_t)j];
    memset(&it, 0, sizeof(it));
    it.p0 = dev_rec;
    it.kind = 2;
    it.m = m;
    it.r0 = (int32_t)(j * (BS / WAVE));
    it.r1 = (int32_t)std::min<int64_t>(A->ntiles_csr, (j + 1) * (BS / WAVE));
  }
  SPMV_HIP(hipMemcpyAsync(items, v.data(), sizeof(BatchItem) * (size_t)n, hipMemcpyHostToDevice, s));
  SPMV_HIP(hipStreamSynchronize(s));  // v is freed on return
  return SPMV_OK;
}

spmv_status_t launch_batch_tile_fix(int dt, int32_t ntm, const void* recs, void* const* ys, hipStream_t s) {
  if (ntm <= 0) return SPMV_OK;
  if (dt == SPMV_F64) launch(k_batch_tile_fix<double>, ntm, BS, s, (const BatchTiles*)recs, ys);
  else launch(k_batch_tile_fix<float>, ntm, BS, s, (const BatchTiles*)recs, ys);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

spmv_status_t batch_items_fill(const spmv_mat_s* A, int32_t m, void* items, hipStream_t s) {
  if (A->fmt == SPMV_FMT_SELL) {
    const int64_t n = batch_item_count(A);
    if (n <= 0) return SPMV_OK;
    int logc = 0;
    while ((1 << logc) < A->C) ++logc;
    k_batch_sell_items<<<(unsigned)std::min<int64_t>(cdiv(n, BS), 1024), BS, 0, s>>>(
        n, A->nchunks, logc, A->M, A->cs, A->perm, A->scol, A->sval, m, (BatchItem*)items);
    SPMV_LAUNCH_CHECK();
    return SPMV_OK;
  }
  if (A->nblk <= 0) return SPMV_OK;
  k_batch_items<<<(unsigned)std::min<int64_t>(cdiv(A->nblk, BS), 1024), BS, 0, s>>>(
      A->nblk, A->blk_row, A->ptr, A->col, A->val, m, (BatchItem*)items);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

size_t batch_item_size() { return sizeof(BatchItem); }

spmv_status_t launch_batched(int dt, int64_t nitems, const void* items, const void* const* xs, void* const* ys,
                             int grid, hipStream_t s) {
  if (nitems <= 0) return SPMV_OK;
  if (dt == SPMV_F64)
    launch(k_csr_batched<double>, grid, BS, s, nitems, (const BatchItem*)items, xs, ys);
  else
    launch(k_csr_batched<float>, grid, BS, s, nitems, (const BatchItem*)items, xs, ys);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

// ------------------------------------------------------------ creation
spmv_status_t mat_from_csr(int64_t M, int64_t N, int64_t nnz, const int32_t* ptr, const int32_t* col, const void* val,
                           spmv_dtype_t dt, int on_dev, uint32_t flags, hipStream_t s, spmv_mat_s* A) {
  A->fmt = SPMV_FMT_CSR;
  A->dt = dt;
  A->M = M;
  A->N = N;
  A->nnz = nnz;
  A->sv = value_size(dt);
  resolve_params(nullptr, &A->params);
  SPMV_TRY(mat_alloc(A, (void**)&A->ptr, sizeof(int32_t) * (M + 1)));
  SPMV_TRY(mat_alloc(A, (void**)&A->col, sizeof(int32_t) * nnz));
  SPMV_TRY(mat_alloc(A, &A->val, (size_t)A->sv * nnz));
  const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  SPMV_HIP(hipMemcpyAsync(A->ptr, ptr, sizeof(int32_t) * (M + 1), kind, s));
  if (nnz) {
    SPMV_HIP(hipMemcpyAsync(A->col, col, sizeof(int32_t) * nnz, kind, s));
    SPMV_HIP(hipMemcpyAsync(A->val, val, (size_t)A->sv * nnz, kind, s));
  }
  // ptr is always checked (the kernels index with it); columns unless told not to
  SPMV_TRY(validate_csr(A, (flags & SPMV_FLAG_NO_CHECK) ? 0 : 1, s));
  SPMV_TRY(csr_build_blocks(A, s));
  A->bytes_fmt = bytes_min(A);
  return SPMV_OK;
}

// a1: COO -> CSR on the device.  Keys row*N + col are radix-sorted stably
// with the input position as payload; each run of equal keys is summed
// in sorted (= input) order by one thread, in FP64, rounded once.
__global__ void k_coo_check(const int32_t* row, const int32_t* col, int64_t n, int64_t M, int64_t N, int* err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (row[i] < 0 || row[i] >= M || col[i] < 0 || col[i] >= N) atomicOr(err, 1);
}

__global__ void k_coo_keys(const int32_t* row, const int32_t* col, int64_t n, int64_t N, uint64_t* key, uint32_t* idx) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    key[i] = (uint64_t)row[i] * (uint64_t)N + (uint64_t)col[i];
    idx[i] = (uint32_t)i;
  }
}

__global__ void k_coo_heads(const uint64_t* key, int64_t n, int32_t* head) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    head[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

template <typename T>
__global__ void k_coo_reduce(const uint64_t* key, const uint32_t* idx, const T* vin, int64_t n, int64_t N,
                             const int32_t* pos, int32_t* col, T* vout, int32_t* urow) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!(i == 0 || key[i] != key[i - 1])) continue;
    double s = (double)vin[idx[i]];
    int64_t j = i + 1;
    for (; j < n && key[j] == key[i]; ++j) s += (double)vin[idx[j]];
    const int32_t u = pos[i];
    col[u] = (int32_t)(key[i] % (uint64_t)N);
    vout[u] = (T)s;
    urow[u] = (int32_t)(key[i] / (uint64_t)N);
  }
}

// ptr[r] = number of unique entries in rows before r: a lower bound in the
// (sorted) row of each unique entry; no atomics, so long rows cost nothing
// extra.
__global__ void k_coo_ptr(int64_t M, int64_t U, const int32_t* urow, int32_t* ptr) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= M; r += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = U;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (urow[mid] < r) lo = mid + 1;
      else hi = mid;
    }
    ptr[r] = (int32_t)lo;
  }
}

static int bits_for(uint64_t v) {
  int b = 0;
  while (b < 64 && (v >> b)) ++b;
  return b;
}

spmv_status_t mat_from_coo(int64_t M, int64_t N, int64_t n, const int32_t* row, const int32_t* col, const void* val,
                           spmv_dtype_t dt, int on_dev, hipStream_t s, spmv_mat_s* A) {
  A->fmt = SPMV_FMT_CSR;
  A->dt = dt;
  A->M = M;
  A->N = N;
  A->sv = value_size(dt);
  resolve_params(nullptr, &A->params);
  const int sv = A->sv;
  DTmp drow, dcol, dval, k1, k2, v1, v2, head, pos, err;
  const int32_t *r_in = row, *c_in = col;
  const void* val_in = val;
  if (!on_dev) {
    SPMV_TRY(drow.alloc(sizeof(int32_t) * n));
    SPMV_TRY(dcol.alloc(sizeof(int32_t) * n));
    SPMV_TRY(dval.alloc((size_t)sv * n));
    if (n) {
      SPMV_HIP(hipMemcpyAsync(drow.p, row, sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
      SPMV_HIP(hipMemcpyAsync(dcol.p, col, sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
      SPMV_HIP(hipMemcpyAsync(dval.p, val, (size_t)sv * n, hipMemcpyHostToDevice, s));
    }
    r_in = drow.as<int32_t>();
    c_in = dcol.as<int32_t>();
    val_in = dval.p;
  }
  const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(cdiv(n, BS), 1), 65536);
  SPMV_TRY(err.alloc(sizeof(int)));
  SPMV_HIP(hipMemsetAsync(err.p, 0, sizeof(int), s));
  if (n) {
    k_coo_check<<<g, BS, 0, s>>>(r_in, c_in, n, M, N, err.as<int>());
    SPMV_LAUNCH_CHECK();
  }
  int h = 0;
  SPMV_TRY(copy_to_host(&h, err.p, sizeof(int), s));
  if (h) return fail(SPMV_ERR_BAD_STRUCTURE, "COO coordinate out of range");
  SPMV_TRY(k1.alloc(sizeof(uint64_t) * n));
  SPMV_TRY(k2.alloc(sizeof(uint64_t) * n));
  SPMV_TRY(v1.alloc(sizeof(uint32_t) * n));
  SPMV_TRY(v2.alloc(sizeof(uint32_t) * n));
  SPMV_TRY(head.alloc(sizeof(int32_t) * (n + 1)));
  SPMV_TRY(pos.alloc(sizeof(int32_t) * (n + 1)));
  uint64_t* keys = k1.as<uint64_t>();
  uint32_t* idx = v1.as<uint32_t>();
  if (n) {
    k_coo_keys<<<g, BS, 0, s>>>(r_in, c_in, n, N, keys, idx);
    SPMV_LAUNCH_CHECK();
    const int kb = bits_for((uint64_t)M * (uint64_t)N - 1);
    SPMV_TRY(radix_sort_pairs(&keys, &idx, k2.as<uint64_t>(), v2.as<uint32_t>(), n, kb, s));
    k_coo_heads<<<g, BS, 0, s>>>(keys, n, head.as<int32_t>());
    SPMV_LAUNCH_CHECK();
  }
  SPMV_TRY(scan_i32_to_i32(head.as<int32_t>(), pos.as<int32_t>(), n, s));
  int32_t U = 0;
  SPMV_TRY(copy_to_host(&U, pos.as<int32_t>() + n, sizeof(int32_t), s));
  A->nnz = U;
  DTmp urow;
  SPMV_TRY(urow.alloc(sizeof(int32_t) * std::max<int64_t>(U, 1)));
  SPMV_TRY(mat_alloc(A, (void**)&A->ptr, sizeof(int32_t) * (M + 1)));
  SPMV_TRY(mat_alloc(A, (void**)&A->col, sizeof(int32_t) * U));
  SPMV_TRY(mat_alloc(A, &A->val, (size_t)sv * U));
  if (n) {
    if (dt == SPMV_F64)
      k_coo_reduce<double><<<g, BS, 0, s>>>(keys, idx, (const double*)val_in, n, N, pos.as<int32_t>(), A->col,
                                            (double*)A->val, urow.as<int32_t>());
    else
      k_coo_reduce<float><<<g, BS, 0, s>>>(keys, idx, (const float*)val_in, n, N, pos.as<int32_t>(), A->col,
                                           (float*)A->val, urow.as<int32_t>());
    SPMV_LAUNCH_CHECK();
  }
  k_coo_ptr<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(M + 1, BS), 65536)), BS, 0, s>>>(
      M, U, urow.as<int32_t>(), A->ptr);
  SPMV_LAUNCH_CHECK();
  SPMV_TRY(csr_build_blocks(A, s));
  A->bytes_fmt = bytes_min(A);
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

}  // namespace spmv
