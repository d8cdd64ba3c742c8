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
#include "common.h"

namespace spmv {

constexpr int CSR_W = 2048;    // rows + nonzeros per row block
constexpr int CSR_CAP = 2560;  // nonzeros a block can stage in LDS
constexpr int CSR_IT = CSR_CAP / BS;
constexpr int CSR_LONG = 4096; // rows at least this long are reduced by a whole block

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
__global__ void k_csr_blocks(const int32_t* ptr, int64_t M, int64_t nblk, int32_t* blk_row) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= nblk; b += (int64_t)gridDim.x * blockDim.x) {
    if (b == nblk) {
      blk_row[b] = (int32_t)M;
      continue;
    }
    const int64_t target = b * CSR_W;
    int64_t lo = 0, hi = M;  // first r in [0, M) with r + ptr[r] >= target, else M
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (mid + ptr[mid] >= target) hi = mid;
      else lo = mid + 1;
    }
    blk_row[b] = (int32_t)lo;
  }
}

spmv_status_t csr_build_blocks(spmv_mat_s* A, hipStream_t s) {
  A->nblk = cdiv(A->M + A->nnz, CSR_W);
  if (A->nblk < 1) A->nblk = 1;
  SPMV_TRY(mat_alloc(A, (void**)&A->blk_row, sizeof(int32_t) * (A->nblk + 1)));
  int64_t g = cdiv(A->nblk + 1, BS);
  if (g > 65536) g = 65536;
  k_csr_blocks<<<(unsigned)g, BS, 0, s>>>(A->ptr, A->M, A->nblk, A->blk_row);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

// ------------------------------------------------------------ kernels
__device__ __forceinline__ int lanes_for(int64_t nz, int64_t rows) {
  const int64_t avg = rows > 0 ? nz / rows : 0;
  if (avg >= 128) return 64;
  if (avg >= 64) return 32;
  if (avg >= 32) return 16;
  if (avg >= 16) return 8;
  if (avg >= 8) return 4;
  if (avg >= 4) return 2;
  return 1;
}

// One row block (all threads of the workgroup call this with the same rows).
template <typename T>
__device__ __forceinline__ void csr_rows_block(int64_t r0, int64_t r1, const int32_t* __restrict__ ptr,
                                               const int32_t* __restrict__ col, const T* __restrict__ val,
                                               const T* __restrict__ x, T* __restrict__ y, double* prod) {
  if (r0 >= r1) return;
  const int t = threadIdx.x;
  const int64_t k0 = ptr[r0], k1 = ptr[r1];
  const int64_t E = k1 - k0;
  if (E <= CSR_CAP) {
    int32_t c[CSR_IT];
    T v[CSR_IT];
#pragma unroll
    for (int j = 0; j < CSR_IT; ++j) {
      const int64_t k = t + j * BS;
      if (k < E) {
        c[j] = ldnt(col + k0 + k);
        v[j] = ldnt(val + k0 + k);
      }
    }
#pragma unroll
    for (int j = 0; j < CSR_IT; ++j) {
      const int64_t k = t + j * BS;
      if (k < E) prod[k] = (double)v[j] * (double)x[c[j]];
    }
    __syncthreads();
    const int V = lanes_for(E, r1 - r0);
    const int g = t / V, lane = t % V, ng = BS / V;
    for (int64_t r = r0 + g; r < r1; r += ng) {
      const int a = ptr[r] - (int32_t)k0, e = ptr[r + 1] - (int32_t)k0;
      double s = 0.0;
      for (int k = a + lane; k < e; k += V) s += prod[k];
      s = group_sum_rt(s, V);
      if (lane == 0) y[r] = (T)s;
    }
    __syncthreads();  // prod may be reused by the caller's next block
    return;
  }
  // long path: a wave per row below CSR_LONG, the whole block above
  const int w = t / WAVE, lane = __lane_id();
  for (int64_t r = r0 + w; r < r1; r += BS / WAVE) {
    const int64_t a = ptr[r], e = ptr[r + 1];
    if (e - a >= CSR_LONG) continue;
    double s = group_sum<64>(row_dot(col, val, x, a, e, lane, WAVE));
    if (lane == 0) y[r] = (T)s;
  }
  for (int64_t r = r0; r < r1; ++r) {
    const int64_t a = ptr[r], e = ptr[r + 1];
    if (e - a < CSR_LONG) continue;
    const double s = block_sum(row_dot(col, val, x, a, e, t, BS), prod);
    if (t == 0) y[r] = (T)s;
  }
  __syncthreads();
}

template <typename T, bool XCD>
__global__ __launch_bounds__(BS) void k_csr_rows(int64_t nblk, const int32_t* __restrict__ blk_row,
                                                 const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                 const T* __restrict__ val, const T* __restrict__ x, T* __restrict__ y) {
  __shared__ double prod[CSR_CAP];
  const uint32_t b = XCD ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  if (b >= nblk) return;
  csr_rows_block<T>(blk_row[b], blk_row[b + 1], ptr, col, val, x, y, prod);
}

template <typename T, int V>
__global__ __launch_bounds__(BS) void k_csr_vector(int64_t M, const int32_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ col, const T* __restrict__ val,
                                                   const T* __restrict__ x, T* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * (BS / V) + threadIdx.x / V;
  const int lane = threadIdx.x % V;
  if (r >= M) return;  // uniform across the V-lane group
  const double s = group_sum<V>(row_dot(col, val, x, ptr[r], ptr[r + 1], lane, V));
  if (lane == 0) y[r] = (T)s;
}

template <typename T>
static spmv_status_t run_csr_t(spmv_mat_s* A, const T* x, T* y, hipStream_t s) {
  if (A->M == 0) return SPMV_OK;
  const int V = A->params.csr_lanes_per_row;
  const int32_t* ptr = A->ptr;
  const T* val = (const T*)A->val;
  if (V == 0) {
    k_csr_rows<T, true><<<(unsigned)A->nblk, BS, 0, s>>>(A->nblk, A->blk_row, ptr, A->col, val, x, y);
  } else {
    const unsigned g = (unsigned)cdiv(A->M, BS / V);
    switch (V) {
      case 1: k_csr_vector<T, 1><<<g, BS, 0, s>>>(A->M, ptr, A->col, val, x, y); break;
      case 2: k_csr_vector<T, 2><<<g, BS, 0, s>>>(A->M, ptr, A->col, val, x, y); break;
      case 4: k_csr_vector<T, 4><<<g, BS, 0, s>>>(A->M, ptr, A->col, val, x, y); break;
      case 8: k_csr_vector<T, 8><<<g, BS, 0, s>>>(A->M, ptr, A->col, val, x, y); break;
      case 16: k_csr_vector<T, 16><<<g, BS, 0, s>>>(A->M, ptr, A->col, val, x, y); break;
      case 32: k_csr_vector<T, 32><<<g, BS, 0, s>>>(A->M, ptr, A->col, val, x, y); break;
      case 64: k_csr_vector<T, 64><<<g, BS, 0, s>>>(A->M, ptr, A->col, val, x, y); break;
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

// ------------------------------------------------------- batched launch
// A work item is one row block of one matrix; items are numbered across
// the batch (prefix of row-block counts), so the list is balanced by
// rows-plus-nonzeros.  A fixed grid strides over the item list.
struct BatchDesc {
  const int32_t* ptr;
  const int32_t* col;
  const void* val;
  const int32_t* blk_row;
  int64_t item0;  // first global item of this matrix
};

template <typename T>
__global__ __launch_bounds__(BS) void k_csr_batched(int32_t n, int64_t nitems, const BatchDesc* __restrict__ desc,
                                                    const void* const* __restrict__ xs, void* const* __restrict__ ys) {
  __shared__ double prod[CSR_CAP];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    int lo = 0, hi = n - 1;  // last matrix with item0 <= it
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (desc[mid].item0 <= it) lo = mid;
      else hi = mid - 1;
    }
    const BatchDesc d = desc[lo];
    const int64_t b = it - d.item0;
    csr_rows_block<T>(d.blk_row[b], d.blk_row[b + 1], d.ptr, d.col, (const T*)d.val, (const T*)xs[lo], (T*)ys[lo],
                      prod);
  }
}

spmv_status_t launch_batched(int dt, int32_t n, int64_t nitems, const void* desc, const void* const* xs,
                             void* const* ys, int grid, hipStream_t s) {
  if (nitems <= 0) return SPMV_OK;
  if (dt == SPMV_F64)
    k_csr_batched<double><<<grid, BS, 0, s>>>(n, nitems, (const BatchDesc*)desc, xs, ys);
  else
    k_csr_batched<float><<<grid, BS, 0, s>>>(n, nitems, (const BatchDesc*)desc, xs, ys);
  SPMV_LAUNCH_CHECK();
  return SPMV_OK;
}

size_t batch_desc_size() { return sizeof(BatchDesc); }
void batch_desc_fill(void* dst, const spmv_mat_s* A, int64_t item0) {
  BatchDesc* d = (BatchDesc*)dst;
  d->ptr = A->ptr;
  d->col = A->col;
  d->val = A->val;
  d->blk_row = A->blk_row;
  d->item0 = item0;
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
                             const int32_t* pos, int32_t* col, T* vout, int32_t* rowcnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!(i == 0 || key[i] != key[i - 1])) continue;
    double s = (double)vin[idx[i]];
    int64_t j = i + 1;
    for (; j < n && key[j] == key[i]; ++j) s += (double)vin[idx[j]];
    const int32_t u = pos[i];
    col[u] = (int32_t)(key[i] % (uint64_t)N);
    vout[u] = (T)s;
    atomicAdd(&rowcnt[key[i] / (uint64_t)N], 1);
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
  DTmp rowcnt;
  SPMV_TRY(rowcnt.alloc(sizeof(int32_t) * (M + 1)));
  SPMV_HIP(hipMemsetAsync(rowcnt.p, 0, sizeof(int32_t) * (M + 1), s));
  SPMV_TRY(mat_alloc(A, (void**)&A->ptr, sizeof(int32_t) * (M + 1)));
  SPMV_TRY(mat_alloc(A, (void**)&A->col, sizeof(int32_t) * U));
  SPMV_TRY(mat_alloc(A, &A->val, (size_t)sv * U));
  if (n) {
    if (dt == SPMV_F64)
      k_coo_reduce<double><<<g, BS, 0, s>>>(keys, idx, (const double*)val_in, n, N, pos.as<int32_t>(), A->col,
                                            (double*)A->val, rowcnt.as<int32_t>());
    else
      k_coo_reduce<float><<<g, BS, 0, s>>>(keys, idx, (const float*)val_in, n, N, pos.as<int32_t>(), A->col,
                                           (float*)A->val, rowcnt.as<int32_t>());
    SPMV_LAUNCH_CHECK();
  }
  SPMV_TRY(scan_i32_to_i32(rowcnt.as<int32_t>(), A->ptr, M, s));
  SPMV_TRY(csr_build_blocks(A, s));
  A->bytes_fmt = bytes_min(A);
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

}  // namespace spmv
