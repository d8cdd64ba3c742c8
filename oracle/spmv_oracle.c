/*
 * CPU oracle for the SpMV format library -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct FP64 C.  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the GPU library never does,
 * and this file shares no code, header or table with it.
 *
 * Paper: "Optimizing Sparse Matrix-Vector Multiplication on Emerging
 * Many-Core Architectures" (arXiv 1805.11938).  Each function names the
 * passage it follows.  Where the paper is silent, the reading taken is
 * stated at the function.
 *
 * Compiled with -O2 -ffp-contract=off, so every multiply and add is rounded
 * separately, in the order written.
 *
 * Conventions: int32 indices; int64 slot offsets; FP64 values; FP32 inputs
 * are promoted to FP64 by the caller before they reach this file.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_BAD_ARG -1
#define ORC_BAD_STRUCTURE -2
#define ORC_OOM -3

/* ===================================================================== */
/* COO -> CSR (Sec. II-B, COO and CSR paragraphs; Table I).               */
/* Reading: entries are ordered by (row, col) with a stable sort, so      */
/* duplicates keep their input order and are summed left to right in     */
/* that order; explicit zeros are kept.                                   */
/* ===================================================================== */

/* stable merge sort of idx[0..n) by key (row, col) */
static void msort(int64_t* idx, int64_t* tmp, int64_t n, const int32_t* row, const int32_t* col) {
  if (n < 2) return;
  int64_t h = n / 2;
  msort(idx, tmp, h, row, col);
  msort(idx + h, tmp, n - h, row, col);
  int64_t i = 0, j = h, k = 0;
  while (i < h && j < n) {
    int64_t a = idx[i], b = idx[j];
    int take_b = (row[b] < row[a]) || (row[b] == row[a] && col[b] < col[a]);
    tmp[k++] = take_b ? idx[j++] : idx[i++];
  }
  while (i < h) tmp[k++] = idx[i++];
  while (j < n) tmp[k++] = idx[j++];
  memcpy(idx, tmp, sizeof(int64_t) * (size_t)n);
}

/* Returns the number of unique entries through *nnz_out; ocol/oval must hold
 * n entries.  Out-of-range coordinates -> ORC_BAD_STRUCTURE. */
int orc_coo_to_csr(int64_t M, int64_t N, int64_t n, const int32_t* row, const int32_t* col, const double* val,
                   int32_t* ptr, int32_t* ocol, double* oval, int64_t* nnz_out) {
  if (M < 0 || N < 0 || n < 0) return ORC_BAD_ARG;
  for (int64_t k = 0; k < n; ++k)
    if (row[k] < 0 || row[k] >= M || col[k] < 0 || col[k] >= N) return ORC_BAD_STRUCTURE;
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!idx || !tmp) { free(idx); free(tmp); return ORC_OOM; }
  for (int64_t k = 0; k < n; ++k) idx[k] = k;
  msort(idx, tmp, n, row, col);
  for (int64_t i = 0; i <= M; ++i) ptr[i] = 0;
  int64_t u = 0;
  for (int64_t k = 0; k < n; ++k) {
    int64_t e = idx[k];
    if (k > 0 && row[idx[k - 1]] == row[e] && col[idx[k - 1]] == col[e]) {
      oval[u - 1] = oval[u - 1] + val[e]; /* duplicate: add in input order */
    } else {
      ocol[u] = col[e];
      oval[u] = val[e];
      ptr[row[e] + 1] += 1;
      ++u;
    }
  }
  for (int64_t i = 0; i < M; ++i) ptr[i + 1] += ptr[i];
  *nnz_out = u;
  free(idx);
  free(tmp);
  return ORC_OK;
}

/* CSR well-formedness (Sec. II-B, CSR paragraph): ptr[0] = 0, ptr
 * non-decreasing, ptr[M] = nnz, columns in range and strictly increasing
 * inside each row. */
int orc_csr_check(int64_t M, int64_t N, int64_t nnz, const int32_t* ptr, const int32_t* col) {
  if (M < 0 || N < 0 || nnz < 0) return ORC_BAD_ARG;
  if (ptr[0] != 0 || ptr[M] != nnz) return ORC_BAD_STRUCTURE;
  for (int64_t i = 0; i < M; ++i) {
    if (ptr[i + 1] < ptr[i]) return ORC_BAD_STRUCTURE;
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
      if (col[k] < 0 || col[k] >= N) return ORC_BAD_STRUCTURE;
      if (k > ptr[i] && col[k] <= col[k - 1]) return ORC_BAD_STRUCTURE;
    }
  }
  return ORC_OK;
}

/* ===================================================================== */
/* y = A x over CSR (Sec. II-A definition; Sec. II-B CSR).                */
/* y_i = sum over k in [ptr[i], ptr[i+1]) of data[k] * x[indices[k]].     */
/* ===================================================================== */
void orc_csr_spmv(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, const double* x,
                  double* y) {
  for (int64_t i = 0; i < M; ++i) {
    double s = 0.0;
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) s += val[k] * x[col[k]];
    y[i] = s;
  }
}

/* The same loop with the rows split statically over OpenMP threads, the
 * paper's threading model for its row-parallel kernels (Sec. III-B, III-D).
 * Results are identical to orc_csr_spmv (each row is still one thread's
 * sequential sum).  Returns the thread count used. */
int orc_csr_spmv_omp(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, const double* x,
                     double* y, int nthreads) {
  int used = 1;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
#pragma omp single
    {
#ifdef _OPENMP
      used = omp_get_num_threads();
#endif
    }
#pragma omp for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
      double s = 0.0;
      for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) s += val[k] * x[col[k]];
      y[i] = s;
    }
  }
  return used;
}

/* Row-wise sum of |a_ij * x_j|: the denominator of the row-wise relative
 * error (any summation order of row i errs by at most gamma_n times it). */
void orc_csr_absspmv(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, const double* x,
                     double* y) {
  for (int64_t i = 0; i < M; ++i) {
    double s = 0.0;
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) s += fabs(val[k] * x[col[k]]);
    y[i] = s;
  }
}

/* SpMM: Y[M x k] = A X[N x k], row-major with leading dimensions ldx/ldy,
 * one column at a time (the definition of Sec. II-A applied per column). */
void orc_csr_spmm(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, int64_t kk,
                  const double* X, int64_t ldx, double* Y, int64_t ldy) {
  for (int64_t c = 0; c < kk; ++c)
    for (int64_t i = 0; i < M; ++i) {
      double s = 0.0;
      for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) s += val[k] * X[(int64_t)col[k] * ldx + c];
      Y[i * ldy + c] = s;
    }
}

/* ===================================================================== */
/* ELL (Sec. II-B, ELL paragraph; Table I).                               */
/* K = the largest row length.  Reading: the M x K arrays are stored      */
/* column-major (slot (i,k) at k*M + i); padding is index -1, value +0.0  */
/* (the table's '*'), so that padding is never mistaken for a real entry  */
/* at column 0 and never reads x.                                         */
/* ===================================================================== */
int64_t orc_max_row_len(int64_t M, const int32_t* ptr) {
  int64_t K = 0;
  for (int64_t i = 0; i < M; ++i)
    if (ptr[i + 1] - ptr[i] > K) K = ptr[i + 1] - ptr[i];
  return K;
}

void orc_csr_to_ell(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, int64_t K,
                    int32_t* ecol, double* eval) {
  for (int64_t i = 0; i < M; ++i) {
    int64_t len = ptr[i + 1] - ptr[i];
    for (int64_t k = 0; k < K; ++k) {
      int64_t s = k * M + i;
      if (k < len) { ecol[s] = col[ptr[i] + k]; eval[s] = val[ptr[i] + k]; }
      else { ecol[s] = -1; eval[s] = 0.0; }
    }
  }
}

void orc_ell_spmv(int64_t M, int64_t K, const int32_t* ecol, const double* eval, const double* x, double* y) {
  for (int64_t i = 0; i < M; ++i) {
    double s = 0.0;
    for (int64_t k = 0; k < K; ++k) {
      int32_t c = ecol[k * M + i];
      if (c >= 0) s += eval[k * M + i] * x[c];
    }
    y[i] = s;
  }
}

/* Inverse: drop the -1 padding; returns nnz. */
int64_t orc_ell_to_csr(int64_t M, int64_t K, const int32_t* ecol, const double* eval, int32_t* ptr, int32_t* col,
                       double* val) {
  int64_t n = 0;
  ptr[0] = 0;
  for (int64_t i = 0; i < M; ++i) {
    for (int64_t k = 0; k < K; ++k) {
      int32_t c = ecol[k * M + i];
      if (c < 0) break;
      col[n] = c;
      val[n] = eval[k * M + i];
      ++n;
    }
    ptr[i + 1] = (int32_t)n;
  }
  return n;
}

/* ===================================================================== */
/* SELL and SELL-C-sigma (Sec. II-B, SELL paragraph; Table I).            */
/* Strips of C adjacent rows, each stored as ELL with its own width (the  */
/* table's `slices`).  SELL-C-sigma first sorts rows by length, not       */
/* globally but inside windows of sigma consecutive rows.                 */
/* Readings: descending length, stable (ties keep row order; Table I's    */
/* C=2, sigma=4 example gives order 1,0,3,2); windows start at row 0;     */
/* the row count is padded to a multiple of C with empty virtual rows     */
/* (perm = -1); inside a strip, slot (p,k) sits at cs[c] + k*C + p        */
/* (column-major), cs = exclusive prefix sum of C * width; padding is     */
/* (-1, +0.0); y is written in the original row order through perm and x */
/* is not permuted.  sigma = 1 means plain SELL.                          */
/* ===================================================================== */

/* perm[M_pad] and widths[nchunks]; returns total slots. */
int64_t orc_sell_layout(int64_t M, int64_t C, int64_t sigma, const int32_t* ptr, int32_t* perm, int32_t* widths,
                        int64_t* cs) {
  int64_t nch = (M + C - 1) / C, Mp = nch * C;
  for (int64_t p = 0; p < Mp; ++p) perm[p] = p < M ? (int32_t)p : -1;
  if (sigma > 1) {
    for (int64_t w0 = 0; w0 < M; w0 += sigma) {
      int64_t w1 = w0 + sigma < M ? w0 + sigma : M;
      /* stable insertion sort by descending length (plain, O(sigma^2)) */
      for (int64_t a = w0 + 1; a < w1; ++a) {
        int32_t r = perm[a];
        int64_t lr = ptr[r + 1] - ptr[r];
        int64_t b = a - 1;
        while (b >= w0 && (ptr[perm[b] + 1] - ptr[perm[b]]) < lr) { perm[b + 1] = perm[b]; --b; }
        perm[b + 1] = r;
      }
    }
  }
  cs[0] = 0;
  for (int64_t c = 0; c < nch; ++c) {
    int64_t w = 0;
    for (int64_t p = c * C; p < (c + 1) * C; ++p)
      if (perm[p] >= 0 && ptr[perm[p] + 1] - ptr[perm[p]] > w) w = ptr[perm[p] + 1] - ptr[perm[p]];
    widths[c] = (int32_t)w;
    cs[c + 1] = cs[c] + C * w;
  }
  return cs[nch];
}

void orc_csr_to_sell(int64_t M, int64_t C, const int32_t* ptr, const int32_t* col, const double* val,
                     const int32_t* perm, const int32_t* widths, const int64_t* cs, int32_t* scol, double* sval) {
  int64_t nch = (M + C - 1) / C;
  for (int64_t c = 0; c < nch; ++c)
    for (int64_t p = 0; p < C; ++p) {
      int32_t r = perm[c * C + p];
      int64_t len = r >= 0 ? ptr[r + 1] - ptr[r] : 0;
      for (int64_t k = 0; k < widths[c]; ++k) {
        int64_t s = cs[c] + k * C + p;
        if (k < len) { scol[s] = col[ptr[r] + k]; sval[s] = val[ptr[r] + k]; }
        else { scol[s] = -1; sval[s] = 0.0; }
      }
    }
}

void orc_sell_spmv(int64_t M, int64_t C, const int32_t* perm, const int32_t* widths, const int64_t* cs,
                   const int32_t* scol, const double* sval, const double* x, double* y) {
  int64_t nch = (M + C - 1) / C;
  for (int64_t c = 0; c < nch; ++c)
    for (int64_t p = 0; p < C; ++p) {
      double s = 0.0;
      for (int64_t k = 0; k < widths[c]; ++k) {
        int64_t q = cs[c] + k * C + p;
        if (scol[q] >= 0) s += sval[q] * x[scol[q]];
      }
      if (perm[c * C + p] >= 0) y[perm[c * C + p]] = s;
    }
}

int64_t orc_sell_to_csr(int64_t M, int64_t C, const int32_t* perm, const int32_t* widths, const int64_t* cs,
                        const int32_t* scol, const double* sval, int32_t* ptr, int32_t* col, double* val) {
  int64_t nch = (M + C - 1) / C;
  int32_t* len = (int32_t*)calloc((size_t)(M > 0 ? M : 1), sizeof(int32_t));
  int64_t* pos = (int64_t*)calloc((size_t)(M > 0 ? M : 1), sizeof(int64_t));
  for (int64_t c = 0; c < nch; ++c)
    for (int64_t p = 0; p < C; ++p) {
      int32_t r = perm[c * C + p];
      if (r < 0) continue;
      pos[r] = c * C + p;
      int64_t k = 0;
      while (k < widths[c] && scol[cs[c] + k * C + p] >= 0) ++k;
      len[r] = (int32_t)k;
    }
  ptr[0] = 0;
  for (int64_t i = 0; i < M; ++i) ptr[i + 1] = ptr[i] + len[i];
  for (int64_t i = 0; i < M; ++i) {
    int64_t c = pos[i] / C, p = pos[i] % C;
    for (int64_t k = 0; k < len[i]; ++k) {
      col[ptr[i] + k] = scol[cs[c] + k * C + p];
      val[ptr[i] + k] = sval[cs[c] + k * C + p];
    }
  }
  int64_t n = ptr[M];
  free(len);
  free(pos);
  return n;
}

/* ===================================================================== */
/* HYB = ELL(K) + COO (Sec. II-B, HYB paragraph; Table I).                */
/* The paper says K, the "typical" row length, comes from the matrix but  */
/* gives no formula.  Reading: K is the largest k >= 0 such that at least */
/* ceil(M/3) rows have length >= k (Table I: lengths 2,3,1,2 -> K = 2).   */
/* The ELL part holds each row's first min(len, K) entries; the COO part  */
/* holds the rest in row-major order.                                     */
/* ===================================================================== */
int64_t orc_hyb_k_rule(int64_t M, const int32_t* ptr) {
  if (M <= 0) return 0;
  int64_t need = (M + 2) / 3, K = 0;
  int64_t maxlen = orc_max_row_len(M, ptr);
  for (int64_t k = 1; k <= maxlen; ++k) {
    int64_t cnt = 0;
    for (int64_t i = 0; i < M; ++i) cnt += (ptr[i + 1] - ptr[i]) >= k;
    if (cnt >= need) K = k; else break;
  }
  return K;
}

int64_t orc_hyb_coo_count(int64_t M, const int32_t* ptr, int64_t K) {
  int64_t n = 0;
  for (int64_t i = 0; i < M; ++i)
    if (ptr[i + 1] - ptr[i] > K) n += ptr[i + 1] - ptr[i] - K;
  return n;
}

void orc_csr_to_hyb(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, int64_t K,
                    int32_t* ecol, double* eval, int32_t* crow, int32_t* ccol, double* cval) {
  int64_t n = 0;
  for (int64_t i = 0; i < M; ++i) {
    int64_t len = ptr[i + 1] - ptr[i];
    for (int64_t k = 0; k < K; ++k) {
      int64_t s = k * M + i;
      if (k < len) { ecol[s] = col[ptr[i] + k]; eval[s] = val[ptr[i] + k]; }
      else { ecol[s] = -1; eval[s] = 0.0; }
    }
    for (int64_t k = K; k < len; ++k) {
      crow[n] = (int32_t)i; ccol[n] = col[ptr[i] + k]; cval[n] = val[ptr[i] + k]; ++n;
    }
  }
}

void orc_hyb_spmv(int64_t M, int64_t K, const int32_t* ecol, const double* eval, int64_t ncoo, const int32_t* crow,
                  const int32_t* ccol, const double* cval, const double* x, double* y) {
  orc_ell_spmv(M, K, ecol, eval, x, y);
  for (int64_t n = 0; n < ncoo; ++n) y[crow[n]] += cval[n] * x[ccol[n]];
}

int64_t orc_hyb_to_csr(int64_t M, int64_t K, const int32_t* ecol, const double* eval, int64_t ncoo,
                       const int32_t* crow, const int32_t* ccol, const double* cval, int32_t* ptr, int32_t* col,
                       double* val) {
  int64_t n = 0, c = 0;
  ptr[0] = 0;
  for (int64_t i = 0; i < M; ++i) {
    for (int64_t k = 0; k < K; ++k) {
      int32_t cc = ecol[k * M + i];
      if (cc < 0) break;
      col[n] = cc; val[n] = eval[k * M + i]; ++n;
    }
    while (c < ncoo && crow[c] == i) { col[n] = ccol[c]; val[n] = cval[c]; ++n; ++c; }
    ptr[i + 1] = (int32_t)n;
  }
  return n;
}

/* ===================================================================== */
/* CSR5 (Sec. II-B, CSR5 paragraph; Table I with omega = sigma = 2).      */
/* The first T = floor(nnz / (omega*sigma)) * omega*sigma nonzeros are    */
/* cut into 2-D tiles of omega lanes x sigma entries; lane l of tile t    */
/* owns the sigma consecutive CSR entries starting at t*w*s + l*s.        */
/* Storage: slot (i, l) of tile t (i < sigma, l < omega) sits at          */
/* t*w*s + i*w + l and holds CSR entry t*w*s + l*s + i.                   */
/* tile_ptr[t] = the row holding entry t*w*s (largest r, ptr[r] <= t*w*s) */
/* and tile_ptr[T] = M.  Descriptor per lane: bit_flag bit i set when     */
/* slot (i, l) is the first entry of a row, and always at (0, 0) of each  */
/* tile (Table I flags the first slot of the second tile although it is   */
/* mid-row); y_off[l] = number of set flags in lanes before l;            */
/* seg_off[l] = number of consecutive following lanes with no flag.       */
/* Readings where the paper is silent: the flags of a lane are packed in  */
/* one 32-bit word (bit i <-> entry i, so sigma <= 32); only each tile's  */
/* first slot is forced, not each lane's; the remaining nnz mod (w*s)     */
/* entries stay in CSR order after the tiles.                             */
/* ===================================================================== */
static int64_t upper_bound_ptr(int64_t M, const int32_t* ptr, int64_t v) {
  int64_t lo = 0, hi = M + 1; /* first j in [0, M+1) with ptr[j] > v */
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (ptr[mid] > v) hi = mid; else lo = mid + 1;
  }
  return lo;
}

int64_t orc_csr5_ntiles(int64_t nnz, int64_t omega, int64_t sigma) { return nnz / (omega * sigma); }

/* Outputs: tile_ptr[T+1], flags[T*omega], y_off[T*omega], seg_off[T*omega],
 * tcol/tval[T*omega*sigma] (the tiled part; the tail is CSR entries
 * T*omega*sigma .. nnz-1 unchanged). */
void orc_csr_to_csr5(int64_t M, int64_t nnz, const int32_t* ptr, const int32_t* col, const double* val,
                     int64_t omega, int64_t sigma, int32_t* tile_ptr, uint32_t* flags, int32_t* y_off,
                     int32_t* seg_off, int32_t* tcol, double* tval) {
  int64_t W = omega * sigma, T = nnz / W;
  /* is entry e the first entry of some row? */
  unsigned char* start = (unsigned char*)calloc((size_t)(nnz > 0 ? nnz : 1), 1);
  for (int64_t i = 0; i < M; ++i)
    if (ptr[i + 1] > ptr[i]) start[ptr[i]] = 1;
  for (int64_t t = 0; t < T; ++t) {
    tile_ptr[t] = (int32_t)(upper_bound_ptr(M, ptr, t * W) - 1);
    for (int64_t l = 0; l < omega; ++l) {
      uint32_t f = 0;
      for (int64_t i = 0; i < sigma; ++i) {
        int64_t e = t * W + l * sigma + i;
        int64_t s = t * W + i * omega + l;
        tcol[s] = col[e];
        tval[s] = val[e];
        if (start[e] || (l == 0 && i == 0)) f |= 1u << i;
      }
      flags[t * omega + l] = f;
    }
    int32_t run = 0;
    for (int64_t l = 0; l < omega; ++l) {
      y_off[t * omega + l] = run;
      for (int64_t i = 0; i < sigma; ++i) run += (flags[t * omega + l] >> i) & 1u;
    }
    for (int64_t l = 0; l < omega; ++l) {
      int32_t n = 0;
      for (int64_t m = l + 1; m < omega && flags[t * omega + m] == 0; ++m) ++n;
      seg_off[t * omega + l] = n;
    }
  }
  tile_ptr[T] = (int32_t)M;
  free(start);
}

/* Interpreter: walks the tiles in storage order and assigns each entry to a
 * row by counting flags: the j-th flag of tile t opens the row that is the
 * j-th non-empty row at or after tile_ptr[t] (forced first flag included);
 * the tail is summed CSR-style.  It reads only the CSR5 arrays plus ptr
 * (the format keeps CSR's ptr, Table I). */
void orc_csr5_spmv(int64_t M, int64_t nnz, const int32_t* ptr, int64_t omega, int64_t sigma,
                   const int32_t* tile_ptr, const uint32_t* flags, const int32_t* tcol, const double* tval,
                   const int32_t* tail_col, const double* tail_val, const double* x, double* y) {
  int64_t W = omega * sigma, T = nnz / W;
  for (int64_t i = 0; i < M; ++i) y[i] = 0.0;
  for (int64_t t = 0; t < T; ++t) {
    int64_t r = tile_ptr[t];
    int64_t nflag = 0;
    for (int64_t l = 0; l < omega; ++l)
      for (int64_t i = 0; i < sigma; ++i) {
        if ((flags[t * omega + l] >> i) & 1u) {
          if (nflag > 0) { /* next non-empty row */
            ++r;
            while (ptr[r + 1] == ptr[r]) ++r;
          }
          ++nflag;
        }
        int64_t s = t * W + i * omega + l;
        y[r] += tval[s] * x[tcol[s]];
      }
  }
  /* tail: entries T*W .. nnz-1 in CSR order */
  for (int64_t i = 0; i < M; ++i) {
    int64_t a = ptr[i] > T * W ? ptr[i] : T * W, b = ptr[i + 1];
    for (int64_t k = a; k < b; ++k) y[i] += tail_val[k - T * W] * x[tail_col[k - T * W]];
  }
}

/* Inverse: undo the in-tile transpose; ptr is unchanged by the format. */
void orc_csr5_to_csr(int64_t nnz, int64_t omega, int64_t sigma, const int32_t* tcol, const double* tval,
                     const int32_t* tail_col, const double* tail_val, int32_t* col, double* val) {
  int64_t W = omega * sigma, T = nnz / W;
  for (int64_t t = 0; t < T; ++t)
    for (int64_t l = 0; l < omega; ++l)
      for (int64_t i = 0; i < sigma; ++i) {
        col[t * W + l * sigma + i] = tcol[t * W + i * omega + l];
        val[t * W + l * sigma + i] = tval[t * W + i * omega + l];
      }
  for (int64_t k = T * W; k < nnz; ++k) { col[k] = tail_col[k - T * W]; val[k] = tail_val[k - T * W]; }
}

/* ===================================================================== */
/* Features (Sec. V-B, Table IV), extended by four structural ones.       */
/* Order: n_rows, n_cols, nnz, nnz_frac = nnz/(M*N), nnz_min, nnz_max,    */
/* nnz_avg, nnz_std (population), variation, ell_pad = M*nnz_max/nnz,    */
/* bandwidth = max |i - j| over nonzeros, gini of the row lengths.        */
/* Readings: Table IV's "variation (matrix regularity)" is taken as the   */
/* coefficient of variation nnz_std / nnz_avg; "percentage of nonzeros"   */
/* is stored as a fraction.  Gini = sum_i (2i - M - 1) L_(i) / (M sum L)  */
/* with lengths sorted ascending and i 1-based; 0 when nnz = 0.           */
/* ===================================================================== */
static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

void orc_features(int64_t M, int64_t N, const int32_t* ptr, const int32_t* col, double* f) {
  int64_t nnz = M > 0 ? ptr[M] : 0;
  double mn = 0.0, mx = 0.0, mean = 0.0, var = 0.0, band = 0.0, gini = 0.0;
  if (M > 0) {
    mn = 1e300;
    for (int64_t i = 0; i < M; ++i) {
      double L = (double)(ptr[i + 1] - ptr[i]);
      if (L < mn) mn = L;
      if (L > mx) mx = L;
      mean += L;
    }
    mean /= (double)M;
    for (int64_t i = 0; i < M; ++i) {
      double d = (double)(ptr[i + 1] - ptr[i]) - mean;
      var += d * d;
    }
    var /= (double)M;
    for (int64_t i = 0; i < M; ++i)
      for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
        double d = fabs((double)i - (double)col[k]);
        if (d > band) band = d;
      }
    if (nnz > 0) {
      int64_t* L = (int64_t*)malloc(sizeof(int64_t) * (size_t)M);
      for (int64_t i = 0; i < M; ++i) L[i] = ptr[i + 1] - ptr[i];
      qsort(L, (size_t)M, sizeof(int64_t), cmp_i64);
      double num = 0.0;
      for (int64_t i = 0; i < M; ++i) num += (double)(2 * (i + 1) - M - 1) * (double)L[i];
      gini = num / ((double)M * (double)nnz);
      free(L);
    }
  }
  double sd = sqrt(var);
  f[0] = (double)M;
  f[1] = (double)N;
  f[2] = (double)nnz;
  f[3] = (M > 0 && N > 0) ? (double)nnz / ((double)M * (double)N) : 0.0;
  f[4] = mn;
  f[5] = mx;
  f[6] = mean;
  f[7] = sd;
  f[8] = mean > 0.0 ? sd / mean : 0.0;
  f[9] = nnz > 0 ? (double)M * mx / (double)nnz : 0.0;
  f[10] = band;
  f[11] = gini;
}
