/*
 * Seeded synthetic sparse-matrix generators.
 *
 * These produce the inputs that both the GPU library and the CPU oracle
 * consume.  They hold none of the SpMV method's arithmetic: they only draw
 * random structure and values.  Structured generators (stencils, banded,
 * block-diagonal, row-length driven) emit rows whose column lists are already
 * sorted and duplicate-free; the R-MAT generator emits raw COO triplets with
 * duplicates, which the library and the oracle each canonicalise on their own.
 *
 * Random numbers come from a counter-based generator: every draw is a pure
 * function of (seed, stream, index), using the SplitMix64 output mix
 * (Steele, Lea and Flood, OOPSLA 2014).  That makes every generator
 * deterministic and trivially parallel (OpenMP over rows or edges).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Draw number `idx` of stream `stream` under `seed`. */
uint64_t syn_u64(uint64_t seed, uint64_t stream, uint64_t idx) {
  uint64_t key = mix64(seed * GOLDEN + mix64(stream + GOLDEN));
  return mix64(key + (idx + 1) * GOLDEN);
}

/* Uniform in [0,1) with 53 random bits. */
static inline double u01(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (double)(syn_u64(seed, stream, idx) >> 11) * (1.0 / 9007199254740992.0);
}

/* Uniform integer in [0, n) by the multiply-shift map (n < 2^63). */
static inline uint64_t uint_below(uint64_t r, uint64_t n) {
  return (uint64_t)(((unsigned __int128)r * (unsigned __int128)n) >> 64);
}

/* Standard normal by Box-Muller from draws 2*idx and 2*idx+1. */
static inline double normal01(uint64_t seed, uint64_t stream, uint64_t idx) {
  double u1 = ((double)(syn_u64(seed, stream, 2 * idx) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
  double u2 = (double)(syn_u64(seed, stream, 2 * idx + 1) >> 11) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

enum { ST_VAL = 1, ST_LEN = 2, ST_COL = 3, ST_FILL = 4, ST_RMAT = 5, ST_X = 6 };

/* ---------------------------------------------------------------- values */

void syn_normal(int64_t n, uint64_t seed, uint64_t stream, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = normal01(seed, ST_VAL * 1000003ULL + stream, (uint64_t)i);
}

void syn_uniform(int64_t n, double lo, double hi, uint64_t seed, uint64_t stream, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    out[i] = lo + (hi - lo) * u01(seed, ST_X * 1000003ULL + stream, (uint64_t)i);
}

/* ------------------------------------------------------------- stencils */

int64_t syn_laplace2d_nnz(int64_t n) { return n <= 0 ? 0 : 5 * n * n - 4 * n; }

/* 2-D 5-point Dirichlet Laplacian on an n x n grid, row r = n*i + j.
 * Diagonal 4, the four grid neighbours -1, no wrap-around. */
void syn_laplace2d(int64_t n, int32_t* ptr, int32_t* col, double* val) {
  int64_t k = 0;
  ptr[0] = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      int64_t r = n * i + j;
      if (i > 0) { col[k] = (int32_t)(r - n); val[k++] = -1.0; }
      if (j > 0) { col[k] = (int32_t)(r - 1); val[k++] = -1.0; }
      col[k] = (int32_t)r; val[k++] = 4.0;
      if (j < n - 1) { col[k] = (int32_t)(r + 1); val[k++] = -1.0; }
      if (i < n - 1) { col[k] = (int32_t)(r + n); val[k++] = -1.0; }
      ptr[r + 1] = (int32_t)k;
    }
}

int64_t syn_stencil27_nnz(int64_t n) { return n <= 0 ? 0 : (3 * n - 2) * (3 * n - 2) * (3 * n - 2); }

static inline int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* 3-D 27-point stencil on an n^3 grid, r = (i*n + j)*n + k; every neighbour
 * with |d| <= 1 per axis, no wrap.  Columns come out sorted.  Values are
 * left to the caller (syn_normal), so only the pattern is built here. */
void syn_stencil27(int64_t n, int32_t* ptr, int32_t* col) {
  int64_t nrow = n * n * n;
  /* row lengths, then a serial scan, then a parallel fill */
  ptr[0] = 0;
  for (int64_t r = 0; r < nrow; ++r) {
    int64_t i = r / (n * n), j = (r / n) % n, k = r % n;
    int64_t ci = clampi(i + 1, 0, n - 1) - clampi(i - 1, 0, n - 1) + 1;
    int64_t cj = clampi(j + 1, 0, n - 1) - clampi(j - 1, 0, n - 1) + 1;
    int64_t ck = clampi(k + 1, 0, n - 1) - clampi(k - 1, 0, n - 1) + 1;
    ptr[r + 1] = (int32_t)(ptr[r] + ci * cj * ck);
  }
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrow; ++r) {
    int64_t i = r / (n * n), j = (r / n) % n, k = r % n;
    int64_t p = ptr[r];
    for (int64_t di = -1; di <= 1; ++di) {
      if (i + di < 0 || i + di >= n) continue;
      for (int64_t dj = -1; dj <= 1; ++dj) {
        if (j + dj < 0 || j + dj >= n) continue;
        for (int64_t dk = -1; dk <= 1; ++dk) {
          if (k + dk < 0 || k + dk >= n) continue;
          col[p++] = (int32_t)(r + di * n * n + dj * n + dk);
        }
      }
    }
  }
}

/* ------------------------------------------------------- row lengths */

/* Truncated Zipf(alpha) on {1..zmax}: CDF table, caller-sized zmax doubles. */
static double* zipf_cdf(double alpha, int64_t zmax) {
  double* cdf = (double*)malloc(sizeof(double) * (size_t)zmax);
  double s = 0.0;
  for (int64_t z = 1; z <= zmax; ++z) { s += pow((double)z, -alpha); cdf[z - 1] = s; }
  for (int64_t z = 0; z < zmax; ++z) cdf[z] /= s;
  cdf[zmax - 1] = 1.0;
  return cdf;
}

static inline int64_t zipf_draw(const double* cdf, int64_t zmax, double u) {
  int64_t lo = 0, hi = zmax - 1; /* smallest z with cdf[z] >= u */
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (cdf[mid] >= u) hi = mid; else lo = mid + 1;
  }
  return lo + 1;
}

static inline int64_t zipf_len(int64_t z, double scale, int64_t lmax) {
  double v = floor(scale * (double)z + 0.5);
  int64_t L = (int64_t)v;
  if (L < 1) L = 1;
  if (L > lmax) L = lmax;
  return L;
}

/* Exact mean of L = min(lmax, max(1, round(scale*Z))), Z ~ Zipf(alpha) on
 * {1..lmax}; used by the caller to solve `scale` for a target mean. */
double syn_zipf_mean(double alpha, double scale, int64_t lmax) {
  double* cdf = zipf_cdf(alpha, lmax);
  double m = 0.0, prev = 0.0;
  for (int64_t z = 1; z <= lmax; ++z) {
    m += (cdf[z - 1] - prev) * (double)zipf_len(z, scale, lmax);
    prev = cdf[z - 1];
  }
  free(cdf);
  return m;
}

/* Zipf row lengths, capped by ncols. */
void syn_lens_zipf(int64_t M, int64_t ncols, double alpha, double scale, int64_t lmax, uint64_t seed,
                   int32_t* len) {
  double* cdf = zipf_cdf(alpha, lmax);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < M; ++i) {
    int64_t L = zipf_len(zipf_draw(cdf, lmax, u01(seed, ST_LEN, (uint64_t)i)), scale, lmax);
    len[i] = (int32_t)(L > ncols ? ncols : L);
  }
  free(cdf);
}

/* Poisson(mean) row lengths by CDF inversion (mean <= ~700), capped by ncols;
 * stands in for Binomial(ncols, mean/ncols) at ncols >> mean. */
void syn_lens_poisson(int64_t M, int64_t ncols, double mean, uint64_t seed, int32_t* len) {
  double p0 = exp(-mean);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < M; ++i) {
    double u = u01(seed, ST_LEN, (uint64_t)i);
    double p = p0, c = p0;
    int64_t k = 0;
    while (u > c && k < ncols) { ++k; p *= mean / (double)k; c += p; if (p == 0.0 && c < u) break; }
    len[i] = (int32_t)(k > ncols ? ncols : k);
  }
}

/* Uniform row lengths in [lo, hi] (inclusive), capped by ncols. */
void syn_lens_uniform_int(int64_t M, int64_t ncols, int64_t lo, int64_t hi, uint64_t seed, int32_t* len) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < M; ++i) {
    int64_t L = lo + (int64_t)uint_below(syn_u64(seed, ST_LEN, (uint64_t)i), (uint64_t)(hi - lo + 1));
    len[i] = (int32_t)(L > ncols ? ncols : L);
  }
}

/* ------------------------------------------------ random column sets */

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* For each row i, draw len_i = ptr[i+1]-ptr[i] distinct columns uniformly
 * from [0, ncols) by Floyd's sampling, then sort them ascending. */
void syn_fill_random_cols(int64_t M, int64_t ncols, const int32_t* ptr, uint64_t seed, int32_t* col) {
#pragma omp parallel
  {
    int64_t cap = 0;
    int64_t* table = NULL;
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < M; ++i) {
      int64_t L = ptr[i + 1] - ptr[i];
      int32_t* out = col + ptr[i];
      if (L == 0) continue;
      int64_t need = 16;
      while (need < 2 * L) need <<= 1;
      if (need > cap) { free(table); cap = need; table = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap); }
      for (int64_t h = 0; h < need; ++h) table[h] = -1;
      int64_t m = 0;
      for (int64_t j = ncols - L; j < ncols; ++j, ++m) {
        int64_t t = (int64_t)uint_below(syn_u64(seed, ST_COL, (uint64_t)ptr[i] + (uint64_t)m), (uint64_t)(j + 1));
        /* insert t, or j if t is already present */
        int64_t pick = t;
        for (int pass = 0; pass < 2; ++pass) {
          uint64_t h = mix64((uint64_t)pick) & (uint64_t)(need - 1);
          int found = 0;
          while (table[h] != -1) {
            if (table[h] == pick) { found = 1; break; }
            h = (h + 1) & (uint64_t)(need - 1);
          }
          if (!found) { table[h] = pick; out[m] = (int32_t)pick; break; }
          pick = j; /* j has never been drawn before (all earlier draws are < j) */
        }
      }
      qsort(out, (size_t)L, sizeof(int32_t), cmp_i32);
    }
    free(table);
  }
}

/* ------------------------------------------- banded / block-diagonal */

/* Banded: row i keeps column j in [i-hw, i+hw] with probability `fill`,
 * always keeping the diagonal when it exists.  Pass col == NULL to count. */
void syn_banded(int64_t M, int64_t N, int64_t hw, double fill, uint64_t seed, int32_t* len_or_null,
                const int32_t* ptr, int32_t* col) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < M; ++i) {
    int64_t lo = i - hw < 0 ? 0 : i - hw, hi = i + hw > N - 1 ? N - 1 : i + hw;
    int64_t c = 0;
    int32_t* out = col ? col + ptr[i] : NULL;
    for (int64_t j = lo; j <= hi; ++j) {
      int keep = (j == i) || u01(seed, ST_FILL, (uint64_t)i * 1048583ULL + (uint64_t)(j - i + hw)) < fill;
      if (keep) { if (out) out[c] = (int32_t)j; ++c; }
    }
    if (len_or_null) len_or_null[i] = (int32_t)c;
  }
}

/* Block-diagonal: blocks of `bs` rows/cols; inside its block, row i keeps
 * each column with probability `dens`, always keeping the diagonal. */
void syn_blockdiag(int64_t M, int64_t N, int64_t bs, double dens, uint64_t seed, int32_t* len_or_null,
                   const int32_t* ptr, int32_t* col) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < M; ++i) {
    int64_t b0 = (i / bs) * bs, b1 = b0 + bs > N ? N : b0 + bs;
    int64_t c = 0;
    int32_t* out = col ? col + ptr[i] : NULL;
    for (int64_t j = b0; j < b1; ++j) {
      int keep = (j == i) || u01(seed, ST_FILL, (uint64_t)i * 1048583ULL + (uint64_t)(j - b0)) < dens;
      if (keep) { if (out) out[c] = (int32_t)j; ++c; }
    }
    if (len_or_null) len_or_null[i] = (int32_t)c;
  }
}

/* --------------------------------------------------------------- R-MAT */

/* R-MAT edge list (Chakrabarti, Zhan, Faloutsos 2004): each edge descends
 * `scale` levels, picking quadrant (0,0),(0,1),(1,0),(1,1) with probability
 * a, b, c, 1-a-b-c; the first level picks the most significant bit.  No
 * noise, no relabelling.  Duplicates are kept: they are the consumer's job. */
void syn_rmat(int64_t scale, int64_t nedges, double a, double b, double c, uint64_t seed, int32_t* row,
              int32_t* col) {
  double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < nedges; ++e) {
    uint64_t r = 0, q = 0;
    for (int64_t l = 0; l < scale; ++l) {
      double u = u01(seed, ST_RMAT, (uint64_t)e * (uint64_t)scale + (uint64_t)l);
      uint64_t rb = u >= ab, cb = (u >= a && u < ab) || u >= abc;
      r = (r << 1) | rb;
      q = (q << 1) | cb;
    }
    row[e] = (int32_t)r;
    col[e] = (int32_t)q;
  }
}

/* Prefix sum of row lengths into a CSR row pointer; returns nnz, or -1 when
 * it would overflow int32. */
int64_t syn_lens_to_ptr(int64_t M, const int32_t* len, int32_t* ptr) {
  int64_t s = 0;
  ptr[0] = 0;
  for (int64_t i = 0; i < M; ++i) {
    s += len[i];
    if (s > 2147483647LL) return -1;
    ptr[i + 1] = (int32_t)s;
  }
  return s;
}
