/*
 * Host-only driver for the AddressSanitizer / UndefinedBehaviorSanitizer build
 * of the CPU oracle (oracle/spmv_oracle.c) and the seeded input generators
 * (paper_1805_11938_amd/synth/synth.c).  tests/test_sanitizers.py compiles the
 * three files with -fsanitize=address,undefined and runs this program: every
 * generator and every oracle routine runs on small matrices of each kind
 * (with empty rows, one long row, duplicates in COO input), round trips are
 * checked, and any out-of-bounds access, leak or undefined operation aborts
 * the run.  Test infrastructure; nothing of the library is linked.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* generators */
void syn_normal(int64_t n, uint64_t seed, uint64_t stream, double* out);
void syn_uniform(int64_t n, double lo, double hi, uint64_t seed, uint64_t stream, double* out);
int64_t syn_laplace2d_nnz(int64_t n);
void syn_laplace2d(int64_t n, int32_t* ptr, int32_t* col, double* val);
int64_t syn_stencil27_nnz(int64_t n);
void syn_stencil27(int64_t n, int32_t* ptr, int32_t* col);
double syn_zipf_mean(double alpha, double scale, int64_t lmax);
void syn_lens_zipf(int64_t M, int64_t ncols, double alpha, double scale, int64_t lmax, uint64_t seed, int32_t* len);
void syn_lens_poisson(int64_t M, int64_t ncols, double mean, uint64_t seed, int32_t* len);
void syn_lens_uniform_int(int64_t M, int64_t ncols, int64_t lo, int64_t hi, uint64_t seed, int32_t* len);
void syn_fill_random_cols(int64_t M, int64_t ncols, const int32_t* ptr, uint64_t seed, int32_t* col);
void syn_banded(int64_t M, int64_t N, int64_t hw, double fill, uint64_t seed, int32_t* len_or_null,
                const int32_t* ptr, int32_t* col);
void syn_blockdiag(int64_t M, int64_t N, int64_t bs, double dens, uint64_t seed, int32_t* len_or_null,
                   const int32_t* ptr, int32_t* col);
void syn_rmat(int64_t scale, int64_t nedges, double a, double b, double c, uint64_t seed, int32_t* row, int32_t* col);
int64_t syn_lens_to_ptr(int64_t M, const int32_t* len, int32_t* ptr);

/* oracle */
int orc_coo_to_csr(int64_t M, int64_t N, int64_t n, const int32_t* row, const int32_t* col, const double* val,
                   int32_t* ptr, int32_t* ocol, double* oval, int64_t* nnz_out);
int orc_csr_check(int64_t M, int64_t N, int64_t nnz, const int32_t* ptr, const int32_t* col);
void orc_csr_spmv(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, const double* x, double* y);
int orc_csr_spmv_omp(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, const double* x, double* y,
                     int nthreads);
void orc_csr_absspmv(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, const double* x,
                     double* y);
void orc_csr_spmm(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, int64_t kk, const double* X,
                  int64_t ldx, double* Y, int64_t ldy);
int64_t orc_max_row_len(int64_t M, const int32_t* ptr);
void orc_csr_to_ell(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, int64_t K, int32_t* ecol,
                    double* eval);
void orc_ell_spmv(int64_t M, int64_t K, const int32_t* ecol, const double* eval, const double* x, double* y);
int64_t orc_ell_to_csr(int64_t M, int64_t K, const int32_t* ecol, const double* eval, int32_t* ptr, int32_t* col,
                       double* val);
int64_t orc_sell_layout(int64_t M, int64_t C, int64_t sigma, const int32_t* ptr, int32_t* perm, int32_t* widths,
                        int64_t* cs);
void orc_csr_to_sell(int64_t M, int64_t C, const int32_t* ptr, const int32_t* col, const double* val,
                     const int32_t* perm, const int32_t* widths, const int64_t* cs, int32_t* scol, double* sval);
void orc_sell_spmv(int64_t M, int64_t C, const int32_t* perm, const int32_t* widths, const int64_t* cs,
                   const int32_t* scol, const double* sval, const double* x, double* y);
int64_t orc_sell_to_csr(int64_t M, int64_t C, const int32_t* perm, const int32_t* widths, const int64_t* cs,
                        const int32_t* scol, const double* sval, int32_t* ptr, int32_t* col, double* val);
int64_t orc_hyb_k_rule(int64_t M, const int32_t* ptr);
int64_t orc_hyb_coo_count(int64_t M, const int32_t* ptr, int64_t K);
void orc_csr_to_hyb(int64_t M, const int32_t* ptr, const int32_t* col, const double* val, int64_t K, int32_t* ecol,
                    double* eval, int32_t* crow, int32_t* ccol, double* cval);
void orc_hyb_spmv(int64_t M, int64_t K, const int32_t* ecol, const double* eval, int64_t ncoo, const int32_t* crow,
                  const int32_t* ccol, const double* cval, const double* x, double* y);
int64_t orc_hyb_to_csr(int64_t M, int64_t K, const int32_t* ecol, const double* eval, int64_t ncoo,
                       const int32_t* crow, const int32_t* ccol, const double* cval, int32_t* ptr, int32_t* col,
                       double* val);
int64_t orc_csr5_ntiles(int64_t nnz, int64_t omega, int64_t sigma);
void orc_csr_to_csr5(int64_t M, int64_t nnz, const int32_t* ptr, const int32_t* col, const double* val, int64_t omega,
                     int64_t sigma, int32_t* tile_ptr, uint32_t* flags, int32_t* y_off, int32_t* seg_off,
                     int32_t* tcol, double* tval);
void orc_csr5_spmv(int64_t M, int64_t nnz, const int32_t* ptr, int64_t omega, int64_t sigma, const int32_t* tile_ptr,
                   const uint32_t* flags, const int32_t* tcol, const double* tval, const int32_t* tail_col,
                   const double* tail_val, const double* x, double* y);
void orc_csr5_to_csr(int64_t nnz, int64_t omega, int64_t sigma, const int32_t* tcol, const double* tval,
                     const int32_t* tail_col, const double* tail_val, int32_t* col, double* val);
void orc_features(int64_t M, int64_t N, const int32_t* ptr, const int32_t* col, double* f);

static int failures = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                         \
    }                                                                     \
  } while (0)

static void* xmalloc(size_t n) {
  void* p = malloc(n ? n : 1);
  if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
  return p;
}

/* worst row-wise relative error of y against yref */
static double rel_err(int64_t M, const double* y, const double* yref, const double* den) {
  double e = 0.0;
  for (int64_t i = 0; i < M; ++i) {
    double d = fabs(y[i] - yref[i]);
    if (den[i] == 0.0) { if (d != 0.0) return INFINITY; continue; }
    if (d / den[i] > e) e = d / den[i];
  }
  return e;
}

static int same_csr(int64_t M, int64_t nnz, const int32_t* p0, const int32_t* c0, const double* v0,
                    const int32_t* p1, const int32_t* c1, const double* v1) {
  return !memcmp(p0, p1, sizeof(int32_t) * (size_t)(M + 1)) && !memcmp(c0, c1, sizeof(int32_t) * (size_t)nnz) &&
         !memcmp(v0, v1, sizeof(double) * (size_t)nnz);
}

/* every format of the oracle on one CSR matrix */
static void exercise(const char* name, int64_t M, int64_t N, const int32_t* ptr, const int32_t* col,
                     const double* val) {
  const int64_t nnz = ptr[M];
  CHECK(orc_csr_check(M, N, nnz, ptr, col) == 0);
  double* x = (double*)xmalloc(sizeof(double) * (size_t)N);
  double* y = (double*)xmalloc(sizeof(double) * (size_t)M);
  double* yr = (double*)xmalloc(sizeof(double) * (size_t)M);
  double* den = (double*)xmalloc(sizeof(double) * (size_t)M);
  int32_t* p2 = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(M + 1));
  int32_t* c2 = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nnz);
  double* v2 = (double*)xmalloc(sizeof(double) * (size_t)nnz);
  syn_uniform(N, -1.0, 1.0, 77, 0, x);
  orc_csr_spmv(M, ptr, col, val, x, yr);
  orc_csr_absspmv(M, ptr, col, val, x, den);
  CHECK(orc_csr_spmv_omp(M, ptr, col, val, x, y, 3) >= 1);
  CHECK(!memcmp(y, yr, sizeof(double) * (size_t)M));
  /* SpMM with padded leading dimensions */
  {
    const int64_t k = 3, ldx = 5, ldy = 4;
    double* X = (double*)xmalloc(sizeof(double) * (size_t)(N * ldx));
    double* Y = (double*)xmalloc(sizeof(double) * (size_t)(M * ldy));
    for (int64_t j = 0; j < N; ++j)
      for (int64_t c = 0; c < ldx; ++c) X[j * ldx + c] = x[j];
    orc_csr_spmm(M, ptr, col, val, k, X, ldx, Y, ldy);
    for (int64_t i = 0; i < M; ++i) CHECK(Y[i * ldy + 2] == yr[i]);
    free(X);
    free(Y);
  }
  /* ELL */
  {
    const int64_t K = orc_max_row_len(M, ptr);
    int32_t* ec = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(M * K));
    double* ev = (double*)xmalloc(sizeof(double) * (size_t)(M * K));
    orc_csr_to_ell(M, ptr, col, val, K, ec, ev);
    orc_ell_spmv(M, K, ec, ev, x, y);
    CHECK(rel_err(M, y, yr, den) <= 1e-14);
    CHECK(orc_ell_to_csr(M, K, ec, ev, p2, c2, v2) == nnz);
    CHECK(same_csr(M, nnz, ptr, col, val, p2, c2, v2));
    free(ec);
    free(ev);
  }
  /* SELL-C-sigma */
  {
    const int64_t Cs[3] = {1, 4, 32}, sigmas[3] = {1, 8, 1 << 20};
    for (int a = 0; a < 3; ++a) {
      const int64_t C = Cs[a], sg = sigmas[a], nch = (M + C - 1) / C;
      int32_t* perm = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(nch * C));
      int32_t* wid = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nch);
      int64_t* cs = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(nch + 1));
      const int64_t ns = orc_sell_layout(M, C, sg, ptr, perm, wid, cs);
      int32_t* sc = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)ns);
      double* sv = (double*)xmalloc(sizeof(double) * (size_t)ns);
      orc_csr_to_sell(M, C, ptr, col, val, perm, wid, cs, sc, sv);
      orc_sell_spmv(M, C, perm, wid, cs, sc, sv, x, y);
      CHECK(rel_err(M, y, yr, den) <= 1e-14);
      CHECK(orc_sell_to_csr(M, C, perm, wid, cs, sc, sv, p2, c2, v2) == nnz);
      CHECK(same_csr(M, nnz, ptr, col, val, p2, c2, v2));
      free(perm);
      free(wid);
      free(cs);
      free(sc);
      free(sv);
    }
  }
  /* HYB with the rule's K and two others */
  {
    const int64_t Ks[3] = {orc_hyb_k_rule(M, ptr), 0, 2};
    for (int a = 0; a < 3; ++a) {
      const int64_t K = Ks[a], nc = orc_hyb_coo_count(M, ptr, K);
      int32_t* ec = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(M * K));
      double* ev = (double*)xmalloc(sizeof(double) * (size_t)(M * K));
      int32_t* cr = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nc);
      int32_t* cc = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nc);
      double* cv = (double*)xmalloc(sizeof(double) * (size_t)nc);
      orc_csr_to_hyb(M, ptr, col, val, K, ec, ev, cr, cc, cv);
      orc_hyb_spmv(M, K, ec, ev, nc, cr, cc, cv, x, y);
      CHECK(rel_err(M, y, yr, den) <= 1e-14);
      CHECK(orc_hyb_to_csr(M, K, ec, ev, nc, cr, cc, cv, p2, c2, v2) == nnz);
      CHECK(same_csr(M, nnz, ptr, col, val, p2, c2, v2));
      free(ec);
      free(ev);
      free(cr);
      free(cc);
      free(cv);
    }
  }
  /* CSR5 at several tile shapes */
  {
    const int64_t ws[3] = {2, 16, 64}, ss[3] = {2, 3, 16};
    for (int a = 0; a < 3; ++a) {
      const int64_t w = ws[a], s = ss[a], T = orc_csr5_ntiles(nnz, w, s), W = w * s;
      int32_t* tp = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(T + 1));
      uint32_t* fl = (uint32_t*)xmalloc(sizeof(uint32_t) * (size_t)(T * w));
      int32_t* yo = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(T * w));
      int32_t* so = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(T * w));
      int32_t* tc = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(T * W));
      double* tv = (double*)xmalloc(sizeof(double) * (size_t)(T * W));
      orc_csr_to_csr5(M, nnz, ptr, col, val, w, s, tp, fl, yo, so, tc, tv);
      orc_csr5_spmv(M, nnz, ptr, w, s, tp, fl, tc, tv, col + T * W, val + T * W, x, y);
      CHECK(rel_err(M, y, yr, den) <= 1e-14);
      orc_csr5_to_csr(nnz, w, s, tc, tv, col + T * W, val + T * W, c2, v2);
      CHECK(!memcmp(c2, col, sizeof(int32_t) * (size_t)nnz) && !memcmp(v2, val, sizeof(double) * (size_t)nnz));
      free(tp);
      free(fl);
      free(yo);
      free(so);
      free(tc);
      free(tv);
    }
  }
  {
    double f[12];
    orc_features(M, N, ptr, col, f);
    CHECK(f[0] == (double)M && f[2] == (double)nnz);
  }
  free(x);
  free(y);
  free(yr);
  free(den);
  free(p2);
  free(c2);
  free(v2);
  fprintf(stderr, "%s: M=%lld nnz=%lld ok\n", name, (long long)M, (long long)nnz);
}

/* CSR from lengths and random distinct columns */
static void random_cols_case(const char* name, int64_t M, int64_t N, int32_t* len) {
  int32_t* ptr = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(M + 1));
  const int64_t nnz = syn_lens_to_ptr(M, len, ptr);
  CHECK(nnz >= 0);
  int32_t* col = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nnz);
  double* val = (double*)xmalloc(sizeof(double) * (size_t)nnz);
  syn_fill_random_cols(M, N, ptr, 5, col);
  syn_normal(nnz, 6, 0, val);
  exercise(name, M, N, ptr, col, val);
  free(ptr);
  free(col);
  free(val);
}

int main(void) {
  /* Laplacian */
  {
    const int64_t n = 9, M = n * n, nnz = syn_laplace2d_nnz(n);
    int32_t* ptr = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(M + 1));
    int32_t* col = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nnz);
    double* val = (double*)xmalloc(sizeof(double) * (size_t)nnz);
    syn_laplace2d(n, ptr, col, val);
    exercise("laplace2d_9", M, M, ptr, col, val);
    free(ptr);
    free(col);
    free(val);
  }
  /* 27-point stencil */
  {
    const int64_t n = 5, M = n * n * n, nnz = syn_stencil27_nnz(n);
    int32_t* ptr = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(M + 1));
    int32_t* col = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nnz);
    double* val = (double*)xmalloc(sizeof(double) * (size_t)nnz);
    syn_stencil27(n, ptr, col);
    syn_normal(nnz, 2, 0, val);
    exercise("stencil27_5", M, M, ptr, col, val);
    free(ptr);
    free(col);
    free(val);
  }
  /* Zipf, Poisson and uniform row lengths with random columns (empty rows included) */
  {
    const int64_t M = 700, N = 650;
    int32_t* len = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)M);
    const double mean = syn_zipf_mean(2.0, 1.5, 600);
    CHECK(mean > 1.0);
    syn_lens_zipf(M, N, 2.0, 1.5, 600, 4, len);
    random_cols_case("zipf_700", M, N, len);
    syn_lens_poisson(M, N, 3.0, 8, len);
    random_cols_case("poisson_700", M, N, len);
    syn_lens_uniform_int(M, N, 0, 40, 9, len);
    random_cols_case("uniform_700", M, N, len);
    free(len);
  }
  /* banded and block-diagonal (count pass, then fill) */
  for (int kind = 0; kind < 2; ++kind) {
    const int64_t M = 500, N = 500;
    int32_t* len = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)M);
    int32_t* ptr = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(M + 1));
    if (kind == 0) syn_banded(M, N, 7, 0.4, 3, len, NULL, NULL);
    else syn_blockdiag(M, N, 24, 0.3, 3, len, NULL, NULL);
    const int64_t nnz = syn_lens_to_ptr(M, len, ptr);
    int32_t* col = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nnz);
    double* val = (double*)xmalloc(sizeof(double) * (size_t)nnz);
    if (kind == 0) syn_banded(M, N, 7, 0.4, 3, NULL, ptr, col);
    else syn_blockdiag(M, N, 24, 0.3, 3, NULL, ptr, col);
    syn_normal(nnz, 4, 0, val);
    exercise(kind == 0 ? "banded_500" : "blockdiag_500", M, N, ptr, col, val);
    free(len);
    free(ptr);
    free(col);
    free(val);
  }
  /* R-MAT edges with duplicates, canonicalised by the oracle */
  {
    const int64_t scale = 9, M = (int64_t)1 << scale, ne = 6000;
    int32_t* row = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)ne);
    int32_t* col = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)ne);
    double* val = (double*)xmalloc(sizeof(double) * (size_t)ne);
    syn_rmat(scale, ne, 0.57, 0.19, 0.19, 10, row, col);
    syn_normal(ne, 12, 0, val);
    int32_t* ptr = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)(M + 1));
    int32_t* oc = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)ne);
    double* ov = (double*)xmalloc(sizeof(double) * (size_t)ne);
    int64_t nnz = 0;
    CHECK(orc_coo_to_csr(M, M, ne, row, col, val, ptr, oc, ov, &nnz) == 0);
    CHECK(nnz > 0 && nnz <= ne);
    exercise("rmat_9", M, M, ptr, oc, ov);
    row[0] = (int32_t)M; /* out of range is refused, not read past */
    CHECK(orc_coo_to_csr(M, M, ne, row, col, val, ptr, oc, ov, &nnz) == -2);
    free(row);
    free(col);
    free(val);
    free(ptr);
    free(oc);
    free(ov);
  }
  /* one long row among empty rows */
  {
    const int64_t M = 40, N = 300;
    int32_t* len = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)M);
    for (int64_t i = 0; i < M; ++i) len[i] = i == 17 ? 300 : 0;
    random_cols_case("one_long_row", M, N, len);
    free(len);
  }
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  fprintf(stderr, "all sanitizer cases passed\n");
  return 0;
}
