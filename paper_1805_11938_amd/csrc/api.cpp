// C-ABI of libspmv: argument checking, handle lifetime, format dispatch and
// array export.  All arithmetic happens in the kernels of the .hip files.
#include <cstdlib>
#include <cstring>
#include <new>

#include "common.h"

namespace spmv {

const char* last_error_cstr();
spmv_status_t mat_from_csr(int64_t M, int64_t N, int64_t nnz, const int32_t* ptr, const int32_t* col, const void* val,
                           spmv_dtype_t dt, int on_dev, uint32_t flags, hipStream_t s, spmv_mat_s* A);
spmv_status_t mat_from_coo(int64_t M, int64_t N, int64_t n, const int32_t* row, const int32_t* col, const void* val,
                           spmv_dtype_t dt, int on_dev, hipStream_t s, spmv_mat_s* A);
spmv_status_t ell_sell_hyb_to_csr(spmv_mat_s* A, int32_t* ptr, int32_t* col, void* val, hipStream_t s);
spmv_status_t csr5_to_csr(spmv_mat_s* A, int32_t* ptr, int32_t* col, void* val, hipStream_t s);

spmv_status_t mat_alloc(spmv_mat_s* A, void** p, size_t bytes) {
  SPMV_TRY(dmalloc(p, bytes));
  A->own(*p);
  return SPMV_OK;
}

void resolve_params(const spmv_params_t* in, spmv_params_t* out) {
  spmv_params_t d;
  d.sell_C = 32;
  d.sell_sigma = 1;
  d.csr_lanes_per_row = 0;
  d.hyb_K = -1;
  d.csr5_omega = 64;
  d.csr5_sigma = 16;
  d.max_bytes = 0;
  d.flags = 0;
  d.bands = 1;
  if (in) {
    if (in->sell_C > 0) d.sell_C = in->sell_C;
    if (in->sell_sigma > 0) d.sell_sigma = in->sell_sigma;
    if (in->csr_lanes_per_row > 0) d.csr_lanes_per_row = in->csr_lanes_per_row;
    d.hyb_K = in->hyb_K;
    if (in->csr5_omega > 0) d.csr5_omega = in->csr5_omega;
    if (in->csr5_sigma > 0) d.csr5_sigma = in->csr5_sigma;
    if (in->max_bytes > 0) d.max_bytes = in->max_bytes;
    d.flags = in->flags;
    if (in->bands > 0) d.bands = in->bands;
  }
  *out = d;
}

int64_t bytes_min(const spmv_mat_s* A) {
  return A->nnz * (A->sv + 4) + 4 * (A->M + 1) + A->N * A->sv + A->M * A->sv;
}

spmv_status_t dispatch_run(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  // the kernels address x, and ELL/SELL columns, with 32-bit byte offsets
  if (A->N * A->sv >= ((int64_t)1 << 32) || A->M * A->sv >= ((int64_t)1 << 32))
    return fail(SPMV_ERR_UNSUPPORTED, "x or y larger than 4 GiB");
  if (!A->sub.empty()) return run_banded(A, x, y, s);
  switch (A->fmt) {
    case SPMV_FMT_CSR: return run_csr(A, x, y, s);
    case SPMV_FMT_CSR5: return run_csr5(A, x, y, s);
    case SPMV_FMT_ELL: return run_ell(A, x, y, s);
    case SPMV_FMT_SELL: return run_sell(A, x, y, s);
    case SPMV_FMT_HYB: return run_hyb(A, x, y, s);
  }
  return fail(SPMV_ERR_INVALID_ARG, "unknown format %d", (int)A->fmt);
}

static spmv_status_t check_sizes(int64_t M, int64_t N, int64_t nnz) {
  const int64_t lim = (int64_t)INT32_MAX;
  if (M < 0 || N < 0 || nnz < 0) return fail(SPMV_ERR_INVALID_ARG, "negative size");
  if (M >= lim || N >= lim || nnz >= lim) return fail(SPMV_ERR_TOO_LARGE, "sizes must be < 2^31 (int32 indices)");
  return SPMV_OK;
}

static void destroy(spmv_mat_s* A) {
  if (!A) return;
  for (void* p : A->owned) dfree(p);
  delete A;
}

template <class F>
static spmv_status_t build_handle(spmv_mat_t* out, F&& f) {
  if (!out) return fail(SPMV_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  spmv_mat_s* A = new (std::nothrow) spmv_mat_s();
  if (!A) return fail(SPMV_ERR_OOM, "host allocation failed");
  spmv_status_t st = f(A);
  if (st != SPMV_OK) {
    destroy(A);
    return st;
  }
  *out = A;
  return SPMV_OK;
}


// a CSR handle of its own (copies of src's arrays) with the kernel variant's
// tables: row blocks, wave units, and, by flag, wave tiles or XCD bands
spmv_status_t convert_csr(spmv_mat_s* src, spmv_mat_s* A, hipStream_t st) {
  const int V = A->params.csr_lanes_per_row;
  if (V < 0 || V > 64 || (V & (V - 1))) return fail(SPMV_ERR_UNSUPPORTED, "csr_lanes_per_row=%d", V);
  SPMV_TRY(mat_alloc(A, (void**)&A->ptr, sizeof(int32_t) * (A->M + 1)));
  SPMV_TRY(mat_alloc(A, (void**)&A->col, sizeof(int32_t) * A->nnz));
  SPMV_TRY(mat_alloc(A, &A->val, (size_t)A->sv * A->nnz));
  SPMV_HIP(hipMemcpyAsync(A->ptr, src->ptr, sizeof(int32_t) * (A->M + 1), hipMemcpyDeviceToDevice, st));
  if (A->nnz) {
    SPMV_HIP(hipMemcpyAsync(A->col, src->col, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToDevice, st));
    SPMV_HIP(hipMemcpyAsync(A->val, src->val, (size_t)A->sv * A->nnz, hipMemcpyDeviceToDevice, st));
  }
  SPMV_TRY(csr_build_blocks(A, st));
  A->bytes_fmt = bytes_min(A);
  if ((A->params.flags & SPMV_FLAG_CSR_TILES) && V == 0) SPMV_TRY(csr_build_tiles(A, st));
  if (A->params.flags & SPMV_FLAG_CSR_BANDS) {
    SPMV_TRY(csr_build_bands(A, st));
    A->bytes_fmt += (int64_t)(A->nbands - 1) * 4 * (A->M + 1);  // one row pointer per band
  }
  SPMV_HIP(hipStreamSynchronize(st));
  return SPMV_OK;
}
}  // namespace spmv

using namespace spmv;

extern "C" {

const char* spmv_status_str(spmv_status_t st) {
  switch (st) {
    case SPMV_OK: return "ok";
    case SPMV_ERR_INVALID_ARG: return "invalid argument";
    case SPMV_ERR_BAD_STRUCTURE: return "bad matrix structure";
    case SPMV_ERR_OOM: return "out of memory";
    case SPMV_ERR_TOO_LARGE: return "too large";
    case SPMV_ERR_UNSUPPORTED: return "unsupported";
    case SPMV_ERR_HIP: return "HIP error";
    case SPMV_ERR_MODEL: return "model error";
  }
  return "unknown status";
}

const char* spmv_last_error(void) { return last_error_cstr(); }

int64_t spmv_mem_in_use(void) { return mem_in_use(); }
int64_t spmv_mem_release(void) { return mem_release(); }

spmv_status_t spmv_mat_from_csr(int64_t M, int64_t N, int64_t nnz, const int32_t* ptr, const int32_t* col,
                                const void* val, spmv_dtype_t dt, int src_on_device, uint32_t flags, spmv_stream_t s,
                                spmv_mat_t* out) {
  SPMV_TRY(check_sizes(M, N, nnz));
  if (dt != SPMV_F64 && dt != SPMV_F32) return fail(SPMV_ERR_INVALID_ARG, "dtype %d", (int)dt);
  if (!ptr || (nnz > 0 && (!col || !val))) return fail(SPMV_ERR_INVALID_ARG, "null array");
  return build_handle(out, [&](spmv_mat_s* A) {
    return mat_from_csr(M, N, nnz, ptr, col, val, dt, src_on_device, flags, hs(s), A);
  });
}

spmv_status_t spmv_mat_from_coo(int64_t M, int64_t N, int64_t n, const int32_t* row, const int32_t* col,
                                const void* val, spmv_dtype_t dt, int src_on_device, spmv_stream_t s, spmv_mat_t* out) {
  SPMV_TRY(check_sizes(M, N, n));
  if (dt != SPMV_F64 && dt != SPMV_F32) return fail(SPMV_ERR_INVALID_ARG, "dtype %d", (int)dt);
  if (n > 0 && (!row || !col || !val)) return fail(SPMV_ERR_INVALID_ARG, "null array");
  return build_handle(out, [&](spmv_mat_s* A) {
    return mat_from_coo(M, N, n, row, col, val, dt, src_on_device, hs(s), A);
  });
}


spmv_status_t spmv_convert(spmv_mat_t csr, spmv_fmt_t fmt, const spmv_params_t* p, spmv_stream_t s, spmv_mat_t* out) {
  if (!csr || csr->fmt != SPMV_FMT_CSR || !csr->sub.empty())
    return fail(SPMV_ERR_INVALID_ARG, "convert needs a CSR handle without column bands");
  if ((int)fmt < 0 || (int)fmt >= SPMV_NUM_FORMATS) return fail(SPMV_ERR_INVALID_ARG, "format %d", (int)fmt);
  hipStream_t st = hs(s);
  return build_handle(out, [&](spmv_mat_s* A) -> spmv_status_t {
    A->fmt = fmt;
    A->dt = csr->dt;
    A->M = csr->M;
    A->N = csr->N;
    A->nnz = csr->nnz;
    A->sv = csr->sv;
    resolve_params(p, &A->params);
    if (A->params.bands > 1 && fmt != SPMV_FMT_HYB) return convert_banded(csr, A, st);
    switch (fmt) {
      case SPMV_FMT_CSR: return convert_csr(csr, A, st);
      case SPMV_FMT_ELL: return convert_ell(csr, A, st);
      case SPMV_FMT_SELL: return convert_sell(csr, A, st);
      case SPMV_FMT_HYB: return convert_hyb(csr, A, st);
      case SPMV_FMT_CSR5: return convert_csr5(csr, A, st);
    }
    return fail(SPMV_ERR_INVALID_ARG, "format");
  });
}

spmv_status_t spmv_to_csr(spmv_mat_t A, int32_t* ptr, int32_t* col, void* val, int dst_on_device, spmv_stream_t s) {
  if (!A || !ptr || (A->nnz && (!col || !val))) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  hipStream_t st = hs(s);
  int32_t *dp = ptr, *dc = col;
  void* dv = val;
  DTmp tp, tc, tv;
  if (!dst_on_device) {
    SPMV_TRY(tp.alloc(sizeof(int32_t) * (A->M + 1)));
    SPMV_TRY(tc.alloc(sizeof(int32_t) * A->nnz));
    SPMV_TRY(tv.alloc((size_t)A->sv * A->nnz));
    dp = tp.as<int32_t>();
    dc = tc.as<int32_t>();
    dv = tv.p;
  }
  if (!A->sub.empty()) {
    SPMV_TRY(banded_to_csr(A, dp, dc, dv, st));
  } else switch (A->fmt) {
    case SPMV_FMT_CSR:
      SPMV_HIP(hipMemcpyAsync(dp, A->ptr, sizeof(int32_t) * (A->M + 1), hipMemcpyDeviceToDevice, st));
      if (A->nnz) {
        SPMV_HIP(hipMemcpyAsync(dc, A->col, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToDevice, st));
        SPMV_HIP(hipMemcpyAsync(dv, A->val, (size_t)A->sv * A->nnz, hipMemcpyDeviceToDevice, st));
      }
      break;
    case SPMV_FMT_CSR5: SPMV_TRY(csr5_to_csr(A, dp, dc, dv, st)); break;
    default: SPMV_TRY(ell_sell_hyb_to_csr(A, dp, dc, dv, st)); break;
  }
  if (!dst_on_device) {
    SPMV_HIP(hipMemcpyAsync(ptr, dp, sizeof(int32_t) * (A->M + 1), hipMemcpyDeviceToHost, st));
    if (A->nnz) {
      SPMV_HIP(hipMemcpyAsync(col, dc, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToHost, st));
      SPMV_HIP(hipMemcpyAsync(val, dv, (size_t)A->sv * A->nnz, hipMemcpyDeviceToHost, st));
    }
    SPMV_HIP(hipStreamSynchronize(st));
  }
  return SPMV_OK;
}

static spmv_status_t lookup(spmv_mat_t A, const char* name, const void** p, size_t* bytes) {
  if (!A || !name) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  if (!strncmp(name, "band", 4) && name[4] >= '0' && name[4] <= '9') {  // "band<b>.<array>" of a banded SELL
    char* rest = nullptr;
    const long b = strtol(name + 4, &rest, 10);
    if (*rest != '.' || b < 0 || b >= (long)A->sub.size())
      return fail(SPMV_ERR_INVALID_ARG, "array '%s' does not exist for this handle", name);
    return lookup(A->sub[b].get(), rest + 1, p, bytes);
  }
  const bool own = A->sub.empty();  // a banded handle keeps its arrays in its bands
  const bool sell = A->fmt == SPMV_FMT_SELL && own;
  const int64_t sv = A->sv, M = A->M, nnz = A->nnz;
  const int64_t TW = A->ntiles * (int64_t)A->omega * A->c5sigma;
  struct Entry {
    const char* n;
    int ok;
    const void* p;
    int64_t b;
  } tab[] = {
      {"ptr", (A->fmt == SPMV_FMT_CSR || A->fmt == SPMV_FMT_CSR5) && own, A->ptr, 4 * (M + 1)},
      {"band_ptr", A->nbands > 0, A->bptr, 4 * (int64_t)A->nbands * (M + 1)},
      {"band_col", A->nbands > 0, A->bcol, 4 * nnz},
      {"band_val", A->nbands > 0, A->bval, sv * nnz},
      {"col", A->fmt == SPMV_FMT_CSR, A->col, 4 * nnz},
      {"val", A->fmt == SPMV_FMT_CSR, A->val, sv * nnz},
      {"ell_col", A->fmt == SPMV_FMT_ELL || A->fmt == SPMV_FMT_HYB, A->ecol, 4 * M * A->K},
      {"ell_val", A->fmt == SPMV_FMT_ELL || A->fmt == SPMV_FMT_HYB, A->eval, sv * M * A->K},
      {"sell_perm", sell && A->perm, A->perm, 4 * A->Mpad},
      {"sell_cs", sell, A->cs, 8 * (A->nchunks + 1)},
      {"sell_col", sell, A->scol, 4 * A->nslots},
      {"sell_val", sell, A->sval, sv * A->nslots},
      {"coo_row", A->fmt == SPMV_FMT_HYB, A->crow, 4 * A->ncoo},
      {"coo_col", A->fmt == SPMV_FMT_HYB, A->ccol, 4 * A->ncoo},
      {"coo_val", A->fmt == SPMV_FMT_HYB, A->cval, sv * A->ncoo},
      {"tile_ptr", A->fmt == SPMV_FMT_CSR5 && own, A->tile_ptr, 4 * (A->ntiles + 1)},
      {"bit_flag", A->fmt == SPMV_FMT_CSR5 && own, A->bit_flag, 4 * A->ntiles * A->omega},
      {"y_off", A->fmt == SPMV_FMT_CSR5 && own, A->y_off, 4 * A->ntiles * A->omega},
      {"seg_off", A->fmt == SPMV_FMT_CSR5 && own, A->seg_off, 4 * A->ntiles * A->omega},
      {"tile_col", A->fmt == SPMV_FMT_CSR5 && own, A->col, 4 * TW},
      {"tile_val", A->fmt == SPMV_FMT_CSR5 && own, A->val, sv * TW},
      {"tail_col", A->fmt == SPMV_FMT_CSR5 && own, A->col ? (const void*)(A->col + TW) : nullptr, 4 * (nnz - TW)},
      {"tail_val", A->fmt == SPMV_FMT_CSR5 && own, A->val ? (const void*)((const char*)A->val + sv * TW) : nullptr,
       sv * (nnz - TW)},
  };
  for (const Entry& e : tab)
    if (!strcmp(e.n, name)) {
      if (!e.ok) return fail(SPMV_ERR_INVALID_ARG, "array '%s' does not exist for this handle", name);
      *p = e.p;
      *bytes = (size_t)e.b;
      return SPMV_OK;
    }
  return fail(SPMV_ERR_INVALID_ARG, "unknown array '%s'", name);
}

spmv_status_t spmv_array_bytes(spmv_mat_t A, const char* name, size_t* bytes) {
  const void* p;
  if (!bytes) return fail(SPMV_ERR_INVALID_ARG, "bytes is null");
  return lookup(A, name, &p, bytes);
}

spmv_status_t spmv_export(spmv_mat_t A, const char* name, void* dst, size_t bytes, spmv_stream_t s) {
  const void* p;
  size_t need;
  SPMV_TRY(lookup(A, name, &p, &need));
  if (bytes < need || (need && !dst)) return fail(SPMV_ERR_INVALID_ARG, "destination too small (%zu < %zu)", bytes, need);
  return copy_to_host(dst, p, need, hs(s));
}

spmv_status_t spmv_mat_info(spmv_mat_t A, spmv_info_t* info) {
  if (!A || !info) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  info->fmt = A->fmt;
  info->dtype = A->dt;
  info->M = A->M;
  info->N = A->N;
  info->nnz = A->nnz;
  info->bytes_fmt = A->bytes_fmt;
  info->bytes_min = bytes_min(A);
  info->pad_slots = A->pad_slots;
  info->aux = A->fmt == SPMV_FMT_HYB    ? A->ncoo
              : A->fmt == SPMV_FMT_CSR5 ? A->ntiles
              : A->fmt == SPMV_FMT_SELL ? A->nchunks
              : A->fmt == SPMV_FMT_ELL  ? A->K
                                        : A->nblk;
  info->params = A->params;
  return SPMV_OK;
}

void spmv_mat_free(spmv_mat_t A) { destroy(A); }

spmv_status_t spmv_run(spmv_fmt_t fmt, spmv_mat_t A, const void* x, void* y, spmv_stream_t s) {
  if (!A) return fail(SPMV_ERR_INVALID_ARG, "null handle");
  if (fmt != A->fmt) return fail(SPMV_ERR_INVALID_ARG, "format %d does not match the handle's %d", (int)fmt, (int)A->fmt);
  if (A->M == 0) return SPMV_OK;
  if (!y || (A->N > 0 && !x)) return fail(SPMV_ERR_INVALID_ARG, "null x or y");
  const char *xb = (const char*)x, *yb = (const char*)y;
  if (x && xb < yb + A->M * A->sv && yb < xb + A->N * A->sv) return fail(SPMV_ERR_INVALID_ARG, "x and y overlap");
  return dispatch_run(A, x, y, hs(s));
}

spmv_status_t spmv_run_timed(spmv_fmt_t fmt, spmv_mat_t A, const void* x, void* y, spmv_stream_t s,
                             void* start_event, void* stop_event) {
  if (!start_event || !stop_event) return fail(SPMV_ERR_INVALID_ARG, "null event");
  return timed_call((hipEvent_t)start_event, (hipEvent_t)stop_event, hs(s),
                    [&] { return spmv_run(fmt, A, x, y, s); });
}

}  // extern "C"
