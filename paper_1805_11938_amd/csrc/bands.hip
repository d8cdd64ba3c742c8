// Column bands (an execution layout of CSR, SELL-C-sigma and CSR5, not a format of
// the paper): the entries are split by column into nb equal bands, each band
// is converted on its own (a matrix of all M rows holding only the band's
// columns) and the bands run one after another.  Each launch then gathers
// from one slice of x, which fits an XCD's L2 when x itself does not, and
// random gathers served from L2 cost about half of those served from the
// Infinity Cache.  Band 0 writes y; every later band adds its product onto
// y (each row's band sum added in FP64, rounded once per band), so the
// bands are summed in band order with no scratch and no summing pass.
#include "common.h"

namespace spmv {

spmv_status_t csr5_to_csr(spmv_mat_s* A, int32_t* ptr, int32_t* col, void* val, hipStream_t s);
spmv_status_t ell_sell_hyb_to_csr(spmv_mat_s* A, int32_t* ptr, int32_t* col, void* val, hipStream_t s);

static unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, BS), 1 << 20));
}

spmv_status_t convert_banded(spmv_mat_s* src, spmv_mat_s* A, hipStream_t s) {
  const int nb = A->params.bands;
  if (A->fmt != SPMV_FMT_SELL && A->fmt != SPMV_FMT_CSR5 && A->fmt != SPMV_FMT_CSR)
    return fail(SPMV_ERR_UNSUPPORTED, "column bands are implemented for CSR, SELL and CSR5");
  if (nb > 64) return fail(SPMV_ERR_UNSUPPORTED, "%d column bands (at most 64)", nb);
  if (A->fmt == SPMV_FMT_CSR && (A->params.flags & (SPMV_FLAG_CSR_WAVES | SPMV_FLAG_CSR_BANDS)))
    return fail(SPMV_ERR_UNSUPPORTED, "CSR over column bands runs as row blocks, wave tiles or V lanes per row");
  const int64_t M = src->M, N = src->N, sv = A->sv;
  const int64_t bw = std::max<int64_t>(1, cdiv(N, nb));
  A->band_w = bw;
  DTmp bp, bc, bv;
  SPMV_TRY(bp.alloc(sizeof(int32_t) * nb * (M + 1)));
  SPMV_TRY(bc.alloc(sizeof(int32_t) * std::max<int64_t>(src->nnz, 1)));
  SPMV_TRY(bv.alloc((size_t)sv * std::max<int64_t>(src->nnz, 1)));
  std::vector<int64_t> off;
  SPMV_TRY(csr_split_bands(src, nb, bw, bp.as<int32_t>(), bc.as<int32_t>(), bv.p, off, s));
  int64_t fmt_bytes = 0;
  for (int b = 0; b < nb; ++b) {
    spmv_mat_s band;  // a CSR view of band b (owns nothing)
    band.fmt = SPMV_FMT_CSR;
    band.dt = src->dt;
    band.sv = src->sv;
    band.M = M;
    band.N = N;
    band.nnz = off[b + 1] - off[b];
    band.ptr = bp.as<int32_t>() + (int64_t)b * (M + 1);
    band.col = bc.as<int32_t>() + off[b];
    band.val = (char*)bv.p + (size_t)sv * off[b];
    std::unique_ptr<spmv_mat_s> sub(new (std::nothrow) spmv_mat_s());
    if (!sub) return fail(SPMV_ERR_OOM, "host allocation failed");
    sub->fmt = A->fmt;
    sub->dt = src->dt;
    sub->sv = src->sv;
    sub->M = M;
    sub->N = N;
    sub->nnz = band.nnz;
    sub->params = A->params;
    sub->params.bands = 1;
    sub->acc = b > 0;  // bands after the first add onto y
    const spmv_status_t st = A->fmt == SPMV_FMT_SELL   ? convert_sell(&band, sub.get(), s)
                             : A->fmt == SPMV_FMT_CSR5 ? convert_csr5(&band, sub.get(), s)
                                                       : convert_csr(&band, sub.get(), s);
    A->owned.insert(A->owned.end(), sub->owned.begin(), sub->owned.end());  // freed with the handle
    sub->owned.clear();
    if (st != SPMV_OK) return st;
    fmt_bytes += sub->bytes_fmt - N * sv - M * sv;  // the band's own arrays
    A->nchunks += sub->nchunks;
    A->ntiles += sub->ntiles;
    A->pad_slots += sub->pad_slots;
    A->C = sub->C;
    A->sigma = sub->sigma;
    A->omega = sub->omega;
    A->c5sigma = sub->c5sigma;
    A->sub.push_back(std::move(sub));
  }
  const int64_t cap = A->params.max_bytes > 0 ? A->params.max_bytes : default_max_bytes();
  if (fmt_bytes > cap)
    return fail(SPMV_ERR_TOO_LARGE, "%d column bands need %lld bytes (cap %lld)", nb, (long long)fmt_bytes,
                (long long)cap);
  // the bands' arrays, x once, y once (y read and written again by each band
  // after the first is traffic of this execution layout, not of the product:
  // not counted)
  A->bytes_fmt = fmt_bytes + N * sv + M * sv;
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

spmv_status_t run_banded(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  for (const auto& b : A->sub) SPMV_TRY(dispatch_run(b.get(), x, y, s));  // in band order on one stream
  return SPMV_OK;
}

// Back to one CSR: row r is band 0's row r, then band 1's, ... (the bands
// are column ranges in order, so the columns stay sorted).
__global__ void k_bands_len(int64_t M, int nb, const int32_t* bptr, int32_t* len) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x) {
    int32_t n = 0;
    for (int b = 0; b < nb; ++b) n += bptr[b * (M + 1) + r + 1] - bptr[b * (M + 1) + r];
    len[r] = n;
  }
}

// one wave per row, the lanes copying consecutive entries of each band
template <typename T>
__global__ void k_bands_merge(int64_t M, int nb, const int32_t* bptr, const int64_t* off, const int32_t* bcol,
                              const T* bval, const int32_t* ptr, int32_t* col, T* val) {
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
  const int lane = __lane_id();
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; r < M; r += nw) {
    int64_t d = ptr[r];
    for (int b = 0; b < nb; ++b) {
      const int64_t a = off[b] + bptr[b * (M + 1) + r], e = off[b] + bptr[b * (M + 1) + r + 1];
      for (int64_t k = a + lane; k < e; k += WAVE) {
        col[d + (k - a)] = bcol[k];
        val[d + (k - a)] = bval[k];
      }
      d += e - a;
    }
  }
}

spmv_status_t banded_to_csr(spmv_mat_s* A, int32_t* ptr, int32_t* col, void* val, hipStream_t s) {
  const int nb = (int)A->sub.size();
  const int64_t M = A->M, sv = A->sv;
  DTmp bp, bc, bv, len, doff;
  SPMV_TRY(bp.alloc(sizeof(int32_t) * nb * (M + 1)));
  SPMV_TRY(bc.alloc(sizeof(int32_t) * std::max<int64_t>(A->nnz, 1)));
  SPMV_TRY(bv.alloc((size_t)sv * std::max<int64_t>(A->nnz, 1)));
  SPMV_TRY(len.alloc(sizeof(int32_t) * std::max<int64_t>(M, 1)));
  std::vector<int64_t> off(nb + 1, 0);
  for (int b = 0; b < nb; ++b) {
    spmv_mat_s* B = A->sub[b].get();
    int32_t* pb = bp.as<int32_t>() + (int64_t)b * (M + 1);
    int32_t* cb = bc.as<int32_t>() + off[b];
    void* vb = (char*)bv.p + (size_t)sv * off[b];
    if (B->fmt == SPMV_FMT_CSR) {
      SPMV_HIP(hipMemcpyAsync(pb, B->ptr, sizeof(int32_t) * (M + 1), hipMemcpyDeviceToDevice, s));
      if (B->nnz) {
        SPMV_HIP(hipMemcpyAsync(cb, B->col, sizeof(int32_t) * B->nnz, hipMemcpyDeviceToDevice, s));
        SPMV_HIP(hipMemcpyAsync(vb, B->val, (size_t)sv * B->nnz, hipMemcpyDeviceToDevice, s));
      }
    } else {
      SPMV_TRY(B->fmt == SPMV_FMT_CSR5 ? csr5_to_csr(B, pb, cb, vb, s) : ell_sell_hyb_to_csr(B, pb, cb, vb, s));
    }
    off[b + 1] = off[b] + B->nnz;
  }
  SPMV_TRY(doff.alloc(sizeof(int64_t) * (nb + 1)));
  SPMV_HIP(hipMemcpyAsync(doff.p, off.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, s));
  if (M) {
    k_bands_len<<<grid_for(M), BS, 0, s>>>(M, nb, bp.as<int32_t>(), len.as<int32_t>());
    SPMV_LAUNCH_CHECK();
  }
  SPMV_TRY(scan_i32_to_i32(len.as<int32_t>(), ptr, M, s));
  if (M) {
    const unsigned gw = (unsigned)std::min<int64_t>(cdiv(M, BS / WAVE), 1 << 20);
    if (A->dt == SPMV_F64)
      k_bands_merge<double><<<gw, BS, 0, s>>>(M, nb, bp.as<int32_t>(), doff.as<int64_t>(), bc.as<int32_t>(),
                                                       (const double*)bv.p, ptr, col, (double*)val);
    else
      k_bands_merge<float><<<gw, BS, 0, s>>>(M, nb, bp.as<int32_t>(), doff.as<int64_t>(), bc.as<int32_t>(),
                                                      (const float*)bv.p, ptr, col, (float*)val);
    SPMV_LAUNCH_CHECK();
  }
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

}  // namespace spmv
