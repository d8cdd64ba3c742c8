// Batched launch, SpMM entry point and the autotuner (host side).
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

#include <algorithm>
#include "common.h"

namespace spmv {
spmv_status_t launch_batched(int dt, int64_t nitems, const void* items, const void* const* xs,
                             void* const* ys, int grid, hipStream_t s);
size_t batch_item_size();
spmv_status_t batch_items_fill(const spmv_mat_s* A, int32_t m, void* items, hipStream_t s);
int64_t batch_item_count(const spmv_mat_s* A);
size_t batch_tiles_size();
spmv_status_t batch_tile_items(const spmv_mat_s* A, int32_t m, void* host_rec, const void* dev_rec, void* items,
                               hipStream_t s);
spmv_status_t launch_batch_tile_fix(int dt, int32_t ntm, const void* recs, void* const* ys, hipStream_t s);
spmv_status_t time_run(spmv_mat_s* A, const void* x, void* y, int warmup, int min_reps, int max_reps, double rel_ci,
                       int64_t scrub_bytes, hipStream_t s, double out[5]);
}  // namespace spmv

using namespace spmv;

struct spmv_batch_s {
  int32_t n = 0;
  spmv_dtype_t dt = SPMV_F64;
  int64_t nitems = 0;
  void* desc = nullptr;   // device: one record per work item (matrix, row and nonzero range)
  void** xy = nullptr;    // device: n x pointers then n y pointers
  int32_t ntm = 0;        // matrices run as CSR wave tiles
  void* tiles = nullptr;  // device: their records (arrays, tile tables, batch index), for the fix-up pass
  std::vector<const void*> last;  // host copy of the pointers last uploaded
};

extern "C" {

spmv_status_t spmv_spmm(spmv_mat_t A, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t k, spmv_stream_t s) {
  if (!A || (A->M && (!X || !Y))) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  return run_spmm(A, X, ldx, Y, ldy, k, hs(s));
}

spmv_status_t spmv_spmm_timed(spmv_mat_t A, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t k,
                              spmv_stream_t s, void* start_event, void* stop_event) {
  if (!start_event || !stop_event) return fail(SPMV_ERR_INVALID_ARG, "null event");
  return timed_call((hipEvent_t)start_event, (hipEvent_t)stop_event, hs(s),
                    [&] { return spmv_spmm(A, X, ldx, Y, ldy, k, s); });
}

spmv_status_t spmv_batch_create(const spmv_mat_t* A, int32_t n, spmv_batch_t* out) {
  if (!A || n <= 0 || !out) return fail(SPMV_ERR_INVALID_ARG, "batch arguments");
  *out = nullptr;
  for (int32_t i = 0; i < n; ++i) {
    if (!A[i] || (A[i]->fmt != SPMV_FMT_CSR && A[i]->fmt != SPMV_FMT_SELL) || !A[i]->sub.empty())
      return fail(SPMV_ERR_INVALID_ARG, "batch matrix %d is not a CSR or SELL handle without column bands", i);
    if (A[i]->dt != A[0]->dt) return fail(SPMV_ERR_INVALID_ARG, "batch mixes dtypes");
    if (A[i]->M >= INT32_MAX) return fail(SPMV_ERR_TOO_LARGE, "batch matrix %d has %lld rows", i, (long long)A[i]->M);
  }
  spmv_batch_s* b = new (std::nothrow) spmv_batch_s();
  if (!b) return fail(SPMV_ERR_OOM, "host allocation failed");
  b->n = n;
  b->dt = A[0]->dt;
  int64_t items = 0;
  for (int32_t i = 0; i < n; ++i) items += batch_item_count(A[i]);  // every item of every matrix, in order
  b->nitems = items;
  const size_t is = batch_item_size();
  spmv_status_t st = dmalloc(&b->desc, is * (size_t)std::max<int64_t>(items, 1));
  if (st == SPMV_OK) st = dmalloc((void**)&b->xy, sizeof(void*) * 2 * n);
  for (int32_t i = 0; i < n; ++i)
    if (A[i]->fmt == SPMV_FMT_CSR && A[i]->ntiles_csr > 0) ++b->ntm;
  const size_t ts = batch_tiles_size();
  std::vector<char> hrec(ts * (size_t)std::max<int32_t>(b->ntm, 1));
  if (st == SPMV_OK && b->ntm > 0) st = dmalloc(&b->tiles, ts * (size_t)b->ntm);
  int64_t at = 0;
  int32_t tm = 0;
  for (int32_t i = 0; i < n && st == SPMV_OK; ++i) {
    if (A[i]->fmt == SPMV_FMT_CSR && A[i]->ntiles_csr > 0) {
      st = batch_tile_items(A[i], i, hrec.data() + ts * tm, (char*)b->tiles + ts * tm, (char*)b->desc + is * at,
                            nullptr);
      ++tm;
    } else {
      st = batch_items_fill(A[i], i, (char*)b->desc + is * at, nullptr);
    }
    at += batch_item_count(A[i]);
  }
  if (st == SPMV_OK && b->ntm > 0 && hipMemcpy(b->tiles, hrec.data(), ts * b->ntm, hipMemcpyHostToDevice) != hipSuccess)
    st = fail(SPMV_ERR_HIP, "batch tile records upload failed");
  if (st == SPMV_OK && hipDeviceSynchronize() != hipSuccess) st = fail(SPMV_ERR_HIP, "batch item table build failed");
  if (st != SPMV_OK) {
    dfree(b->desc);
    dfree(b->xy);
    dfree(b->tiles);
    delete b;
    return st;
  }
  *out = b;
  return SPMV_OK;
}

spmv_status_t spmv_batch_run(spmv_batch_t b, const void* const* x, void* const* y, spmv_stream_t s) {
  if (!b || !x || !y) return fail(SPMV_ERR_INVALID_ARG, "null argument");
  std::vector<const void*> ptrs(2 * b->n);
  for (int32_t i = 0; i < b->n; ++i) {
    if (!x[i] || !y[i] || x[i] == y[i]) return fail(SPMV_ERR_INVALID_ARG, "bad x/y pointer for matrix %d", i);
    ptrs[i] = x[i];
    ptrs[b->n + i] = y[i];
  }
  hipStream_t st = hs(s);
  if (ptrs != b->last) {  // upload the pointer table only when it changes
    SPMV_HIP(hipStreamSynchronize(st));
    SPMV_HIP(hipMemcpy(b->xy, ptrs.data(), sizeof(void*) * 2 * b->n, hipMemcpyHostToDevice));
    b->last = ptrs;
  }
  if (b->nitems > INT32_MAX) return fail(SPMV_ERR_TOO_LARGE, "batch of %lld row blocks", (long long)b->nitems);
  const int grid = (int)std::max<int64_t>(b->nitems, 1);  // one workgroup per item
  SPMV_TRY(launch_batched(b->dt, b->nitems, b->desc, (const void* const*)b->xy, b->xy + b->n, grid, st));
  return launch_batch_tile_fix(b->dt, b->ntm, b->tiles, b->xy + b->n, st);
}

spmv_status_t spmv_batch_run_timed(spmv_batch_t b, const void* const* x, void* const* y, spmv_stream_t s,
                                   void* start_event, void* stop_event) {
  if (!start_event || !stop_event) return fail(SPMV_ERR_INVALID_ARG, "null event");
  return timed_call((hipEvent_t)start_event, (hipEvent_t)stop_event, hs(s),
                    [&] { return spmv_batch_run(b, x, y, s); });
}

void spmv_batch_free(spmv_batch_t b) {
  if (!b) return;
  dfree(b->desc);
  dfree(b->xy);
  dfree(b->tiles);
  delete b;
}

// ------------------------------------------------------------ autotuner
// Exhaustive search over a small grid per format; each candidate is
// converted and timed with the same protocol as spmv_time (median of the
// confidence-interval rule).  Only performance depends on the choice.
// Results are cached per (structure hash, shape, dtype, format, byte cap,
// caller's flags) for the life of the process: tuning depends on the
// sparsity structure, not on the values.  The flags are part of the key
// because the candidates keep those the grid does not set (e.g.
// SPMV_FLAG_SELL_SLICES), so callers asking for different flags are tuned
// separately.
typedef std::tuple<uint64_t, int64_t, int64_t, int64_t, int, int, int64_t, uint32_t> TuneKey;
static std::mutex g_tune_mu;
static std::map<TuneKey, std::pair<spmv_params_t, double>> g_tune_cache;

spmv_status_t spmv_autotune(spmv_mat_t csr, spmv_fmt_t fmt, const void* x, void* y, int64_t scrub_bytes, int reps,
                            spmv_params_t* inout, double* ms_out, spmv_stream_t s) {
  if (!csr || csr->fmt != SPMV_FMT_CSR || !csr->sub.empty() || !inout) return fail(SPMV_ERR_INVALID_ARG, "autotune arguments");
  if (csr->M && (!y || (csr->N && !x))) return fail(SPMV_ERR_INVALID_ARG, "null x or y");
  if (reps < 3) reps = 3;
  hipStream_t st = hs(s);
  spmv_params_t base;
  resolve_params(inout, &base);
  base.bands = 1;  // the candidates below set their own
  uint64_t h = 0;
  SPMV_TRY(structure_hash(csr, &h, st));
  const TuneKey key(h, csr->M, csr->N, csr->nnz, (int)csr->dt, (int)fmt, base.max_bytes, base.flags);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *inout = it->second.first;
      if (ms_out) *ms_out = it->second.second;
      return SPMV_OK;
    }
  }
  // x larger than one XCD's 4 MiB L2: SELL and CSR5 over 2 and 4 column
  // bands (8 too above 32 MiB) are candidates.  Random gathers from a slice
  // that fits the L2s cost about half those served from the Infinity Cache,
  // but each band adds launches and an M-long partial product; measured,
  // they paid off on x of 16 MB and more, not at 8 MB.
  std::vector<int> xbands;
  {
    const int64_t xb = csr->N * (int64_t)csr->sv;
    if (csr->M && xb > ((int64_t)4 << 20)) xbands = {2, 4};
    if (csr->M && xb > ((int64_t)32 << 20)) xbands.push_back(8);
  }
  std::vector<spmv_params_t> cand;
  auto add = [&](auto&& f) {
    spmv_params_t p = base;
    f(p);
    cand.push_back(p);
  };
  switch (fmt) {
    case SPMV_FMT_CSR:
      add([](spmv_params_t& p) {
        p.csr_lanes_per_row = 0;
        p.flags &= ~(SPMV_FLAG_CSR_WAVES | SPMV_FLAG_LINEAR | SPMV_FLAG_CSR_BANDS | SPMV_FLAG_CSR_TILES);
      });
      add([](spmv_params_t& p) { p.csr_lanes_per_row = 0; p.flags |= SPMV_FLAG_CSR_WAVES; });
      add([](spmv_params_t& p) { p.csr_lanes_per_row = 0; p.flags = (p.flags & ~SPMV_FLAG_CSR_WAVES) | SPMV_FLAG_LINEAR; });
      add([](spmv_params_t& p) {
        p.csr_lanes_per_row = 0;
        p.flags = (p.flags & ~(SPMV_FLAG_CSR_WAVES | SPMV_FLAG_LINEAR)) | SPMV_FLAG_CSR_BANDS;
      });
      add([](spmv_params_t& p) {
        p.csr_lanes_per_row = 0;
        p.flags = (p.flags & ~(SPMV_FLAG_CSR_WAVES | SPMV_FLAG_LINEAR | SPMV_FLAG_CSR_BANDS)) | SPMV_FLAG_CSR_TILES;
      });
      for (int V : {4, 8, 16, 32}) add([V](spmv_params_t& p) { p.csr_lanes_per_row = V; });
      // x larger than 4 MiB: row blocks and wave tiles over 2 and 4 column
      // bands.  Measured, 2 bands paid off from about 8 MB of x on (a 4 MB
      // slice fits an XCD's L2) and 4 bands on x of 128 MB (a 32 MB slice
      // stays in the Infinity Cache); more bands lost to the extra passes.
      if (csr->M && csr->N * (int64_t)csr->sv > ((int64_t)4 << 20))
        for (int nb : {2, 4})
          for (uint32_t tiles : {0u, (uint32_t)SPMV_FLAG_CSR_TILES})
            add([nb, tiles](spmv_params_t& p) {
              p.csr_lanes_per_row = 0;
              p.flags = (p.flags & ~(SPMV_FLAG_CSR_WAVES | SPMV_FLAG_LINEAR | SPMV_FLAG_CSR_BANDS | SPMV_FLAG_CSR_TILES)) | tiles;
              p.bands = nb;
            });
      break;
    case SPMV_FMT_CSR5:
      for (int sg : {4, 8, 16, 32}) add([sg](spmv_params_t& p) { p.csr5_omega = 64; p.csr5_sigma = sg; p.bands = 1; });
      // over bands the short tiles win (zipf_1M over 2 bands: sigma 8 153.5 us,
      // 4 154.2, 16 164.5: more waves in flight for the band's gathers)
      for (int nb : xbands)
        for (int sg : {4, 8, 16, 32})
          add([sg, nb](spmv_params_t& p) { p.csr5_omega = 64; p.csr5_sigma = sg; p.bands = nb; });
      break;
    case SPMV_FMT_ELL:
      add([](spmv_params_t& p) { p.flags &= ~SPMV_FLAG_SPLIT4; });
      add([](spmv_params_t& p) { p.flags |= SPMV_FLAG_SPLIT4; });
      break;
    case SPMV_FMT_SELL:
      // sigma in {1, C, 8C, 256C} and one window over all rows (a global
      // sort by length, which removes nearly all padding of skewed rows)
      for (int C : {8, 16, 32, 64}) {
        const int64_t all = std::max<int64_t>(csr->M, 1);
        for (int64_t sg : {(int64_t)1, (int64_t)C, (int64_t)8 * C, (int64_t)256 * C, all}) {
          if (sg == all && all <= (int64_t)256 * C) continue;  // 256C already covers every row
          add([C, sg](spmv_params_t& p) {
            p.sell_C = C;
            p.sell_sigma = (int32_t)sg;
            p.bands = 1;
            p.flags &= ~(SPMV_FLAG_SPLIT4 | SPMV_FLAG_SPLIT6);
          });
          // C = 64: also four and six waves per chunk
          if (C == 64)
            for (uint32_t sp : {(uint32_t)SPMV_FLAG_SPLIT4, (uint32_t)SPMV_FLAG_SPLIT6})
              add([C, sg, sp](spmv_params_t& p) {
                p.sell_C = C;
                p.sell_sigma = (int32_t)sg;
                p.bands = 1;
                p.flags = (p.flags & ~(SPMV_FLAG_SPLIT4 | SPMV_FLAG_SPLIT6)) | sp;
              });
        }
      }
      if (!xbands.empty()) {
        const int32_t all = (int32_t)std::min<int64_t>(csr->M, INT32_MAX);
        for (int nb : xbands)
          for (int C : {32, 64})
            add([C, all, nb](spmv_params_t& p) {
              p.sell_C = C;
              p.sell_sigma = all;
              p.bands = nb;
              p.flags &= ~(SPMV_FLAG_SPLIT4 | SPMV_FLAG_SPLIT6);
            });
      }
      break;
    case SPMV_FMT_HYB: {
      // K from the rule, and the 50/75/90/99th percentiles of the row lengths
      std::vector<int32_t> lens(csr->M);
      std::vector<int32_t> hp(csr->M + 1);
      if (csr->M) {
        SPMV_HIP(hipMemcpyAsync(hp.data(), csr->ptr, sizeof(int32_t) * (csr->M + 1), hipMemcpyDeviceToHost, st));
        SPMV_HIP(hipStreamSynchronize(st));
        for (int64_t i = 0; i < csr->M; ++i) lens[i] = hp[i + 1] - hp[i];
        std::sort(lens.begin(), lens.end());
      }
      // and, when x exceeds 4 MiB, each K with the COO tail over 2 and 4
      // column bands (8 too when x exceeds 32 MiB).  Measured: 2 bands took
      // zipf_1M's HYB from 191 to 159 us (8 MB of x), 4 bands rmat24's from
      // 3.59 to 2.17 ms (134 MB); on x of about 8 MB with shorter tails, and
      // in FP32 at 4 MB, bands lost.
      // and K = 0, 1, 2: a short ELL part and nearly all entries in the
      // banded tail (zipf_1M over 2 bands: K 1 158 us against 165 at K 3)
      std::vector<int32_t> Ks{-1};
      for (double q : {0.5, 0.75, 0.9, 0.99}) Ks.push_back(csr->M ? lens[(size_t)(q * (double)(csr->M - 1))] : 0);
      for (int32_t k : {0, 1, 2})
        if (std::find(Ks.begin(), Ks.end(), k) == Ks.end()) Ks.push_back(k);
      std::vector<int> nbs{1};
      const int64_t xbytes = csr->N * (int64_t)csr->sv;
      if (csr->M && xbytes > ((int64_t)4 << 20)) nbs.insert(nbs.end(), {2, 4});
      if (csr->M && xbytes > ((int64_t)32 << 20)) nbs.push_back(8);
      for (int nb : nbs)
        for (int32_t K : Ks)
          for (uint32_t sp : {0u, (uint32_t)SPMV_FLAG_SPLIT4})
            add([K, nb, sp](spmv_params_t& p) {
              p.hyb_K = K;
              p.bands = nb;
              p.flags = (p.flags & ~SPMV_FLAG_SPLIT4) | sp;
            });
      break;
    }
    default: return fail(SPMV_ERR_INVALID_ARG, "format %d", (int)fmt);
  }
  // Every candidate is timed with `reps` launches; the three fastest are then
  // timed again with three times as many, and the fastest of that round wins
  // (one lucky median among dozens of candidates otherwise decides: rmat24's
  // CSR over 2 bands was timed at 2.52 ms by the first round and runs at
  // 2.78 ms, against 2.61 ms over 4 bands).
  std::vector<std::pair<double, spmv_params_t>> scored;
  for (const spmv_params_t& p : cand) {
    spmv_mat_t B = nullptr;
    spmv_status_t cst = spmv_convert(csr, fmt, &p, s, &B);
    if (cst == SPMV_ERR_TOO_LARGE || cst == SPMV_ERR_UNSUPPORTED) continue;
    if (cst != SPMV_OK) return cst;
    double out[5];
    spmv_status_t tst = time_run(B, x, y, 2, reps, reps, 0.0, scrub_bytes, st, out);
    const spmv_params_t used = B->params;
    spmv_mat_free(B);
    if (tst != SPMV_OK) return tst;
    scored.emplace_back(out[0], used);
  }
  if (scored.empty()) return fail(SPMV_ERR_TOO_LARGE, "no candidate of format %d fits the byte cap", (int)fmt);
  std::stable_sort(scored.begin(), scored.end(),
                   [](const std::pair<double, spmv_params_t>& a, const std::pair<double, spmv_params_t>& b) {
                     return a.first < b.first;
                   });
  double best = scored[0].first;
  spmv_params_t bestp = scored[0].second;
  if (scored.size() > 1) {
    best = 1e300;
    const int r3 = 3 * std::max(reps, 1);
    for (size_t i = 0; i < std::min<size_t>(3, scored.size()); ++i) {
      spmv_mat_t B = nullptr;
      SPMV_TRY(spmv_convert(csr, fmt, &scored[i].second, s, &B));
      double out[5];
      spmv_status_t tst = time_run(B, x, y, 2, r3, r3, 0.0, scrub_bytes, st, out);
      spmv_mat_free(B);
      if (tst != SPMV_OK) return tst;
      if (out[0] < best) {
        best = out[0];
        bestp = scored[i].second;
      }
    }
  }
  *inout = bestp;
  if (ms_out) *ms_out = best;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_cache[key] = std::make_pair(bestp, best);
  return SPMV_OK;
}

void spmv_autotune_cache_clear(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_cache.clear();
}

}  // extern "C"
