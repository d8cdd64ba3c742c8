/*
 * spmv.h -- C-ABI of libspmv.so, an MI355X (gfx950) SpMV library over the
 * five storage formats studied in arXiv 1805.11938 ("Optimizing Sparse
 * Matrix-Vector Multiplication on Emerging Many-Core Architectures").
 *
 * The operation (Sec. II-A): y = A x, A sparse M x N, x and y dense.
 * Formats (Sec. II-B, Table I): CSR, CSR5, ELL, SELL / SELL-C-sigma,
 * HYB = ELL + COO.  Adaptive format selection from static matrix features
 * (Sec. V): features, min-max scaling and a learned classifier.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Status codes, never exceptions; spmv_last_error() gives a message for
 *   the calling thread's last failure.
 * - Indices are int32 (M, N, nnz < 2^31); slot offsets inside padded
 *   formats are int64.  Values are FP64 or FP32 (spmv_dtype_t); the
 *   kernels accumulate in FP64 for both.
 * - Streams are hipStream_t passed as void* (NULL = the null stream).
 *   Calls that only enqueue device work are asynchronous on that stream;
 *   calls that return host data (features, select, to_csr/export to host,
 *   timing) synchronise it.  Library-internal allocations use hipMalloc.
 * - Matrix handles (spmv_mat_t) own their device arrays: creation copies
 *   the caller's arrays, so the caller may free them afterwards.  Runs of
 *   distinct handles on different streams are independent.  Three kinds of
 *   handle keep per-handle device scratch that every run rewrites -- CSR5
 *   (tile carries), SELL with column slices (partial sums and slice counts) and CSR built
 *   with SPMV_FLAG_CSR_WAVES (long-row segment sums) -- so two runs of the
 *   *same* such handle must not overlap (same stream, or synchronise).
 *   x, y, X, Y stay owned by the caller: device pointers of the handle's
 *   dtype.
 * - y is overwritten (beta = 0).  x and y must not overlap.
 */
#ifndef SPMV_H
#define SPMV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Format = class index of the selector (Sec. V-B, Table II column order). */
typedef enum { SPMV_FMT_CSR = 0, SPMV_FMT_CSR5 = 1, SPMV_FMT_ELL = 2, SPMV_FMT_SELL = 3, SPMV_FMT_HYB = 4 } spmv_fmt_t;
#define SPMV_NUM_FORMATS 5

typedef enum { SPMV_F64 = 0, SPMV_F32 = 1 } spmv_dtype_t;

typedef enum {
  SPMV_OK = 0,
  SPMV_ERR_INVALID_ARG = -1,   /* null handle/pointer, bad size, x == y, fmt mismatch */
  SPMV_ERR_BAD_STRUCTURE = -2, /* malformed CSR/COO (ptr not monotone, col out of range, unsorted/duplicate col) */
  SPMV_ERR_OOM = -3,           /* device allocation failed, or SPMV_MEM_CAP_BYTES exceeded */
  SPMV_ERR_TOO_LARGE = -4,     /* padded format would exceed the byte cap (ELL / SELL / HYB) or int limits */
  SPMV_ERR_UNSUPPORTED = -5,   /* parameter combination the kernels do not implement */
  SPMV_ERR_HIP = -6,           /* a HIP runtime call failed */
  SPMV_ERR_MODEL = -7          /* model file missing, corrupt, or of the wrong version */
} spmv_status_t;

typedef struct spmv_mat_s* spmv_mat_t;
typedef struct spmv_model_s* spmv_model_t;
typedef struct spmv_batch_s* spmv_batch_t;
typedef void* spmv_stream_t; /* hipStream_t */

/* Tuning parameters (Sec. II-B names omega, sigma for CSR5, C and sigma for
 * SELL-C-sigma, and HYB's K).  Zero / -1 fields take the defaults below. */
typedef struct {
  int32_t sell_C;            /* chunk height C in {8,16,32,64}; default 32 */
  int32_t sell_sigma;        /* sort window sigma >= 1 (1 = plain SELL); default 1 */
  int32_t csr_lanes_per_row; /* 0 = nnz-balanced row blocks (default); V in {1,2,4,..,64} = V lanes per row */
  int32_t hyb_K;             /* ELL width of HYB; -1 = the one-third rule (default) */
  int32_t csr5_omega;        /* tile width; must divide 64 for spmv_run; default 64 */
  int32_t csr5_sigma;        /* tile height 1..32; default 16 */
  int64_t max_bytes;         /* byte cap of the converted format; 0 = default (SPMV_MAX_BYTES env or 64 GiB) */
  uint32_t flags;            /* SPMV_FLAG_* */
  int32_t bands;             /* CSR, SELL and CSR5: split the columns into this many equal bands (1..64), each
                                converted to the format on its own over all M rows and run one after
                                another, so each launch gathers from one slice of x that fits the L2; band 0
                                writes y and each later band adds its row sums onto y (in FP64, rounded once
                                per band), so the bands are summed in band order.  CSR over bands: row
                                blocks, wave tiles or V lanes per row (SPMV_FLAG_CSR_WAVES or
                                SPMV_FLAG_CSR_BANDS -> UNSUPPORTED).  HYB: the
                                COO tail is ordered by band (then row, column) and each band's pass adds
                                onto y after the previous one.  0 or 1 = no split (default); ELL returns
                                UNSUPPORTED for bands > 1 */
} spmv_params_t;

#define SPMV_FLAG_NO_CHECK 1u /* skip the column checks of spmv_mat_from_csr (ptr is always checked) */
#define SPMV_FLAG_CSR_WAVES 2u /* CSR: per-wave row units (+ long-row segments) instead of workgroup row blocks */
#define SPMV_FLAG_LINEAR 4u    /* CSR row blocks, ELL and HYB's ELL part: workgroups take rows in launch order
                                  instead of each XCD taking a contiguous range of rows */
#define SPMV_FLAG_SELL_SLICES 8u /* SELL: every chunk as column-slice items (default: chunks at most 32 wide
                                    take one pass per stored row; wider chunks are cut into slices of 64
                                    slots, run in the same launch, whose partial sums a fix-up adds) */
#define SPMV_FLAG_CSR_BANDS 16u /* CSR: split the columns into 8 bands, one per XCD, so each XCD's L2 holds its
                                   eighth of x; per-band partial sums are added by a second pass */
#define SPMV_FLAG_CSR_TILES 32u /* CSR: one wave per tile of 1,024 consecutive nonzeros (segmented scan in
                                   registers, no workgroup barrier), rows crossing tiles finished by an ordered
                                   fix-up pass; for irregular rows.  Ignored with csr_lanes_per_row > 0 or
                                   SPMV_FLAG_CSR_BANDS; with bands > 1 each column band runs as tiles */
#define SPMV_FLAG_SPLIT4 64u    /* ELL with K <= 32 and SELL chunks of C = 64 at most 32 wide: four waves share
                                  each 64 rows, each taking a quarter of every row's slots; the four sums are
                                  added in wave order (fewer registers per wave, more loads in flight per CU) */
#define SPMV_FLAG_SPLIT6 128u   /* SELL chunks of C = 64 at most 32 wide: six waves share each chunk, each taking
                                  a sixth of every row's slots, sums added in wave order (over SPLIT4 when both
                                  are set; other formats and chunk heights ignore it) */

typedef struct {
  int32_t fmt, dtype;
  int64_t M, N, nnz;
  int64_t bytes_fmt;     /* bytes one spmv_run streams: format arrays incl. padding/metadata, x once, y once */
  int64_t bytes_min;     /* compulsory CSR bytes nnz*(sv+4) + 4(M+1) + N*sv + M*sv (format independent) */
  int64_t pad_slots;     /* stored slots that hold padding (ELL / SELL / HYB-ELL) */
  int64_t aux;           /* HYB: COO entries; CSR5: tiles; SELL: chunks; ELL: K; CSR: row blocks */
  spmv_params_t params;  /* the parameters the handle was built with (defaults resolved) */
} spmv_info_t;

const char* spmv_status_str(spmv_status_t st);
const char* spmv_last_error(void);
/* Device bytes the library currently holds: live handles, batches, models and
 * the workspaces it keeps (not the caller's buffers).  With the environment
 * variable SPMV_MEM_CAP_BYTES set (read once per process), an allocation that
 * would take this above the cap fails with SPMV_ERR_OOM.
 * Arrays the library frees (a destroyed handle, a conversion's temporaries)
 * are kept for its later allocations on the same device, up to
 * SPMV_CACHE_BYTES (read once per process; default 16 GiB, 0 keeps none);
 * kept blocks are not counted here. */
int64_t spmv_mem_in_use(void);
/* Hands every kept free block back to HIP (hipFree); returns the bytes
 * released.  Safe at any time: handles and their arrays are not affected. */
int64_t spmv_mem_release(void);

/* ------------------------------------------------------------ creation */

/* CSR matrix from caller arrays (Sec. II-B, CSR): ptr[M+1] with ptr[0] = 0
 * and ptr[M] = nnz, col[nnz] strictly increasing inside each row, val[nnz]
 * of dtype dt.  src_on_device: 0 = host arrays, 1 = device arrays.  The
 * structure is checked on the device unless SPMV_FLAG_NO_CHECK is passed in
 * flags: BAD_STRUCTURE on failure.  Synchronises s. */
spmv_status_t spmv_mat_from_csr(int64_t M, int64_t N, int64_t nnz, const int32_t* ptr, const int32_t* col,
                                const void* val, spmv_dtype_t dt, int src_on_device, uint32_t flags,
                                spmv_stream_t s, spmv_mat_t* out);

/* CSR matrix from raw COO triplets (Sec. II-B, COO; Sec. III-D reads Matrix
 * Market into COO before converting): on the device, the n triplets are
 * stably sorted by (row, col), duplicates are summed left to right in input
 * order, explicit zeros are kept.  Out-of-range coordinates -> BAD_STRUCTURE.
 * Synchronises s. */
spmv_status_t spmv_mat_from_coo(int64_t M, int64_t N, int64_t n, const int32_t* row, const int32_t* col,
                                const void* val, spmv_dtype_t dt, int src_on_device, spmv_stream_t s,
                                spmv_mat_t* out);

/* Convert a CSR handle to fmt (Sec. II-B; Table I): a new handle.  p may be
 * NULL (defaults).  ELL/SELL/HYB above the byte cap -> TOO_LARGE.  The source
 * must be a CSR handle without column bands (INVALID_ARG otherwise); so must
 * the handles given to spmv_autotune and spmv_features (INVALID_ARG) and to
 * spmv_spmm (UNSUPPORTED); spmv_batch_create also takes SELL handles.
 * Conversion runs on the device; it synchronises s (sizes come back). */
spmv_status_t spmv_convert(spmv_mat_t csr, spmv_fmt_t fmt, const spmv_params_t* p, spmv_stream_t s,
                           spmv_mat_t* out);

/* Inverse conversion of any handle back to CSR arrays (bit-exact round
 * trip).  dst_on_device: 0 = host buffers (synchronises s), 1 = device. */
spmv_status_t spmv_to_csr(spmv_mat_t A, int32_t* ptr, int32_t* col, void* val, int dst_on_device, spmv_stream_t s);

/* Copy a named internal array to host memory (golden tests).  Names:
 * "ptr","col","val" (CSR; CSR5 keeps CSR's ptr); "ell_col","ell_val"
 * (ELL and HYB, column-major M x K); "sell_perm","sell_cs","sell_col",
 * "sell_val"; "coo_row","coo_col","coo_val" (HYB; with bands > 1 ordered by
 * band, then row and column); "tile_ptr","bit_flag",
 * "y_off","seg_off","tile_col","tile_val","tail_col","tail_val" (CSR5);
 * "band_ptr","band_col","band_val" (CSR built with SPMV_FLAG_CSR_BANDS:
 * 8 row-pointer arrays of M+1, then the bands' entries band after band).
 * A CSR, SELL or CSR5 handle built with bands > 1 has no arrays of its own;
 * band b's are "band<b>.col", "band<b>.sell_col", "band<b>.tile_ptr" etc. (band b holds
 * the columns [b*ceil(N/bands), (b+1)*ceil(N/bands)).
 * spmv_array_bytes reports the size; export fails with INVALID_ARG when
 * bytes is smaller.  Synchronises s. */
spmv_status_t spmv_array_bytes(spmv_mat_t A, const char* name, size_t* bytes);
spmv_status_t spmv_export(spmv_mat_t A, const char* name, void* dst, size_t bytes, spmv_stream_t s);

spmv_status_t spmv_mat_info(spmv_mat_t A, spmv_info_t* info);
void spmv_mat_free(spmv_mat_t A);

/* ------------------------------------------------------------------ run */

/* y = A x (Sec. II-A) with the kernel of A's format.  fmt must equal A's
 * format (INVALID_ARG otherwise).  x: N values, y: M values, device memory,
 * A's dtype. */
spmv_status_t spmv_run(spmv_fmt_t fmt, spmv_mat_t A, const void* x, void* y, spmv_stream_t s);

/* Not in the paper: Sec. II-A's y = A x applied to k right-hand sides at once.
 * Y = A X for k right-hand sides, row-major: X[j*ldx + c], Y[i*ldy + c],
 * c < k <= 64, ldx >= k, ldy >= k.  A must be a CSR handle
 * (SPMV_ERR_UNSUPPORTED otherwise); columns c >= k of Y are not touched. */
spmv_status_t spmv_spmm(spmv_mat_t A, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t k, spmv_stream_t s);

/* Not in the paper (it runs one matrix at a time; Sec. III-D splits one SpMV
 * into tasks -- rows, block rows, tiles -- and this extends the tasks over many
 * matrices).  Batched launch: n handles of one dtype, each a CSR handle
 * without column bands (its row blocks become items; built with
 * SPMV_FLAG_CSR_TILES, its wave tiles, four per item), or a SELL-C-sigma
 * handle without column bands (groups of 256 / C chunks become items, one
 * stored row per thread, slots summed 8 at a time), processed by ONE kernel
 * launch, one workgroup per item of a work list built at creation; the
 * hardware dispatcher hands out the items, so the grid is not persistent.
 * When wave-tile handles are present, a second, small kernel adds the partial
 * sums of their rows that cross tiles, in tile order (each such handle's tile
 * scratch is shared with its spmv_run: runs of one handle must not overlap).  create builds the device work list (INVALID_ARG
 * for other handles, mixed dtypes or a null handle; the handles must outlive
 * the batch); run takes host arrays of n device pointers x[i] (N_i values)
 * and y[i] (M_i values), and y[i] is overwritten. */
spmv_status_t spmv_batch_create(const spmv_mat_t* A, int32_t n, spmv_batch_t* out);
spmv_status_t spmv_batch_run(spmv_batch_t b, const void* const* x, void* const* y, spmv_stream_t s);
void spmv_batch_free(spmv_batch_t b);

/* ---------------------------------------------------------- measurement */

/* Timed variants of spmv_run, spmv_spmm and spmv_batch_run (the byte and
 * time model of the measurements: Sec. III-D, Alg. 1 times repeated runs
 * and reports time and bandwidth).  start_event / stop_event are
 * hipEvent_t created by the caller (with timing enabled).  The call's first
 * kernel records start_event as it begins and its last kernel records
 * stop_event as it ends (the kernels are launched with hipExtLaunchKernel),
 * so hipEventElapsedTime(start, stop) is the run's kernel time without the
 * dispatch latency of separate event records.  A call that launches no
 * kernel (M = 0) records both events on s.  Errors as the untimed calls;
 * SPMV_ERR_INVALID_ARG for a null event. */
spmv_status_t spmv_run_timed(spmv_fmt_t fmt, spmv_mat_t A, const void* x, void* y, spmv_stream_t s,
                             void* start_event, void* stop_event);
spmv_status_t spmv_spmm_timed(spmv_mat_t A, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t k,
                              spmv_stream_t s, void* start_event, void* stop_event);
spmv_status_t spmv_batch_run_timed(spmv_batch_t b, const void* const* x, void* const* y, spmv_stream_t s,
                                   void* start_event, void* stop_event);

/* Timing in the manner of Sec. V-B: repeat until the 95% confidence
 * interval of the mean is narrower than rel_ci (0.05 = the paper's 5%
 * gap), with at least min_reps and at most max_reps launches, after
 * `warmup` untimed ones.  Each launch is bracketed by HIP events on s;
 * scrub_bytes > 0 runs a cache-scrub kernel over that many bytes before
 * every launch, outside the events (cold L2 / Infinity Cache).
 * out[0..4] = median ms, mean ms, CI half-width ms, reps, min ms. */
spmv_status_t spmv_time(spmv_fmt_t fmt, spmv_mat_t A, const void* x, void* y, int warmup, int min_reps,
                        int max_reps, double rel_ci, int64_t scrub_bytes, spmv_stream_t s, double out[5]);

/* Enqueue the cache scrub on s (reads scrub_bytes of a library buffer, so
 * the caches hold clean lines of it afterwards). */
spmv_status_t spmv_scrub(int64_t scrub_bytes, spmv_stream_t s);

/* Device-to-device copy probe: returns the GB/s of a plain copy kernel
 * reading and writing `bytes` each (median of reps). */
spmv_status_t spmv_copy_probe(int64_t bytes, int reps, spmv_stream_t s, double* gbps);

/* Random-gather probe: a perfectly balanced SpMV of `rows` rows with 16
 * entries each whose columns are uniform over [0, nx) (a seeded SplitMix64
 * hash), column and value arrays slot-major (coalesced), every load of a row
 * in flight at once.  Its time is the floor for gathering 16 * rows entries
 * from an x of nx values of dtype dt, the bound of launches limited by
 * scattered gathers rather than by HBM bytes.  Allocates and frees its own
 * buffers; times `reps` launches, each after a read-only scrub of
 * scrub_bytes (0 = none), and writes the median in ms.  Synchronises s.
 * INVALID_ARG unless 1 <= nx < 2^31 and 1 <= rows <= 2^27. */
spmv_status_t spmv_gather_probe(int64_t nx, int64_t rows, spmv_dtype_t dt, int reps, int64_t scrub_bytes,
                                spmv_stream_t s, double* ms);

/* Not in the paper (it fixes each format's parameters; Sec. II-B names them).
 * Autotuner: time every candidate of fmt's grid on x/y (reps launches each),
 * time the three fastest again with 3 * reps launches, and write the fastest
 * of that round into *inout.  CSR: row blocks, wave units, linear order, XCD
 * bands, wave tiles, V lanes per row, and, when x exceeds 4 MiB, row blocks
 * and wave tiles over 2 and 4 column bands.  CSR5: sigma in {4, 8, 16, 32};
 * when x exceeds 4 MiB each of them also over 2 and 4 column bands (8 too
 * above 32 MiB).  ELL: one wave or four waves per 64 rows.  SELL: C in {8,
 * 16, 32, 64} x sigma in {1, C, 8C, 256C, M} (M: one window over all rows),
 * C = 64 also with four and with six waves per chunk, and, when x exceeds
 * 4 MiB, C 32 and 64 with sigma = M over 2 and 4 column bands (8 above 32
 * MiB).  HYB: K in {rule, p50, p75, p90, p99, 0, 1, 2}, each with one or four
 * waves per 64 rows of the ELL part and with the COO tail over 2 and 4 column
 * bands when x exceeds 4 MiB (8 above 32 MiB).  ms_out (optional) receives
 * the best median.  The
 * result is cached for the life of the process, keyed by a 64-bit hash of
 * the sparsity structure (ptr, col), the shape, dtype, format, byte cap and
 * the caller's flags (the candidates keep the flags the grid does not set):
 * a second call for the same structure returns the cached choice without
 * timing (spmv_autotune_cache_clear empties the cache). */
spmv_status_t spmv_autotune(spmv_mat_t csr, spmv_fmt_t fmt, const void* x, void* y, int64_t scrub_bytes, int reps,
                            spmv_params_t* inout, double* ms_out, spmv_stream_t s);
void spmv_autotune_cache_clear(void);

/* ------------------------------------------------------------ selection */

/* The 12 static features of A (Sec. V-B, Table IV, plus nnz, ELL padding
 * ratio, bandwidth and Gini of row lengths), in FP64:
 * n_rows, n_cols, nnz, nnz_frac, nnz_min, nnz_max, nnz_avg, nnz_std,
 * variation (= std/avg), ell_pad (= M*max/nnz), bandwidth (max |i-j|),
 * gini.  Computed on the device; A must be CSR.  Synchronises s. */
spmv_status_t spmv_features(spmv_mat_t A, double out[12], spmv_stream_t s);

/* MLP selector, 12 -> 64 -> 64 -> 5, FP32, ReLU (Sec. V-D lists an MLP
 * among the classifiers).  Parameter vector (5317 floats): W1[12x64],
 * b1[64], W2[64x64], b2[64], W3[64x5], b3[5], W row-major (fan_in, fan_out).
 * A model also holds the feature scaler (per-feature min and max of the
 * training set after the log transform, Sec. V-B "Feature Scaling"). */
#define SPMV_MLP_NPARAM 5317
spmv_status_t spmv_model_create(const float* params, const double fmin[12], const double fmax[12],
                                spmv_model_t* out);
spmv_status_t spmv_model_load(const char* path, spmv_model_t* out);
spmv_status_t spmv_model_save(spmv_model_t m, const char* path);
spmv_status_t spmv_model_params(spmv_model_t m, float* params_out, double fmin[12], double fmax[12]);
void spmv_model_free(spmv_model_t m);

/* Predict the format for raw features (Sec. V-A: features -> scaled ->
 * model -> label): transform + scaling + forward + argmax on the device.
 * scores (optional) receives the 5 logits.  Ties go to the lower index. */
spmv_status_t spmv_select(spmv_model_t m, const double features[12], spmv_fmt_t* best, float scores[5]);

/* Training kernels, exported for gradient checks.  All pointers are device
 * memory, FP32.  X: B x 12 scaled features (row-major); params: 5317.
 * forward: Z (B x 5 logits), A1/A2 (B x 64 pre-activations, may be NULL).
 * backward: labels[B] int32 in 0..4; grads (5317) = d(mean CE)/d(params);
 * loss (1 float, optional).  adam: one step t >= 1 on params with moments
 * m, v (5317 each). */
spmv_status_t spmv_mlp_forward(const float* params, const float* X, int32_t B, float* Z, float* A1, float* A2,
                               spmv_stream_t s);
spmv_status_t spmv_mlp_backward(const float* params, const float* X, const int32_t* labels, int32_t B,
                                float* grads, float* loss, spmv_stream_t s);
spmv_status_t spmv_mlp_adam(float* params, const float* grads, float* m, float* v, int32_t t, float lr, float beta1,
                            float beta2, float eps, spmv_stream_t s);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid hipMalloc):
 * spmv_mlp_backward without any allocation.  Same arguments, kernels and
 * results as spmv_mlp_backward, but its scratch (activations, deltas and
 * per-sample losses of up to SPMV_NOALLOC_MAX_BATCH samples, 4.3 MB) is one
 * static array in the library's device code, which each GPU holds from the
 * first call on it until the process ends.  B > SPMV_NOALLOC_MAX_BATCH ->
 * SPMV_ERR_TOO_LARGE.  Only enqueues work on s (no synchronisation), so grads
 * and loss are ready when s reaches this point.  Every call on one GPU shares
 * that GPU's scratch: calls that may overlap on one GPU (different streams,
 * or host threads) race and must be serialised by the caller. */
#define SPMV_NOALLOC_MAX_BATCH 4096
spmv_status_t spmv_mlp_backward_noalloc(const float* params, const float* X, const int32_t* labels, int32_t B,
                                        float* grads, float* loss, spmv_stream_t s);
/* Feature transform + min-max scaling on the device: F (n x 12 FP64 raw
 * features) -> X (n x 12 FP32 scaled).  fmin/fmax: host arrays. */
spmv_status_t spmv_scale_features(const double* F, int32_t n, const double fmin[12], const double fmax[12],
                                  float* X, spmv_stream_t s);
/* Scaler fit: per-feature minimum and maximum of the transformed features
 * of F (n x 12 FP64 raw features, device), returned to the host. */
spmv_status_t spmv_feature_range(const double* F, int32_t n, double fmin[12], double fmax[12], spmv_stream_t s);
/* Whole training run: epochs x (n / batch) Adam steps over device data X
 * (n x 12 scaled), labels (n); order (epochs x n int32, device) gives the
 * sample order of every epoch; the last partial batch is used as is.
 * params (device, 5317) are trained in place; loss_out (host, epochs,
 * optional) receives each epoch's mean training loss.  Synchronises s. */
spmv_status_t spmv_mlp_train(float* params, const float* X, const int32_t* labels, int32_t n, const int32_t* order,
                             int32_t epochs, int32_t batch, float lr, spmv_stream_t s, float* loss_out);

#ifdef __cplusplus
}
#endif
#endif /* SPMV_H */
