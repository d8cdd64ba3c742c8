// Internal declarations of libspmv (gfx950).  Not part of the C-ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "spmv.h"

namespace spmv {

constexpr int BS = 256;    // threads per workgroup for the streaming kernels (4 wave64s)
constexpr int WAVE = 64;

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
spmv_status_t fail(spmv_status_t st, const char* fmt, ...);

#define SPMV_HIP(expr)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return ::spmv::fail(SPMV_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),  \
                          __FILE__, __LINE__);                                                  \
  } while (0)

#define SPMV_TRY(expr)                   \
  do {                                   \
    spmv_status_t st_ = (expr);          \
    if (st_ != SPMV_OK) return st_;      \
  } while (0)

#define SPMV_LAUNCH_CHECK() SPMV_HIP(hipGetLastError())

// --------------------------------------------------------------- memory
// Device allocations go through these so that SPMV_MEM_CAP_BYTES can cap
// the library's live device memory (OOM is then reported, never a fault).
spmv_status_t dmalloc(void** p, size_t bytes);
void dfree(void* p);
int64_t mem_in_use();  // bytes the library holds from dmalloc (kept free blocks not counted)
int64_t mem_release(); // hands every kept free block back to HIP; returns the bytes released

// A scoped device buffer for temporaries inside conversions.  Its release
// waits for the device first, so no queued kernel can still be using it.
struct DTmp {
  void* p = nullptr;
  ~DTmp() {
    if (p) {
      (void)hipDeviceSynchronize();
      dfree(p);
    }
  }
  spmv_status_t alloc(size_t bytes) { return dmalloc(&p, bytes); }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

inline hipStream_t hs(spmv_stream_t s) { return reinterpret_cast<hipStream_t>(s); }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int value_size(spmv_dtype_t dt) { return dt == SPMV_F64 ? 8 : 4; }
int64_t default_max_bytes();
// Workgroups that fit on the device at once when each CU holds per_cu of them
// (persistent kernels size their grid with it).
int64_t resident_blocks(int per_cu);
spmv_status_t structure_hash(const spmv_mat_s* A, uint64_t* out, hipStream_t s);

// Kernel-bound timing.  While a RunTiming is armed on the calling thread,
// every kernel of a run path is launched through hipExtLaunchKernel: the
// first records `start` as it begins and each records `stop` as it ends
// (the last one's value stays), so stop - start spans exactly the kernels
// of one run, without the dispatch latency that separate event markers add.
struct RunTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local RunTiming* g_timing;

struct TimingArm {
  RunTiming t;
  RunTiming* prev;
  TimingArm(hipEvent_t a, hipEvent_t b) : prev(g_timing) {
    t.start = a;
    t.stop = b;
    g_timing = &t;
  }
  ~TimingArm() { g_timing = prev; }
};

// Runs f() with kernel-bound timing armed; a call that launched no kernel
// (an empty matrix) records both events on the stream.
template <typename F>
inline spmv_status_t timed_call(hipEvent_t a, hipEvent_t b, hipStream_t s, F&& f) {
  TimingArm arm(a, b);
  const spmv_status_t st = f();
  if (st == SPMV_OK && arm.t.start) {
    SPMV_HIP(hipEventRecord(a, s));
    SPMV_HIP(hipEventRecord(b, s));
  }
  return st;
}

template <typename... KArgs, typename... Args>
inline void launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t s, Args... args) {
  if (g_timing) {
    hipEvent_t a = g_timing->start;
    g_timing->start = nullptr;
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, g_timing->stop, 0, static_cast<KArgs>(args)...);
  } else {
    kernel<<<grid, block, 0, s>>>(static_cast<KArgs>(args)...);
  }
}

}  // namespace spmv

struct spmv_mat_s {
  spmv_fmt_t fmt = SPMV_FMT_CSR;
  spmv_dtype_t dt = SPMV_F64;
  int64_t M = 0, N = 0, nnz = 0;
  spmv_params_t params{};
  int sv = 8;
  std::vector<void*> owned;  // freed by spmv_mat_free

  // CSR arrays (CSR; CSR5 keeps ptr and stores col/val tile-transposed)
  int32_t* ptr = nullptr;
  int32_t* col = nullptr;
  void* val = nullptr;
  int32_t* blk_row = nullptr;  // CSR row blocks: block b owns rows [blk_row[b], blk_row[b+1])
  int64_t nblk = 0;
  int32_t* unit_row = nullptr; // CSR wave units: unit u owns rows [unit_row[u], unit_row[u+1])
  int64_t nunits = 0;
  int64_t ntiles_csr = 0;      // CSR wave tiles (SPMV_FLAG_CSR_TILES): tiles of TILE_E nonzeros
  int32_t* ct_start = nullptr;  // ntiles+1: first row starting at or after the tile's first entry (M at the end)
  int32_t* ct_cont = nullptr;   // ntiles+1: row holding the tile's first entry
  double* ct_head = nullptr;    // per tile: run scratch of the tile reduction (as the HYB COO pass)
  double* ct_tail = nullptr;
  int32_t* ct_trow = nullptr;
  int32_t* ct_info = nullptr;
  int64_t nseg = 0, nlong = 0; // CSR long rows cut into segments
  int32_t maxlen = -1;         // CSR: the longest row (-1: not known)
  int2* segs = nullptr;        // (row, first nonzero) per segment
  int4* longs = nullptr;       // (row, first segment, segment count) per long row
  double* seg_part = nullptr;  // segment partial sums (run scratch)
  // CSR column bands (SPMV_FLAG_CSR_BANDS): band b holds the entries with
  // col in [b*band_w, (b+1)*band_w) as a CSR of all M rows
  int32_t nbands = 0;
  int64_t band_w = 0;
  int32_t* bptr = nullptr;        // nbands x (M+1), each relative to its band's first entry
  int32_t* bcol = nullptr;        // nnz, band after band
  void* bval = nullptr;
  int32_t* bblk = nullptr;        // row blocks of every band, concatenated
  double* bpart = nullptr;        // nbands x M partial sums (run scratch)
  std::vector<int64_t> band_off;  // host: first entry of each band (nbands+1)
  std::vector<int64_t> band_nblk; // host: row blocks per band
  std::vector<int64_t> band_blk0; // host: first row block of each band in bblk

  // ELL, and the ELL part of HYB: column-major M x K, slot (i,k) at k*M + i
  int64_t K = 0;
  int32_t* ecol = nullptr;
  void* eval = nullptr;

  // SELL-C-sigma
  int32_t C = 0, sigma = 1;
  int64_t nchunks = 0, nslots = 0, Mpad = 0;
  int32_t* perm = nullptr;  // Mpad entries (nullptr when sigma == 1)
  int64_t* cs = nullptr;    // nchunks + 1 slot offsets
  int32_t* scol = nullptr;
  void* sval = nullptr;
  int64_t nitems = 0, nwide = 0;  // column-slice work items; chunks split into more than SELL_FUSE slices
  int32_t sell_maxw = 0;          // widest chunk (= longest row)
  int64_t kc_first = 0;           // chunks [kc_first, nchunks) are at most SELL_KC_MAX wide (one-pass kernel);
  int32_t kc_w = 0;               // the widest of them; chunks before kc_first go through the slice items
  int2* items = nullptr;          // (chunk, first column) per item
  int4* wide = nullptr;           // (chunk, first item, item count) per split chunk
  double* part = nullptr;         // nitems * C partial sums (run scratch, split chunks only)
  int32_t* wcnt = nullptr;        // per item: slices of its split chunk done (at the chunk's first item)

  // HYB COO part (row-major) and the per-tile scratch of its pass
  int64_t ncoo = 0;
  int32_t* crow = nullptr;
  int32_t* ccol = nullptr;
  void* cval = nullptr;
  double* coo_head = nullptr;   // per COO tile: partial sum of its first row when begun earlier (run scratch)
  double* coo_tail = nullptr;   // per COO tile: partial sum of its last row when it continues (run scratch)
  int32_t* coo_trow = nullptr;  // per COO tile: that last row
  int32_t* coo_tinfo = nullptr; // per COO tile: CT_TAIL / CT_SPAN / 0
  // HYB with bands > 1: the COO entries are ordered by column band, then by
  // row and column; band b's are [coo_boff[b], coo_boff[b+1]) (host, bands+1)
  std::vector<int64_t> coo_boff;

  // CSR5
  int32_t omega = 0, c5sigma = 0;
  int64_t ntiles = 0;
  int32_t* tile_ptr = nullptr;   // ntiles + 1 (last = M)
  uint32_t* bit_flag = nullptr;  // ntiles * omega packed words
  int32_t* y_off = nullptr;
  int32_t* seg_off = nullptr;
  int32_t* tile_row = nullptr;   // ntiles + 1: tile_ptr[0..T-1] and the row holding the first tail entry
  int32_t tail_rlo = 0;          // first row r with ptr[r] >= T*omega*sigma
  int32_t c5_tail_row = 0;       // row holding the first tail entry (M when there is no tail)
  int has_empty = 0;
  int32_t* nzrow = nullptr;      // non-empty rows, ascending (only when has_empty)
  int32_t* erows = nullptr;      // empty rows, ascending (only when has_empty)
  int64_t nerows = 0;
  int32_t* tile_nzbase = nullptr;
  int64_t nchains = 0;
  int32_t* chains = nullptr;     // (row, t_begin, t_end) triples for the carry fix-up
  int64_t nchains_short = 0;     // the first nchains_short chains span at most C5_SHORT tiles
  double* carry = nullptr;       // ntiles + 1 partial sums (run scratch)

  // Column bands (params.bands > 1, CSR, SELL and CSR5): sub[b] is the handle's
  // format built from the entries with col in [b*band_w, (b+1)*band_w), over
  // all M rows; this handle holds no format arrays of its own
  std::vector<std::unique_ptr<spmv_mat_s>> sub;
  int32_t acc = 0;  // a column band after the first: its run adds its product onto y instead of writing it

  int64_t bytes_fmt = 0, pad_slots = 0;

  void* own(void* p) {
    if (p) owned.push_back(p);
    return p;
  }
};

struct spmv_model_s {
  float* d_params = nullptr;  // device, SPMV_MLP_NPARAM
  double fmin[12], fmax[12];
  float h_params[SPMV_MLP_NPARAM];
};

namespace spmv {

// ----------------------------------------------------------- primitives
// Exclusive scan of n inputs into out[0..n]; out[n] is the total.
spmv_status_t scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, hipStream_t s);
spmv_status_t scan_i64_to_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
spmv_status_t scan_i32_to_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on the low key_bits bits.
// On return *keys / *vals point at whichever buffer holds the result (the
// input buffers or the given alternates).
spmv_status_t radix_sort_pairs(uint64_t** keys, uint32_t** vals, uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                               int key_bits, hipStream_t s);
spmv_status_t device_max_i32(const int32_t* ptr_lens_src, int64_t M, int lens_from_ptr, int32_t* out_host,
                             hipStream_t s);
spmv_status_t copy_to_host(void* dst, const void* src, size_t bytes, hipStream_t s);
spmv_status_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);

// ------------------------------------------------------------- builders
spmv_status_t csr_build_blocks(spmv_mat_s* A, hipStream_t s);
spmv_status_t csr_build_bands(spmv_mat_s* A, hipStream_t s);
spmv_status_t csr_build_tiles(spmv_mat_s* A, hipStream_t s);
// Splits src's entries by column band (band b: col in [b*bw, (b+1)*bw)) into
// nb CSRs of all M rows: bptr is nb x (M+1), each relative to its band's first
// entry off[b]; bcol / bval hold the bands one after another.
spmv_status_t csr_split_bands(const spmv_mat_s* src, int nb, int64_t bw, int32_t* bptr, int32_t* bcol, void* bval,
                              std::vector<int64_t>& off, hipStream_t s);
spmv_status_t convert_ell(spmv_mat_s* src, spmv_mat_s* A, hipStream_t s);
spmv_status_t convert_sell(spmv_mat_s* src, spmv_mat_s* A, hipStream_t s);
spmv_status_t convert_hyb(spmv_mat_s* src, spmv_mat_s* A, hipStream_t s);
spmv_status_t convert_csr5(spmv_mat_s* src, spmv_mat_s* A, hipStream_t s);
spmv_status_t to_csr_device(spmv_mat_s* A, int32_t* ptr, int32_t* col, void* val, hipStream_t s);

// ---------------------------------------------------------------- kernels
spmv_status_t run_csr(spmv_mat_s* A, const void* x, void* y, hipStream_t s);
spmv_status_t run_ell(spmv_mat_s* A, const void* x, void* y, hipStream_t s);
spmv_status_t run_sell(spmv_mat_s* A, const void* x, void* y, hipStream_t s);
spmv_status_t run_hyb(spmv_mat_s* A, const void* x, void* y, hipStream_t s);
spmv_status_t run_csr5(spmv_mat_s* A, const void* x, void* y, hipStream_t s);
spmv_status_t run_spmm(spmv_mat_s* A, const void* X, int64_t ldx, void* Y, int64_t ldy, int k, hipStream_t s);
spmv_status_t dispatch_run(spmv_mat_s* A, const void* x, void* y, hipStream_t s);
spmv_status_t convert_banded(spmv_mat_s* src, spmv_mat_s* A, hipStream_t s);
spmv_status_t convert_csr(spmv_mat_s* src, spmv_mat_s* A, hipStream_t s);
spmv_status_t run_banded(spmv_mat_s* A, const void* x, void* y, hipStream_t s);
spmv_status_t banded_to_csr(spmv_mat_s* A, int32_t* ptr, int32_t* col, void* val, hipStream_t s);

spmv_status_t mat_alloc(spmv_mat_s* A, void** p, size_t bytes);
void resolve_params(const spmv_params_t* in, spmv_params_t* out);
int64_t bytes_min(const spmv_mat_s* A);

}  // namespace spmv

// ------------------------------------------------------ device helpers
#ifdef __HIPCC__
namespace spmv {

template <typename T>
__device__ __forceinline__ T ldnt(const T* p) {
  return __builtin_nontemporal_load(p);
}

// Loads at a wave-uniform base plus a 32-bit per-lane element offset: the
// compiler can then use the scalar-base addressing form (one VGPR per
// address instead of a 64-bit pair), which keeps more loads in flight.
template <typename T>
__device__ __forceinline__ T ld32(const T* base, uint32_t idx) {
  return *(const T*)((const char*)base + idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T ldnt32(const T* base, uint32_t idx) {
  return __builtin_nontemporal_load((const T*)((const char*)base + idx * (uint32_t)sizeof(T)));
}

// y[i] = s, or y[i] + s (rounded once to the value type) when add is set --
// the runs of column bands after the first add onto the previous bands' sum.
template <typename TY>
__device__ __forceinline__ void put_y(TY* y, int64_t i, double s, int add) {
  y[i] = add ? (TY)((double)y[i] + s) : (TY)s;
}

// Keeps the compiler from moving work across this point: used after a batch
// of independent loads so that all of them are issued before the first wait.
__device__ __forceinline__ void issue_fence() { __builtin_amdgcn_sched_barrier(0); }

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }

// Sum over aligned groups of G lanes (G a power of two <= 64).
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double group_sum_rt(double v, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// MI355X dispatches workgroups round-robin over its 8 XCDs (each with its
// own L2).  This bijection gives each XCD a contiguous range of logical
// blocks, so neighbouring row blocks (which share x) share an L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t bid, uint32_t n) {
  const uint32_t q = n >> 3, r = n & 7u, x = bid & 7u, loc = bid >> 3;
  return x < r ? x * (q + 1) + loc : r * (q + 1) + (x - r) * q + loc;
}

// Sum of a 256-thread block (called by all threads; result valid in all).
__device__ __forceinline__ double block_sum(double v, double* sh /* >= 4 doubles of LDS */) {
  v = group_sum<64>(v);
  __syncthreads();
  if (__lane_id() == 0) sh[threadIdx.x / WAVE] = v;
  __syncthreads();
  double r = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return r;
}

// sum of val[k] * x[col[k]] over k = a + first, a + first + stride, ... < e
// (four independent loads per step, non-temporal loads of the matrix streams)
template <typename T>
__device__ __forceinline__ double row_dot(const int32_t* __restrict__ col, const T* __restrict__ val,
                                          const T* __restrict__ x, int64_t a, int64_t e, int first, int stride) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t k = a + first;
  for (; k + 3 * stride < e; k += 4 * stride) {
    const int32_t c0 = ldnt(col + k), c1 = ldnt(col + k + stride), c2 = ldnt(col + k + 2 * stride),
                  c3 = ldnt(col + k + 3 * stride);
    const T v0 = ldnt(val + k), v1 = ldnt(val + k + stride), v2 = ldnt(val + k + 2 * stride),
            v3 = ldnt(val + k + 3 * stride);
    const T x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
    s0 += (double)v0 * (double)x0;
    s1 += (double)v1 * (double)x1;
    s2 += (double)v2 * (double)x2;
    s3 += (double)v3 * (double)x3;
  }
  for (; k < e; k += stride) s0 += (double)ldnt(val + k) * (double)x[ldnt(col + k)];
  return (s0 + s1) + (s2 + s3);
}

// ------------------------------------------------- wave tiles of entries
// A wave reduces TILE_S * 64 consecutive entries in row order (lane l holds
// entries s*64 + l, s < TILE_S): the caller has loaded, for each place, the
// column, the value and the row (TILE_NONE past the last entry), and passes
// the row that continues into the tile from before (rprev, else -1) and the
// row that continues after it (rnext, else -2).  Rows are reduced by a
// segmented scan over the lanes of each slice, carried from slice to slice.
// A row that ends in the tile and began in it is written to y (added to the
// value y holds when ADD, whose load goes out with the gathers); a row
// crossing tile boundaries leaves tail_part in the tile where it starts and
// head_part in each later tile it reaches, and k_tile_fix finishes it.
// Cross-lane steps of the tile reduction, as DPP moves (ALU, no LDS round
// trip): within-row shifts (row_shr:d), the row broadcasts of lanes 15 and
// 31 that carry a scan across the four 16-lane rows, and whole-wave shifts
// by one lane.  A lane with no source (or in a row the mask leaves out)
// reads `old`.
enum : int { DPP_ROW_SR1 = 0x111, DPP_ROW_SR2 = 0x112, DPP_ROW_SR4 = 0x114, DPP_ROW_SR8 = 0x118,
             DPP_WF_SL1 = 0x130, DPP_WF_SR1 = 0x138, DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143 };

template <int CTRL, int ROWS>
__device__ __forceinline__ int32_t dpp_i(int32_t v, int32_t old) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {  // old = +0.0
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)(uint32_t)b, CTRL, ROWS, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)(uint32_t)(b >> 32), CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(b >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// one step of a segmented inclusive scan: add the source's partial unless a
// row already started at or before this lane within the window
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_step(double& v, int32_t& f) {
  const double vn = dpp_d<CTRL, ROWS>(v);
  const int32_t fn = dpp_i<CTRL, ROWS>(f, 0);
  if (!f) {
    v += vn;
    f = fn;
  }
}
// segmented inclusive scan of v over the 64 lanes, f = 1 where a row starts;
// returns with f = 1 where a row started at or before the lane
__device__ __forceinline__ void seg_scan64(double& v, int32_t& f) {
  seg_step<DPP_ROW_SR1, 0xf>(v, f);
  seg_step<DPP_ROW_SR2, 0xf>(v, f);
  seg_step<DPP_ROW_SR4, 0xf>(v, f);
  seg_step<DPP_ROW_SR8, 0xf>(v, f);
  seg_step<DPP_ROW_BCAST15, 0xa>(v, f);
  seg_step<DPP_ROW_BCAST31, 0xc>(v, f);
}
// inclusive running maximum over the 64 lanes (values >= -1)
__device__ __forceinline__ int32_t max_scan64(int32_t v) {
  constexpr int32_t LOW = -2147483647 - 1;
  int32_t u;
  u = dpp_i<DPP_ROW_SR1, 0xf>(v, LOW); v = u > v ? u : v;
  u = dpp_i<DPP_ROW_SR2, 0xf>(v, LOW); v = u > v ? u : v;
  u = dpp_i<DPP_ROW_SR4, 0xf>(v, LOW); v = u > v ? u : v;
  u = dpp_i<DPP_ROW_SR8, 0xf>(v, LOW); v = u > v ? u : v;
  u = dpp_i<DPP_ROW_BCAST15, 0xa>(v, LOW); v = u > v ? u : v;
  u = dpp_i<DPP_ROW_BCAST31, 0xc>(v, LOW); v = u > v ? u : v;
  return v;
}

constexpr int TILE_S = 16;
constexpr int TILE_E = WAVE * TILE_S;
constexpr int32_t TILE_NONE = 0x7fffffff;
constexpr int32_t TILE_TAIL = 1;  // the tile's last row starts in it and continues into the next tile
constexpr int32_t TILE_SPAN = 2;  // one row covers the whole tile and continues on both sides

template <typename T, bool ADD>
__device__ __forceinline__ void wave_tile_reduce(int64_t t, int nv, const int32_t (&rr)[TILE_S],
                                                 const int32_t (&cc)[TILE_S], const T (&vv)[TILE_S],
                                                 int32_t rprev, int32_t rnext, const T* __restrict__ x,
                                                 T* __restrict__ y, double* __restrict__ head_part,
                                                 double* __restrict__ tail_part, int32_t* __restrict__ tail_row,
                                                 int32_t* __restrict__ tinfo) {
  const int l = __lane_id();
  // a place ends its row when the next entry is another row
  bool en[TILE_S];
#pragma unroll
  for (int s = 0; s < TILE_S; ++s) {
    const int32_t dn = dpp_i<DPP_WF_SL1, 0xf>(rr[s], 0);  // lane l + 1's row (lane 63: none)
    const int32_t n0 = __builtin_amdgcn_readlane(rr[s + 1 < TILE_S ? s + 1 : s], 0);  // next slice's first row
    const int32_t nx = l < WAVE - 1 ? dn : (s + 1 < TILE_S ? n0 : rnext);
    en[s] = rr[s] != TILE_NONE && rr[s] != nx;
  }
  T xg[TILE_S], yg[TILE_S];
#pragma unroll
  for (int s = 0; s < TILE_S; ++s) xg[s] = ld32(x, (uint32_t)cc[s]);
  if (ADD) {
#pragma unroll
    for (int s = 0; s < TILE_S; ++s) yg[s] = en[s] && rr[s] != rprev ? y[rr[s]] : (T)0;
  }
  issue_fence();
  double carry = 0.0, last_v = 0.0;
  int32_t prev_last = rprev;
#pragma unroll
  for (int s = 0; s < TILE_S; ++s) {
    const int32_t r = rr[s];
    const int32_t up = dpp_i<DPP_WF_SR1, 0xf>(r, 0);  // lane l - 1's row (lane 0: none)
    const int32_t rp = l > 0 ? up : prev_last;
    double v = r != TILE_NONE ? (double)vv[s] * (double)xg[s] : 0.0;
    int32_t f = r != rp;  // a row starts here
    seg_scan64(v, f);     // segmented inclusive scan over the slice
    if (!f) v += carry;   // the row continues from the previous slice
    if (en[s]) {
      if (r == rprev) head_part[t] = v;  // the tile's first row, begun in an earlier tile
      else y[r] = ADD ? (T)((double)yg[s] + v) : (T)v;
    }
    if (s * WAVE + l == nv - 1) last_v = v;
    carry = readlane_d(v, WAVE - 1);
    prev_last = __builtin_amdgcn_readlane(r, WAVE - 1);
  }
  // the last entry's row, if it continues into the next tile
  const int ll = __builtin_amdgcn_readfirstlane((nv - 1) % WAVE), sl = (nv - 1) / WAVE;
  int32_t last_r = TILE_NONE;
#pragma unroll
  for (int s = 0; s < TILE_S; ++s)
    if (s == sl) last_r = __builtin_amdgcn_readlane(rr[s], ll);
  last_v = readlane_d(last_v, ll);
  if (l == 0) {
    int32_t info = 0;
    if (last_r == rnext) {
      if (last_r == rprev) {
        head_part[t] = last_v;
        info = TILE_SPAN;
      } else {
        tail_part[t] = last_v;
        tail_row[t] = last_r;
        info = TILE_TAIL;
      }
    }
    tinfo[t] = info;
  }
}

// one thread per tile whose last row continues: the row's partial sums in
// tile order, then into y (added to it when ADD)
template <typename T, bool ADD>
__global__ void k_tile_fix(int64_t ntiles, const double* __restrict__ head_part, const double* __restrict__ tail_part,
                           const int32_t* __restrict__ tail_row, const int32_t* __restrict__ tinfo,
                           T* __restrict__ y) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * blockDim.x) {
    if (tinfo[t] != TILE_TAIL) continue;
    const int32_t r = tail_row[t];
    const double yo = ADD ? (double)y[r] : 0.0;  // loaded before the partials, not after them
    double tot = tail_part[t];
    for (int64_t u = t + 1;; ++u) {
      tot += head_part[u];
      if (tinfo[u] != TILE_SPAN) break;
    }
    y[r] = ADD ? (T)(yo + tot) : (T)tot;
  }
}

}  // namespace spmv
#endif
