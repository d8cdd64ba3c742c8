// CSR5 (Sec. II-B, CSR5 paragraph; Table I): the nonzeros are cut into
// equal 2-D tiles of omega lanes x sigma entries, each lane owning sigma
// consecutive CSR entries; in memory the tile is transposed (slot (i, l) at
// t*omega*sigma + i*omega + l) so that for each i the omega lanes load
// omega consecutive slots.  Descriptors: tile_ptr (row of the tile's first
// entry), per-lane bit_flag (bit i = entry i starts a row; the tile's first
// slot is always flagged), y_off (flags in earlier lanes) and seg_off
// (following flag-free lanes).  The nnz mod omega*sigma tail stays in CSR
// order after the tiles.  CSR's ptr is kept.
//
// GPU design.  omega divides 64, so a wave64 holds 64/omega tiles; with the
// default omega = 64 a wave is one tile.  Each lane sums its entries,
// splitting at flags; rows that close inside the lane are written at once.
// The open tail of a lane is completed by a reverse segmented scan over the
// lanes of its tile (shuffles, log2(omega) steps), which is what y_off and
// seg_off encode for SIMD units without cross-lane shuffles: the kernel
// recomputes both from bit_flag with shuffles instead of loading them.  A
// tile whose first entry continues a row begun in an earlier tile writes
// that partial sum to carry[t]; a fix-up kernel adds each row's carries in
// tile order (one wave per row), so results are deterministic.  The tail
// is summed CSR-style by one extra workgroup.  Matrices with empty rows
// map the j-th flag of a tile to a row through the list of non-empty rows,
// and the writer of each non-empty row also zeroes the empty rows just
// before it.
#include "common.h"

namespace spmv {

static unsigned grid_n(int64_t n) {
  int64_t g = cdiv(n, BS);
  if (g < 1) g = 1;
  if (g > (1 << 20)) g = 1 << 20;
  return (unsigned)g;
}

// ----------------------------------------------------------- conversion
// first j in [0, M] with ptr[j] > v, minus 1 = the row holding entry v
__device__ __forceinline__ int64_t row_of_entry(const int32_t* ptr, int64_t M, int64_t v) {
  int64_t lo = 0, hi = M + 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (ptr[mid] > v) hi = mid;
    else lo = mid + 1;
  }
  return lo - 1;
}

__global__ void k_c5_tileptr(int64_t M, int64_t nnz, int64_t T, int64_t W, const int32_t* ptr, int32_t* tile_ptr,
                             int32_t* tile_row) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= T; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = t * W;
    const int64_t r = v < nnz ? row_of_entry(ptr, M, v) : M;
    tile_ptr[t] = (int32_t)(t < T ? r : M);
    tile_row[t] = (int32_t)r;
  }
}

__global__ void k_c5_starts(int64_t M, const int32_t* ptr, unsigned char* start) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x)
    if (ptr[r + 1] > ptr[r]) start[ptr[r]] = 1;
}

__global__ void k_c5_flags(int64_t T, int omega, int sigma, const unsigned char* start, uint32_t* flags) {
  const int64_t n = T * omega;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = q / omega, l = q % omega;
    const int64_t e0 = t * omega * sigma + l * sigma;
    uint32_t f = l == 0 ? 1u : 0u;
    for (int i = 0; i < sigma; ++i)
      if (start[e0 + i]) f |= 1u << i;
    flags[q] = f;
  }
}

__global__ void k_c5_desc(int64_t T, int omega, const uint32_t* flags, int32_t* y_off, int32_t* seg_off) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t* f = flags + t * omega;
    int32_t run = 0;
    for (int l = 0; l < omega; ++l) {
      y_off[t * omega + l] = run;
      run += __popc(f[l]);
    }
    int32_t empty_after = 0;  // flag-free lanes following lane l, counted from the right
    for (int l = omega - 1; l >= 0; --l) {
      seg_off[t * omega + l] = empty_after;
      empty_after = f[l] == 0 ? empty_after + 1 : 0;
    }
  }
}

template <typename T>
__global__ void k_c5_transpose(int64_t nnz, int64_t TW, int omega, int sigma, const int32_t* col, const T* val,
                               int32_t* ocol, T* oval) {
  const int64_t W = (int64_t)omega * sigma;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
    int64_t e = q;
    if (q < TW) {
      const int64_t t = q / W, rem = q % W, i = rem / omega, l = rem % omega;
      e = t * W + l * sigma + i;
    }
    ocol[q] = col[e];
    oval[q] = val[e];
  }
}

template <typename T>
__global__ void k_c5_untranspose(int64_t nnz, int64_t TW, int omega, int sigma, const int32_t* tcol, const T* tval,
                                 int32_t* col, T* val) {
  const int64_t W = (int64_t)omega * sigma;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t q = e;
    if (e < TW) {
      const int64_t t = e / W, rem = e % W, l = rem / sigma, i = rem % sigma;
      q = t * W + i * omega + l;
    }
    col[e] = tcol[q];
    val[e] = tval[q];
  }
}

__global__ void k_c5_nonempty(int64_t M, const int32_t* ptr, int32_t* nz) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x)
    nz[r] = ptr[r + 1] > ptr[r] ? 1 : 0;
}

__global__ void k_c5_nzrow(int64_t M, const int32_t* ptr, const int32_t* rank, int32_t* nzrow) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x)
    if (ptr[r + 1] > ptr[r]) nzrow[rank[r]] = (int32_t)r;
}

__global__ void k_c5_erows(int64_t M, const int32_t* ptr, const int32_t* rank, int32_t* erows) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x)
    if (ptr[r + 1] == ptr[r]) erows[r - rank[r]] = (int32_t)r;
}

__global__ void k_c5_nzbase(int64_t T, const int32_t* tile_ptr, const int32_t* rank, int32_t* base) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += (int64_t)gridDim.x * blockDim.x)
    base[t] = rank[tile_ptr[t]];
}

// tile t (1 <= t <= Tlast) continues a row begun earlier iff that row starts before t*W
__global__ void k_c5_chain_heads(int64_t Tlast, int64_t W, const int32_t* ptr, const int32_t* tile_row,
                                 int32_t* head) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= Tlast; t += (int64_t)gridDim.x * blockDim.x) {
    int32_t h = 0;
    if (t > 0) {
      const bool cont = ptr[tile_row[t]] < t * W;
      const bool prev_cont = (t - 1 > 0) && ptr[tile_row[t - 1]] < (t - 1) * W;
      h = cont && !(prev_cont && tile_row[t - 1] == tile_row[t]);
    }
    head[t] = h;
  }
}

__global__ void k_c5_chains(int64_t Tlast, const int32_t* head, const int32_t* pos, const int32_t* tile_row,
                            int32_t* chains) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= Tlast; t += (int64_t)gridDim.x * blockDim.x) {
    if (!head[t]) continue;
    const int32_t r = tile_row[t];
    int64_t lo = t, hi = Tlast + 1;  // first u > t with tile_row[u] > r
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (tile_row[mid] > r) hi = mid;
      else lo = mid + 1;
    }
    const int64_t c = pos[t];
    chains[3 * c] = r;
    chains[3 * c + 1] = (int32_t)t;
    chains[3 * c + 2] = (int32_t)(lo - 1);
  }
}

__global__ void k_c5_tail_rlo(int64_t M, int64_t TW, const int32_t* ptr, int32_t* out) {
  int64_t lo = 0, hi = M;  // first r in [0, M) with ptr[r] >= TW, else M
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (ptr[mid] >= TW) hi = mid;
    else lo = mid + 1;
  }
  *out = (int32_t)lo;
}

// The carry fix-up takes chains of at most C5_SHORT tiles one per thread and
// longer ones one per wave: short tiles (small sigma) make many short chains,
// for which a wave each leaves 60 of 64 lanes idle (zipf_1M, sigma 4 over two
// bands: 6.3 us per band pass with a wave per chain).  The chains are put
// short first (each group in tile order); A->nchains_short counts them.
constexpr int C5_SHORT = 32;

static spmv_status_t c5_split_chains(spmv_mat_s* A, hipStream_t s) {
  const int64_t n = A->nchains;
  std::vector<int32_t> h((size_t)n * 3), o;
  SPMV_TRY(copy_to_host(h.data(), A->chains, sizeof(int32_t) * h.size(), s));
  o.reserve(h.size());
  for (int pass = 0; pass < 2; ++pass)
    for (int64_t c = 0; c < n; ++c) {
      const bool shrt = h[3 * c + 2] - h[3 * c + 1] < C5_SHORT;
      if (shrt == (pass == 0)) o.insert(o.end(), {h[3 * c], h[3 * c + 1], h[3 * c + 2]});
      if (pass == 0 && shrt) ++A->nchains_short;
    }
  SPMV_HIP(hipMemcpyAsync(A->chains, o.data(), sizeof(int32_t) * o.size(), hipMemcpyHostToDevice, s));
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

spmv_status_t convert_csr5(spmv_mat_s* src, spmv_mat_s* A, hipStream_t s) {
  const int64_t M = src->M, nnz = src->nnz;
  const int omega = A->params.csr5_omega, sigma = A->params.csr5_sigma;
  if (omega < 1 || omega > 64) return fail(SPMV_ERR_UNSUPPORTED, "CSR5 omega=%d (1..64)", omega);
  if (sigma < 1 || sigma > 32) return fail(SPMV_ERR_UNSUPPORTED, "CSR5 sigma=%d (1..32)", sigma);
  const int64_t W = (int64_t)omega * sigma, T = nnz / W, TW = T * W;
  A->omega = omega;
  A->c5sigma = sigma;
  A->ntiles = T;
  // ptr is shared in content with CSR: keep a private copy
  SPMV_TRY(mat_alloc(A, (void**)&A->ptr, sizeof(int32_t) * (M + 1)));
  SPMV_HIP(hipMemcpyAsync(A->ptr, src->ptr, sizeof(int32_t) * (M + 1), hipMemcpyDeviceToDevice, s));
  SPMV_TRY(mat_alloc(A, (void**)&A->col, sizeof(int32_t) * nnz));
  SPMV_TRY(mat_alloc(A, &A->val, (size_t)A->sv * nnz));
  SPMV_TRY(mat_alloc(A, (void**)&A->tile_ptr, sizeof(int32_t) * (T + 1)));
  SPMV_TRY(mat_alloc(A, (void**)&A->tile_row, sizeof(int32_t) * (T + 1)));
  SPMV_TRY(mat_alloc(A, (void**)&A->bit_flag, sizeof(uint32_t) * T * omega));
  SPMV_TRY(mat_alloc(A, (void**)&A->y_off, sizeof(int32_t) * T * omega));
  SPMV_TRY(mat_alloc(A, (void**)&A->seg_off, sizeof(int32_t) * T * omega));
  SPMV_TRY(mat_alloc(A, (void**)&A->carry, sizeof(double) * (T + 1)));
  k_c5_tileptr<<<grid_n(T + 1), BS, 0, s>>>(M, nnz, T, W, src->ptr, A->tile_ptr, A->tile_row);
  SPMV_LAUNCH_CHECK();
  SPMV_TRY(copy_to_host(&A->c5_tail_row, A->tile_row + T, sizeof(int32_t), s));
  if (nnz) {
    if (A->dt == SPMV_F64)
      k_c5_transpose<double><<<grid_n(nnz), BS, 0, s>>>(nnz, TW, omega, sigma, src->col, (const double*)src->val,
                                                        A->col, (double*)A->val);
    else
      k_c5_transpose<float><<<grid_n(nnz), BS, 0, s>>>(nnz, TW, omega, sigma, src->col, (const float*)src->val, A->col,
                                                       (float*)A->val);
    SPMV_LAUNCH_CHECK();
  }
  if (T) {
    DTmp start;
    SPMV_TRY(start.alloc(nnz));
    SPMV_HIP(hipMemsetAsync(start.p, 0, nnz, s));
    k_c5_starts<<<grid_n(M), BS, 0, s>>>(M, src->ptr, start.as<unsigned char>());
    SPMV_LAUNCH_CHECK();
    k_c5_flags<<<grid_n(T * omega), BS, 0, s>>>(T, omega, sigma, start.as<unsigned char>(), A->bit_flag);
    SPMV_LAUNCH_CHECK();
    k_c5_desc<<<grid_n(T), BS, 0, s>>>(T, omega, A->bit_flag, A->y_off, A->seg_off);
    SPMV_LAUNCH_CHECK();
    SPMV_HIP(hipStreamSynchronize(s));
  }
  // empty rows
  DTmp nz, rank;
  SPMV_TRY(nz.alloc(sizeof(int32_t) * std::max<int64_t>(M, 1)));
  SPMV_TRY(rank.alloc(sizeof(int32_t) * (M + 1)));
  if (M) {
    k_c5_nonempty<<<grid_n(M), BS, 0, s>>>(M, src->ptr, nz.as<int32_t>());
    SPMV_LAUNCH_CHECK();
  }
  SPMV_TRY(scan_i32_to_i32(nz.as<int32_t>(), rank.as<int32_t>(), M, s));
  int32_t nnzrows = 0;
  SPMV_TRY(copy_to_host(&nnzrows, rank.as<int32_t>() + M, sizeof(int32_t), s));
  A->has_empty = nnzrows < M;
  if (A->has_empty) {
    SPMV_TRY(mat_alloc(A, (void**)&A->nzrow, sizeof(int32_t) * std::max<int32_t>(nnzrows, 1)));
    SPMV_TRY(mat_alloc(A, (void**)&A->tile_nzbase, sizeof(int32_t) * std::max<int64_t>(T, 1)));
    k_c5_nzrow<<<grid_n(M), BS, 0, s>>>(M, src->ptr, rank.as<int32_t>(), A->nzrow);
    SPMV_LAUNCH_CHECK();
    A->nerows = M - nnzrows;
    SPMV_TRY(mat_alloc(A, (void**)&A->erows, sizeof(int32_t) * A->nerows));
    k_c5_erows<<<grid_n(M), BS, 0, s>>>(M, src->ptr, rank.as<int32_t>(), A->erows);
    SPMV_LAUNCH_CHECK();
    if (T) {
      k_c5_nzbase<<<grid_n(T), BS, 0, s>>>(T, A->tile_ptr, rank.as<int32_t>(), A->tile_nzbase);
      SPMV_LAUNCH_CHECK();
    }
  }
  // tail start row, and the carry chains
  DTmp rlo;
  SPMV_TRY(rlo.alloc(sizeof(int32_t)));
  k_c5_tail_rlo<<<1, 1, 0, s>>>(M, TW, src->ptr, rlo.as<int32_t>());
  SPMV_LAUNCH_CHECK();
  SPMV_TRY(copy_to_host(&A->tail_rlo, rlo.p, sizeof(int32_t), s));
  const int64_t Tlast = TW < nnz ? T : T - 1;  // last index with a tile_row of its own
  A->nchains = 0;
  A->nchains_short = 0;
  if (Tlast >= 1) {
    DTmp head, pos;
    SPMV_TRY(head.alloc(sizeof(int32_t) * (Tlast + 1)));
    SPMV_TRY(pos.alloc(sizeof(int32_t) * (Tlast + 2)));
    k_c5_chain_heads<<<grid_n(Tlast + 1), BS, 0, s>>>(Tlast, W, src->ptr, A->tile_row, head.as<int32_t>());
    SPMV_LAUNCH_CHECK();
    SPMV_TRY(scan_i32_to_i32(head.as<int32_t>(), pos.as<int32_t>(), Tlast + 1, s));
    int32_t nch = 0;
    SPMV_TRY(copy_to_host(&nch, pos.as<int32_t>() + Tlast + 1, sizeof(int32_t), s));
    A->nchains = nch;
    SPMV_TRY(mat_alloc(A, (void**)&A->chains, sizeof(int32_t) * 3 * std::max<int32_t>(nch, 1)));
    if (nch) {
      k_c5_chains<<<grid_n(Tlast + 1), BS, 0, s>>>(Tlast, head.as<int32_t>(), pos.as<int32_t>(), A->tile_row,
                                                   A->chains);
      SPMV_LAUNCH_CHECK();
      SPMV_TRY(c5_split_chains(A, s));
    }
    SPMV_HIP(hipStreamSynchronize(s));
  }
  A->bytes_fmt = nnz * (4 + A->sv) + T * omega * 4 + (T + 1) * 4 + A->N * A->sv + A->M * A->sv +
                 (A->has_empty ? (int64_t)nnzrows * 8 + T * 4 + A->nerows * 4 : 0);
  SPMV_HIP(hipStreamSynchronize(s));
  return SPMV_OK;
}

spmv_status_t csr5_to_csr(spmv_mat_s* A, int32_t* ptr, int32_t* col, void* val, hipStream_t s) {
  SPMV_HIP(hipMemcpyAsync(ptr, A->ptr, sizeof(int32_t) * (A->M + 1), hipMemcpyDeviceToDevice, s));
  if (A->nnz) {
    const int64_t TW = A->ntiles * A->omega * A->c5sigma;
    if (A->dt == SPMV_F64)
      k_c5_untranspose<double><<<grid_n(A->nnz), BS, 0, s>>>(A->nnz, TW, A->omega, A->c5sigma, A->col,
                                                             (const double*)A->val, col, (double*)val);
    else
      k_c5_untranspose<float><<<grid_n(A->nnz), BS, 0, s>>>(A->nnz, TW, A->omega, A->c5sigma, A->col,
                                                            (const float*)A->val, col, (float*)val);
    SPMV_LAUNCH_CHECK();
  }
  return SPMV_OK;
}

// ------------------------------------------------------------------ SpMV
struct C5Args {
  int64_t ntiles, nb_main, nnz, M;
  int omega, sigma;
  const int32_t* ptr;
  const int32_t* tile_ptr;
  const uint32_t* flags;
  const int32_t* col;
  const int32_t* nzrow;
  const int32_t* nzbase;
  int32_t tail_rlo, tail_row;
  double* carry;
  const int32_t* erows;  // the empty rows (written 0 unless adding)
  int64_t nerows;
  int add;  // add the rows' sums onto y (a column band after the first)
};

template <typename T, bool EMPTY>
__device__ __forceinline__ void c5_write(const C5Args& a, int64_t t, int64_t row0, int64_t nzb, bool cont, int j,
                                         double s, T* __restrict__ y) {
  if (j == 0 && cont) {
    a.carry[t] = s;
    return;
  }
  if (!EMPTY) {
    put_y(y, row0 + j, s, a.add);
    return;
  }
  put_y(y, a.nzrow[nzb + j], s, a.add);  // empty rows are zeroed by k_csr5 (left alone when adding)
}

// The tail (entries past the last full tile) in CSR order.  Its leading
// continuation goes to carry[ntiles] (the last workgroup); the rows that
// start in it -- possibly many, when trailing rows are empty -- are spread
// over every wave of the grid, one row per wave at a time.
template <typename T>
__device__ void c5_tail(const C5Args& a, const T* __restrict__ val, const T* __restrict__ x, T* __restrict__ y) {
  __shared__ double sh[4];
  const int64_t TW = a.ntiles * (int64_t)a.omega * a.sigma;
  const int t = threadIdx.x, lane = __lane_id();
  if (blockIdx.x == gridDim.x - 1 && TW < a.nnz) {
    const int64_t rs = a.ptr[a.tail_row], re = a.ptr[a.tail_row + 1];
    if (rs < TW) {
      const double s = block_sum(row_dot(a.col, val, x, TW, re < a.nnz ? re : a.nnz, t, BS), sh);
      if (t == 0) a.carry[a.ntiles] = s;
    }
  }
  const int64_t nw = (int64_t)gridDim.x * (BS / WAVE);
  for (int64_t r = a.tail_rlo + (int64_t)blockIdx.x * (BS / WAVE) + t / WAVE; r < a.M; r += nw) {
    const double s = group_sum<64>(row_dot(a.col, val, x, a.ptr[r], a.ptr[r + 1], lane, WAVE));
    if (lane == 0) put_y(y, r, s, a.add);
  }
}

// One tile (omega lanes).  t and row0 are wave-uniform when W64.  PY: the
// tile adds onto y with the old values of each lane's first rows loaded
// beside its streams (see below).
template <typename T, int SIG, bool EMPTY, bool W64, bool PY = false>
__device__ __forceinline__ void c5_tile(const C5Args& a, int64_t t, int l, const T* __restrict__ val,
                                        const T* __restrict__ x, T* __restrict__ y) {
  const int omega = W64 ? WAVE : a.omega;
  const int sigma = SIG > 0 ? SIG : a.sigma;
  const int64_t W = (int64_t)omega * sigma, base = t * W;
  const uint32_t F = a.flags[t * omega + l];
  const int64_t row0 = W64 ? (int64_t)__builtin_amdgcn_readfirstlane(a.tile_ptr[t]) : (int64_t)a.tile_ptr[t];
  const bool cont = a.ptr[row0] < base;
  const int64_t nzb = EMPTY ? a.nzbase[t] : 0;
  // y_off: flags in earlier lanes of the tile.  (The lane scans stay on
  // cross-lane shuffles: DPP versions of both scans left the stencil's time
  // unchanged and, by raising occupancy, made the sigma = 32 tiles over two
  // column bands of a Zipf matrix slower, 174 -> 189 us.)
  const int pc = __popc(F);
  int inc = pc;
  for (int d = 1; d < omega; d <<= 1) {
    const int u = __shfl_up(inc, d, omega);
    if (l >= d) inc += u;
  }
  const int yoff = inc - pc;
  double acc = 0.0, head = 0.0;
  bool seen = false;
  int lf = 0;
  // Adding onto y (PY, a column band after the first): the lane writes rows
  // yoff, yoff + 1, ... in that order, so their old values (and, with empty
  // rows, their row numbers) for the first C5_PY of them are loaded beside
  // the tile's streams instead of one dependent load per row written
  // (zipf_1M, sigma = 16 over two bands: 169.5 -> 165 us).
  constexpr int C5_PY = 4;
  double yp[C5_PY] = {0.0, 0.0, 0.0, 0.0};
  int32_t rp[C5_PY] = {0, 0, 0, 0};
  int nw = 0;  // rows (or the carry) written so far
  auto put = [&](int j, double sum) {
    if (PY && SIG > 0 && nw < C5_PY && !(j == 0 && cont)) {  // (the prefetch is in the SIG > 0 path)
      const int64_t r = EMPTY ? (int64_t)rp[0] : row0 + j;
      y[r] = (T)(yp[0] + sum);
    } else {
      c5_write<T, EMPTY>(a, t, row0, nzb, cont, j, sum, y);
    }
    if (PY) {
#pragma unroll
      for (int u = 0; u + 1 < C5_PY; ++u) {
        yp[u] = yp[u + 1];
        rp[u] = rp[u + 1];
      }
      ++nw;
    }
  };
  if (SIG > 0) {
    int32_t c[SIG > 0 ? SIG : 1];
    T v[SIG > 0 ? SIG : 1], xv[SIG > 0 ? SIG : 1];
    const int32_t* cb = a.col + base;  // tile base (wave-uniform when W64)
    const T* vb = val + base;
#pragma unroll
    for (int i = 0; i < SIG; ++i) {
      c[i] = ldnt32(cb, (uint32_t)(i * omega + l));
      v[i] = ldnt32(vb, (uint32_t)(i * omega + l));
    }
    if (PY) {
      if (EMPTY) {
#pragma unroll
        for (int u = 0; u < C5_PY; ++u)
          if (u < pc) rp[u] = a.nzrow[nzb + yoff + u];
      }
#pragma unroll
      for (int u = 0; u < C5_PY; ++u)
        if (u < pc && !(yoff + u == 0 && cont)) yp[u] = (double)y[EMPTY ? (int64_t)rp[u] : row0 + yoff + u];
    }
    issue_fence();
#pragma unroll
    for (int i = 0; i < SIG; ++i) xv[i] = ld32(x, (uint32_t)c[i]);
    issue_fence();
#pragma unroll
    for (int i = 0; i < SIG; ++i) {
      if ((F >> i) & 1u) {
        if (seen) put(yoff + lf - 1, acc);
        else head = acc;
        seen = true;
        acc = 0.0;
        ++lf;
      }
      acc += (double)v[i] * (double)xv[i];
    }
  } else {
    for (int i = 0; i < sigma; ++i) {
      const int32_t ci = ldnt(a.col + base + (int64_t)i * omega + l);
      const T vi = ldnt(val + base + (int64_t)i * omega + l);
      if ((F >> i) & 1u) {
        if (seen) c5_write<T, EMPTY>(a, t, row0, nzb, cont, yoff + lf - 1, acc, y);
        else head = acc;
        seen = true;
        acc = 0.0;
        ++lf;
      }
      acc += (double)vi * (double)x[ci];
    }
  }
  if (!seen) head = acc;
  // reverse segmented scan over the tile's lanes: R_l = head_l + (lane l
  // flag-free ? R_{l+1} : 0), so R_{l+1} completes lane l's open segment
  double Rv = head;
  int Rs = seen ? 1 : 0;
  for (int d = 1; d < omega; d <<= 1) {
    const double ov = __shfl_down(Rv, d, omega);
    const int os = __shfl_down(Rs, d, omega);
    if (l + d < omega && !Rs) {
      Rv += ov;
      Rs = os;
    }
  }
  double S = __shfl_down(Rv, 1, omega);
  if (l == omega - 1) S = 0.0;
  if (seen) put(yoff + lf - 1, acc + S);
}

// Each lane group takes its tile (the loop covers grids smaller than the
// tile count); then the grid sums the CSR-ordered tail.
template <typename T, int SIG, bool EMPTY, bool W64, bool PY = false>
__global__ __launch_bounds__(BS) void k_csr5(C5Args a, const T* __restrict__ val, const T* __restrict__ x,
                                             T* __restrict__ y) {
  const int omega = W64 ? WAVE : a.omega;
  const int tpb = BS / omega;
  const int l = threadIdx.x % omega;
  const int64_t step = (int64_t)gridDim.x * tpb;
  const int64_t first = W64 ? (int64_t)blockIdx.x * tpb + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE)
                            : (int64_t)blockIdx.x * tpb + threadIdx.x / omega;
  if (EMPTY && !a.add)  // no tile writes an empty row: zero them beside the tiles
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < a.nerows; i += (int64_t)gridDim.x * BS)
      y[a.erows[i]] = (T)0;
  for (int64_t t = first; t < a.ntiles; t += step) c5_tile<T, SIG, EMPTY, W64, PY>(a, t, l, val, x, y);
  c5_tail<T>(a, val, x, y);
}

template <typename T>
__global__ __launch_bounds__(BS) void k_csr5_fix(int64_t nchains, const int32_t* __restrict__ chains,
                                                 const double* __restrict__ carry, T* __restrict__ y) {
  const int64_t c = (int64_t)blockIdx.x * (BS / WAVE) + threadIdx.x / WAVE;
  if (c >= nchains) return;
  const int32_t row = chains[3 * c], tb = chains[3 * c + 1], te = chains[3 * c + 2];
  double s = 0.0;
  for (int64_t u = tb + __lane_id(); u <= te; u += WAVE) s += carry[u];
  s = group_sum<64>(s);
  if (__lane_id() == 0) y[row] = (T)((double)y[row] + s);
}

// one thread per chain of at most C5_SHORT tiles: its carries in tile order
// (four loads in flight), then added onto the row
template <typename T>
__global__ __launch_bounds__(BS) void k_csr5_fix_short(int64_t nchains, const int32_t* __restrict__ chains,
                                                       const double* __restrict__ carry, T* __restrict__ y) {
  const int64_t c = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (c >= nchains) return;
  const int32_t row = chains[3 * c], tb = chains[3 * c + 1], te = chains[3 * c + 2];
  double s = 0.0;
  int32_t u = tb;
  for (; u + 3 <= te; u += 4) {
    const double a = carry[u], b = carry[u + 1], d = carry[u + 2], e = carry[u + 3];
    s = (((s + a) + b) + d) + e;
  }
  for (; u <= te; ++u) s += carry[u];
  y[row] = (T)((double)y[row] + s);
}

template <typename T, bool EMPTY, bool W64, bool PY = false>
static void launch_c5w(const C5Args& a, unsigned grid, const T* val, const T* x, T* y, hipStream_t s) {
  switch (a.sigma) {
    case 4: launch(k_csr5<T, 4, EMPTY, W64, PY>, grid, BS, s, a, val, x, y); break;
    case 8: launch(k_csr5<T, 8, EMPTY, W64, PY>, grid, BS, s, a, val, x, y); break;
    case 16: launch(k_csr5<T, 16, EMPTY, W64, PY>, grid, BS, s, a, val, x, y); break;
    case 32: launch(k_csr5<T, 32, EMPTY, W64, PY>, grid, BS, s, a, val, x, y); break;
    default: launch(k_csr5<T, 0, EMPTY, W64, PY>, grid, BS, s, a, val, x, y); break;
  }
}

template <typename T, bool EMPTY>
static void launch_c5(const C5Args& a, unsigned grid, const T* val, const T* x, T* y, hipStream_t s) {
  // adding onto y: the old values prefetched (sigma 4, 8 and 16; with sigma =
  // 32 the extra registers cost more than the dependent loads they save)
  if (a.omega == WAVE && a.add && (a.sigma == 4 || a.sigma == 8 || a.sigma == 16))
    launch_c5w<T, EMPTY, true, true>(a, grid, val, x, y, s);
  else if (a.omega == WAVE) launch_c5w<T, EMPTY, true>(a, grid, val, x, y, s);
  else launch_c5w<T, EMPTY, false>(a, grid, val, x, y, s);
}

template <typename T>
static spmv_status_t run_csr5_t(spmv_mat_s* A, const T* x, T* y, hipStream_t s) {
  if (A->M == 0) return SPMV_OK;
  if (A->omega < 1 || 64 % A->omega != 0)
    return fail(SPMV_ERR_UNSUPPORTED, "CSR5 SpMV needs omega dividing 64 (got %d)", A->omega);
  C5Args a;
  a.ntiles = A->ntiles;
  a.nb_main = cdiv(A->ntiles, BS / A->omega);
  a.nnz = A->nnz;
  a.M = A->M;
  a.omega = A->omega;
  a.sigma = A->c5sigma;
  a.ptr = A->ptr;
  a.tile_ptr = A->tile_ptr;
  a.flags = A->bit_flag;
  a.col = A->col;
  a.nzrow = A->nzrow;
  a.nzbase = A->tile_nzbase;
  a.tail_rlo = A->tail_rlo;
  a.tail_row = A->c5_tail_row;
  a.carry = A->carry;
  a.erows = A->erows;
  a.nerows = A->nerows;
  a.add = A->acc;
  // one workgroup per BS / omega tiles: the dispatcher balances them (a
  // persistent grid of 8 workgroups per CU was 4% slower on the stencil)
  const unsigned grid = (unsigned)std::max<int64_t>(1, a.nb_main);
  if (A->has_empty) launch_c5<T, true>(a, grid, (const T*)A->val, x, y, s);
  else launch_c5<T, false>(a, grid, (const T*)A->val, x, y, s);
  SPMV_LAUNCH_CHECK();
  if (A->nchains_short > 0) {  // a thread per short chain
    launch(k_csr5_fix_short<T>, (unsigned)cdiv(A->nchains_short, BS), BS, s, A->nchains_short, A->chains, A->carry,
           y);
    SPMV_LAUNCH_CHECK();
  }
  if (A->nchains > A->nchains_short) {  // a wave per long chain
    const int64_t nl = A->nchains - A->nchains_short;
    launch(k_csr5_fix<T>, (unsigned)cdiv(nl, BS / WAVE), BS, s, nl, A->chains + 3 * A->nchains_short, A->carry, y);
    SPMV_LAUNCH_CHECK();
  }
  return SPMV_OK;
}

spmv_status_t run_csr5(spmv_mat_s* A, const void* x, void* y, hipStream_t s) {
  if (A->dt == SPMV_F64) return run_csr5_t<double>(A, (const double*)x, (double*)y, s);
  return run_csr5_t<float>(A, (const float*)x, (float*)y, s);
}

}  // namespace spmv
