// Structure work done once per handle: CSR validation, row statistics and the
// split-row plan, an exclusive scan, and the transposed structure built by a
// stable LSD radix sort on column index.  All integer work, bit-exact.
#include "internal.hpp"

namespace spmm {
namespace {

// ---------------------------------------------------------------------------
// Validation.  Status bits: 1 rowptr[0] != 0, 2 rowptr decreases, 4 rowptr[rows]
// != nnz, 8 rowptr outside [0, nnz], 16 column out of range, 32 columns not
// strictly increasing within a row.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) validate_rowptr_kernel(const int32_t* rowptr, int64_t rows, int64_t nnz,
                                                                 uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i > rows) return;
  uint32_t bad = 0;
  const int64_t a = rowptr[i];
  if (i == 0 && a != 0) bad |= 1u;
  if (a < 0 || a > nnz) bad |= 8u;
  if (i < rows && (int64_t)rowptr[i + 1] < a) bad |= 2u;
  if (i == rows && a != nnz) bad |= 4u;
  if (bad) atomicOr(status, bad);
}

// One wave per row; only launched once rowptr is known to be valid.
__global__ void __launch_bounds__(kBlock) validate_colind_kernel(const int32_t* rowptr, const int32_t* colind,
                                                                 int64_t rows, int64_t cols, uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (i >= rows) return;
  const int64_t p0 = rowptr[i], p1 = rowptr[i + 1];
  uint32_t bad = 0;
  for (int64_t p = p0 + lane; p < p1; p += 64) {
    const int32_t c = colind[p];
    if (c < 0 || c >= cols) bad |= 16u;
    if (p > p0 && colind[p - 1] >= c) bad |= 32u;
  }
  if (bad) atomicOr(status, bad);
}

// ---------------------------------------------------------------------------
// Row statistics and the split-row plan.
// A split row of combined length L is cut into units of max(segment, ceil(sqrt(L)))
// non-zeros of one k-tile: a unit then costs about as many dependent load rounds as
// the fix-up that sums the row's units, so neither becomes the tail.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t unit_length(int64_t len, int32_t segment) {
  int64_t r = (int64_t)sqrtf((float)len);
  while (r * r < len) ++r;
  return r > segment ? r : segment;
}

__global__ void __launch_bounds__(kBlock) plan_count_kernel(PlanCountParams P) {
  __shared__ unsigned long long s_stats[35];
  for (int t = threadIdx.x; t < 35; t += kBlock) s_stats[t] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < P.rows) {
    int64_t len = 0, units = 0;
    for (int k = 0; k < P.num_k; ++k) len += (int64_t)P.rowptr[k][i + 1] - P.rowptr[k][i];
    const int64_t sl = unit_length(len, P.segment);
    for (int k = 0; k < P.num_k; ++k) {
      const int64_t l = (int64_t)P.rowptr[k][i + 1] - P.rowptr[k][i];
      units += (l + sl - 1) / sl;
    }
    const bool split = len > P.long_row;
    P.nseg[i] = split ? (int32_t)units : 0;
    P.islong[i] = split ? 1 : 0;
    atomicMax(&s_stats[0], (unsigned long long)len);
    if (len == 0) atomicAdd(&s_stats[1], 1ull);
    const int bits = len == 0 ? 0 : 64 - __clzll((unsigned long long)len);
    atomicAdd(&s_stats[2 + bits], 1ull);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 35; t += kBlock) {
    if (s_stats[t] == 0) continue;
    if (t == 0)
      atomicMax(&P.stats[0], s_stats[0]);
    else
      atomicAdd(&P.stats[t], s_stats[t]);
  }
}

__global__ void __launch_bounds__(kBlock) plan_emit_kernel(PlanEmitParams P) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= P.rows || !P.islong[i]) return;
  int32_t o = P.seg_off[i];
  P.lrow[P.long_off[i]] = LongRow{(int32_t)i, o, o + P.nseg[i], 0};
  int64_t len = 0;
  for (int k = 0; k < P.num_k; ++k) len += (int64_t)P.rowptr[k][i + 1] - P.rowptr[k][i];
  const int32_t sl = (int32_t)unit_length(len, P.segment);
  for (int k = 0; k < P.num_k; ++k) {
    const int32_t p0 = P.rowptr[k][i], p1 = P.rowptr[k][i + 1];
    for (int64_t p = p0; p < p1; p += sl) {  // 64-bit: p + sl may pass 2^31 for a large unit
      const int64_t e = (p1 - p > sl) ? p + sl : p1;
      P.seg[o++] = Seg{(int32_t)i, k, (int32_t)p, (int32_t)e};
    }
  }
}

// ---------------------------------------------------------------------------
// Exclusive scan: 4096 elements per workgroup (16 per thread, blocked),
// recursive over workgroup sums.
// ---------------------------------------------------------------------------
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int32_t block_exclusive(int32_t v, int32_t* s_warp, int32_t* total) {
  // inclusive scan within the wave
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_warp[w] = x;
  __syncthreads();
  int32_t before = 0, all = 0;
#pragma unroll
  for (int q = 0; q < kBlock / 64; ++q) {
    if (q < w) before += s_warp[q];
    all += s_warp[q];
  }
  *total = all;
  return before + x - v;
}

__global__ void __launch_bounds__(kBlock) scan_reduce_kernel(const int32_t* in, int64_t n, int32_t* sums) {
  __shared__ int32_t s_warp[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t t = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q)
    if (base + q < n) t += in[base + q];
  int32_t total;
  block_exclusive(t, s_warp, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock) scan_tile_kernel(const int32_t* in, int32_t* out, int64_t n,
                                                           const int32_t* offsets, int32_t* total_out) {
  __shared__ int32_t s_warp[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t t = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = (base + q < n) ? in[base + q] : 0;
    t += v[q];
  }
  int32_t total;
  int32_t run = block_exclusive(t, s_warp, &total);
  const int32_t off = offsets ? offsets[blockIdx.x] : 0;
  run += off;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    if (base + q < n) out[base + q] = run;
    run += v[q];
  }
  if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total_out = off + total;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key = column, value = CSR position), 8-bit digits.
// Each workgroup owns a tile of 4096 consecutive entries, visited in 16 rounds
// of 256 so that thread order is entry order inside a round; an entry's rank
// is (digit count of earlier rounds) + (earlier waves of this round) + (earlier
// lanes of its wave holding the same digit).  The last makes every pass stable.
// ---------------------------------------------------------------------------
constexpr int kRsRounds = 16;
constexpr int kRsTile = kBlock * kRsRounds;

__global__ void __launch_bounds__(kBlock) radix_hist_kernel(const int32_t* keys, int64_t n, int shift,
                                                            int32_t* hist, int64_t nb) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsRounds; ++r) {
    const int64_t idx = base + (int64_t)r * kBlock + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kBlock) radix_scatter_kernel(const int32_t* kin, const int32_t* vin, int64_t n,
                                                               int shift, const int32_t* offs, int64_t nb,
                                                               int32_t* kout, int32_t* vout) {
  __shared__ int32_t s_base[256];
  __shared__ int32_t s_run[256];
  __shared__ int32_t s_wcnt[kBlock / 64][256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  s_base[tid] = offs[(int64_t)tid * nb + blockIdx.x];
  s_run[tid] = 0;
#pragma unroll
  for (int q = 0; q < kBlock / 64; ++q) s_wcnt[q][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsRounds; ++r) {
    const int64_t idx = base + (int64_t)r * kBlock + tid;
    const bool valid = idx < n;
    const int32_t key = valid ? kin[idx] : 0;
    const int32_t val = valid ? (vin ? vin[idx] : (int32_t)idx) : 0;
    const int d = (key >> shift) & 255;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot((d >> b) & 1);
      m &= ((d >> b) & 1) ? bb : ~bb;
    }
    const int rank = __popcll(m & lt);
    if (valid && rank == 0) s_wcnt[w][d] = __popcll(m);
    __syncthreads();
    if (valid) {
      int32_t pos = s_base[d] + s_run[d] + rank;
      for (int q = 0; q < w; ++q) pos += s_wcnt[q][d];
      vout[pos] = val;
      if (kout) kout[pos] = key;
    }
    __syncthreads();
    int32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) {
      sum += s_wcnt[q][tid];
      s_wcnt[q][tid] = 0;
    }
    s_run[tid] += sum;
    __syncthreads();
  }
}

// rowid[p] = row of CSR position p; one wave per row.
__global__ void __launch_bounds__(kBlock) expand_rows_kernel(const int32_t* rowptr, int64_t rows, int32_t* rowid) {
  const int64_t i = (int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
  if (i >= rows) return;
  const int lane = threadIdx.x & 63;
  for (int64_t p = (int64_t)rowptr[i] + lane; p < rowptr[i + 1]; p += 64) rowid[p] = (int32_t)i;
}

// cnt[c] += uses of column c (one device atomic per non-zero; integer sums, so the
// result does not depend on the order).
__global__ void __launch_bounds__(kBlock) count_columns_kernel(const int32_t* colind, int64_t nnz, int32_t* cnt) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p < nnz) atomicAdd(&cnt[colind[p]], 1);
}

__global__ void __launch_bounds__(kBlock) gather_rows_kernel(const int32_t* rowid, const int32_t* perm, int64_t nnz,
                                                             int32_t* colindT) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q < nnz) colindT[q] = rowid[perm[q]];
}

inline unsigned blocks_for(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_validate_rowptr(const int32_t* rowptr, int64_t rows, int64_t nnz, uint32_t* status,
                                  hipStream_t s) {
  hipLaunchKernelGGL(validate_rowptr_kernel, dim3(blocks_for(rows + 1, kBlock)), dim3(kBlock), 0, s, rowptr,
                     rows, nnz, status);
  return hipGetLastError();
}

hipError_t launch_validate_colind(const int32_t* rowptr, const int32_t* colind, int64_t rows, int64_t cols,
                                  uint32_t* status, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(validate_colind_kernel, dim3(blocks_for(rows, kBlock / 64)), dim3(kBlock), 0, s, rowptr,
                     colind, rows, cols, status);
  return hipGetLastError();
}

hipError_t launch_plan_count(const PlanCountParams& P, hipStream_t s) {
  if (P.rows == 0) return hipSuccess;
  hipLaunchKernelGGL(plan_count_kernel, dim3(blocks_for(P.rows, kBlock)), dim3(kBlock), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_plan_emit(const PlanEmitParams& P, hipStream_t s) {
  if (P.rows == 0) return hipSuccess;
  hipLaunchKernelGGL(plan_emit_kernel, dim3(blocks_for(P.rows, kBlock)), dim3(kBlock), 0, s, P);
  return hipGetLastError();
}

int64_t scan_temp_elems(int64_t n) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb <= 1) return 0;
  return 2 * nb + scan_temp_elems(nb);
}

hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* total, int32_t* temp,
                          hipStream_t s) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (n == 0) {
    if (total) return hipMemsetAsync(total, 0, sizeof(int32_t), s);
    return hipSuccess;
  }
  if (nb == 1) {
    hipLaunchKernelGGL(scan_tile_kernel, dim3(1), dim3(kBlock), 0, s, in, out, n, (const int32_t*)nullptr, total);
    return hipGetLastError();
  }
  int32_t* sums = temp;
  int32_t* offs = temp + nb;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive(sums, offs, nb, total, temp + 2 * nb, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_tile_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, (const int32_t*)offs,
                     (int32_t*)nullptr);
  return hipGetLastError();
}

hipError_t launch_count_columns(const int32_t* colind, int64_t nnz, int32_t* cnt, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(count_columns_kernel, dim3(blocks_for(nnz, kBlock)), dim3(kBlock), 0, s, colind, nnz, cnt);
  return hipGetLastError();
}

int64_t transpose_temp_bytes(int64_t rows, int64_t cols, int64_t nnz) {
  (void)rows;
  const int64_t nb = (nnz + kRsTile - 1) / kRsTile;
  const int64_t hist = 256 * (nb > 0 ? nb : 1);
  const int64_t scan = scan_temp_elems(hist > cols ? hist : cols);
  return 4 * (4 * nnz + hist + scan + 8) + 256;
}

hipError_t build_transpose(const int32_t* rowptr, const int32_t* colind, int64_t rows, int64_t cols, int64_t nnz,
                           int32_t* rowid, int32_t* rowptrT, int32_t* colindT, int32_t* perm, void* temp,
                           hipStream_t s) {
  hipError_t e;
  // rowptrT: column counts, then exclusive scan with the total in rowptrT[cols].
  e = hipMemsetAsync(rowptrT, 0, sizeof(int32_t) * (cols + 1), s);
  if (e != hipSuccess) return e;
  if (rows > 0) {
    hipLaunchKernelGGL(expand_rows_kernel, dim3(blocks_for(rows, kBlock / 64)), dim3(kBlock), 0, s, rowptr, rows,
                       rowid);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  int32_t* t = static_cast<int32_t*>(temp);
  int32_t* k0 = t;
  int32_t* k1 = t + nnz;
  int32_t* v0 = t + 2 * nnz;
  int32_t* v1 = t + 3 * nnz;
  const int64_t nb = (nnz + kRsTile - 1) / kRsTile;
  int32_t* hist = t + 4 * nnz;
  int32_t* scan_tmp = hist + 256 * (nb > 0 ? nb : 1);
  e = launch_count_columns(colind, nnz, rowptrT, s);
  if (e != hipSuccess) return e;
  e = scan_exclusive(rowptrT, rowptrT, cols, rowptrT + cols, scan_tmp, s);
  if (e != hipSuccess) return e;
  if (nnz == 0) return hipSuccess;
  // Radix passes over the bits that column indices < cols can occupy.
  int bits = 0;
  while (bits < 31 && ((int64_t)1 << bits) < cols) ++bits;
  const int passes = bits == 0 ? 1 : (bits + 7) / 8;
  const int32_t* kin = colind;
  const int32_t* vin = nullptr;  // first pass: value = position
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = 8 * pass;
    const bool last = pass == passes - 1;
    int32_t* kout = last ? nullptr : (pass % 2 == 0 ? k0 : k1);
    int32_t* vout = last ? perm : (pass % 2 == 0 ? v0 : v1);
    hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, kin, nnz, shift, hist, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = scan_exclusive(hist, hist, 256 * nb, nullptr, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, kin, vin, nnz, shift,
                       (const int32_t*)hist, nb, kout, vout);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    kin = kout;
    vin = vout;
  }
  hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for(nnz, kBlock)), dim3(kBlock), 0, s, rowid, perm, nnz,
                     colindT);
  return hipGetLastError();
}

}  // namespace spmm
