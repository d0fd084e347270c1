// Local sparse-times-sparse product C = A B (CSR x CSR -> CSR), the local step of
// the paper's SpGEMM experiments (Section 6.2 multiplies C = A A with the same
// distributed algorithms; each GPU runs a local SpGEMM per tile pair).
//
// Row-wise (Gustavson) product: row i of C is the sum over p in row i of A of
// a_p times row colA[p] of B.  Two phases, both binned by row:
//  * symbolic (at plan creation): the number of products of each row, then the
//    number of distinct output columns: rows with few products in a wave-local LDS
//    hash set, the others in a workgroup-wide bitmap over all N columns (LDS when
//    it fits, else a global slot), new bits counted as they are set;
//  * numeric: rows with few output entries accumulate in a wave-local LDS hash
//    table, medium rows in a workgroup-wide LDS table, both bitonic-sorted by column
//    afterwards; long rows accumulate in a dense global row (values + bitmap) owned
//    by one workgroup, then compacted in column order (sorted for free) and cleared.
// Every product (p, q) of a row is visited once: the row's A entries are taken 64
// (a wave) or 1024 (a workgroup) at a time, the lengths of their B rows are
// prefix-summed, and each lane takes products t, t + lanes, ... locating its A entry
// by binary search in the prefix, so that short B rows still fill every lane.
// Output columns are sorted and the pattern is exact; values are FP32 sums whose
// order inside a row follows the atomics (no fixed order).
#include <algorithm>
#include <new>
#include <vector>

#include "internal.hpp"
#include "spmm.h"

namespace spmm {
namespace {

constexpr int kWG = 1024;            // threads of the workgroup-wide kernels
constexpr int kWGWaves = kWG / 64;

__device__ __forceinline__ uint32_t hash_slot(int32_t col, int shift) {
  return ((uint32_t)col * 2654435761u) >> shift;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int64_t wave_sum64(int64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int lo = __shfl_xor((int)(uint32_t)x, o, 64);
    const int hi = __shfl_xor((int)(x >> 32), o, 64);
    x += (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
  }
  return x;
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

struct SgOperands {
  const int32_t* rowptrA;
  const int32_t* colA;
  const float* valA;
  const int32_t* rowptrB;
  const int32_t* colB;
  const float* valB;
  int64_t M, N;
};

// Products of every row: sum over p in row i of the length of B row colA[p].
__global__ void __launch_bounds__(kBlock) row_products_kernel(SgOperands O, int64_t* fl) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); i < O.M;
       i += (int64_t)gridDim.x * (kBlock / 64)) {
    int64_t acc = 0;
    for (int64_t p = O.rowptrA[i] + lane; p < O.rowptrA[i + 1]; p += 64) {
      const int32_t k = O.colA[p];
      acc += O.rowptrB[k + 1] - O.rowptrB[k];
    }
    acc = wave_sum64(acc);
    if (lane == 0) fl[i] = acc;
  }
}

// First position in colB[lo, hi) whose column is >= x (colB is sorted within a row).
__device__ __forceinline__ int32_t lower_bound(const int32_t* colB, int32_t lo, int32_t hi, int32_t x) {
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (colB[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Visit products with one wave: f(col, a * b).  The wave takes A entries in chunks of
// 64 starting at a0 and advancing by `step` (64 for a wave on its own; 64 x waves when
// the waves of a workgroup share a row), up to a1.  With WIN, only the products whose
// column lies in [c0, c1): each B row is cut to that range, by the split table when
// given (bsplit[k * stride + win] = first position at column >= win * window) or by
// binary search.  s_pref/s_start/s_aval hold 64 entries each (this wave's).
template <bool VALS, bool WIN = false, typename F>
__device__ __forceinline__ void wave_products(const SgOperands& O, int32_t a0, int32_t a1, int32_t* s_pref,
                                              int32_t* s_start, float* s_aval, F&& f, int32_t step = 64,
                                              int32_t c0 = 0, int32_t c1 = 0, const int32_t* bsplit = nullptr,
                                              int64_t stride = 0, int win = 0) {
  const int lane = threadIdx.x & 63;
  for (int32_t c = a0; c < a1; c += step) {
    const int n = min(64, a1 - c);
    int32_t st = 0, len = 0;
    float av = 0.0f;
    if (lane < n) {
      const int32_t k = O.colA[c + lane];
      st = O.rowptrB[k];
      int32_t en = O.rowptrB[k + 1];
      if constexpr (WIN) {
        if (bsplit) {
          const int32_t* sp = bsplit + (int64_t)k * stride + win;
          st = sp[0];
          en = sp[1];
        } else {
          st = lower_bound(O.colB, st, en, c0);
          en = lower_bound(O.colB, st, en, c1);
        }
      }
      len = en - st;
      if constexpr (VALS) av = O.valA[c + lane];
    }
    int32_t incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    s_pref[lane] = incl - len;
    s_start[lane] = st;
    if constexpr (VALS) s_aval[lane] = av;
    const int32_t tot = __builtin_amdgcn_readlane(incl, 63);
    wave_sync_lds();
    // four products per lane per pass: their searches and loads are independent, so
    // their latencies overlap
    for (int32_t t0 = lane; t0 < tot; t0 += 4 * 64) {
      int32_t col[4];
      float prod[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t t = t0 + u * 64;
        const int32_t tc = t < tot ? t : tot - 1;
        int pi = 0;
#pragma unroll
        for (int sp = 32; sp > 0; sp >>= 1)
          if (s_pref[pi + sp] <= tc) pi += sp;
        const int32_t q = s_start[pi] + (tc - s_pref[pi]);
        col[u] = O.colB[q];
        prod[u] = VALS ? s_aval[pi] * O.valB[q] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (t0 + u * 64 < tot) f(col[u], prod[u]);
    }
    wave_sync_lds();
  }
}

// Exclusive scan of one value per thread over a kWG-thread workgroup; returns the
// total.  s_tmp holds kWGWaves ints.
__device__ __forceinline__ int32_t block_scan(int32_t v, int32_t* excl, int32_t* s_tmp) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_tmp[w] = incl;
  __syncthreads();
  int32_t base = 0, total = 0;
  for (int u = 0; u < kWGWaves; ++u) {
    const int32_t x = s_tmp[u];
    if (u < w) base += x;
    total += x;
  }
  __syncthreads();
  *excl = base + incl - v;
  return total;
}

// Visit the products of the workgroup's B-row segments: thread tid < n holds segment
// [st, st + len) of B (len = 0 elsewhere) scaled by av; f(col, av * b) for each entry.
// The lengths are prefix-summed, each wave takes one contiguous share (1/kWGWaves) of
// the products and its lanes take consecutive ones (lane l: l, l + 64, ...): one binary
// search in the prefix per lane, then a forward step over segment boundaries, four
// loads in flight; the 64 loads of an instruction are consecutive entries of one or two
// B rows, so they coalesce.  Ends with a barrier.
// LDS: s_pref[kWG + 1], s_start[kWG], s_aval[kWG], s_tmp[kWGWaves].
template <bool VALS, typename F>
__device__ __forceinline__ void walk_products(const SgOperands& O, int32_t st, int32_t len, float av,
                                              int32_t* s_pref, int32_t* s_start, float* s_aval, int32_t* s_tmp,
                                              F&& f) {
  const int tid = threadIdx.x;
  int32_t excl;
  const int32_t tot = block_scan(len, &excl, s_tmp);
  s_pref[tid] = excl;
  s_start[tid] = st;
  if constexpr (VALS) s_aval[tid] = av;
  if (tid == 0) s_pref[kWG] = tot;
  __syncthreads();
  // each wave takes a contiguous share of the products; its lanes take consecutive
  // products (lane l: l, l + 64, ...), so the B loads of a wave are contiguous
  constexpr int kWaves = kWG / 64;
  const int lane = tid & 63, wv = tid >> 6;
  const int32_t per_wave = (((tot + kWaves - 1) / kWaves) + 63) & ~63;
  const int32_t w0 = wv * per_wave;
  const int32_t w1 = min(w0 + per_wave, tot);
  int32_t t = w0 + lane;
  if (t < w1) {
    int pi = 0;
#pragma unroll
    for (int step = kWG / 2; step > 0; step >>= 1)
      if (s_pref[pi + step] <= t) pi += step;
    int32_t next = s_pref[pi + 1];
    int32_t base = s_start[pi] - s_pref[pi];
    float a = VALS ? s_aval[pi] : 0.0f;
    while (t < w1) {
      int32_t qs[4];
      float as[4];
      int cnt = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        qs[u] = 0;
        as[u] = 0.0f;
        if (t < w1) {
          while (t >= next) {  // forward to the segment holding t
            ++pi;
            next = s_pref[pi + 1];
            base = s_start[pi] - s_pref[pi];
            if constexpr (VALS) a = s_aval[pi];
          }
          qs[u] = base + t;
          as[u] = a;
          t += 64;
          cnt = u + 1;
        }
      }
      int32_t col[4];
      float prod[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t qq = qs[u < cnt ? u : 0];
        col[u] = O.colB[qq];
        prod[u] = VALS ? as[u] * O.valB[qq] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (u < cnt) f(col[u], prod[u]);
    }
  }
  __syncthreads();
}

// Visit the products of A entries [a0, a1) with the whole workgroup: f(col, a * b);
// with WIN, only the products whose column lies in [c0, c1), each B row cut to that
// range by the split table when given (bsplit[k * stride + win] = first position at
// column >= win * window) or by binary search.  kWG A entries at a time.
template <bool VALS, bool WIN, typename F>
__device__ __forceinline__ void block_products(const SgOperands& O, int32_t a0, int32_t a1, int32_t* s_pref,
                                               int32_t* s_start, float* s_aval, int32_t* s_tmp, F&& f,
                                               int32_t c0 = 0, int32_t c1 = 0, const int32_t* bsplit = nullptr,
                                               int64_t stride = 0, int win = 0) {
  const int tid = threadIdx.x;
  for (int32_t c = a0; c < a1; c += kWG) {
    const int n = min(kWG, a1 - c);
    int32_t st = 0, len = 0;
    float av = 0.0f;
    if (tid < n) {
      const int32_t k = O.colA[c + tid];
      st = O.rowptrB[k];
      int32_t en = O.rowptrB[k + 1];
      if constexpr (WIN) {
        if (bsplit) {
          const int32_t* sp = bsplit + (int64_t)k * stride + win;
          st = sp[0];
          en = sp[1];
        } else {
          st = lower_bound(O.colB, st, en, c0);
          en = lower_bound(O.colB, st, en, c1);
        }
      }
      len = en - st;
      if constexpr (VALS) av = O.valA[c + tid];
    }
    walk_products<VALS>(O, st, len, av, s_pref, s_start, s_aval, s_tmp, f);
  }
}

// ---------------------------------------------------------------- symbolic

// Rows with at most TS/2 products: distinct columns in a wave-local hash set.
template <int TS>
__global__ void __launch_bounds__(kBlock) sym_wave_kernel(SgOperands O, const int32_t* rows, int64_t n_rows,
                                                          int32_t* nnz_row) {
  constexpr int W = kBlock / 64;
  constexpr int SHIFT = 32 - __builtin_ctz(TS);
  __shared__ int32_t s_tab[W][TS];
  __shared__ int32_t s_pref[W][64], s_start[W][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t* tab = s_tab[w];
  for (int64_t r = (int64_t)blockIdx.x * W + w; r < n_rows; r += (int64_t)gridDim.x * W) {
    const int32_t i = rows[r];
    for (int j = lane; j < TS; j += 64) tab[j] = -1;
    wave_sync_lds();
    int cnt = 0;
    wave_products<false>(O, O.rowptrA[i], O.rowptrA[i + 1], s_pref[w], s_start[w], nullptr,
                         [&](int32_t col, float) {
                           uint32_t h = hash_slot(col, SHIFT);
                           for (int probe = 0; probe < TS; ++probe) {  // the table is at most half full
                             const int32_t old = atomicCAS(&tab[h], -1, col);
                             if (old == -1) {
                               ++cnt;
                               break;
                             }
                             if (old == col) break;
                             h = (h + 1) & (TS - 1);
                           }
                         });
    cnt = wave_sum(cnt);
    if (lane == 0) nnz_row[i] = cnt;
    wave_sync_lds();
  }
}

// Other rows: one workgroup per row, a bitmap over the N output columns (LDS when
// `words` fit, else the workgroup's global slot), counting bits as they turn on.
// With wcnt, also the entries per column window of 2^(win_words_log2 + 5) columns:
// wcnt[r * n_win + w] for the r-th row of the list (they place long rows' windows).
template <bool GLOBAL>
__global__ void __launch_bounds__(kWG) sym_bitmap_kernel(SgOperands O, const int32_t* rows, int64_t n_rows,
                                                         int32_t* nnz_row, uint32_t* gbits, int64_t slot_words,
                                                         int32_t* wcnt, int n_win, int win_words_log2) {
  extern __shared__ int32_t s_dyn[];
  int32_t* s_pref = s_dyn;
  int32_t* s_start = s_pref + kWG + 1;
  int32_t* s_tmp = s_start + kWG;
  int32_t* s_cnt = s_tmp + kWGWaves;
  int32_t* s_wc = s_cnt + kWGWaves;  // n_win counters when wcnt is given
  uint32_t* bits = GLOBAL ? gbits + (int64_t)blockIdx.x * slot_words
                          : reinterpret_cast<uint32_t*>(s_wc + (wcnt ? n_win : 0));
  const int64_t words = (O.N + 31) / 32;
  const int tid = threadIdx.x;
  if constexpr (!GLOBAL) {
    for (int64_t j = tid; j < words; j += kWG) bits[j] = 0u;
  }
  if (wcnt)
    for (int w = tid; w < n_win; w += kWG) s_wc[w] = 0;
  __syncthreads();
  for (int64_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
    const int32_t i = rows[r];
    int cnt = 0;
    block_products<false, false>(O, O.rowptrA[i], O.rowptrA[i + 1], s_pref, s_start, nullptr, s_tmp,
                                 [&](int32_t col, float) {
                                   const uint32_t bit = 1u << (col & 31);
                                   uint32_t old;
                                   if constexpr (GLOBAL)
                                     old = __hip_atomic_fetch_or(bits + (col >> 5), bit, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
                                   else
                                     old = atomicOr(bits + (col >> 5), bit);
                                   if (!(old & bit)) ++cnt;
                                 });
    cnt = wave_sum(cnt);
    if ((tid & 63) == 0) s_cnt[tid >> 6] = cnt;
    if constexpr (GLOBAL) __threadfence();
    __syncthreads();
    if (tid == 0) {
      int total = 0;
      for (int u = 0; u < kWGWaves; ++u) total += s_cnt[u];
      nnz_row[i] = total;
    }
    // window counts, and clear for the next row
    for (int64_t j = tid; j < words; j += kWG) {
      uint32_t word;
      if constexpr (GLOBAL) {
        word = __hip_atomic_load(bits + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(bits + j, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        word = bits[j];
        bits[j] = 0u;
      }
      if (wcnt && word) atomicAdd(&s_wc[j >> win_words_log2], __popc(word));
    }
    if constexpr (GLOBAL) __threadfence();
    __syncthreads();
    if (wcnt) {
      for (int w = tid; w < n_win; w += kWG) {
        wcnt[r * n_win + w] = s_wc[w];
        s_wc[w] = 0;
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- numeric

struct SgOut {
  const int32_t* rowptrC;
  int32_t* colC;
  float* valC;
};

// Sort the first P (a power of two) (key, value) pairs by key with bitonic merges;
// `lanes` threads starting at thread `t0` take part; sync() orders the stages.
template <typename Sync>
__device__ __forceinline__ void bitonic_sort(int32_t* key, float* val, int P, int t0, int lanes, Sync&& sync) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = t0; t < P / 2; t += lanes) {
        // t-th pair of this stage: lower index a, partner a + j (j is a power of two)
        const int a = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int b = a + j;
        const bool up = (a & k) == 0;
        const int32_t ka = key[a], kb = key[b];
        if ((ka > kb) == up) {
          key[a] = kb;
          key[b] = ka;
          const float va = val[a];
          val[a] = val[b];
          val[b] = va;
        }
      }
      sync();
    }
  }
}

// x from lane (lane xor j).  j = 1, 2: one DPP quad permutation; j = 4: the quad
// permutation xor 3, then the half-row mirror (lane i of 8 reads 7 - i = i xor 7);
// j = 8: the half-row mirror, then the row mirror (i xor 15): register moves that
// leave the LDS pipe alone.  j = 16, 32: a lane shuffle.
__device__ __forceinline__ int32_t lane_xor(int32_t x, int j) {
  constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kQuadXor3 = 0x1B;  // quad_perm [1,0,3,2], [2,3,0,1], [3,2,1,0]
  constexpr int kRowMirror = 0x140, kRowHalfMirror = 0x141;
  switch (j) {  // a constant once the sorting network is unrolled
    case 1:
      return __builtin_amdgcn_mov_dpp(x, kQuadXor1, 0xF, 0xF, true);
    case 2:
      return __builtin_amdgcn_mov_dpp(x, kQuadXor2, 0xF, 0xF, true);
    case 4:
      return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(x, kQuadXor3, 0xF, 0xF, true), kRowHalfMirror, 0xF,
                                      0xF, true);
    case 8:
      return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(x, kRowHalfMirror, 0xF, 0xF, true), kRowMirror, 0xF,
                                      0xF, true);
    default:
      return __shfl_xor(x, j, 64);
  }
}

// Bitonic sort of P = 64 KPL (key, value) pairs held in one wave's registers: element
// e = r * 64 + lane sits in register r of that lane.  Stages whose partner distance j
// is 64 or more pair two registers of one lane; shorter ones pair two lanes (one
// shuffle per register), and both lanes of a pair compare the same two keys, so they
// agree on which keeps the smaller.  Keys are distinct apart from the padding, whose
// pairs never swap.  No LDS and no barrier.
template <int KPL>
__device__ __forceinline__ void wave_sort_regs(int32_t (&k)[KPL], float (&v)[KPL], int lane) {
  constexpr int P = 64 * KPL;
#pragma unroll
  for (int kk = 2; kk <= P; kk <<= 1) {
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) {
      if (j >= 64) {
        const int jr = j >> 6;
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
          if (r & jr) continue;
          const int r2 = r | jr;
          const bool up = ((r * 64 + lane) & kk) == 0;
          if ((k[r] > k[r2]) == up) {
            const int32_t tk = k[r];
            k[r] = k[r2];
            k[r2] = tk;
            const float tv = v[r];
            v[r] = v[r2];
            v[r2] = tv;
          }
        }
      } else {
        const bool lower = (lane & j) == 0;
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
          const bool up = ((r * 64 + lane) & kk) == 0;
          const int32_t pk = lane_xor(k[r], j);
          const float pv = __int_as_float(lane_xor(__float_as_int(v[r]), j));
          const bool take = (lower == up) ? (pk < k[r]) : (pk > k[r]);
          if (take) {
            k[r] = pk;
            v[r] = pv;
          }
        }
      }
    }
  }
}

// Sort the first 64 KPL (key, value) slots of a wave's table in registers and write
// the first cnt of them to C at base (element e by lane e mod 64: coalesced).
template <int KPL>
__device__ __forceinline__ void sort_emit_wave(const int32_t* key, const float* val, int lane, const SgOut& Co,
                                               int32_t base, int32_t cnt) {
  int32_t k[KPL];
  float v[KPL];
#pragma unroll
  for (int r = 0; r < KPL; ++r) {
    k[r] = key[r * 64 + lane];
    v[r] = val[r * 64 + lane];
  }
  wave_sort_regs<KPL>(k, v, lane);
#pragma unroll
  for (int r = 0; r < KPL; ++r) {
    const int e = r * 64 + lane;
    if (e < cnt) {
      Co.colC[base + e] = k[r];
      Co.valC[base + e] = v[r];
    }
  }
}

__device__ __forceinline__ int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Rows with at most TS/2 output entries: a wave-local hash table of (column, sum).
template <int TS>
__global__ void __launch_bounds__(kBlock) num_wave_kernel(SgOperands O, SgOut Co, const int32_t* rows,
                                                          int64_t n_rows) {
  constexpr int W = kBlock / 64;
  constexpr int SHIFT = 32 - __builtin_ctz(TS);
  __shared__ int32_t s_key[W][TS];
  __shared__ float s_val[W][TS];
  __shared__ int32_t s_pref[W][64], s_start[W][64];
  __shared__ float s_aval[W][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t* key = s_key[w];
  float* val = s_val[w];
  for (int64_t r = (int64_t)blockIdx.x * W + w; r < n_rows; r += (int64_t)gridDim.x * W) {
    const int32_t i = rows[r];
    for (int j = lane; j < TS; j += 64) {
      key[j] = -1;
      val[j] = 0.0f;
    }
    wave_sync_lds();
    wave_products<true>(O, O.rowptrA[i], O.rowptrA[i + 1], s_pref[w], s_start[w], s_aval[w],
                        [&](int32_t col, float prod) {
                          uint32_t h = hash_slot(col, SHIFT);
                          for (int probe = 0; probe < TS; ++probe) {  // at most half full
                            const int32_t old = atomicCAS(&key[h], -1, col);
                            if (old == -1 || old == col) {
                              atomicAdd(&val[h], prod);
                              break;
                            }
                            h = (h + 1) & (TS - 1);
                          }
                        });
    // Move the occupied slots to the front, in place, 64 slots at a time (each chunk is
    // read before it is written, and lands at or below its own slots), then sort only
    // the smallest power of two that holds them.
    int n = 0;
    for (int c0 = 0; c0 < TS; c0 += 64) {
      const int32_t k = key[c0 + lane];
      const float v = val[c0 + lane];
      const bool occ = k >= 0;
      const uint64_t m = __ballot(occ);
      const int pos = n + __popcll(m & ((1ull << lane) - 1));
      wave_sync_lds();
      if (occ) {
        key[pos] = k;
        val[pos] = v;
      }
      n += __popcll(m);
      wave_sync_lds();
    }
    // sort the smallest power of two (at least 64, at most TS / 2) that holds them, in
    // registers
    const int P = n <= 64 ? 64 : pow2_at_least(n);
    for (int j = n + lane; j < P; j += 64) key[j] = 0x7fffffff;  // padding sorts last
    wave_sync_lds();
    const int32_t base = Co.rowptrC[i], cnt = min(Co.rowptrC[i + 1] - base, n);
    if (P == 64) {
      sort_emit_wave<1>(key, val, lane, Co, base, cnt);
    } else if (P == 128) {
      sort_emit_wave<2>(key, val, lane, Co, base, cnt);
    } else if constexpr (TS >= 512) {
      if (P == 256) {
        sort_emit_wave<4>(key, val, lane, Co, base, cnt);
      } else if constexpr (TS >= 1024) {
        sort_emit_wave<8>(key, val, lane, Co, base, cnt);
      }
    }
    wave_sync_lds();
  }
}

// Rows of at most CAP output entries whose sorted columns the plan keeps (pattern,
// indexed like C): one wave per row; the columns go to the wave's LDS beside their
// sums, each product finds its column by binary search and adds into its sum with one
// LDS atomic, and the row is written in order, coalesced: no hash inserts, no
// compaction and no sort.
template <int CAP>
__global__ void __launch_bounds__(kBlock) num_wave_kept_kernel(SgOperands O, SgOut Co, const int32_t* rows,
                                                               int64_t n_rows, const int32_t* pattern) {
  constexpr int W = kBlock / 64;
  __shared__ int32_t s_key[W][CAP];
  __shared__ float s_val[W][CAP];
  __shared__ int32_t s_pref[W][64], s_start[W][64];
  __shared__ float s_aval[W][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t* keys = s_key[w];
  float* sums = s_val[w];
  for (int64_t r = (int64_t)blockIdx.x * W + w; r < n_rows; r += (int64_t)gridDim.x * W) {
    const int32_t i = rows[r];
    const int32_t base = Co.rowptrC[i];
    const int32_t n = min(Co.rowptrC[i + 1] - base, CAP);
    for (int j = lane; j < n; j += 64) {
      keys[j] = pattern[base + j];
      sums[j] = 0.0f;
    }
    int hb = 1;  // the largest power of two not above n
    while (hb * 2 <= n) hb *= 2;
    wave_sync_lds();
    wave_products<true>(O, O.rowptrA[i], O.rowptrA[i + 1], s_pref[w], s_start[w], s_aval[w],
                        [&](int32_t col, float prod) {
                          int pos = -1;  // the last key below col
                          for (int step = hb; step > 0; step >>= 1)
                            if (pos + step < n && keys[pos + step] < col) pos += step;
                          if (pos + 1 < n) atomicAdd(&sums[pos + 1], prod);
                        });
    wave_sync_lds();
    for (int j = lane; j < n; j += 64) {
      Co.colC[base + j] = keys[j];
      Co.valC[base + j] = sums[j];
    }
    wave_sync_lds();
  }
}

// Rows with at most tg/2 output entries: one workgroup per row, an LDS hash table
// of up to 2^tg_log2 slots (a power of two; dynamic LDS), sized per row.  Output
// order: with BM, a bitmap over all N columns (in LDS after the table) marks each new
// key, and a walk over it writes the row in column order, looking each value up in
// the table; without BM (N too wide for LDS), the occupied slots are compacted and
// bitonic-sorted.
template <bool BM>
__global__ void __launch_bounds__(kWG) num_block_kernel(SgOperands O, SgOut Co, const int32_t* rows,
                                                        int64_t n_rows, int tg_log2) {
  extern __shared__ int32_t s_dyn[];
  const int tg_max = 1 << tg_log2;
  int32_t* key = s_dyn;
  float* val = reinterpret_cast<float*>(key + tg_max);
  int32_t* s_pref = reinterpret_cast<int32_t*>(val + tg_max);
  int32_t* s_start = s_pref + kWG + 1;
  float* s_aval = reinterpret_cast<float*>(s_start + kWG);
  int32_t* s_tmp = reinterpret_cast<int32_t*>(s_aval + kWG);
  uint32_t* bits = reinterpret_cast<uint32_t*>(s_tmp + kWGWaves);  // BM: ceil(N / 32) words
  const int64_t words = (O.N + 31) / 32;
  const int tid = threadIdx.x;
  if constexpr (BM) {
    for (int64_t j = tid; j < words; j += kWG) bits[j] = 0u;
  }
  for (int64_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
    const int32_t i = rows[r];
    // this row's table: a power of two of at least twice its entries (>= kWG)
    const int32_t nrow = Co.rowptrC[i + 1] - Co.rowptrC[i];
    int tl = tg_log2 < 10 ? tg_log2 : 10;
    while (tl < tg_log2 && (1 << tl) < 2 * nrow) ++tl;
    const int tg = 1 << tl;
    const int shift = 32 - tl;
    for (int j = tid; j < tg; j += kWG) {
      key[j] = -1;
      val[j] = 0.0f;
    }
    __syncthreads();
    block_products<true, false>(O, O.rowptrA[i], O.rowptrA[i + 1], s_pref, s_start, s_aval, s_tmp,
                        [&](int32_t col, float prod) {
                          uint32_t h = hash_slot(col, shift);
                          for (int probe = 0; probe < tg; ++probe) {  // at most half full
                            const int32_t old = atomicCAS(&key[h], -1, col);
                            if (old == -1 || old == col) {
                              atomicAdd(&val[h], prod);
                              if (BM && old == -1) atomicOr(bits + (col >> 5), 1u << (col & 31));
                              break;
                            }
                            h = (h + 1) & (uint32_t)(tg - 1);
                          }
                        });
    const int32_t base = Co.rowptrC[i];
    if constexpr (BM) {
      // walk the bitmap in column order; each set bit's value comes from the table
      const int32_t end = Co.rowptrC[i + 1];
      int32_t out = base;
      for (int64_t w0 = 0; w0 < words; w0 += kWG) {
        const int64_t wi = w0 + tid;
        uint32_t word = wi < words ? bits[wi] : 0u;
        int32_t excl;
        const int32_t tot = block_scan(__popc(word), &excl, s_tmp);
        int32_t pos = out + excl;
        while (word) {
          const int b = __ffs(word) - 1;
          word &= word - 1;
          const int32_t col = (int32_t)(wi * 32 + b);
          uint32_t h = hash_slot(col, shift);
          float v = 0.0f;
          for (int probe = 0; probe < tg; ++probe) {
            if (key[h] == col) {
              v = val[h];
              break;
            }
            h = (h + 1) & (uint32_t)(tg - 1);
          }
          if (pos < end) {
            Co.colC[pos] = col;
            Co.valC[pos] = v;
          }
          ++pos;
        }
        if (wi < words) bits[wi] = 0u;
        out += tot;
      }
      __syncthreads();
    } else {
      // compact the occupied slots to the front (chunks of kWG, read before written),
      // then sort the smallest power of two that holds them
      int n = 0;
      for (int c0 = 0; c0 < tg; c0 += kWG) {
        const int j = c0 + tid;
        int32_t k = -1;
        float v = 0.0f;
        if (j < tg) {
          k = key[j];
          v = val[j];
        }
        const int occ = k >= 0 ? 1 : 0;
        int32_t excl;
        const int32_t tot = block_scan(occ, &excl, s_tmp);  // synchronises: all reads are done
        if (occ) {
          key[n + excl] = k;
          val[n + excl] = v;
        }
        n += tot;
        __syncthreads();
      }
      const int P = pow2_at_least(n);
      for (int j = n + tid; j < P; j += kWG) key[j] = 0x7fffffff;
      __syncthreads();
      bitonic_sort(key, val, P, tid, kWG, [] { __syncthreads(); });
      const int32_t cnt = min(Co.rowptrC[i + 1] - base, n);
      for (int j = tid; j < cnt; j += kWG) {
        Co.colC[base + j] = key[j];
        Co.valC[base + j] = val[j];
      }
      __syncthreads();
    }
  }
}

// Rows of at most `cap` output entries whose sorted columns the plan keeps (pattern,
// indexed like C): one workgroup per row; the columns go to LDS beside their sums,
// each product finds its column by binary search and adds into its sum with one LDS
// atomic, and the row is written in order, coalesced.  No table to clear, no bitmap.
__global__ void __launch_bounds__(kWG) num_block_kept_kernel(SgOperands O, SgOut Co, const int32_t* rows,
                                                             int64_t n_rows, int cap, const int32_t* pattern) {
  extern __shared__ int32_t s_dyn[];
  int32_t* keys = s_dyn;
  float* sums = reinterpret_cast<float*>(keys + cap);
  int32_t* s_pref = reinterpret_cast<int32_t*>(sums + cap);
  int32_t* s_start = s_pref + kWG + 1;
  float* s_aval = reinterpret_cast<float*>(s_start + kWG);
  int32_t* s_tmp = reinterpret_cast<int32_t*>(s_aval + kWG);
  const int tid = threadIdx.x;
  for (int64_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
    const int32_t i = rows[r];
    const int32_t base = Co.rowptrC[i];
    const int32_t n = min(Co.rowptrC[i + 1] - base, cap);
    for (int j = tid; j < n; j += kWG) {
      keys[j] = pattern[base + j];
      sums[j] = 0.0f;
    }
    int hb = 1;  // the largest power of two not above n
    while (hb * 2 <= n) hb *= 2;
    __syncthreads();
    block_products<true, false>(O, O.rowptrA[i], O.rowptrA[i + 1], s_pref, s_start, s_aval, s_tmp,
                                [&](int32_t col, float prod) {
                                  int pos = -1;  // the last key below col
                                  for (int step = hb; step > 0; step >>= 1)
                                    if (pos + step < n && keys[pos + step] < col) pos += step;
                                  if (pos + 1 < n) atomicAdd(&sums[pos + 1], prod);
                                });
    for (int j = tid; j < n; j += kWG) {
      Co.colC[base + j] = keys[j];
      Co.valC[base + j] = sums[j];
    }
    __syncthreads();
  }
}

// Long rows, one (row, column window) item per workgroup at a time: the window's
// 2^win_log2 sums and its bitmap live in LDS (zeroed once, and cleared entry by
// entry as the compaction reads them), products accumulate with LDS atomics, and
// the bitmap walk writes the window's entries in column order at the item's offset.
struct SgItem {
  int32_t row, win, out, cnt;
};

// A long row's non-empty windows: items[first, first + count).
struct SgRow {
  int32_t row, first, count, pad;
};

// bsplit[k * (n_win + 1) + w]: first position of B row k at column >= w * 2^win_log2
// (w = n_win: the row's end).
__global__ void __launch_bounds__(kBlock) bsplit_kernel(const int32_t* rowptrB, const int32_t* colB, int64_t K,
                                                        int n_win, int win_log2, int32_t* bsplit) {
  const int64_t stride = n_win + 1;
  for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < K * stride; x += (int64_t)gridDim.x * kBlock) {
    const int64_t k = x / stride;
    const int w = (int)(x - k * stride);
    const int32_t lo = rowptrB[k], hi = rowptrB[k + 1];
    bsplit[x] = w == n_win ? hi : lower_bound(colB, lo, hi, (int32_t)((int64_t)w << win_log2));
  }
}

// Write a window's entries in column order at [out, out + cnt) from its LDS sums and
// bitmap (ww words), clearing both as they are read.  Ends with a barrier.
__device__ __forceinline__ void window_emit(const SgOut& Co, float* acc, uint32_t* bits, int ww, int32_t c0,
                                            int32_t out, int32_t cnt, int32_t* s_tmp) {
  const int tid = threadIdx.x;
  const int32_t end = out + cnt;
  for (int w0 = 0; w0 < ww; w0 += kWG) {
    const int wi = w0 + tid;
    uint32_t word = wi < ww ? bits[wi] : 0u;
    int32_t excl;
    const int32_t tot = block_scan(__popc(word), &excl, s_tmp);
    int32_t pos = out + excl;
    while (word) {
      const int b = __ffs(word) - 1;
      word &= word - 1;
      const int x = wi * 32 + b;
      if (pos < end) {
        Co.colC[pos] = c0 + x;
        Co.valC[pos] = acc[x];
      }
      acc[x] = 0.0f;
      ++pos;
    }
    if (wi < ww) bits[wi] = 0u;
    out += tot;
  }
  __syncthreads();
}

// A window's entries at [out, out + cnt) in the order of its stored columns src[0, cnt):
// each sum is read and cleared by the one thread that writes its entry (the columns of
// a window are distinct), coalesced global reads and writes.  Ends with a barrier.
__device__ __forceinline__ void window_emit_values(const SgOut& Co, float* acc, const int32_t* src, int32_t c0,
                                                   int32_t out, int32_t cnt) {
  for (int32_t e = threadIdx.x; e < cnt; e += kWG) {
    const int32_t col = src[e];
    const int32_t x = col - c0;
    Co.colC[out + e] = col;
    Co.valC[out + e] = acc[x];
    acc[x] = 0.0f;
  }
  __syncthreads();
}

// Long rows without a split table: one (row, window) item per workgroup at a time, each
// B row cut to the window by binary search.
__global__ void __launch_bounds__(kWG) num_window_kernel(SgOperands O, SgOut Co, const SgItem* items,
                                                         int64_t n_items, int win_log2, const int32_t* bsplit,
                                                         int n_win) {
  extern __shared__ int32_t s_dyn[];
  const int W = 1 << win_log2;
  const int ww = W >> 5;
  float* acc = reinterpret_cast<float*>(s_dyn);
  uint32_t* bits = reinterpret_cast<uint32_t*>(acc + W);
  int32_t* s_pref = reinterpret_cast<int32_t*>(bits + ww);
  int32_t* s_start = s_pref + kWG + 1;
  float* s_aval = reinterpret_cast<float*>(s_start + kWG);
  int32_t* s_tmp = reinterpret_cast<int32_t*>(s_aval + kWG);
  const int tid = threadIdx.x;
  for (int j = tid; j < W; j += kWG) acc[j] = 0.0f;
  for (int j = tid; j < ww; j += kWG) bits[j] = 0u;
  __syncthreads();
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const SgItem item = items[it];
    const int32_t c0 = item.win << win_log2;
    const int32_t c1 = (int32_t)min((int64_t)c0 + W, O.N);
    block_products<true, true>(O, O.rowptrA[item.row], O.rowptrA[item.row + 1], s_pref, s_start, s_aval, s_tmp,
                               [&](int32_t col, float prod) {
                                 const int32_t x = col - c0;
                                 atomicOr(bits + (x >> 5), 1u << (x & 31));
                                 atomicAdd(acc + x, prod);
                               },
                               c0, c1, bsplit, (int64_t)n_win + 1, item.win);
    window_emit(Co, acc, bits, ww, c0, item.out, item.cnt, s_tmp);
  }
}

// Long rows with a split table: one row per workgroup at a time, its non-empty windows
// (items[first, first + count), in column order) one after the other.  A row of at
// most kWG A entries keeps each entry's B row and value in a register across its
// windows and prefetches the next window's split-table bounds while the current window
// accumulates, so a window costs its products and its compaction, not a chain of
// dependent loads; longer rows take each window through block_products.
// MODE kRowFull: sums and bitmap by LDS atomics, entries written from the bitmap.
// kRowValues: sums only, entries written in the order of C's kept columns (one LDS
// atomic per product instead of two, and no bitmap walk).
constexpr int kRowFull = 0, kRowValues = 1;

template <int MODE>
__device__ __forceinline__ void window_add(float* acc, uint32_t* bits, int32_t x, float prod) {
  if constexpr (MODE == kRowFull) atomicOr(bits + (x >> 5), 1u << (x & 31));
  atomicAdd(acc + x, prod);
}

template <int MODE>
__device__ __forceinline__ void window_finish(const SgOut& Co, float* acc, uint32_t* bits, int ww, int32_t c0,
                                              const SgItem& item, int32_t* pattern, int32_t* s_tmp) {
  if constexpr (MODE == kRowFull) window_emit(Co, acc, bits, ww, c0, item.out, item.cnt, s_tmp);
  if constexpr (MODE == kRowValues) window_emit_values(Co, acc, pattern + item.out, c0, item.out, item.cnt);
}

template <int MODE>
__global__ void __launch_bounds__(kWG) num_rowwin_kernel(SgOperands O, SgOut Co, const SgItem* items,
                                                         const SgRow* rows, int64_t n_rows, int win_log2,
                                                         const int32_t* bsplit, int n_win, int32_t* pattern) {
  extern __shared__ int32_t s_dyn[];
  const int W = 1 << win_log2;
  const int ww = W >> 5;
  float* acc = reinterpret_cast<float*>(s_dyn);
  uint32_t* bits = reinterpret_cast<uint32_t*>(acc + W);
  int32_t* s_pref = reinterpret_cast<int32_t*>(bits + ww);
  int32_t* s_start = s_pref + kWG + 1;
  float* s_aval = reinterpret_cast<float*>(s_start + kWG);
  int32_t* s_tmp = reinterpret_cast<int32_t*>(s_aval + kWG);
  const int tid = threadIdx.x;
  const int64_t stride = (int64_t)n_win + 1;
  for (int j = tid; j < W; j += kWG) acc[j] = 0.0f;
  for (int j = tid; j < ww; j += kWG) bits[j] = 0u;
  __syncthreads();
  for (int64_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
    const SgRow R = rows[r];
    const int32_t a0 = O.rowptrA[R.row], a1 = O.rowptrA[R.row + 1];
    if (a1 - a0 <= kWG) {
      const bool mine = tid < a1 - a0;
      int32_t k = 0;
      float av = 0.0f;
      if (mine) {
        k = O.colA[a0 + tid];
        av = O.valA[a0 + tid];
      }
      const int32_t* sp = bsplit + (int64_t)k * stride;
      SgItem item = items[R.first];
      int32_t st = 0, en = 0;
      if (mine) {
        st = sp[item.win];
        en = sp[item.win + 1];
      }
      for (int32_t j = 0; j < R.count; ++j) {
        SgItem nxt = item;
        int32_t nst = 0, nen = 0;
        if (j + 1 < R.count) {
          nxt = items[R.first + j + 1];
          if (mine) {
            nst = sp[nxt.win];
            nen = sp[nxt.win + 1];
          }
        }
        const int32_t c0 = item.win << win_log2;
        walk_products<true>(O, st, en - st, av, s_pref, s_start, s_aval, s_tmp,
                            [&](int32_t col, float prod) { window_add<MODE>(acc, bits, col - c0, prod); });
        window_finish<MODE>(Co, acc, bits, ww, c0, item, pattern, s_tmp);
        item = nxt;
        st = nst;
        en = nen;
      }
    } else {
      for (int32_t j = 0; j < R.count; ++j) {
        const SgItem item = items[R.first + j];
        const int32_t c0 = item.win << win_log2;
        const int32_t c1 = (int32_t)min((int64_t)c0 + W, O.N);
        block_products<true, true>(O, a0, a1, s_pref, s_start, s_aval, s_tmp,
                                   [&](int32_t col, float prod) { window_add<MODE>(acc, bits, col - c0, prod); },
                                   c0, c1, bsplit, stride, item.win);
        window_finish<MODE>(Co, acc, bits, ww, c0, item, pattern, s_tmp);
      }
    }
  }
}

// Long rows: workgroup b owns slot b (N floats + a bitmap of N bits, all zero
// between rows) and takes rows b, b + grid, ...; products accumulate with
// workgroup-scope atomics (only this workgroup touches the slot), then the bitmap is
// walked in column order to write the row and clear what it set.
__global__ void __launch_bounds__(kWG) num_dense_kernel(SgOperands O, SgOut Co, const int32_t* rows,
                                                        int64_t n_rows, float* gvals, uint32_t* gbits,
                                                        int64_t slot_words) {
  __shared__ int32_t s_pref[kWG + 1], s_start[kWG];
  __shared__ float s_aval[kWG];
  __shared__ int32_t s_tmp[kWGWaves];
  float* vals = gvals + (int64_t)blockIdx.x * slot_words * 32;
  uint32_t* bits = gbits + (int64_t)blockIdx.x * slot_words;
  const int64_t words = (O.N + 31) / 32;
  const int tid = threadIdx.x;
  for (int64_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
    const int32_t i = rows[r];
    block_products<true, false>(O, O.rowptrA[i], O.rowptrA[i + 1], s_pref, s_start, s_aval, s_tmp,
                         [&](int32_t col, float prod) {
                           __hip_atomic_fetch_or(bits + (col >> 5), 1u << (col & 31), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
                           __hip_atomic_fetch_add(vals + col, prod, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                         });
    __threadfence();
    __syncthreads();
    int32_t out = Co.rowptrC[i];
    const int32_t end = Co.rowptrC[i + 1];  // writes stay inside the row even if the counts disagreed
    for (int64_t w0 = 0; w0 < words; w0 += kWG) {
      const int64_t wi = w0 + tid;
      uint32_t word = 0;
      if (wi < words) word = __hip_atomic_load(bits + wi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int32_t excl;
      const int32_t tot = block_scan(__popc(word), &excl, s_tmp);
      int32_t pos = out + excl;
      while (word) {
        const int b = __ffs(word) - 1;
        word &= word - 1;
        const int64_t col = wi * 32 + b;
        if (pos < end) {
          Co.colC[pos] = (int32_t)col;
          Co.valC[pos] = __hip_atomic_load(vals + col, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __hip_atomic_store(vals + col, 0.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ++pos;
      }
      if (wi < words) __hip_atomic_store(bits + wi, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      out += tot;
    }
    __threadfence();
    __syncthreads();
  }
}

// Numeric classes: wave tables of 256 / 512 / 1024 slots (0..2), workgroup tables of
// 2K / 4K / 8K / 16K slots (3..6, each launched with just the LDS it needs), long
// rows (7).  Symbolic classes: wave sets of 256 / 512 / 1024 slots, bitmap.
constexpr int kNumClasses = 8;
constexpr int kLongClass = 7;
constexpr int kSymClasses = 4;
constexpr int kMaxWindows = 4096;   // column windows per long row (else the dense slots)
constexpr int64_t kSplitBudget = (int64_t)1 << 26;  // B-row window split table entries (else binary search)

int64_t grid_for(int64_t items, int64_t per_block) {
  return std::max<int64_t>(1, std::min<int64_t>((items + per_block - 1) / per_block, kMaxGridBlocks));
}

}  // namespace
}  // namespace spmm

using spmm::kLongClass;
using spmm::kNumClasses;
using spmm::kSymClasses;

struct spgemm_s {
  int64_t M = 0, K = 0, N = 0;
  spmm_csr A = {}, B = {};
  int device = 0;
  int64_t nnz_c = 0, products = 0;
  int32_t* rowptrC = nullptr;   // device, M + 1
  int32_t* rows = nullptr;      // device: rows grouped by numeric class
  int64_t cls_off[kNumClasses] = {}, cls_cnt[kNumClasses] = {};
  int tg_log2 = 0;              // workgroup table of 2^tg_log2 slots
  size_t lds_block = 0;         // its dynamic LDS bytes
  size_t lds_max = 0;           // dynamic LDS a workgroup may use on this device
  float* slot_vals = nullptr;   // dense slots: n_slots x (slot_words * 32) floats
  uint32_t* slot_bits = nullptr;
  int64_t slot_words = 0;
  int n_slots = 0;
  int win_log2 = 0;             // long rows by column windows of 2^win_log2 (0: dense slots)
  size_t lds_window = 0;        // the window kernel's dynamic LDS bytes
  spmm::SgItem* items = nullptr;  // device: (row, window, offset, count) of the long rows
  int64_t n_items = 0;
  spmm::SgRow* wrows = nullptr;   // device, with a split table: each long row's run of items
  int64_t n_wrows = 0;
  int32_t* bsplit = nullptr;      // device: B rows' window split positions (nullable)
  int n_win = 0;
  int32_t* pattern = nullptr;     // device: C's columns, indexed like C (nullable)
  int64_t pattern_entries = 0;
  bool pattern_ready = false;     // filled by a compute call outside graph capture
  ~spgemm_s() {
    if (pattern) (void)hipFree(pattern);
    if (rowptrC) (void)hipFree(rowptrC);
    if (rows) (void)hipFree(rows);
    if (items) (void)hipFree(items);
    if (wrows) (void)hipFree(wrows);
    if (bsplit) (void)hipFree(bsplit);
    if (slot_vals) (void)hipFree(slot_vals);
    if (slot_bits) (void)hipFree(slot_bits);
  }
};

namespace {

#define SG_TRY(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return spmm::set_error(SPMM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

template <typename T>
hipError_t dmalloc(T** p, int64_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)(n > 0 ? n : 1));
}

spmm::SgOperands operands(const spgemm_s* h) {
  spmm::SgOperands O;
  O.rowptrA = h->A.rowptr;
  O.colA = h->A.colind;
  O.valA = h->A.values;
  O.rowptrB = h->B.rowptr;
  O.colB = h->B.colind;
  O.valB = h->B.values;
  O.M = h->M;
  O.N = h->N;
  return O;
}

constexpr size_t kBlockFixedLds = sizeof(int32_t) * (size_t)(3 * spmm::kWG + 1 + 2 * spmm::kWGWaves);

// Dense slots for `want` concurrent rows (values + bitmap over N columns), zeroed.
spmm_status ensure_slots(spgemm_s* h, int want, hipStream_t s) {
  if (want <= h->n_slots) return SPMM_OK;
  if (h->slot_vals) (void)hipFree(h->slot_vals);
  if (h->slot_bits) (void)hipFree(h->slot_bits);
  h->slot_vals = nullptr;
  h->slot_bits = nullptr;
  h->n_slots = 0;
  h->slot_words = (h->N + 31) / 32;
  if (dmalloc(&h->slot_vals, (int64_t)want * h->slot_words * 32) != hipSuccess ||
      dmalloc(&h->slot_bits, (int64_t)want * h->slot_words) != hipSuccess)
    return spmm::set_error(SPMM_ERR_ALLOC, "device allocation of %d dense SpGEMM rows failed", want);
  SG_TRY(hipMemsetAsync(h->slot_vals, 0, sizeof(float) * (size_t)want * h->slot_words * 32, s));
  SG_TRY(hipMemsetAsync(h->slot_bits, 0, sizeof(uint32_t) * (size_t)want * h->slot_words, s));
  h->n_slots = want;
  return SPMM_OK;
}

// Slots for rows handled one workgroup each: a few per CU, within 1 GiB.
int slot_count(const spgemm_s* h, int64_t rows, int cus) {
  const double slot_bytes = 4.0 * (double)((h->N + 31) / 32) * 33.0;
  const int64_t by_mem = std::max<int64_t>(1, (int64_t)((double)(1ll << 30) / slot_bytes));
  return (int)std::max<int64_t>(1, std::min<int64_t>({rows, (int64_t)cus * 2, by_mem}));
}

}  // namespace

extern "C" {

spmm_status spgemm_create(int64_t M, const spmm_csr* A, const spmm_csr* B, unsigned flags, void* stream,
                          spgemm_t* out) {
  spmm::TraceRange trace_range("spgemm_create");
  if (!out) return spmm::set_error(SPMM_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (!A || !B) return spmm::set_error(SPMM_ERR_INVALID_ARG, "A/B is null");
  if (M < 0 || M >= ((int64_t)1 << 31)) return spmm::set_error(SPMM_ERR_INVALID_ARG, "M out of range");
  if (A->cols < 0 || A->cols >= ((int64_t)1 << 31) || B->cols < 0 || B->cols >= ((int64_t)1 << 31))
    return spmm::set_error(SPMM_ERR_INVALID_ARG, "column count out of range");
  if (A->nnz < 0 || B->nnz < 0) return spmm::set_error(SPMM_ERR_INVALID_ARG, "negative nnz");
  if (A->nnz > spmm::kMaxNnz || B->nnz > spmm::kMaxNnz)
    return spmm::set_error(SPMM_ERR_UNSUPPORTED, "nnz > 2^31 - 2^16 needs 64-bit indices");
  if (!A->rowptr || !B->rowptr) return spmm::set_error(SPMM_ERR_INVALID_ARG, "rowptr is null");
  if ((A->nnz > 0 && (!A->colind || !A->values)) || (B->nnz > 0 && (!B->colind || !B->values)))
    return spmm::set_error(SPMM_ERR_INVALID_ARG, "colind/values null");
  if (flags & ~(SPMM_TILE_VALIDATE | SPGEMM_BITMAP_ONLY))
    return spmm::set_error(SPMM_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (flags & SPMM_TILE_VALIDATE) {
    const spmm_status st = spmm::validate_csr(A->rowptr, A->colind, M, A->cols, A->nnz, s);
    if (st != SPMM_OK) return st;
    const spmm_status st2 = spmm::validate_csr(B->rowptr, B->colind, A->cols, B->cols, B->nnz, s);
    if (st2 != SPMM_OK) return st2;
  }
  spgemm_s* h = new (std::nothrow) spgemm_s();
  if (!h) return spmm::set_error(SPMM_ERR_ALLOC, "host allocation failed");
  h->M = M;
  h->K = A->cols;
  h->N = B->cols;
  h->A = *A;
  h->B = *B;
  (void)hipGetDevice(&h->device);
  auto body = [&]() -> spmm_status {
    int cus = 0, lds_max = 0;
    SG_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    SG_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
    const spmm::SgOperands O = operands(h);
    // products per row
    int64_t* d_fl = nullptr;
    int32_t* d_nnz = nullptr;
    int32_t* d_rows = nullptr;
    std::vector<int64_t> fl((size_t)M);
    std::vector<int32_t> nz((size_t)M);
    auto cleanup = [&]() {
      if (d_fl) (void)hipFree(d_fl);
      if (d_nnz) (void)hipFree(d_nnz);
      if (d_rows) (void)hipFree(d_rows);
    };
    auto run = [&]() -> spmm_status {
      if (dmalloc(&d_fl, M) != hipSuccess || dmalloc(&d_nnz, M) != hipSuccess || dmalloc(&d_rows, M) != hipSuccess ||
          dmalloc(&h->rowptrC, M + 1) != hipSuccess || dmalloc(&h->rows, M) != hipSuccess)
        return spmm::set_error(SPMM_ERR_ALLOC, "device allocation of the SpGEMM plan failed");
      if (M > 0) {
        hipLaunchKernelGGL(spmm::row_products_kernel, dim3((unsigned)spmm::grid_for(M, spmm::kBlock / 64)),
                           dim3(spmm::kBlock), 0, s, O, d_fl);
        SG_TRY(hipGetLastError());
        SG_TRY(hipMemcpyAsync(fl.data(), d_fl, sizeof(int64_t) * (size_t)M, hipMemcpyDeviceToHost, s));
        SG_TRY(hipStreamSynchronize(s));
      }
      // symbolic classes by products
      std::vector<int32_t> list((size_t)M);
      int64_t off[kSymClasses + 1] = {}, cnt[kSymClasses] = {};
      auto sym_cls = [&](int64_t f) { return f == 0 ? -1 : f <= 128 ? 0 : f <= 256 ? 1 : f <= 512 ? 2 : 3; };
      for (int64_t i = 0; i < M; ++i) {
        h->products += fl[(size_t)i];
        const int c = sym_cls(fl[(size_t)i]);
        if (c >= 0) ++cnt[c];
        else nz[(size_t)i] = 0;
      }
      for (int c = 0; c < kSymClasses; ++c) off[c + 1] = off[c] + cnt[c];
      {
        int64_t pos[kSymClasses];
        for (int c = 0; c < kSymClasses; ++c) pos[c] = off[c];
        for (int64_t i = 0; i < M; ++i) {
          const int c = sym_cls(fl[(size_t)i]);
          if (c >= 0) list[(size_t)pos[c]++] = (int32_t)i;
        }
      }
      const std::vector<int32_t> list_sym(list);
      if (M > 0) {
        SG_TRY(hipMemsetAsync(d_nnz, 0, sizeof(int32_t) * (size_t)M, s));
        SG_TRY(hipMemcpyAsync(d_rows, list.data(), sizeof(int32_t) * (size_t)M, hipMemcpyHostToDevice, s));
      }
      if (cnt[0]) hipLaunchKernelGGL(spmm::sym_wave_kernel<256>, dim3((unsigned)spmm::grid_for(cnt[0], 4)),
                                     dim3(spmm::kBlock), 0, s, O, d_rows + off[0], cnt[0], d_nnz);
      if (cnt[1]) hipLaunchKernelGGL(spmm::sym_wave_kernel<512>, dim3((unsigned)spmm::grid_for(cnt[1], 4)),
                                     dim3(spmm::kBlock), 0, s, O, d_rows + off[1], cnt[1], d_nnz);
      if (cnt[2]) hipLaunchKernelGGL(spmm::sym_wave_kernel<1024>, dim3((unsigned)spmm::grid_for(cnt[2], 4)),
                                     dim3(spmm::kBlock), 0, s, O, d_rows + off[2], cnt[2], d_nnz);
      SG_TRY(hipGetLastError());
      // Column windows for the long rows: the largest power of two (at most 32K columns)
      // whose sums and bitmap fit in LDS next to the product scratch; window counts
      // come from the symbolic bitmap pass when there are at most kMaxWindows windows.
      {
        int wl = 10;
        while (wl < 15 && kBlockFixedLds + (size_t)4 * (((size_t)1 << (wl + 1)) + ((size_t)1 << (wl - 4))) <=
                              (size_t)lds_max)
          ++wl;
        const int64_t n_win = (h->N + ((int64_t)1 << wl) - 1) >> wl;
        h->win_log2 = (n_win <= spmm::kMaxWindows && h->N > 0) ? wl : 0;
        h->lds_window = kBlockFixedLds + (size_t)4 * (((size_t)1 << wl) + ((size_t)1 << (wl - 5)));
      }
      const int n_win = h->win_log2 ? (int)((h->N + ((int64_t)1 << h->win_log2) - 1) >> h->win_log2) : 0;
      std::vector<int32_t> wc;
      int32_t* d_wc = nullptr;
      if (cnt[3]) {
        const int64_t words = (h->N + 31) / 32;
        if (n_win) {
          if (dmalloc(&d_wc, cnt[3] * (int64_t)n_win) != hipSuccess)
            return spmm::set_error(SPMM_ERR_ALLOC, "device allocation of window counts failed");
        }
        const size_t lds_fixed = kBlockFixedLds + sizeof(int32_t) * (size_t)n_win;
        const size_t lds = lds_fixed + sizeof(uint32_t) * (size_t)words;
        const int wwl = h->win_log2 ? h->win_log2 - 5 : 0;
        if (lds <= (size_t)lds_max) {
          (void)hipFuncSetAttribute(reinterpret_cast<const void*>(spmm::sym_bitmap_kernel<false>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
          const int64_t grid = std::min<int64_t>(cnt[3], (int64_t)cus * 8);
          hipLaunchKernelGGL(spmm::sym_bitmap_kernel<false>, dim3((unsigned)grid), dim3(spmm::kWG), lds, s, O,
                             d_rows + off[3], cnt[3], d_nnz, (uint32_t*)nullptr, (int64_t)0, d_wc, n_win, wwl);
        } else {
          const spmm_status st = ensure_slots(h, slot_count(h, cnt[3], cus), s);
          if (st != SPMM_OK) {
            if (d_wc) (void)hipFree(d_wc);
            return st;
          }
          (void)hipFuncSetAttribute(reinterpret_cast<const void*>(spmm::sym_bitmap_kernel<true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_fixed);
          hipLaunchKernelGGL(spmm::sym_bitmap_kernel<true>, dim3((unsigned)h->n_slots), dim3(spmm::kWG), lds_fixed,
                             s, O, d_rows + off[3], cnt[3], d_nnz, h->slot_bits, h->slot_words, d_wc, n_win, wwl);
        }
        hipError_t le = hipGetLastError();
        if (le == hipSuccess && d_wc) {
          wc.resize((size_t)cnt[3] * (size_t)n_win);
          le = hipMemcpyAsync(wc.data(), d_wc, sizeof(int32_t) * wc.size(), hipMemcpyDeviceToHost, s);
          if (le == hipSuccess) le = hipStreamSynchronize(s);
        }
        if (d_wc) (void)hipFree(d_wc);
        SG_TRY(le);
      }
      if (M > 0) {
        SG_TRY(hipMemcpyAsync(nz.data(), d_nnz, sizeof(int32_t) * (size_t)M, hipMemcpyDeviceToHost, s));
        SG_TRY(hipStreamSynchronize(s));
      }
      // row pointer of C
      std::vector<int32_t> rp((size_t)M + 1);
      int64_t total = 0;
      for (int64_t i = 0; i < M; ++i) {
        rp[(size_t)i] = (int32_t)total;
        total += nz[(size_t)i];
        if (total >= ((int64_t)1 << 31)) return spmm::set_error(SPMM_ERR_UNSUPPORTED, "C would hold >= 2^31 entries");
      }
      rp[(size_t)M] = (int32_t)total;
      h->nnz_c = total;
      SG_TRY(hipMemcpyAsync(h->rowptrC, rp.data(), sizeof(int32_t) * rp.size(), hipMemcpyHostToDevice, s));
      // numeric classes by output entries
      int tg_log2 = 8;
      while (tg_log2 < 16 && kBlockFixedLds + 8 * ((size_t)1 << (tg_log2 + 1)) <= (size_t)lds_max) ++tg_log2;
      h->tg_log2 = tg_log2;
      h->lds_block = kBlockFixedLds + 8 * ((size_t)1 << tg_log2);
      // A workgroup table writes its row in column order through an LDS bitmap over C's
      // columns when that fits beside it; where it does not and the long-row windows
      // are few, the row goes to the windows instead of the sorting table.
      const size_t bm_bytes = sizeof(uint32_t) * (size_t)((h->N + 31) / 32);
      auto num_cls = [&](int64_t n) {
        if (n == 0) return -1;
        if (n <= 512) return n <= 128 ? 0 : n <= 256 ? 1 : 2;
        for (int c = 3; c < kLongClass; ++c) {
          const int tl = c + 8;  // table of 2^tl slots holds up to 2^(tl-1) entries
          if (tl <= tg_log2 && n <= ((int64_t)1 << (tl - 1))) {
            const bool bm = kBlockFixedLds + 8 * ((size_t)1 << tl) + bm_bytes <= (size_t)lds_max;
            return (bm || !h->win_log2 || n_win > 16) ? c : kLongClass;
          }
        }
        return kLongClass;
      };
      for (int c = 0; c < kNumClasses; ++c) h->cls_cnt[c] = 0;
      for (int64_t i = 0; i < M; ++i) {
        const int c = num_cls(nz[(size_t)i]);
        if (c >= 0) ++h->cls_cnt[c];
      }
      h->cls_off[0] = 0;
      for (int c = 1; c < kNumClasses; ++c) h->cls_off[c] = h->cls_off[c - 1] + h->cls_cnt[c - 1];
      {
        int64_t pos[kNumClasses];
        for (int c = 0; c < kNumClasses; ++c) pos[c] = h->cls_off[c];
        for (int64_t i = 0; i < M; ++i) {
          const int c = num_cls(nz[(size_t)i]);
          if (c >= 0) list[(size_t)pos[c]++] = (int32_t)i;
        }
      }
      if (M > 0)
        SG_TRY(hipMemcpyAsync(h->rows, list.data(), sizeof(int32_t) * (size_t)M, hipMemcpyHostToDevice, s));
      h->lds_max = (size_t)lds_max;
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(spmm::num_block_kernel<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
      for (const void* f : {reinterpret_cast<const void*>(spmm::num_block_kernel<true>),
                            reinterpret_cast<const void*>(spmm::num_block_kept_kernel)})
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
      if (h->cls_cnt[kLongClass] && h->win_log2) {
        // (row, window) items of the long rows, with their output offsets, largest first
        std::vector<int64_t> bitmap_index((size_t)M, -1);
        for (int64_t r = 0; r < cnt[3]; ++r) bitmap_index[(size_t)list_sym[(size_t)(off[3] + r)]] = r;
        std::vector<spmm::SgItem> items;
        for (int64_t t = 0; t < h->cls_cnt[kLongClass]; ++t) {
          const int32_t i = list[(size_t)(h->cls_off[kLongClass] + t)];
          const int64_t r = bitmap_index[(size_t)i];
          if (r < 0) return spmm::set_error(SPMM_ERR_HIP, "internal: long row %d has no window counts", i);
          int32_t out = rp[(size_t)i];
          for (int w = 0; w < n_win; ++w) {
            const int32_t c = wc[(size_t)r * n_win + w];
            if (c > 0) items.push_back(spmm::SgItem{i, w, out, c});
            out += c;
          }
          if (out != rp[(size_t)i + 1]) return spmm::set_error(SPMM_ERR_HIP, "internal: window counts of row %d", i);
        }
        h->n_win = n_win;
        const int64_t split_entries = h->K * ((int64_t)n_win + 1);
        if (split_entries <= spmm::kSplitBudget && dmalloc(&h->bsplit, split_entries) == hipSuccess) {
          hipLaunchKernelGGL(spmm::bsplit_kernel, dim3((unsigned)spmm::grid_for(split_entries, spmm::kBlock)),
                             dim3(spmm::kBlock), 0, s, h->B.rowptr, h->B.colind, h->K, n_win, h->win_log2,
                             h->bsplit);
          SG_TRY(hipGetLastError());
          // row-ordered items (each row's windows in column order), rows largest first
          std::vector<spmm::SgRow> wr;
          for (size_t a = 0; a < items.size();) {
            size_t b = a;
            while (b < items.size() && items[b].row == items[a].row) ++b;
            wr.push_back(spmm::SgRow{items[a].row, (int32_t)a, (int32_t)(b - a), 0});
            a = b;
          }
          std::stable_sort(wr.begin(), wr.end(), [&](const spmm::SgRow& x, const spmm::SgRow& y) {
            return rp[(size_t)x.row + 1] - rp[(size_t)x.row] > rp[(size_t)y.row + 1] - rp[(size_t)y.row];
          });
          h->n_wrows = (int64_t)wr.size();
          if (dmalloc(&h->wrows, h->n_wrows) != hipSuccess)
            return spmm::set_error(SPMM_ERR_ALLOC, "device allocation of the window rows failed");
          if (h->n_wrows)
            SG_TRY(hipMemcpyAsync(h->wrows, wr.data(), sizeof(spmm::SgRow) * wr.size(), hipMemcpyHostToDevice, s));
          for (const void* f : {reinterpret_cast<const void*>(spmm::num_rowwin_kernel<spmm::kRowFull>),
                                reinterpret_cast<const void*>(spmm::num_rowwin_kernel<spmm::kRowValues>)})
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds_window);
          SG_TRY(hipStreamSynchronize(s));  // wr is read before it goes out of scope
        } else {
          // (row, window) items largest first
          std::stable_sort(items.begin(), items.end(),
                           [](const spmm::SgItem& x, const spmm::SgItem& y) { return x.cnt > y.cnt; });
          (void)hipFuncSetAttribute(reinterpret_cast<const void*>(spmm::num_window_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds_window);
        }
        h->n_items = (int64_t)items.size();
        if (dmalloc(&h->items, h->n_items) != hipSuccess)
          return spmm::set_error(SPMM_ERR_ALLOC, "device allocation of the window items failed");
        if (h->n_items)
          SG_TRY(hipMemcpyAsync(h->items, items.data(), sizeof(spmm::SgItem) * items.size(), hipMemcpyHostToDevice, s));
      } else if (h->cls_cnt[kLongClass]) {
        const spmm_status st = ensure_slots(h, slot_count(h, h->cls_cnt[kLongClass], cus), s);
        if (st != SPMM_OK) return st;
      }
      // Room for C's columns, indexed like C, kept from the first compute call on (which
      // finds them as before and copies them here): later calls add each product with
      // one LDS atomic (by binary search over a row's kept columns, or into its window's
      // sums) and write the entries in the kept order, instead of finding the columns
      // again with hash inserts, sorts, bitmap atomics and bitmap walks.  They cover
      // every row but the long rows that take no split table; kept when these rows hold
      // at least a quarter of C and nnz(C) indices take at most a quarter of the free
      // device memory.
      int64_t kept = 0;
      for (int c = 0; c <= kLongClass; ++c) {
        if (c == kLongClass && !h->wrows) break;
        for (int64_t t = 0; t < h->cls_cnt[c]; ++t) {
          const int32_t i = list[(size_t)(h->cls_off[c] + t)];
          kept += rp[(size_t)i + 1] - rp[(size_t)i];
        }
      }
      if (!(flags & SPGEMM_BITMAP_ONLY) && kept > 0 && kept * 4 >= h->nnz_c) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && (size_t)h->nnz_c * 4 <= free_b / 4) {
          if (dmalloc(&h->pattern, h->nnz_c) == hipSuccess) {
            h->pattern_entries = kept;
          } else {
            h->pattern = nullptr;
            (void)hipGetLastError();  // no pattern: compute finds the columns on every call
          }
        }
      }
      SG_TRY(hipStreamSynchronize(s));
      return SPMM_OK;
    };
    const spmm_status st = run();
    cleanup();
    return st;
  };
  const spmm_status st = spmm::guarded(body);
  if (st != SPMM_OK) {
    delete h;
    return st;
  }
  *out = h;
  return SPMM_OK;
}

spmm_status spgemm_destroy(spgemm_t plan) {
  if (!plan) return spmm::set_error(SPMM_ERR_INVALID_ARG, "plan is null");
  (void)hipDeviceSynchronize();
  delete plan;
  return SPMM_OK;
}

spmm_status spgemm_info(spgemm_t plan, int64_t* nnz_c, int64_t* products) {
  if (!plan) return spmm::set_error(SPMM_ERR_INVALID_ARG, "plan is null");
  if (nnz_c) *nnz_c = plan->nnz_c;
  if (products) *products = plan->products;
  return SPMM_OK;
}

spmm_status spgemm_pattern_entries(spgemm_t plan, int64_t* entries) {
  if (!plan || !entries) return spmm::set_error(SPMM_ERR_INVALID_ARG, "null argument");
  *entries = plan->pattern_entries;
  return SPMM_OK;
}

spmm_status spgemm_rowptr(spgemm_t plan, int32_t* rowptrC, void* stream) {
  if (!plan || !rowptrC) return spmm::set_error(SPMM_ERR_INVALID_ARG, "null argument");
  SG_TRY(hipMemcpyAsync(rowptrC, plan->rowptrC, sizeof(int32_t) * (size_t)(plan->M + 1), hipMemcpyDeviceToDevice,
                        static_cast<hipStream_t>(stream)));
  return SPMM_OK;
}

spmm_status spgemm_compute(spgemm_t plan, int32_t* colindC, float* valuesC, void* stream) {
  spmm::TraceRange trace_range("spgemm_compute");
  if (!plan) return spmm::set_error(SPMM_ERR_INVALID_ARG, "plan is null");
  if (plan->nnz_c > 0 && (!colindC || !valuesC)) return spmm::set_error(SPMM_ERR_INVALID_ARG, "colindC/valuesC null");
  int dev = 0;
  SG_TRY(hipGetDevice(&dev));
  if (dev != plan->device) return spmm::set_error(SPMM_ERR_INVALID_ARG, "current device differs from the plan's");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const spmm::SgOperands O = operands(plan);
  spmm::SgOut Co{plan->rowptrC, colindC, valuesC};
  const int32_t* rows = plan->rows;
  const int64_t* off = plan->cls_off;
  const int64_t* cnt = plan->cls_cnt;
  // C's kept columns, once a call has filled them; before that, the columns are found
  // as the rows are computed and copied into the plan at the end of the call
  const bool kept = plan->pattern && plan->pattern_ready;
  if (kept) {
    const int32_t* P = plan->pattern;
    if (cnt[0]) hipLaunchKernelGGL(spmm::num_wave_kept_kernel<128>, dim3((unsigned)spmm::grid_for(cnt[0], 4)),
                                   dim3(spmm::kBlock), 0, s, O, Co, rows + off[0], cnt[0], P);
    if (cnt[1]) hipLaunchKernelGGL(spmm::num_wave_kept_kernel<256>, dim3((unsigned)spmm::grid_for(cnt[1], 4)),
                                   dim3(spmm::kBlock), 0, s, O, Co, rows + off[1], cnt[1], P);
    if (cnt[2]) hipLaunchKernelGGL(spmm::num_wave_kept_kernel<512>, dim3((unsigned)spmm::grid_for(cnt[2], 4)),
                                   dim3(spmm::kBlock), 0, s, O, Co, rows + off[2], cnt[2], P);
  } else {
    if (cnt[0]) hipLaunchKernelGGL(spmm::num_wave_kernel<256>, dim3((unsigned)spmm::grid_for(cnt[0], 4)),
                                   dim3(spmm::kBlock), 0, s, O, Co, rows + off[0], cnt[0]);
    if (cnt[1]) hipLaunchKernelGGL(spmm::num_wave_kernel<512>, dim3((unsigned)spmm::grid_for(cnt[1], 4)),
                                   dim3(spmm::kBlock), 0, s, O, Co, rows + off[1], cnt[1]);
    if (cnt[2]) hipLaunchKernelGGL(spmm::num_wave_kernel<1024>, dim3((unsigned)spmm::grid_for(cnt[2], 4)),
                                   dim3(spmm::kBlock), 0, s, O, Co, rows + off[2], cnt[2]);
  }
  SG_TRY(hipGetLastError());
  for (int c = 3; c < kLongClass; ++c) {
    if (!cnt[c]) continue;
    const int tl = c + 8;
    const size_t lds = kBlockFixedLds + 8 * ((size_t)1 << tl);
    const size_t lds_bm = lds + sizeof(uint32_t) * (size_t)((plan->N + 31) / 32);
    const int64_t grid = std::min<int64_t>(cnt[c], 65536);
    if (kept)
      hipLaunchKernelGGL(spmm::num_block_kept_kernel, dim3((unsigned)grid), dim3(spmm::kWG),
                         kBlockFixedLds + 4 * ((size_t)1 << tl), s, O, Co, rows + off[c], cnt[c], 1 << (tl - 1),
                         plan->pattern);
    else if (lds_bm <= plan->lds_max)
      hipLaunchKernelGGL(spmm::num_block_kernel<true>, dim3((unsigned)grid), dim3(spmm::kWG), lds_bm, s, O, Co,
                         rows + off[c], cnt[c], tl);
    else
      hipLaunchKernelGGL(spmm::num_block_kernel<false>, dim3((unsigned)grid), dim3(spmm::kWG), lds, s, O, Co,
                         rows + off[c], cnt[c], tl);
    SG_TRY(hipGetLastError());
  }
  if (cnt[kLongClass] && plan->win_log2) {
    if (plan->n_items) {
      int cus = 0;
      SG_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      if (plan->wrows) {
        const int64_t grid = std::min<int64_t>(plan->n_wrows, (int64_t)cus * 2);
        if (kept)
          hipLaunchKernelGGL(spmm::num_rowwin_kernel<spmm::kRowValues>, dim3((unsigned)grid), dim3(spmm::kWG),
                             plan->lds_window, s, O, Co, plan->items, plan->wrows, plan->n_wrows, plan->win_log2,
                             plan->bsplit, plan->n_win, plan->pattern);
        else
          hipLaunchKernelGGL(spmm::num_rowwin_kernel<spmm::kRowFull>, dim3((unsigned)grid), dim3(spmm::kWG),
                             plan->lds_window, s, O, Co, plan->items, plan->wrows, plan->n_wrows, plan->win_log2,
                             plan->bsplit, plan->n_win, (int32_t*)nullptr);
      } else {
        const int64_t grid = std::min<int64_t>(plan->n_items, (int64_t)cus * 2);
        hipLaunchKernelGGL(spmm::num_window_kernel, dim3((unsigned)grid), dim3(spmm::kWG), plan->lds_window, s, O,
                           Co, plan->items, plan->n_items, plan->win_log2, plan->bsplit, plan->n_win);
      }
      SG_TRY(hipGetLastError());
    }
  } else if (cnt[kLongClass]) {
    hipLaunchKernelGGL(spmm::num_dense_kernel, dim3((unsigned)plan->n_slots), dim3(spmm::kWG), 0, s, O, Co,
                       rows + off[kLongClass], cnt[kLongClass], plan->slot_vals, plan->slot_bits, plan->slot_words);
    SG_TRY(hipGetLastError());
  }
  if (plan->pattern && !kept && plan->nnz_c > 0) {
    // keep the columns this call wrote; not while the stream is being captured (the
    // copy would only run at replay, so later eager calls could not rely on it)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    SG_TRY(hipStreamIsCapturing(s, &cs));
    if (cs == hipStreamCaptureStatusNone) {
      SG_TRY(hipMemcpyAsync(plan->pattern, colindC, sizeof(int32_t) * (size_t)plan->nnz_c, hipMemcpyDeviceToDevice,
                            s));
      plan->pattern_ready = true;
    }
  }
  return SPMM_OK;
}

}  // extern "C"
