// Forward local SpMM over a tile row (C = [C] + sum_k A_k B_k, k from k_offset):
// the tile product of Section 2.1 with the k order of Algorithm 2 (Section 3.3).
//
// Work decomposition (one launch + one fix-up launch):
//   * row-split part: a group of G lanes owns one output row and a window of
//     G*V columns; it walks the row's non-zeros in every k-tile (k' order),
//     gathering B_k rows with one V-element vector load per lane, and keeps the
//     FP32 accumulators in registers across all k-tiles, so C is written once.
//     Column index and value of each non-zero are loaded once per group
//     (coalesced, G at a time) and broadcast across the group (readlane for a
//     full wave, ds_bpermute otherwise).
//   * split-row part: rows whose combined length exceeds a threshold are cut
//     into units of at most `segment` non-zeros of one k-tile; each unit writes
//     an FP32 partial row.  These workgroups come first in the grid so that the
//     long work starts early.
//   * fix-up: one group per split row sums its units' partials in a fixed
//     order (k' order, then position) and stores C once.  Deterministic: no
//     atomics, so replays are bit-identical.
#include "elem.hpp"
#include "fwd_common.hpp"
#include "internal.hpp"

namespace spmm {
namespace {

template <int G, int V, typename E, bool HOT>
__global__ void __launch_bounds__(kBlock) fwd_main(FwdParams P) {
  constexpr int GPB = kBlock / G;  // groups per workgroup
  const int gl = threadIdx.x & (G - 1);
  const int64_t c0 = (int64_t)blockIdx.y * (G * V) + (int64_t)gl * V;
  const bool active = c0 < P.N;
  const int64_t cl = active ? c0 : 0;  // lanes past N load column 0 and store nothing
  const int64_t unit_blocks = (P.n_seg + GPB - 1) / GPB;
  float acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = 0.0f;

  if ((int64_t)blockIdx.x < unit_blocks) {
    // Split-row unit: partial sum over one k-tile range.
    const int64_t s = group_uniform<G>((int64_t)blockIdx.x * GPB + threadIdx.x / G);
    if (s >= P.n_seg) return;
    const Seg d = P.seg[s];
    const TileDev& t = P.t[d.k];
    accumulate_range<G, V, E, HOT>(t, d.p0, d.p1, static_cast<const char*>(t.B) + cl * (int64_t)sizeof(typename E::T),
                                    (uint32_t)(t.ldb * (int64_t)sizeof(typename E::T)), gl, acc,
                                    static_cast<const char*>(t.hot) + cl * (int64_t)sizeof(typename E::T),
                                    (uint32_t)(t.ldh * (int64_t)sizeof(typename E::T)));
    if (active) store_f32v<V>(P.partial + s * P.ldp + c0, acc);
    return;
  }

  const int64_t row = group_uniform<G>(((int64_t)blockIdx.x - unit_blocks) * GPB + threadIdx.x / G);
  if (row >= P.rows) return;
  int64_t len = 0;
  for (int k = 0; k < P.num_k; ++k) len += P.t[k].rowptr[row + 1] - P.t[k].rowptr[row];
  if (len > P.long_row) return;  // written by the fix-up
  for (int kk = 0; kk < P.num_k; ++kk) {
    int k = kk + P.k_offset;
    if (k >= P.num_k) k -= P.num_k;
    const TileDev& t = P.t[k];
    accumulate_range<G, V, E, HOT>(t, t.rowptr[row], t.rowptr[row + 1],
                                    static_cast<const char*>(t.B) + cl * (int64_t)sizeof(typename E::T),
                                    (uint32_t)(t.ldb * (int64_t)sizeof(typename E::T)), gl, acc,
                                    static_cast<const char*>(t.hot) + cl * (int64_t)sizeof(typename E::T),
                                    (uint32_t)(t.ldh * (int64_t)sizeof(typename E::T)));
  }
  if (!active) return;
  typename E::T* c = static_cast<typename E::T*>(P.C) + row * P.ldc + c0;
  if (P.accumulate) {
    float old[V];
    load_vec<E, V>(c, old);
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] += old[e];
  }
  store_vec_nt<E, V>(c, acc);
}

// Stream variant: one wave owns R <= 64 consecutive rows (one per lane for the
// bookkeeping) and walks the concatenation of their non-zeros, over all
// k-tiles in k' order, 64 entries at a time.  Every entry's B row address and
// value are formed by the lane that loaded it, then consumed in order by the
// whole wave (readlane: the address is wave-uniform, each lane loads its V
// columns); accumulators are flushed to C when an entry closes its row.  So
// the B loads of many short rows are in flight together, and the per-row
// order of summation (k' order, then CSR position) is the row-split one.
// Rows longer than the split threshold are left to the units and the fix-up.
template <int V>
constexpr int stream_unroll() {
  return V >= 8 ? 4 : (V >= 4 ? 8 : 16);
}

template <int V, typename E, bool ACC>
__device__ __forceinline__ void store_row(const FwdParams& P, int64_t row, int64_t c0, bool active,
                                          float (&acc)[V]) {
  if (!active) return;
  typename E::T* c = static_cast<typename E::T*>(P.C) + row * P.ldc + c0;
  if constexpr (ACC) {
    float old[V];
    load_vec<E, V>(c, old);
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] += old[e];
  }
  store_vec_nt<E, V>(c, acc);
}

template <int V, typename E, bool ACC, bool HOT>
__global__ void __launch_bounds__(kBlock) fwd_stream(FwdParams P) {
  constexpr int GPB = kBlock / 64;
  constexpr int U = stream_unroll<V>();
  using T = typename E::T;
  extern __shared__ int32_t s_mem[];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int K = P.num_k;
  const int64_t c0 = (int64_t)blockIdx.y * (64 * V) + (int64_t)lane * V;
  const bool active = c0 < P.N;
  const int64_t cl = active ? c0 : 0;
  const int64_t unit_blocks = (P.n_seg + GPB - 1) / GPB;
  float acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = 0.0f;

  if ((int64_t)blockIdx.x < unit_blocks) {
    const int64_t s = group_uniform<64>((int64_t)blockIdx.x * GPB + w);
    if (s >= P.n_seg) return;
    const Seg d = P.seg[s];
    const TileDev& t = P.t[d.k];
    accumulate_range<64, V, E, HOT>(t, d.p0, d.p1, static_cast<const char*>(t.B) + cl * (int64_t)sizeof(T),
                                     (uint32_t)(t.ldb * (int64_t)sizeof(T)), lane, acc,
                                     static_cast<const char*>(t.hot) + cl * (int64_t)sizeof(T),
                                     (uint32_t)(t.ldh * (int64_t)sizeof(T)));
    if (active) store_f32v<V>(P.partial + s * P.ldp + c0, acc);
    return;
  }

  const int R = P.stream_rows;  // rows per wave (1..64); lanes >= R carry no row
  const int64_t r0 = group_uniform<64>((((int64_t)blockIdx.x - unit_blocks) * GPB + w) * R);
  if (r0 >= P.rows) return;
  int32_t* s_pref = s_mem + w * (65 + 128 * K);  // exclusive prefix of streamed lengths, [64] = total
  int32_t* s_beg = s_pref + 65;                   // [kk][lane]: first CSR position of the row in tile kk
  int32_t* s_koff = s_beg + 64 * K;               // [kk][lane]: offset of tile kk inside the row
  const int64_t row = r0 + lane;
  const bool inrow = lane < R && row < P.rows;
  // A row's length over up to 16 k-tiles can pass 2^31: summed in 64 bits.  Streamed rows
  // are at most long_row long (checked against 2^31 / 64 at creation), so the 64-lane
  // prefix below and every in-row offset fit in 32 bits; offsets of split rows are never read.
  int64_t L = 0;
  for (int kk = 0; kk < K; ++kk) {
    int k = kk + P.k_offset;
    if (k >= K) k -= K;
    int32_t b = 0, l = 0;
    if (inrow) {
      b = P.t[k].rowptr[row];
      l = P.t[k].rowptr[row + 1] - b;
    }
    s_beg[kk * 64 + lane] = b;
    s_koff[kk * 64 + lane] = (int32_t)L;
    L += l;
  }
  const int32_t Ls = (L > P.long_row) ? 0 : (int32_t)L;  // split rows are not streamed
  int32_t incl = Ls;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  s_pref[lane] = incl - Ls;
  if (lane == 63) s_pref[64] = incl;
  const int32_t total = __builtin_amdgcn_readlane(incl, 63);
  // The bookkeeping above is read back by other lanes of this wave only.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // Empty rows: C = 0, or untouched when accumulating.
  if constexpr (!ACC) {
    uint64_t em = __ballot(inrow && L == 0);
    float z[V];
#pragma unroll
    for (int e = 0; e < V; ++e) z[e] = 0.0f;
    while (em) {
      const int i = __ffsll((long long)em) - 1;
      em &= em - 1;
      if (active) store_vec_nt<E, V>(static_cast<T*>(P.C) + (r0 + i) * P.ldc + c0, z);
    }
  }

  for (int32_t qc = 0; qc < total; qc += 64) {
    const int n = min(64, total - qc);
    const int32_t q = qc + lane;
    // Row of entry q: the last lane i with s_pref[i] <= q.
    int ri = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
      const int cand = ri + step;
      if (cand <= 63 && s_pref[cand] <= q) ri = cand;
    }
    const int32_t o = q - s_pref[ri];
    int kk = 0;
    for (int t = 1; t < K; ++t)
      if (s_koff[t * 64 + ri] <= o) kk = t;
    int k = kk + P.k_offset;
    if (k >= K) k -= K;
    const int32_t p = s_beg[kk * 64 + ri] + (o - s_koff[kk * 64 + ri]);
    const int32_t* colp = P.t[0].colind;
    const float* valp = P.t[0].values;
    const char* bp = static_cast<const char*>(P.t[0].B);
    int64_t ldbb = P.t[0].ldb;
    const char* hp = static_cast<const char*>(P.t[0].hot);
    int64_t ldhh = P.t[0].ldh;
    for (int t = 1; t < K; ++t) {
      if (k == t) {
        colp = P.t[t].colind;
        valp = P.t[t].values;
        bp = static_cast<const char*>(P.t[t].B);
        ldbb = P.t[t].ldb;
        hp = static_cast<const char*>(P.t[t].hot);
        ldhh = P.t[t].ldh;
      }
    }
    uint64_t addr = 0;
    float val = 0.0f;
    int end = 0;
    if (lane < n) {
      const uint32_t col = (uint32_t)__builtin_nontemporal_load(colp + p);
      val = __builtin_nontemporal_load(valp + p);
      addr = reinterpret_cast<uint64_t>(entry_row<HOT>(col, bp, (uint32_t)(ldbb * (int64_t)sizeof(T)), hp,
                                                        (uint32_t)(ldhh * (int64_t)sizeof(T))));
      end = (q + 1 == s_pref[ri + 1]) ? 1 : 0;
    }
    const uint32_t alo = (uint32_t)addr, ahi = (uint32_t)(addr >> 32);
    const uint64_t coff = (uint64_t)(cl * (int64_t)sizeof(T));
    // Double-buffered: the loads of the next U entries are issued before the
    // current U are consumed.  Entries past n repeat the last one (never summed).
    auto issue = [&](float (&b)[U][V], int u0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int jj = min(u0 + u, n - 1);
        const uint64_t a = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)ahi, jj) << 32) |
                           (uint32_t)__builtin_amdgcn_readlane((int)alo, jj);
        load_vec_at<E, V>(a + coff, b[u]);
      }
    };
    auto consume = [&](const float (&b)[U][V], int u0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int jj = min(u0 + u, n - 1);
        const bool ok = u0 + u < n;
        const float v = ok ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(val), jj)) : 0.0f;
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] = fmaf(v, ok ? b[u][e] : 0.0f, acc[e]);
        if (ok && __builtin_amdgcn_readlane(end, jj)) {
          const int r = __builtin_amdgcn_readlane(ri, jj);
          store_row<V, E, ACC>(P, r0 + r, c0, active, acc);
#pragma unroll
          for (int e = 0; e < V; ++e) acc[e] = 0.0f;
        }
      }
    };
    float bA[U][V], bB[U][V];
    issue(bA, 0);
    for (int u0 = 0;;) {
      if (u0 + U < n) issue(bB, u0 + U);
      consume(bA, u0);
      u0 += U;
      if (u0 >= n) break;
      if (u0 + U < n) issue(bA, u0 + U);
      consume(bB, u0);
      u0 += U;
      if (u0 >= n) break;
    }
  }
}

// acc += partial rows [a, b) in order, eight loads in flight.
template <int V>
__device__ __forceinline__ void sum_partials(const FwdParams& P, int a, int b, int64_t c0, float (&acc)[V]) {
  for (int s = a; s < b; s += 8) {
    float x[8][V];
#pragma unroll
    for (int u = 0; u < 8; ++u) load_f32v<V>(P.partial + (int64_t)min(s + u, b - 1) * P.ldp + c0, x[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (s + u < b) {
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] += x[u][e];
      }
  }
}

// One group per split row: the row's units are stored by k-tile (0..K-1), so the
// k' order (k = (k' + k_offset) mod K) is the units of k >= k_offset, then the rest.
template <int G, int V, typename E>
__global__ void __launch_bounds__(kBlock) fwd_fixup(FwdParams P) {
  constexpr int GPB = kBlock / G;
  const int gl = threadIdx.x & (G - 1);
  const int64_t c0 = (int64_t)blockIdx.y * (G * V) + (int64_t)gl * V;
  const int64_t r = group_uniform<G>((int64_t)blockIdx.x * GPB + threadIdx.x / G);
  if (r >= P.n_long || c0 >= P.N) return;
  const LongRow lr = P.lrow[r];
  int m = lr.s0;
  if (P.k_offset > 0) {  // first unit with k >= k_offset
    int lo = lr.s0, hi = lr.s1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (P.seg[mid].k < P.k_offset) lo = mid + 1; else hi = mid;
    }
    m = lo;
  }
  float acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = 0.0f;
  sum_partials<V>(P, m, lr.s1, c0, acc);
  sum_partials<V>(P, lr.s0, m, c0, acc);
  typename E::T* c = static_cast<typename E::T*>(P.C) + (int64_t)lr.row * P.ldc + c0;
  if (P.accumulate) {
    float old[V];
    load_vec<E, V>(c, old);
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] += old[e];
  }
  store_vec<E, V>(c, acc);
}

template <int G, int V, typename E, bool HOT>
hipError_t launch_gvh(const FwdParams& P0, bool stream, hipStream_t s) {
  FwdParams P = P0;
  constexpr int GPB = kBlock / G;
  const int64_t unit_blocks = (P.n_seg + GPB - 1) / GPB;
  const int64_t windows = (P.N + G * V - 1) / (G * V);
  if (stream) {
    // stream_rows rows per wave, GPB waves per workgroup
    const int64_t row_blocks = (P.rows + (int64_t)P.stream_rows * GPB - 1) / ((int64_t)P.stream_rows * GPB);
    P.row_blocks = row_blocks;
    const size_t lds = sizeof(int32_t) * (size_t)GPB * (65 + 128 * (size_t)P.num_k);
    dim3 grid((unsigned)(unit_blocks + row_blocks), (unsigned)windows);
    if (P.accumulate)
      hipLaunchKernelGGL((fwd_stream<V, E, true, HOT>), grid, dim3(kBlock), lds, s, P);
    else
      hipLaunchKernelGGL((fwd_stream<V, E, false, HOT>), grid, dim3(kBlock), lds, s, P);
  } else {
    const int64_t row_blocks = (P.rows + GPB - 1) / GPB;
    P.row_blocks = row_blocks;
    dim3 grid((unsigned)(unit_blocks + row_blocks), (unsigned)windows);
    hipLaunchKernelGGL((fwd_main<G, V, E, HOT>), grid, dim3(kBlock), 0, s, P);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (P.n_long > 0) {
    dim3 grid((unsigned)((P.n_long + GPB - 1) / GPB), (unsigned)windows);
    hipLaunchKernelGGL((fwd_fixup<G, V, E>), grid, dim3(kBlock), 0, s, P);
    return hipGetLastError();
  }
  return hipSuccess;
}

// Kernels that read staged hot rows are separate instances, so that handles without
// staging pay nothing for the address select.
template <int G, int V, typename E>
hipError_t launch_gv(const FwdParams& P, bool stream, hipStream_t s) {
  return P.hot ? launch_gvh<G, V, E, true>(P, stream, s) : launch_gvh<G, V, E, false>(P, stream, s);
}

template <typename E, int V>
hipError_t launch_v(const FwdParams& P, const Variant& v, hipStream_t s) {
  if (v.stream) {
    FwdParams Q = P;
    Q.stream_rows = (v.rows >= 1 && v.rows <= 64) ? v.rows : 64;
    return launch_gv<64, V, E>(Q, true, s);
  }
  switch (v.G) {
    case 4: return launch_gv<4, V, E>(P, false, s);
    case 8: return launch_gv<8, V, E>(P, false, s);
    case 16: return launch_gv<16, V, E>(P, false, s);
    case 32: return launch_gv<32, V, E>(P, false, s);
    case 64: return launch_gv<64, V, E>(P, false, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename E, int V>
hipError_t launch_fixup_v(const FwdParams& P, int G, hipStream_t s) {
  if (P.n_long == 0) return hipSuccess;
  const int64_t windows = (P.N + (int64_t)G * V - 1) / ((int64_t)G * V);
  const int64_t rows_blocks = (P.n_long * G + kBlock - 1) / kBlock;
  dim3 grid((unsigned)rows_blocks, (unsigned)windows);
  switch (G) {
    case 4: hipLaunchKernelGGL((fwd_fixup<4, V, E>), grid, dim3(kBlock), 0, s, P); break;
    case 8: hipLaunchKernelGGL((fwd_fixup<8, V, E>), grid, dim3(kBlock), 0, s, P); break;
    case 16: hipLaunchKernelGGL((fwd_fixup<16, V, E>), grid, dim3(kBlock), 0, s, P); break;
    case 32: hipLaunchKernelGGL((fwd_fixup<32, V, E>), grid, dim3(kBlock), 0, s, P); break;
    case 64: hipLaunchKernelGGL((fwd_fixup<64, V, E>), grid, dim3(kBlock), 0, s, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fixup(const FwdParams& P, int G, int V, DT dt, hipStream_t s) {
  if (dt == DT::F32) {
    switch (V) {
      case 1: return launch_fixup_v<F32E, 1>(P, G, s);
      case 2: return launch_fixup_v<F32E, 2>(P, G, s);
      case 4: return launch_fixup_v<F32E, 4>(P, G, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (V) {
    case 1: return launch_fixup_v<BF16E, 1>(P, G, s);
    case 2: return launch_fixup_v<BF16E, 2>(P, G, s);
    case 4: return launch_fixup_v<BF16E, 4>(P, G, s);
    case 8: return launch_fixup_v<BF16E, 8>(P, G, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fwd(const FwdParams& P, Variant v, DT dt, hipStream_t s) {
  if (dt == DT::F32) {
    switch (v.V) {
      case 1: return launch_v<F32E, 1>(P, v, s);
      case 2: return launch_v<F32E, 2>(P, v, s);
      case 4: return launch_v<F32E, 4>(P, v, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (v.V) {
    case 1: return launch_v<BF16E, 1>(P, v, s);
    case 2: return launch_v<BF16E, 2>(P, v, s);
    case 4: return launch_v<BF16E, 4>(P, v, s);
    case 8: return launch_v<BF16E, 8>(P, v, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace spmm
