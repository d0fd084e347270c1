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
#include "internal.hpp"

namespace spmm {
namespace {

template <int G>
__device__ __forceinline__ int group_bcast(int x, int src) {
  if constexpr (G == 64) {
    return __builtin_amdgcn_readlane(x, src);
  } else {
    const int lane = threadIdx.x & 63;
    return __builtin_amdgcn_ds_bpermute(((lane & ~(G - 1)) + src) << 2, x);
  }
}

template <int G>
__device__ __forceinline__ int64_t group_uniform(int64_t x) {
  if constexpr (G == 64) {
    // A full wave shares the value; make it scalar so row data moves through SGPRs.
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
  } else {
    return x;
  }
}

template <int V>
constexpr int unroll_for() {
  return V >= 8 ? 4 : 8;
}

// acc += sum over p in [p0, p1) of val(p) * B[col(p), c0 .. c0+V), where
// brow = B + c0 (bytes) and B rows are ldb_bytes apart (< 2^32, checked by the host).
// Full batches of U non-zeros issue U independent row loads before any FMA; the
// last partial batch is predicated without branches (clamped source, zeroed terms).
template <int G, int V, typename E>
__device__ __forceinline__ void accumulate_range(const TileDev& t, int p0, int p1, const char* brow,
                                                 uint32_t ldb_bytes, int gl, float (&acc)[V]) {
  constexpr int U = unroll_for<V>();
  using T = typename E::T;
  for (int pc = p0; pc < p1; pc += G) {
    const int cnt = min(G, p1 - pc);
    int my_col = 0;
    float my_val = 0.0f;
    if (gl < cnt) {
      my_col = __builtin_nontemporal_load(t.colind + pc + gl);
      my_val = t.perm ? t.values[t.perm[pc + gl]] : __builtin_nontemporal_load(t.values + pc + gl);
    }
    int j = 0;
    for (; j + U <= cnt; j += U) {
      float b[U][V];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t col = (uint32_t)group_bcast<G>(my_col, j + u);
        load_vec<E, V>(reinterpret_cast<const T*>(brow + (uint64_t)col * ldb_bytes), b[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float v = __int_as_float(group_bcast<G>(__float_as_int(my_val), j + u));
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] = fmaf(v, b[u][e], acc[e]);
      }
    }
    if (j < cnt) {
      float b[U][V];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = min(j + u, cnt - 1);
        const uint32_t col = (uint32_t)group_bcast<G>(my_col, src);
        load_vec<E, V>(reinterpret_cast<const T*>(brow + (uint64_t)col * ldb_bytes), b[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = min(j + u, cnt - 1);
        const bool ok = j + u < cnt;
        const float v = __int_as_float(group_bcast<G>(__float_as_int(my_val), src));
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] = fmaf(ok ? v : 0.0f, ok ? b[u][e] : 0.0f, acc[e]);
      }
    }
  }
}

template <int G, int V, typename E>
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
    accumulate_range<G, V, E>(t, d.p0, d.p1,
                              static_cast<const char*>(t.B) + cl * (int64_t)sizeof(typename E::T),
                              (uint32_t)(t.ldb * (int64_t)sizeof(typename E::T)), gl, acc);
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
    accumulate_range<G, V, E>(t, t.rowptr[row], t.rowptr[row + 1],
                              static_cast<const char*>(t.B) + cl * (int64_t)sizeof(typename E::T),
                              (uint32_t)(t.ldb * (int64_t)sizeof(typename E::T)), gl, acc);
  }
  if (!active) return;
  typename E::T* c = static_cast<typename E::T*>(P.C) + row * P.ldc + c0;
  if (P.accumulate) {
    float old[V];
    load_vec<E, V>(c, old);
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] += old[e];
  }
  store_vec<E, V>(c, acc);
}

template <int G, int V, typename E>
__global__ void __launch_bounds__(kBlock) fwd_fixup(FwdParams P) {
  constexpr int GPB = kBlock / G;
  const int gl = threadIdx.x & (G - 1);
  const int64_t c0 = (int64_t)blockIdx.y * (G * V) + (int64_t)gl * V;
  const int64_t r = group_uniform<G>((int64_t)blockIdx.x * GPB + threadIdx.x / G);
  if (r >= P.n_long || c0 >= P.N) return;
  const LongRow lr = P.lrow[r];
  float acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = 0.0f;
  for (int kk = 0; kk < P.num_k; ++kk) {
    int k = kk + P.k_offset;
    if (k >= P.num_k) k -= P.num_k;
    for (int s = lr.s0; s < lr.s1; ++s) {
      if (P.seg[s].k != k) continue;
      float x[V];
      load_f32v<V>(P.partial + (int64_t)s * P.ldp + c0, x);
#pragma unroll
      for (int e = 0; e < V; ++e) acc[e] += x[e];
    }
  }
  typename E::T* c = static_cast<typename E::T*>(P.C) + (int64_t)lr.row * P.ldc + c0;
  if (P.accumulate) {
    float old[V];
    load_vec<E, V>(c, old);
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] += old[e];
  }
  store_vec<E, V>(c, acc);
}

template <int G, int V, typename E>
hipError_t launch_gv(const FwdParams& P0, hipStream_t s) {
  FwdParams P = P0;
  constexpr int GPB = kBlock / G;
  const int64_t unit_blocks = (P.n_seg + GPB - 1) / GPB;
  const int64_t row_blocks = (P.rows + GPB - 1) / GPB;
  const int64_t windows = (P.N + G * V - 1) / (G * V);
  P.row_blocks = row_blocks;
  if (unit_blocks + row_blocks > 0) {
    dim3 grid((unsigned)(unit_blocks + row_blocks), (unsigned)windows);
    hipLaunchKernelGGL((fwd_main<G, V, E>), grid, dim3(kBlock), 0, s, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (P.n_long > 0) {
    dim3 grid((unsigned)((P.n_long + GPB - 1) / GPB), (unsigned)windows);
    hipLaunchKernelGGL((fwd_fixup<G, V, E>), grid, dim3(kBlock), 0, s, P);
    return hipGetLastError();
  }
  return hipSuccess;
}

template <typename E, int V>
hipError_t launch_v(const FwdParams& P, int G, hipStream_t s) {
  switch (G) {
    case 4: return launch_gv<4, V, E>(P, s);
    case 8: return launch_gv<8, V, E>(P, s);
    case 16: return launch_gv<16, V, E>(P, s);
    case 32: return launch_gv<32, V, E>(P, s);
    case 64: return launch_gv<64, V, E>(P, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_fwd(const FwdParams& P, Variant v, DT dt, hipStream_t s) {
  if (dt == DT::F32) {
    switch (v.V) {
      case 1: return launch_v<F32E, 1>(P, v.G, s);
      case 2: return launch_v<F32E, 2>(P, v.G, s);
      case 4: return launch_v<F32E, 4>(P, v.G, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (v.V) {
    case 1: return launch_v<BF16E, 1>(P, v.G, s);
    case 2: return launch_v<BF16E, 2>(P, v.G, s);
    case 4: return launch_v<BF16E, 4>(P, v.G, s);
    case 8: return launch_v<BF16E, 8>(P, v.G, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace spmm
