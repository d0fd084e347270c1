// Device building blocks shared by the forward kernels (fwd.hip) and the
// batched persistent kernel (batch.hip).
#pragma once

#include "elem.hpp"
#include "internal.hpp"

namespace spmm {

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

// Address of column window c0 of the B row an entry names: B row `col`, or, for a
// tagged entry (bit 31 set), staged row col & ~kHotTag of the hot block.  brow / hrow
// already include the window offset c0 (bytes).
template <bool HOT>
__device__ __forceinline__ const char* entry_row(uint32_t col, const char* brow, uint32_t ldb_bytes,
                                                 const char* hrow, uint32_t ldh_bytes) {
  if constexpr (HOT) {
    const bool h = (col & kHotTag) != 0;
    return (h ? hrow : brow) + (uint64_t)(col & ~kHotTag) * (h ? ldh_bytes : ldb_bytes);
  } else {
    return brow + (uint64_t)col * ldb_bytes;
  }
}

// acc += sum over p in [p0, p1) of val(p) * B[col(p), c0 .. c0+V), where
// brow = B + c0 (bytes) and B rows are ldb_bytes apart (< 2^32, checked by the host);
// with HOT, tagged entries read the staged row at hrow + slot * ldh_bytes instead.
// Full batches of U non-zeros issue U independent row loads before any FMA; the
// last partial batch is predicated without branches (clamped source, zeroed terms).
template <int G, int V, typename E, bool HOT = false>
__device__ __forceinline__ void accumulate_range(const TileDev& t, int p0, int p1, const char* brow,
                                                 uint32_t ldb_bytes, int gl, float (&acc)[V],
                                                 const char* hrow = nullptr, uint32_t ldh_bytes = 0) {
  constexpr int U = unroll_for<V>();
  using T = typename E::T;
  for (int pc = p0; pc < p1; pc += G) {
    const int cnt = min(G, p1 - pc);
    int my_col = 0;
    float my_val = 0.0f;
    if (gl < cnt) {
      my_col = __builtin_nontemporal_load(t.colind + pc + gl);
      my_val = __builtin_nontemporal_load(t.values + pc + gl);
    }
    int j = 0;
    for (; j + U <= cnt; j += U) {
      float b[U][V];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t col = (uint32_t)group_bcast<G>(my_col, j + u);
        load_vec<E, V>(reinterpret_cast<const T*>(entry_row<HOT>(col, brow, ldb_bytes, hrow, ldh_bytes)), b[u]);
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
        load_vec<E, V>(reinterpret_cast<const T*>(entry_row<HOT>(col, brow, ldb_bytes, hrow, ldh_bytes)), b[u]);
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

// Register-lean form of accumulate_range for the persistent batched kernel: one
// predicated code path with U loads in flight (every batch clamps its sources to
// the last entry and zeroes the terms past the end).
template <int G, int V, typename E, int U>
__device__ __forceinline__ void accumulate_range_lean(const TileDev& t, int p0, int p1, const char* brow,
                                                      uint32_t ldb_bytes, int gl, float (&acc)[V]) {
  using T = typename E::T;
  for (int pc = p0; pc < p1; pc += G) {
    const int cnt = min(G, p1 - pc);
    int my_col = 0;
    float my_val = 0.0f;
    if (gl < cnt) {
      my_col = __builtin_nontemporal_load(t.colind + pc + gl);
      my_val = __builtin_nontemporal_load(t.values + pc + gl);
    }
    for (int j = 0; j < cnt; j += U) {
      float b[U][V];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t col = (uint32_t)group_bcast<G>(my_col, min(j + u, cnt - 1));
        load_vec<E, V>(reinterpret_cast<const T*>(brow + (uint64_t)col * ldb_bytes), b[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = j + u < cnt;
        const float v = __int_as_float(group_bcast<G>(__float_as_int(my_val), min(j + u, cnt - 1)));
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] = fmaf(ok ? v : 0.0f, ok ? b[u][e] : 0.0f, acc[e]);
      }
    }
  }
}

}  // namespace spmm
