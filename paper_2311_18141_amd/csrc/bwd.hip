// Backward of C = A B with respect to A's stored values: the sampled dense-dense
// product on A's pattern,  dA[p] = <dC[row(p), :], B[colind[p], :]>, with dC and B
// in FP32 or BF16 (FP32 products and sums; dA in FP32, as A's values).
// (dB = A^T dC reuses the forward kernels on the transposed structure.)
//
// A group of G lanes owns U consecutive non-zeros.  Lane l < U of the group reads the
// row and column of non-zero l (one coalesced load each) and the group broadcasts
// them; each lane then loads V consecutive columns of the U rows of B (and of dC,
// loaded once per distinct row), so U rows of B are in flight per group.  Partial
// dot products accumulate in FP32 and every group reduces with a fixed butterfly, so
// the result does not depend on scheduling.  One launch covers the columns
// [c_begin, c_end); the host may split N into column slices launched one after the
// other (each adding to dA), so that one slice of B stays cache-resident.
#include <algorithm>

#include "elem.hpp"
#include "fwd_common.hpp"
#include "internal.hpp"

namespace spmm {
namespace {

template <int G>
__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <int G, int V, int U, typename E>
__global__ void __launch_bounds__(kBlock) sddmm_kernel(SddmmParams P) {
  static_assert(U <= G, "one lane per non-zero reads the structure");
  using T = typename E::T;
  const T* Bp = static_cast<const T*>(P.B);
  const T* dCp = static_cast<const T*>(P.dC);
  constexpr int GPB = kBlock / G;
  const int gl = threadIdx.x & (G - 1);
  // grid-stride over groups of U non-zeros (the grid is capped below 2^32 threads)
  for (int64_t p0 = ((int64_t)blockIdx.x * GPB + threadIdx.x / G) * U; p0 < P.nnz;
       p0 += (int64_t)gridDim.x * GPB * U) {
    const int cnt = (int)(P.nnz - p0 < U ? P.nnz - p0 : U);
    int my_r = 0, my_c = 0;
    if (gl < cnt) {
      my_r = __builtin_nontemporal_load(P.rowid + p0 + gl);
      my_c = __builtin_nontemporal_load(P.colind + p0 + gl);
    }
    int r[U], c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int src = u < cnt ? u : cnt - 1;  // a short tail repeats its last non-zero
      r[u] = group_bcast<G>(my_r, src);
      c[u] = group_bcast<G>(my_c, src);
    }
    float acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0f;
    for (int64_t col = P.c_begin + (int64_t)gl * V; col < P.c_end; col += G * V) {
      float x[U][V], y[U][V];
#pragma unroll
      for (int u = 0; u < U; ++u) load_vec<E, V>(Bp + (int64_t)c[u] * P.ldb + col, y[u]);
      load_vec<E, V>(dCp + (int64_t)r[0] * P.lddc + col, x[0]);
#pragma unroll
      for (int u = 1; u < U; ++u) {
        if (r[u] != r[u - 1]) {
          load_vec<E, V>(dCp + (int64_t)r[u] * P.lddc + col, x[u]);
        } else {
#pragma unroll
          for (int e = 0; e < V; ++e) x[u][e] = x[u - 1][e];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int e = 0; e < V; ++e) acc[u] = fmaf(x[u][e], y[u][e], acc[u]);
      }
    }
    float mine = 0.0f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float t = group_sum<G>(acc[u]);
      if (gl == u) mine = t;
    }
    if (gl < cnt) {
      float* out = P.dA + p0 + gl;
      *out = P.accumulate ? *out + mine : mine;
    }
  }
}

template <typename E, int V, int U>
hipError_t launch_sddmm_vu(const SddmmParams& P, int G, hipStream_t s) {
  auto go = [&](auto kern, int gpb) {
    const int64_t per_block = (int64_t)gpb * U;
    const int64_t blocks = std::min<int64_t>((P.nnz + per_block - 1) / per_block, kMaxGridBlocks);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kBlock), 0, s, P);
    return hipGetLastError();
  };
  switch (G) {
    case 4: if constexpr (U <= 4) return go(sddmm_kernel<4, V, U, E>, kBlock / 4); else return hipErrorInvalidValue;
    case 8: return go(sddmm_kernel<8, V, U, E>, kBlock / 8);
    case 16: return go(sddmm_kernel<16, V, U, E>, kBlock / 16);
    case 32: return go(sddmm_kernel<32, V, U, E>, kBlock / 32);
    case 64: return go(sddmm_kernel<64, V, U, E>, kBlock / 64);
    default: return hipErrorInvalidValue;
  }
}

template <typename E, int V>
hipError_t launch_sddmm_v(const SddmmParams& P, int G, int U, hipStream_t s) {
  switch (U) {
    case 1: return launch_sddmm_vu<E, V, 1>(P, G, s);
    case 2: return launch_sddmm_vu<E, V, 2>(P, G, s);
    case 4: return launch_sddmm_vu<E, V, 4>(P, G, s);
    case 8: return launch_sddmm_vu<E, V, 8>(P, G, s);
    default: return hipErrorInvalidValue;
  }
}

// out[q] = values[perm[q]]: A's values in the transposed structure's order, so that the
// dB pass reads them coalesced (every load here is independent, so the random reads
// of `values` overlap freely).
__global__ void __launch_bounds__(kBlock) gather_values_kernel(const int32_t* perm, const float* values, float* out,
                                                                int64_t nnz) {
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * kBlock)
    out[q] = values[__builtin_nontemporal_load(perm + q)];
}

// C[r, c] += P[r, c] over a rows x N block; one thread per V consecutive elements.
template <int V, typename E>
__global__ void __launch_bounds__(kBlock) accumulate_kernel(typename E::T* C, int64_t ldc, const typename E::T* Pt,
                                                            int64_t ldp, int64_t rows, int64_t N) {
  const int64_t per_row = N / V;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < rows * per_row; i += (int64_t)gridDim.x * kBlock) {
    const int64_t r = i / per_row, c = (i - r * per_row) * V;
    float x[V], y[V];
    load_vec<E, V>(C + r * ldc + c, x);
    load_vec<E, V>(Pt + r * ldp + c, y);
#pragma unroll
    for (int e = 0; e < V; ++e) x[e] += y[e];
    store_vec<E, V>(C + r * ldc + c, x);
  }
}

template <typename E, int V>
hipError_t launch_acc(void* C, int64_t ldc, const void* Pt, int64_t ldp, int64_t rows, int64_t N, hipStream_t s) {
  const int64_t n = rows * (N / V);
  if (n == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, kMaxGridBlocks);
  hipLaunchKernelGGL((accumulate_kernel<V, E>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                     static_cast<typename E::T*>(C), ldc, static_cast<const typename E::T*>(Pt), ldp, rows, N);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_accumulate(void* C, int64_t ldc, const void* Pt, int64_t ldp, int64_t rows, int64_t N, DT dt,
                             int V, hipStream_t s) {
  if (dt == DT::F32) {
    switch (V) {
      case 4: return launch_acc<F32E, 4>(C, ldc, Pt, ldp, rows, N, s);
      case 2: return launch_acc<F32E, 2>(C, ldc, Pt, ldp, rows, N, s);
      default: return launch_acc<F32E, 1>(C, ldc, Pt, ldp, rows, N, s);
    }
  }
  switch (V) {
    case 8: return launch_acc<BF16E, 8>(C, ldc, Pt, ldp, rows, N, s);
    case 4: return launch_acc<BF16E, 4>(C, ldc, Pt, ldp, rows, N, s);
    case 2: return launch_acc<BF16E, 2>(C, ldc, Pt, ldp, rows, N, s);
    default: return launch_acc<BF16E, 1>(C, ldc, Pt, ldp, rows, N, s);
  }
}

hipError_t launch_gather_values(const int32_t* perm, const float* values, float* out, int64_t nnz, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((nnz + kBlock - 1) / kBlock, kMaxGridBlocks);
  hipLaunchKernelGGL(gather_values_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, perm, values, out, nnz);
  return hipGetLastError();
}

hipError_t launch_sddmm(const SddmmParams& P, int G, int V, int U, DT dt, hipStream_t s) {
  if (dt == DT::F32) {
    switch (V) {
      case 1: return launch_sddmm_v<F32E, 1>(P, G, U, s);
      case 2: return launch_sddmm_v<F32E, 2>(P, G, U, s);
      case 4: return launch_sddmm_v<F32E, 4>(P, G, U, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (V) {
    case 1: return launch_sddmm_v<BF16E, 1>(P, G, U, s);
    case 2: return launch_sddmm_v<BF16E, 2>(P, G, U, s);
    case 4: return launch_sddmm_v<BF16E, 4>(P, G, U, s);
    case 8: return launch_sddmm_v<BF16E, 8>(P, G, U, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace spmm
