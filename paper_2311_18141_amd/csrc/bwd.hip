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

// Sums of U values over a group of G lanes, scattered: after log2(U) halving steps
// (the lane bit at each step's distance decides which half of its values a lane keeps
// and which it sends to its partner) every lane holds one partial sum, of value
// u = lane / (G / U); plain butterfly steps over the remaining G / U lanes complete it.
// U - 1 + log2(G / U) exchanges for U sums, in a fixed order.
template <int G, int U>
__device__ __forceinline__ float group_sum_scatter(float (&d)[U], int gl) {
  static_assert(U <= G, "at most one value per lane");
#pragma unroll
  for (int c = U, o = G / 2; c > 1; c >>= 1, o >>= 1) {
    const bool hi = (gl & o) != 0;
#pragma unroll
    for (int k = 0; k < c / 2; ++k) {
      const float keep = hi ? d[k + c / 2] : d[k];
      const float send = hi ? d[k] : d[k + c / 2];
      d[k] = keep + __shfl_xor(send, o, 64);
    }
  }
  float x = d[0];
#pragma unroll
  for (int o = G / U / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Fused backward over the transposed structure.  A group of G lanes owns one row j of
// A^T (one column of A) and one window of G * V columns (blockIdx.y; one window when
// G * V >= N): it keeps its part of B[j, :] in registers,
// walks the row's entries G at a time (lane l loads entry l's original row, position
// and value, the value read through the position), and for each batch of U entries
// gathers the U rows of dC once: each row feeds the dB accumulators (acc += a * dC[i, :])
// and a partial dot product with B[j, :]; the group sums the U dot products with one
// scattered reduction and the lane holding entry u's sum stores dA at its position (with
// several windows: the window's partial dot product at the entry's transposed position,
// summed over the windows by bwd_dA_sum).  Rows longer than long_row come as the
// transposed plan's units (first in the grid): a unit's dB partial row goes to the
// workspace for the fix-up, its dA entries are final (or partial per window as above).
template <int G, int V, int U, typename E>
__global__ void __launch_bounds__(kBlock) bwd_fused(BwdFusedParams P) {
  static_assert(U <= G, "one lane per entry reads the structure");
  using T = typename E::T;
  constexpr int GPB = kBlock / G;
  const int gl = threadIdx.x & (G - 1);
  const int win = (int)blockIdx.y;
  const int64_t c0 = (int64_t)win * (G * V) + (int64_t)gl * V;
  const bool active = c0 < P.N;
  const int64_t cl = active ? c0 : 0;  // lanes past N read column 0 and contribute nothing
  const int64_t unit_blocks = (P.n_seg + GPB - 1) / GPB;
  const int64_t grp = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
  int64_t j, s = -1;
  int p0, p1;
  if ((int64_t)blockIdx.x < unit_blocks) {
    s = group_uniform<G>(grp);
    if (s >= P.n_seg) return;
    const Seg d = P.seg[s];
    j = d.row;
    p0 = d.p0;
    p1 = d.p1;
  } else {
    j = group_uniform<G>(grp - unit_blocks * GPB);
    if (j >= P.cols) return;
    p0 = P.rowptrT[j];
    p1 = P.rowptrT[j + 1];
    if (p1 - p0 > P.long_row) return;  // done by the units and the fix-up
  }
  float bj[V], acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) {
    bj[e] = 0.0f;
    acc[e] = 0.0f;
  }
  if (p1 > p0 && active) load_vec<E, V>(static_cast<const T*>(P.B) + j * P.ldb + cl, bj);
  const T* dCp = static_cast<const T*>(P.dC) + cl;
  constexpr int kPer = G / U;  // lanes per reduced sum
  for (int pc = p0; pc < p1; pc += G) {
    const int cnt = min(G, p1 - pc);
    int my_i = 0, my_p = 0;
    float my_a = 0.0f;
    if (gl < cnt) {
      my_i = __builtin_nontemporal_load(P.colindT + pc + gl);
      my_p = __builtin_nontemporal_load(P.perm + pc + gl);
      my_a = P.values[my_p];
    }
    for (int jj = 0; jj < cnt; jj += U) {
      float x[U][V];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = group_bcast<G>(my_i, min(jj + u, cnt - 1));
        load_vec<E, V>(dCp + (int64_t)i * P.lddc, x[u]);
      }
      float d[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = jj + u < cnt;
        const float a = __int_as_float(group_bcast<G>(__float_as_int(my_a), min(jj + u, cnt - 1)));
        float t = 0.0f;
#pragma unroll
        for (int e = 0; e < V; ++e) {
          t = fmaf(x[u][e], bj[e], t);
          acc[e] = fmaf(ok ? a : 0.0f, ok ? x[u][e] : 0.0f, acc[e]);
        }
        d[u] = t;
      }
      const float sum = group_sum_scatter<G, U>(d, gl);
      // position of entry jj + u (u = gl / kPer), from the lane of the group that loaded it
      const int u = gl / kPer;
      const int src = (int)(threadIdx.x & 63 & ~(G - 1)) + min(jj + u, cnt - 1);
      const int p = __builtin_amdgcn_ds_bpermute(src << 2, my_p);
      if ((gl & (kPer - 1)) == 0 && jj + u < cnt) {
        if (P.n_win == 1)
          P.dA[p] = sum;
        else
          P.dA_part[(int64_t)win * P.nnz + pc + jj + u] = sum;
      }
    }
  }
  if (!active) return;
  if (s >= 0) {
    store_f32v<V>(P.partial + s * P.ldp + c0, acc);
  } else {
    store_vec_nt<E, V>(static_cast<T*>(P.dB) + j * P.lddb + c0, acc);
  }
}

// dA[perm[q]] = the sum over the windows of the partial dot products of entry q of the
// transposed structure, in window order.
__global__ void __launch_bounds__(kBlock) bwd_dA_sum(const float* part, int n_win, int64_t nnz, const int32_t* perm,
                                                     float* dA) {
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * kBlock) {
    float x = part[q];
    for (int w = 1; w < n_win; ++w) x += part[(int64_t)w * nnz + q];
    dA[__builtin_nontemporal_load(perm + q)] = x;
  }
}

template <typename E, int V, int U>
hipError_t launch_fused_vu(const BwdFusedParams& P, int G, hipStream_t s) {
  auto go = [&](auto kern, int gpb) {
    const int64_t blocks = (P.n_seg + gpb - 1) / gpb + (P.cols + gpb - 1) / gpb;
    if (blocks == 0) return hipSuccess;
    if (blocks >= ((int64_t)1 << 31) || P.n_win < 1 || P.n_win > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks, (unsigned)P.n_win), dim3(kBlock), 0, s, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || P.n_win == 1 || P.nnz == 0) return e;
    const int64_t sb = std::min<int64_t>((P.nnz + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(bwd_dA_sum, dim3((unsigned)sb), dim3(kBlock), 0, s, P.dA_part, P.n_win, P.nnz, P.perm, P.dA);
    return hipGetLastError();
  };
  switch (G) {
    case 4: if constexpr (U <= 4) return go(bwd_fused<4, V, U, E>, kBlock / 4); else return hipErrorInvalidValue;
    case 8: return go(bwd_fused<8, V, U, E>, kBlock / 8);
    case 16: return go(bwd_fused<16, V, U, E>, kBlock / 16);
    case 32: return go(bwd_fused<32, V, U, E>, kBlock / 32);
    case 64: return go(bwd_fused<64, V, U, E>, kBlock / 64);
    default: return hipErrorInvalidValue;
  }
}

template <typename E, int V>
hipError_t launch_fused_v(const BwdFusedParams& P, int G, int U, hipStream_t s) {
  switch (U) {
    case 1: return launch_fused_vu<E, V, 1>(P, G, s);
    case 2: return launch_fused_vu<E, V, 2>(P, G, s);
    case 4: return launch_fused_vu<E, V, 4>(P, G, s);
    case 8: return launch_fused_vu<E, V, 8>(P, G, s);
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

hipError_t launch_bwd_fused(const BwdFusedParams& P, int G, int V, int U, DT dt, hipStream_t s) {
  if (dt == DT::F32) {
    switch (V) {
      case 1: return launch_fused_v<F32E, 1>(P, G, U, s);
      case 2: return launch_fused_v<F32E, 2>(P, G, U, s);
      case 4: return launch_fused_v<F32E, 4>(P, G, U, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (V) {
    case 1: return launch_fused_v<BF16E, 1>(P, G, U, s);
    case 2: return launch_fused_v<BF16E, 2>(P, G, U, s);
    case 4: return launch_fused_v<BF16E, 4>(P, G, U, s);
    case 8: return launch_fused_v<BF16E, 8>(P, G, U, s);
    default: return hipErrorInvalidValue;
  }
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
