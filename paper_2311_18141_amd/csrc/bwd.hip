// Backward of C = A B with respect to A's stored values: the sampled dense-dense
// product on A's pattern,  dA[p] = <dC[row(p), :], B[colind[p], :]>.
// (dB = A^T dC reuses the forward kernels on the transposed structure.)
//
// A group of G lanes owns one non-zero; each lane loads V consecutive columns of
// dC's row and B's row per step (coalesced within the group), accumulates the
// partial dot product in FP32 and the group reduces with a fixed butterfly, so
// the result does not depend on scheduling.  One launch covers the columns
// [c_begin, c_end); the host may split N into column slices launched one after
// the other (each adding to dA), so that one slice of B stays cache-resident.
#include "elem.hpp"
#include "internal.hpp"

namespace spmm {
namespace {

template <int G>
__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <int G, int V>
__global__ void __launch_bounds__(kBlock) sddmm_kernel(SddmmParams P) {
  constexpr int GPB = kBlock / G;
  const int gl = threadIdx.x & (G - 1);
  const int64_t p = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
  if (p >= P.nnz) return;
  const int64_t i = __builtin_nontemporal_load(P.rowid + p);
  const int64_t j = __builtin_nontemporal_load(P.colind + p);
  const float* g = P.dC + i * P.lddc;
  const float* b = P.B + j * P.ldb;
  float acc = 0.0f;
  for (int64_t c = P.c_begin + (int64_t)gl * V; c < P.c_end; c += G * V) {
    float x[V], y[V];
    load_f32v<V>(g + c, x);
    load_f32v<V>(b + c, y);
#pragma unroll
    for (int e = 0; e < V; ++e) acc = fmaf(x[e], y[e], acc);
  }
  acc = group_sum<G>(acc);
  if (gl == 0) P.dA[p] = P.accumulate ? P.dA[p] + acc : acc;
}

template <int V>
hipError_t launch_sddmm_v(const SddmmParams& P, int G, hipStream_t s) {
  auto go = [&](auto kern, int gpb) {
    const int64_t blocks = (P.nnz + gpb - 1) / gpb;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kBlock), 0, s, P);
    return hipGetLastError();
  };
  switch (G) {
    case 4: return go(sddmm_kernel<4, V>, kBlock / 4);
    case 8: return go(sddmm_kernel<8, V>, kBlock / 8);
    case 16: return go(sddmm_kernel<16, V>, kBlock / 16);
    case 32: return go(sddmm_kernel<32, V>, kBlock / 32);
    case 64: return go(sddmm_kernel<64, V>, kBlock / 64);
    default: return hipErrorInvalidValue;
  }
}

// C[r, c] += P[r, c] over a rows x N block; one thread per V consecutive elements.
template <int V, typename E>
__global__ void __launch_bounds__(kBlock) accumulate_kernel(typename E::T* C, int64_t ldc, const typename E::T* Pt,
                                                            int64_t ldp, int64_t rows, int64_t N) {
  const int64_t per_row = N / V;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= rows * per_row) return;
  const int64_t r = i / per_row, c = (i - r * per_row) * V;
  float x[V], y[V];
  load_vec<E, V>(C + r * ldc + c, x);
  load_vec<E, V>(Pt + r * ldp + c, y);
#pragma unroll
  for (int e = 0; e < V; ++e) x[e] += y[e];
  store_vec<E, V>(C + r * ldc + c, x);
}

template <typename E, int V>
hipError_t launch_acc(void* C, int64_t ldc, const void* Pt, int64_t ldp, int64_t rows, int64_t N, hipStream_t s) {
  const int64_t n = rows * (N / V);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((accumulate_kernel<V, E>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
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

hipError_t launch_sddmm(const SddmmParams& P, Variant v, hipStream_t s) {
  switch (v.V) {
    case 1: return launch_sddmm_v<1>(P, v.G, s);
    case 2: return launch_sddmm_v<2>(P, v.G, s);
    case 4: return launch_sddmm_v<4>(P, v.G, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace spmm
