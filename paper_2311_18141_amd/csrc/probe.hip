// Gather micro-benchmark: the memory access of the forward kernels (whole rows of a
// dense table named by random row indices, 16-byte vector loads, several rows in flight
// per wave) without the arithmetic, so that its rate is the ceiling the caches and HBM
// set for such gathers at a given table size and row width.  The loaded words are
// XOR-folded into one 32-bit result (order-free, so the CPU can check it).
#include "internal.hpp"

namespace spmm {
namespace {

constexpr int kProbeUnroll = 8;

__global__ void __launch_bounds__(kBlock) probe_init_kernel(uint32_t* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = 0u;
}

// lanes_per_row = min(64, row_bytes / 16) lanes share one row; each lane loads
// row_bytes / 16 / lanes_per_row 16-byte vectors of it.  Waves stride over the index
// array 64 indices at a time, fetching the next 64 while the rows of the current ones
// load; one XOR per workgroup goes to memory.  Indices outside [0, rows) are skipped.
__global__ void __launch_bounds__(kBlock) probe_gather_kernel(const char* table, int64_t rows, int64_t row_bytes,
                                                              const int32_t* idx, int64_t n, uint32_t* out) {
  __shared__ uint32_t s_acc[kBlock / 64];
  const int lane = threadIdx.x & 63;
  const int vecs = (int)(row_bytes / 16);
  const int L = vecs < 64 ? vecs : 64;
  const int R = 64 / L;                 // rows per load instruction
  const int per_lane = vecs / L;        // vectors per lane per row
  const int sub = lane / L, pos = lane % L;
  const bool active = sub < R;          // L need not divide 64
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64;
  const int64_t stride = (int64_t)gridDim.x * kBlock;  // 64 indices per wave per step
  uint32_t acc = 0u;
  int64_t base = wave * 64;
  int32_t my = base + lane < n ? idx[base + lane] : -1;
  for (; base < n; base += stride) {
    const int64_t nb = base + stride;
    const int32_t nxt = nb + lane < n ? idx[nb + lane] : -1;
    for (int j = 0; j < 64; j += R * kProbeUnroll) {
      // every slot loads (a skipped one reads row 0, always present) and masks its
      // term: no branch between the loads, so all of them are in flight together
      int32_t r[kProbeUnroll];
      uint32_t m[kProbeUnroll];
#pragma unroll
      for (int u = 0; u < kProbeUnroll; ++u) {
        const int src = j + u * R + sub;
        const int32_t row = __shfl(my, src < 64 ? src : 63, 64);
        const bool ok = active && src < 64 && row >= 0 && row < rows;
        r[u] = ok ? row : 0;
        m[u] = ok ? 0xFFFFFFFFu : 0u;
      }
      for (int e = 0; e < per_lane; ++e) {
        uint4 v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u)
          v[u] = *reinterpret_cast<const uint4*>(table + (int64_t)r[u] * row_bytes + ((int64_t)e * L + pos) * 16);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) acc ^= (v[u].x ^ v[u].y ^ v[u].z ^ v[u].w) & m[u];
      }
    }
    my = nxt;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, o, 64);
  if (lane == 0) s_acc[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t x = 0u;
    for (int w = 0; w < kBlock / 64; ++w) x ^= s_acc[w];
    if (x) atomicXor(out, x);
  }
}

}  // namespace
}  // namespace spmm

extern "C" spmm_status spmm_gather_probe(const void* table, int64_t rows, int64_t row_bytes, const int32_t* idx,
                                         int64_t n, uint32_t* out, void* stream) {
  if (!out) return spmm::set_error(SPMM_ERR_INVALID_ARG, "out is null");
  if (rows < 1 || !table) return spmm::set_error(SPMM_ERR_INVALID_ARG, "table is empty or null");
  if (row_bytes < 16 || row_bytes > 4096 || (row_bytes % 16) != 0 ||
      (row_bytes > 1024 && (row_bytes % 1024) != 0))
    return spmm::set_error(SPMM_ERR_INVALID_ARG, "row_bytes=%lld: a multiple of 16 up to 1024, or of 1024 up to 4096",
                           (long long)row_bytes);
  if (n < 0 || (n > 0 && !idx)) return spmm::set_error(SPMM_ERR_INVALID_ARG, "bad index array");
  if ((reinterpret_cast<uintptr_t>(table) % 16) != 0) return spmm::set_error(SPMM_ERR_INVALID_ARG, "table not 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(spmm::probe_init_kernel, dim3(1), dim3(spmm::kBlock), 0, s, out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && n > 0) {
    const int64_t waves = (n + 63) / 64;
    int64_t blocks = (waves + 3) / 4;
    if (blocks > 2048) blocks = 2048;  // 8 workgroups of 4 waves per CU; the rest by striding
    hipLaunchKernelGGL(spmm::probe_gather_kernel, dim3((unsigned)blocks), dim3(spmm::kBlock), 0, s,
                       static_cast<const char*>(table), rows, row_bytes, idx, n, out);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return spmm::set_error(SPMM_ERR_HIP, "gather probe: %s", hipGetErrorString(e));
  return SPMM_OK;
}
