// Hot-row staging for the forward: on skewed matrices (R-MAT, Section 6's
// synthetic inputs) a few columns carry most non-zeros, and the B rows of those
// columns sit at addresses whose low bits are mostly zero, so the gathers crowd
// into a few memory channels.  The handle tags the non-zeros of each k-tile's most
// used columns in its own copy of colind; on every call the tagged rows are copied
// into one contiguous block of the workspace, where consecutive rows fall on
// different channels, and the forward reads them there.  The values read are the
// same B rows, so results are bit-identical to the untagged forward.
#include "internal.hpp"

namespace spmm {
namespace {

template <typename W>
__global__ void __launch_bounds__(kBlock) hot_stage_kernel(HotStageParams P) {
  const int64_t per_row = P.row_bytes / (int64_t)sizeof(W);
  const int64_t total = P.off[P.num_k] * per_row;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int64_t slot = i / per_row;
    const int64_t w = i - slot * per_row;
    int k = 0;
    for (int j = 1; j < P.num_k; ++j)
      if (P.off[j] <= slot) k = j;
    const char* src = static_cast<const char*>(P.B[k]) + (int64_t)P.src[slot] * P.ldb_bytes[k];
    const W x = reinterpret_cast<const W*>(src)[w];
    reinterpret_cast<W*>(P.dst + slot * P.ldh_bytes)[w] = x;
  }
}

__global__ void __launch_bounds__(kBlock) tag_hot_kernel(const int32_t* colind, int64_t nnz, const int32_t* slot_of,
                                                         int32_t* out) {
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * kBlock) {
    const int32_t c = colind[p];
    const int32_t h = slot_of[c];
    out[p] = h >= 0 ? (int32_t)(kHotTag | (uint32_t)h) : c;
  }
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return (unsigned)(b < kMaxGridBlocks ? (b > 0 ? b : 1) : kMaxGridBlocks);
}

}  // namespace

hipError_t launch_hot_stage(const HotStageParams& P, int width_bytes, hipStream_t s) {
  const int64_t slots = P.off[P.num_k];
  if (slots == 0 || P.row_bytes == 0) return hipSuccess;
  switch (width_bytes) {
    case 16:
      hipLaunchKernelGGL(hot_stage_kernel<uint4>, dim3(grid_for(slots * (P.row_bytes / 16))), dim3(kBlock), 0, s, P);
      break;
    case 4:
      hipLaunchKernelGGL(hot_stage_kernel<uint32_t>, dim3(grid_for(slots * (P.row_bytes / 4))), dim3(kBlock), 0, s, P);
      break;
    case 2:
      hipLaunchKernelGGL(hot_stage_kernel<uint16_t>, dim3(grid_for(slots * (P.row_bytes / 2))), dim3(kBlock), 0, s, P);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tag_hot(const int32_t* colind, int64_t nnz, const int32_t* slot_of, int32_t* out, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(tag_hot_kernel, dim3(grid_for(nnz)), dim3(kBlock), 0, s, colind, nnz, slot_of, out);
  return hipGetLastError();
}

}  // namespace spmm
