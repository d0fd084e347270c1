// spmm_fwd_noalloc: the forward for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Its scratch (the split-row partial rows and the staged hot rows that
// spmm_fwd takes as a caller workspace) is a file-scope device array of fixed size,
// one copy per GPU, held until the process ends.
//
// Host code never passes the array's name to a kernel or a copy: on the host that
// name is only a stand-in for the symbol.  The device address of each GPU's copy is
// looked up once per device, with that device current, by hipGetSymbolAddress, and
// that address is what the forward receives as its workspace.
#include <mutex>

#include "internal.hpp"
#include "spmm.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up on the first call on each device).
spmm_status scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return spmm::set_error(SPMM_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return spmm::set_error(SPMM_ERR_UNSUPPORTED, "device %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return spmm::set_error(SPMM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                             hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return SPMM_OK;
}

}  // namespace

extern "C" {

size_t spmm_noalloc_scratch_bytes(void) { return kScratchBytes; }

spmm_status spmm_fwd_noalloc(spmm_tile_t A, int k_offset, const void* const* B, const int64_t* ldb,
                             spmm_dtype b_dtype, void* C, int64_t ldc, spmm_dtype c_dtype, int64_t N, int accumulate,
                             void* stream) {
  // The checks spmm_fwd makes before any HIP call, repeated here because the scratch
  // lookup below is one.
  if (!A) return spmm::set_error(SPMM_ERR_INVALID_ARG, "A is null");
  if (!B || !ldb) return spmm::set_error(SPMM_ERR_INVALID_ARG, "B/ldb array is null");
  if (N < 1) return spmm::set_error(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  if ((b_dtype != SPMM_F32 && b_dtype != SPMM_BF16) || (c_dtype != SPMM_F32 && c_dtype != SPMM_BF16))
    return spmm::set_error(SPMM_ERR_INVALID_ARG, "unknown dtype");
  size_t need = 0;
  spmm_status st = spmm_fwd_workspace_bytes(A, N, &need);
  if (st != SPMM_OK) return st;
  if (need > kScratchBytes)
    return spmm::set_error(SPMM_ERR_WORKSPACE,
                           "this forward needs %zu bytes of scratch; spmm_fwd_noalloc holds %zu (use spmm_fwd "
                           "with a workspace)", need, kScratchBytes);
  void* ws = nullptr;
  if (need > 0 && (st = scratch_ptr(&ws)) != SPMM_OK) return st;
  return spmm_fwd(A, k_offset, B, ldb, b_dtype, C, ldc, c_dtype, N, accumulate, ws, need > 0 ? kScratchBytes : 0,
                  stream);
}

}  // extern "C"
