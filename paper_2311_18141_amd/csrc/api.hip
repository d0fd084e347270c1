// C ABI of libspmm (declared in include/spmm.h): argument checks, handle
// creation (validation, split-row plan, transposed structure) and dispatch of
// the forward / backward kernels on the caller's stream.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "internal.hpp"
#include "spmm.h"

using spmm::DT;
using spmm::kMaxK;

namespace {

thread_local std::string g_err;

spmm_status fail(spmm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(SPMM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int32_t kDefaultLongRow = 1024;
constexpr int32_t kDefaultSegment = 512;

// Device allocation owned by a handle.
template <typename T>
hipError_t dalloc(T** p, int64_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)(n > 0 ? n : 1));
}

struct Plan {
  spmm::Seg* seg = nullptr;
  int64_t n_seg = 0;
  spmm::LongRow* lrow = nullptr;
  int64_t n_long = 0;
  unsigned long long stats[35] = {};
};

void free_plan(Plan& p) {
  if (p.seg) (void)hipFree(p.seg);
  if (p.lrow) (void)hipFree(p.lrow);
  p.seg = nullptr;
  p.lrow = nullptr;
}

// Row statistics and split-row plan for K tiles sharing `rows` rows (synchronous).
spmm_status build_plan(const int32_t* const* rowptr, int K, int64_t rows, int32_t long_row, int32_t segment,
                       hipStream_t s, Plan* out) {
  const int64_t scan_tmp = spmm::scan_temp_elems(rows);
  // layout (int32 units): nseg | islong | seg_off | long_off | totals[2] | scan temp | stats (u64, aligned)
  const int64_t n32 = 4 * rows + 2 + scan_tmp;
  const size_t bytes = sizeof(int32_t) * (size_t)n32 + 16 + sizeof(unsigned long long) * 35;
  char* tmp = nullptr;
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(&tmp), bytes));
  int32_t* nseg = reinterpret_cast<int32_t*>(tmp);
  int32_t* islong = nseg + rows;
  int32_t* seg_off = islong + rows;
  int32_t* long_off = seg_off + rows;
  int32_t* totals = long_off + rows;
  int32_t* stmp = totals + 2;
  unsigned long long* stats =
      reinterpret_cast<unsigned long long*>(tmp + ((sizeof(int32_t) * (size_t)n32 + 15) & ~(size_t)15));
  spmm_status st = SPMM_OK;
  auto run = [&]() -> spmm_status {
    HIP_TRY(hipMemsetAsync(totals, 0, 2 * sizeof(int32_t), s));
    HIP_TRY(hipMemsetAsync(stats, 0, 35 * sizeof(unsigned long long), s));
    spmm::PlanCountParams pc{};
    for (int k = 0; k < K; ++k) pc.rowptr[k] = rowptr[k];
    pc.num_k = K;
    pc.rows = rows;
    pc.long_row = long_row;
    pc.segment = segment;
    pc.nseg = nseg;
    pc.islong = islong;
    pc.stats = stats;
    HIP_TRY(spmm::launch_plan_count(pc, s));
    HIP_TRY(spmm::scan_exclusive(nseg, seg_off, rows, totals, stmp, s));
    HIP_TRY(spmm::scan_exclusive(islong, long_off, rows, totals + 1, stmp, s));
    int32_t host_tot[2];
    HIP_TRY(hipMemcpyAsync(host_tot, totals, sizeof host_tot, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(out->stats, stats, sizeof out->stats, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out->n_seg = host_tot[0];
    out->n_long = host_tot[1];
    if (dalloc(&out->seg, out->n_seg) != hipSuccess || dalloc(&out->lrow, out->n_long) != hipSuccess)
      return fail(SPMM_ERR_ALLOC, "device allocation of the split-row plan failed");
    if (out->n_long > 0) {
      spmm::PlanEmitParams pe{};
      for (int k = 0; k < K; ++k) pe.rowptr[k] = rowptr[k];
      pe.num_k = K;
      pe.rows = rows;
      pe.segment = segment;
      pe.nseg = nseg;
      pe.seg_off = seg_off;
      pe.islong = islong;
      pe.long_off = long_off;
      pe.seg = out->seg;
      pe.lrow = out->lrow;
      HIP_TRY(spmm::launch_plan_emit(pe, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return SPMM_OK;
  };
  st = run();
  (void)hipFree(tmp);
  if (st != SPMM_OK) free_plan(*out);
  return st;
}

size_t partial_ld(int64_t N) { return (size_t)((N + 7) / 8 * 8); }

const char* env_str(const char* name) {
  const char* v = getenv(name);
  return (v && *v) ? v : nullptr;
}

// Kernel variant for width N: the widest aligned vector (16 bytes at most) and
// the smallest power-of-two group (4..64 lanes) that covers the row in one window.
spmm::Variant pick_variant(int64_t N, DT dt, uintptr_t align_or) {
  const int esize = dt == DT::F32 ? 4 : 2;
  int V = 16 / esize;
  while (V > 1 && ((N % V) != 0 || (align_or % (uintptr_t)(V * esize)) != 0)) V /= 2;
  const int64_t need = (N + V - 1) / V;
  int G = 4;
  while (G < 64 && G < need) G *= 2;
  spmm::Variant v{G, V};
  if (const char* f = env_str("SPMM_FWD_VARIANT")) {  // "G,V" for measurement sweeps
    int g = 0, vv = 0;
    if (sscanf(f, "%d,%d", &g, &vv) == 2 && (g == 4 || g == 8 || g == 16 || g == 32 || g == 64) &&
        (vv == 1 || vv == 2 || vv == 4 || (vv == 8 && dt == DT::BF16)) && (N % vv) == 0 &&
        (align_or % (uintptr_t)(vv * esize)) == 0)
      v = spmm::Variant{g, vv};
  }
  return v;
}

}  // namespace

struct spmm_tile_s {
  int64_t rows = 0;
  int num_k = 0;
  spmm_csr t[kMaxK] = {};
  int32_t long_row = kDefaultLongRow;
  int32_t segment = kDefaultSegment;
  Plan plan;
  spmm_tile_stats stats = {};
  bool has_t = false;
  int32_t* rowid = nullptr;
  int32_t* rowptrT = nullptr;
  int32_t* colindT = nullptr;
  int32_t* perm = nullptr;
  Plan planT;
  int device = 0;

  ~spmm_tile_s() {
    free_plan(plan);
    free_plan(planT);
    if (rowid) (void)hipFree(rowid);
    if (rowptrT) (void)hipFree(rowptrT);
    if (colindT) (void)hipFree(colindT);
    if (perm) (void)hipFree(perm);
  }
};

extern "C" {

const char* spmm_status_string(spmm_status status) {
  switch (status) {
    case SPMM_OK: return "SPMM_OK";
    case SPMM_ERR_INVALID_ARG: return "SPMM_ERR_INVALID_ARG";
    case SPMM_ERR_BAD_CSR: return "SPMM_ERR_BAD_CSR";
    case SPMM_ERR_UNSUPPORTED: return "SPMM_ERR_UNSUPPORTED";
    case SPMM_ERR_WORKSPACE: return "SPMM_ERR_WORKSPACE";
    case SPMM_ERR_HIP: return "SPMM_ERR_HIP";
    case SPMM_ERR_ALLOC: return "SPMM_ERR_ALLOC";
  }
  return "unknown spmm_status";
}

const char* spmm_last_error(void) { return g_err.c_str(); }

spmm_status spmm_tile_create(int64_t rows, int num_k, const spmm_csr* tiles, const spmm_tile_opts* opts,
                             void* stream, spmm_tile_t* out) {
  if (!out) return fail(SPMM_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (rows < 0 || rows >= ((int64_t)1 << 31)) return fail(SPMM_ERR_INVALID_ARG, "rows=%lld out of range", (long long)rows);
  if (num_k < 1 || num_k > kMaxK) return fail(SPMM_ERR_INVALID_ARG, "num_k=%d outside [1, %d]", num_k, kMaxK);
  if (!tiles) return fail(SPMM_ERR_INVALID_ARG, "tiles is null");
  const unsigned flags = opts ? opts->flags : 0u;
  if (flags & ~(SPMM_TILE_VALIDATE | SPMM_TILE_TRANSPOSE)) return fail(SPMM_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
  int32_t long_row = (opts && opts->long_row > 0) ? opts->long_row : kDefaultLongRow;
  int32_t segment = (opts && opts->segment > 0) ? opts->segment : kDefaultSegment;
  if (opts && (opts->long_row < 0 || opts->segment < 0)) return fail(SPMM_ERR_INVALID_ARG, "negative long_row/segment");
  int64_t units_bound = 0;
  for (int k = 0; k < num_k; ++k) {
    const spmm_csr& t = tiles[k];
    if (t.cols < 0 || t.cols >= ((int64_t)1 << 31)) return fail(SPMM_ERR_INVALID_ARG, "tile %d: cols out of range", k);
    if (t.nnz < 0) return fail(SPMM_ERR_INVALID_ARG, "tile %d: negative nnz", k);
    if (t.nnz >= ((int64_t)1 << 31)) return fail(SPMM_ERR_UNSUPPORTED, "tile %d: nnz >= 2^31 needs 64-bit indices", k);
    if (!t.rowptr) return fail(SPMM_ERR_INVALID_ARG, "tile %d: rowptr is null", k);
    if (t.nnz > 0 && (!t.colind || !t.values)) return fail(SPMM_ERR_INVALID_ARG, "tile %d: colind/values null", k);
    units_bound += t.nnz / segment + rows;
  }
  if (units_bound >= ((int64_t)1 << 31)) return fail(SPMM_ERR_UNSUPPORTED, "split-row plan would exceed 2^31 units");
  if ((flags & SPMM_TILE_TRANSPOSE) && num_k != 1)
    return fail(SPMM_ERR_UNSUPPORTED, "SPMM_TILE_TRANSPOSE needs a single tile (num_k = 1)");

  hipStream_t s = static_cast<hipStream_t>(stream);
  spmm_tile_s* h = new (std::nothrow) spmm_tile_s();
  if (!h) return fail(SPMM_ERR_ALLOC, "host allocation failed");
  h->rows = rows;
  h->num_k = num_k;
  h->long_row = long_row;
  h->segment = segment;
  for (int k = 0; k < num_k; ++k) h->t[k] = tiles[k];
  (void)hipGetDevice(&h->device);

  auto body = [&]() -> spmm_status {
    if (flags & SPMM_TILE_VALIDATE) {
      uint32_t* status = nullptr;
      HIP_TRY(hipMalloc(reinterpret_cast<void**>(&status), sizeof(uint32_t)));
      spmm_status vst = SPMM_OK;
      for (int k = 0; k < num_k && vst == SPMM_OK; ++k) {
        uint32_t bits = 0;
        auto check = [&](bool cols_pass) -> spmm_status {
          HIP_TRY(hipMemsetAsync(status, 0, sizeof(uint32_t), s));
          if (!cols_pass)
            HIP_TRY(spmm::launch_validate_rowptr(tiles[k].rowptr, rows, tiles[k].nnz, status, s));
          else
            HIP_TRY(spmm::launch_validate_colind(tiles[k].rowptr, tiles[k].colind, rows, tiles[k].cols, status, s));
          HIP_TRY(hipMemcpyAsync(&bits, status, sizeof bits, hipMemcpyDeviceToHost, s));
          HIP_TRY(hipStreamSynchronize(s));
          return SPMM_OK;
        };
        if ((vst = check(false)) != SPMM_OK) break;
        if (bits) {
          vst = fail(SPMM_ERR_BAD_CSR, "tile %d: row pointer invalid (bits 0x%x: 1 first!=0, 2 decreasing, "
                     "4 last!=nnz, 8 out of [0,nnz])", k, bits);
          break;
        }
        if ((vst = check(true)) != SPMM_OK) break;
        if (bits)
          vst = fail(SPMM_ERR_BAD_CSR, "tile %d: column indices invalid (bits 0x%x: 16 out of range, "
                     "32 not strictly increasing in a row)", k, bits);
      }
      (void)hipFree(status);
      if (vst != SPMM_OK) return vst;
    }
    const int32_t* rps[kMaxK];
    for (int k = 0; k < num_k; ++k) rps[k] = tiles[k].rowptr;
    spmm_status st = build_plan(rps, num_k, rows, long_row, segment, s, &h->plan);
    if (st != SPMM_OK) return st;
    if (flags & SPMM_TILE_TRANSPOSE) {
      const spmm_csr& t = tiles[0];
      if (dalloc(&h->rowid, t.nnz) != hipSuccess || dalloc(&h->rowptrT, t.cols + 1) != hipSuccess ||
          dalloc(&h->colindT, t.nnz) != hipSuccess || dalloc(&h->perm, t.nnz) != hipSuccess)
        return fail(SPMM_ERR_ALLOC, "device allocation of the transposed structure failed");
      void* temp = nullptr;
      HIP_TRY(hipMalloc(&temp, (size_t)spmm::transpose_temp_bytes(rows, t.cols, t.nnz)));
      hipError_t e = spmm::build_transpose(t.rowptr, t.colind, rows, t.cols, t.nnz, h->rowid, h->rowptrT,
                                           h->colindT, h->perm, temp, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      (void)hipFree(temp);
      if (e != hipSuccess) return fail(SPMM_ERR_HIP, "transpose: %s", hipGetErrorString(e));
      const int32_t* rpT[1] = {h->rowptrT};
      st = build_plan(rpT, 1, t.cols, long_row, segment, s, &h->planT);
      if (st != SPMM_OK) return st;
      h->has_t = true;
    }
    return SPMM_OK;
  };
  spmm_status st = body();
  if (st != SPMM_OK) {
    delete h;
    return st;
  }
  spmm_tile_stats& S = h->stats;
  S.rows = rows;
  S.num_k = num_k;
  for (int k = 0; k < num_k; ++k) {
    S.nnz_total += tiles[k].nnz;
    S.nnz_per_k[k] = tiles[k].nnz;
  }
  S.max_row = (int64_t)h->plan.stats[0];
  S.empty_rows = (int64_t)h->plan.stats[1];
  for (int b = 0; b < 33; ++b) S.hist_log2[b] = (int64_t)h->plan.stats[2 + b];
  S.long_rows = h->plan.n_long;
  S.segments = h->plan.n_seg;
  S.has_transpose = h->has_t ? 1 : 0;
  S.long_rows_t = h->planT.n_long;
  S.segments_t = h->planT.n_seg;
  *out = h;
  return SPMM_OK;
}

spmm_status spmm_tile_destroy(spmm_tile_t tile) {
  if (!tile) return fail(SPMM_ERR_INVALID_ARG, "tile is null");
  delete tile;
  return SPMM_OK;
}

spmm_status spmm_tile_get_stats(spmm_tile_t tile, spmm_tile_stats* out) {
  if (!tile || !out) return fail(SPMM_ERR_INVALID_ARG, "null argument");
  *out = tile->stats;
  return SPMM_OK;
}

spmm_status spmm_tile_export_transpose(spmm_tile_t tile, int32_t* rowptrT, int32_t* colindT, int32_t* perm,
                                       void* stream) {
  if (!tile || !rowptrT) return fail(SPMM_ERR_INVALID_ARG, "null argument");
  if (!tile->has_t) return fail(SPMM_ERR_UNSUPPORTED, "handle was created without SPMM_TILE_TRANSPOSE");
  const int64_t nnz = tile->t[0].nnz;
  if (nnz > 0 && (!colindT || !perm)) return fail(SPMM_ERR_INVALID_ARG, "null colindT/perm");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(rowptrT, tile->rowptrT, sizeof(int32_t) * (size_t)(tile->t[0].cols + 1),
                         hipMemcpyDeviceToDevice, s));
  if (nnz > 0) {
    HIP_TRY(hipMemcpyAsync(colindT, tile->colindT, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(perm, tile->perm, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
  }
  return SPMM_OK;
}

spmm_status spmm_fwd_workspace_bytes(spmm_tile_t A, int64_t N, size_t* bytes) {
  if (!A || !bytes) return fail(SPMM_ERR_INVALID_ARG, "null argument");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  *bytes = sizeof(float) * partial_ld(N) * (size_t)A->plan.n_seg;
  return SPMM_OK;
}

spmm_status spmm_bwd_workspace_bytes(spmm_tile_t A, int64_t N, size_t* bytes) {
  if (!A || !bytes) return fail(SPMM_ERR_INVALID_ARG, "null argument");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  *bytes = sizeof(float) * partial_ld(N) * (size_t)A->planT.n_seg;
  return SPMM_OK;
}

spmm_status spmm_fwd(spmm_tile_t A, int k_offset, const void* const* B, const int64_t* ldb, spmm_dtype b_dtype,
                     void* C, int64_t ldc, spmm_dtype c_dtype, int64_t N, int accumulate, void* workspace,
                     size_t ws_bytes, void* stream) {
  if (!A) return fail(SPMM_ERR_INVALID_ARG, "A is null");
  if (!B || !ldb) return fail(SPMM_ERR_INVALID_ARG, "B/ldb array is null");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  if ((b_dtype != SPMM_F32 && b_dtype != SPMM_BF16) || (c_dtype != SPMM_F32 && c_dtype != SPMM_BF16))
    return fail(SPMM_ERR_INVALID_ARG, "unknown dtype");
  if (b_dtype != c_dtype) return fail(SPMM_ERR_UNSUPPORTED, "B and C must have the same dtype");
  if (ldc < N) return fail(SPMM_ERR_INVALID_ARG, "ldc=%lld < N=%lld", (long long)ldc, (long long)N);
  if (!C && A->rows > 0) return fail(SPMM_ERR_INVALID_ARG, "C is null");
  const DT dt = b_dtype == SPMM_F32 ? DT::F32 : DT::BF16;
  const int esize = dt == DT::F32 ? 4 : 2;
  const int K = A->num_k;
  uintptr_t align_or = reinterpret_cast<uintptr_t>(C) | (uintptr_t)(ldc * esize);
  for (int k = 0; k < K; ++k) {
    if (!B[k] && A->t[k].cols > 0) return fail(SPMM_ERR_INVALID_ARG, "B[%d] is null", k);
    if (ldb[k] < N) return fail(SPMM_ERR_INVALID_ARG, "ldb[%d]=%lld < N", k, (long long)ldb[k]);
    if (ldb[k] * esize >= ((int64_t)1 << 32)) return fail(SPMM_ERR_UNSUPPORTED, "ldb[%d] * element size >= 2^32", k);
    align_or |= reinterpret_cast<uintptr_t>(B[k]) | (uintptr_t)(ldb[k] * esize);
  }
  const size_t need = sizeof(float) * partial_ld(N) * (size_t)A->plan.n_seg;
  if (need > 0) {
    if (!workspace || ws_bytes < need)
      return fail(SPMM_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    if (reinterpret_cast<uintptr_t>(workspace) % 16) return fail(SPMM_ERR_WORKSPACE, "workspace must be 16-byte aligned");
  }
  if ((N + 63) / 64 > 65535) return fail(SPMM_ERR_UNSUPPORTED, "N too large for one launch");
  if (A->rows == 0) return SPMM_OK;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != A->device) return fail(SPMM_ERR_INVALID_ARG, "current device %d differs from the handle's %d", dev, A->device);

  spmm::FwdParams P{};
  for (int k = 0; k < K; ++k) {
    P.t[k].rowptr = A->t[k].rowptr;
    P.t[k].colind = A->t[k].colind;
    P.t[k].values = A->t[k].values;
    P.t[k].perm = nullptr;
    P.t[k].B = B[k];
    P.t[k].ldb = ldb[k];
  }
  P.num_k = K;
  P.k_offset = (int)(((k_offset % K) + K) % K);
  P.rows = A->rows;
  P.N = N;
  P.C = C;
  P.ldc = ldc;
  P.accumulate = accumulate ? 1 : 0;
  P.long_row = A->long_row;
  P.seg = A->plan.seg;
  P.n_seg = A->plan.n_seg;
  P.lrow = A->plan.lrow;
  P.n_long = A->plan.n_long;
  P.partial = static_cast<float*>(workspace);
  P.ldp = (int64_t)partial_ld(N);
  const spmm::Variant v = pick_variant(N, dt, align_or);
  HIP_TRY(spmm::launch_fwd(P, v, dt, static_cast<hipStream_t>(stream)));
  return SPMM_OK;
}

spmm_status spmm_bwd(spmm_tile_t A, const float* dC, int64_t lddc, const float* B, int64_t ldb, int64_t N,
                     float* dA_values, float* dB, int64_t lddb, void* workspace, size_t ws_bytes, void* stream) {
  if (!A) return fail(SPMM_ERR_INVALID_ARG, "A is null");
  if (A->num_k != 1) return fail(SPMM_ERR_UNSUPPORTED, "spmm_bwd needs a single-tile handle");
  if (!A->has_t) return fail(SPMM_ERR_UNSUPPORTED, "handle was created without SPMM_TILE_TRANSPOSE");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  if (!dC && A->rows > 0) return fail(SPMM_ERR_INVALID_ARG, "dC is null");
  if (lddc < N) return fail(SPMM_ERR_INVALID_ARG, "lddc < N");
  if (dA_values && !B && A->t[0].cols > 0) return fail(SPMM_ERR_INVALID_ARG, "B is null");
  if (dA_values && ldb < N) return fail(SPMM_ERR_INVALID_ARG, "ldb < N");
  if (dB && lddb < N) return fail(SPMM_ERR_INVALID_ARG, "lddb < N");
  if (lddc * 4 >= ((int64_t)1 << 32)) return fail(SPMM_ERR_UNSUPPORTED, "lddc * 4 >= 2^32");
  const spmm_csr& t = A->t[0];
  const size_t need = dB ? sizeof(float) * partial_ld(N) * (size_t)A->planT.n_seg : 0;
  if (need > 0) {
    if (!workspace || ws_bytes < need)
      return fail(SPMM_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    if (reinterpret_cast<uintptr_t>(workspace) % 16) return fail(SPMM_ERR_WORKSPACE, "workspace must be 16-byte aligned");
  }
  if ((N + 63) / 64 > 65535) return fail(SPMM_ERR_UNSUPPORTED, "N too large for one launch");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != A->device) return fail(SPMM_ERR_INVALID_ARG, "current device %d differs from the handle's %d", dev, A->device);
  hipStream_t s = static_cast<hipStream_t>(stream);

  if (dA_values && t.nnz > 0) {
    spmm::SddmmParams P{};
    P.rowid = A->rowid;
    P.colind = t.colind;
    P.nnz = t.nnz;
    P.dC = dC;
    P.lddc = lddc;
    P.B = B;
    P.ldb = ldb;
    P.N = N;
    P.dA = dA_values;
    const uintptr_t a = reinterpret_cast<uintptr_t>(dC) | reinterpret_cast<uintptr_t>(B) | (uintptr_t)(lddc * 4) |
                        (uintptr_t)(ldb * 4);
    int V = 4;
    while (V > 1 && ((N % V) != 0 || (a % (uintptr_t)(V * 4)) != 0)) V /= 2;
    const int64_t need_lanes = (N + V - 1) / V;
    int G = 4;
    while (G < 16 && G * 2 <= need_lanes) G *= 2;
    HIP_TRY(spmm::launch_sddmm(P, spmm::Variant{G, V}, s));
  }
  if (dB && t.cols > 0) {
    spmm::FwdParams P{};
    P.t[0].rowptr = A->rowptrT;
    P.t[0].colind = A->colindT;
    P.t[0].values = t.values;
    P.t[0].perm = A->perm;
    P.t[0].B = dC;
    P.t[0].ldb = lddc;
    P.num_k = 1;
    P.k_offset = 0;
    P.rows = t.cols;
    P.N = N;
    P.C = dB;
    P.ldc = lddb;
    P.accumulate = 0;
    P.long_row = A->long_row;
    P.seg = A->planT.seg;
    P.n_seg = A->planT.n_seg;
    P.lrow = A->planT.lrow;
    P.n_long = A->planT.n_long;
    P.partial = static_cast<float*>(workspace);
    P.ldp = (int64_t)partial_ld(N);
    const uintptr_t a = reinterpret_cast<uintptr_t>(dC) | reinterpret_cast<uintptr_t>(dB) | (uintptr_t)(lddc * 4) |
                        (uintptr_t)(lddb * 4);
    HIP_TRY(spmm::launch_fwd(P, pick_variant(N, DT::F32, a), DT::F32, s));
  }
  return SPMM_OK;
}

}  // extern "C"
