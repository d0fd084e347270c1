// C ABI of libspmm (declared in include/spmm.h): argument checks, handle
// creation (validation, split-row plan, transposed structure) and dispatch of
// the forward / backward kernels on the caller's stream.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <algorithm>
#include <array>
#include <vector>

#include <dlfcn.h>

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

constexpr int32_t kDefaultLongRow = 128;
constexpr int32_t kDefaultSegment = 64;
// Largest split threshold: 64 rows of at most this length sum below 2^31.
constexpr int32_t kMaxLongRow = ((int64_t)1 << 31) / 64 - 1;
// Hot-row staging, library default: up to one B row per kHotColsPerRow columns of the
// k-tile, at least kDefaultHotRows and at most kHotRowsCap, each used by at least
// kHotMinUses non-zeros, for tiles of at least kHotMinNnz non-zeros in total, and only
// where the staged rows serve at least 1/8 of the k-tile's non-zeros and at least
// kHotConcentration times their share of its columns (a skewed column distribution).
// Measured: on the R-MAT scale-22 row block (k-tiles of 2^20 columns) 4K to 64K rows per
// k-tile ran within 3% of each other; on R-MAT scale 23 (one tile of 2^23 columns) 64K
// rows ran 2.7% (BF16) and 2.8% (FP32) faster than 16K, 128K no faster in FP32.
constexpr int32_t kDefaultHotRows = 16384;
constexpr int32_t kHotRowsCap = 65536;
constexpr int64_t kHotColsPerRow = 128;
constexpr int32_t kMaxHotRows = 1 << 24;
constexpr int32_t kHotMinUses = 16;
constexpr int64_t kHotMinNnz = (int64_t)1 << 20;
constexpr int64_t kHotConcentration = 8;
// The rule looks only at k-tiles of at most this many columns (the selection keeps two
// host arrays of one int32 per column).
constexpr int64_t kHotMaxCols = (int64_t)1 << 27;

// Device allocation owned by a handle.
template <typename T>
hipError_t dalloc(T** p, int64_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)(n > 0 ? n : 1));
}

struct Plan {
  int32_t long_row = 0;
  int32_t segment = 0;
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
  out->long_row = long_row;
  out->segment = segment;
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

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Rows per wave of the stream kernel: enough waves to fill the GPU for short tiles,
// 64 (one per lane) for large ones.
int stream_rows_for(int64_t rows) {
  int R = 64;
  while (R > 4 && (rows / R) < 4096) R /= 2;
  return R;
}

// Kernel variant for width N when the handle has no entry, by the width, the dtype and
// the share of empty rows (`empty` of `rows`; < 0: unknown, taken as many; "many" is
// more than 1/8, R-MAT's, whose short and empty rows a wave of the stream kernel
// streams past).  FP32: windows of 64 columns (256 bytes of each B row), of 128 for
// N >= 256 and, on tiles with many empty rows, for N a multiple of 128; the stream
// kernel on tiles with many empty rows, else a full-wave row-split group.  BF16: a
// full-wave row-split group over the fewest windows of at most 256 columns, each on the
// narrowest vector giving that count (the stream kernel at N = 64 on tiles with many
// empty rows).  Below 64 a row-split group with the widest aligned vector and the
// smallest power-of-two group covering N.
spmm::Variant pick_variant(int64_t N, DT dt, uintptr_t align_or, int64_t rows, int64_t empty) {
  const int esize = dt == DT::F32 ? 4 : 2;
  int V = 16 / esize;
  while (V > 1 && ((N % V) != 0 || (align_or % (uintptr_t)(V * esize)) != 0)) V /= 2;
  const bool sparse = empty < 0 || empty * 8 > rows;
  if (N >= 64 && dt == DT::BF16) {
    // BF16: full-wave row-split groups over the fewest windows of at most 256 columns
    // (512 bytes of each B row), each on the narrowest vector that gives that count.
    // The autotuner's picks on the heavy-tailed matrix (N = 128..1024) and on three
    // R-MAT matrices (N = 128, 192, 256): at N = 128 one 128-column window beat the
    // stream kernel by 13-29%, at N = 192 one 4-wide window beat two 2-wide ones by
    // 35-38%.  At N = 64 (or one-element vectors) tiles with many empty rows keep the
    // stream kernel, which streams past them.
    const int64_t windows = (N + 255) / 256;
    int Vb = 1;
    while (Vb * 2 <= V && (N + 64 * Vb - 1) / (64 * Vb) > windows) Vb *= 2;
    if (Vb == 1 && sparse) return spmm::Variant{64, 1, true, stream_rows_for(rows)};
    return spmm::Variant{64, Vb, false};
  }
  if (N >= 256 && V >= 2) {
    // FP32 at N >= 256: windows of 128 columns (512 bytes), the autotuner's picks at
    // N = 256..1024 on the heavy-tailed matrix and at N = 256 on R-MAT: about 5% faster
    // than 256-byte windows (on the 512 uneven tiles the row-split group's per-tile loop
    // took 37.4 ms against 41.3 ms with the stream kernel)
    return sparse ? spmm::Variant{64, 2, true, stream_rows_for(rows)} : spmm::Variant{64, 2, false};
  }
  if (N >= 64) {
    // FP32 windows of 64 columns (256 bytes): the grid walks the windows one after the
    // other, so a narrower window keeps a smaller slice of B in the caches (faster than
    // one window over all of N on the heavy-tailed matrix).  On tiles with many empty
    // rows, the stream kernel, over 128-column windows when they tile N exactly: on three
    // R-MAT matrices at N = 128 they beat 64-column windows by 9-14% (at N = 192 a ragged
    // second window lost 3-5%).  Without many empty rows the row-split group: on the 512
    // uneven tiles (uniform columns, 4 to 256 per row) the per-tile loop took 34.7 ms
    // with it against 60.0 ms with the stream kernel (32.2 autotuned)
    if (!sparse) return spmm::Variant{64, 1, false};
    const int Vs = (V >= 2 && N % 128 == 0) ? 2 : 1;
    return spmm::Variant{64, Vs, true, stream_rows_for(rows)};
  }
  const int64_t need = (N + V - 1) / V;
  int G = 4;
  while (G < 64 && G < need) G *= 2;
  return spmm::Variant{G, V, false};
}

bool pow2_lanes(int g) { return g == 4 || g == 8 || g == 16 || g == 32 || g == 64; }

// The forward launches one grid row per column window of G * V columns; a launch's grid
// has at most 65535 rows.  (The library's own choices use windows of at least 64
// columns, and N is checked against 64 * 65535.)
bool fits_grid(int64_t N, const spmm::Variant& v) { return (N + (int64_t)v.G * v.V - 1) / ((int64_t)v.G * v.V) <= 65535; }

}  // namespace

namespace spmm {

namespace {
struct Roctx {
  int (*push)(const char*) = nullptr;
  int (*pop)() = nullptr;
};

// Opened once, on the first range, and only when SPMM_TRACE asks for it.
const Roctx& roctx() {
  static const Roctx r = [] {
    Roctx x;
    const char* e = std::getenv("SPMM_TRACE");
    if (!e || !*e || std::strcmp(e, "0") == 0) return x;
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_LOCAL);
    if (!h) return x;
    auto push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
    auto pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (push && pop) {
      x.push = push;
      x.pop = pop;
    }
    return x;
  }();
  return r;
}
}  // namespace

TraceRange::TraceRange(const char* name) : on(roctx().push != nullptr) {
  if (on) roctx().push(name);
}

TraceRange::~TraceRange() {
  if (on) roctx().pop();
}

spmm_status set_error(spmm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

spmm_status validate_csr(const int32_t* rowptr, const int32_t* colind, int64_t rows, int64_t cols, int64_t nnz,
                         hipStream_t s) {
  uint32_t* status = nullptr;
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(&status), sizeof(uint32_t)));
  uint32_t bits = 0;
  auto run = [&](bool cols_pass) -> spmm_status {
    HIP_TRY(hipMemsetAsync(status, 0, sizeof(uint32_t), s));
    if (!cols_pass)
      HIP_TRY(launch_validate_rowptr(rowptr, rows, nnz, status, s));
    else
      HIP_TRY(launch_validate_colind(rowptr, colind, rows, cols, status, s));
    HIP_TRY(hipMemcpyAsync(&bits, status, sizeof bits, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SPMM_OK;
  };
  spmm_status st = run(false);
  if (st == SPMM_OK && bits)
    st = fail(SPMM_ERR_BAD_CSR, "row pointer invalid (bits 0x%x: 1 first!=0, 2 decreasing, 4 last!=nnz, "
              "8 out of [0,nnz])", bits);
  if (st == SPMM_OK) {
    st = run(true);
    if (st == SPMM_OK && bits)
      st = fail(SPMM_ERR_BAD_CSR, "column indices invalid (bits 0x%x: 16 out of range, 32 not strictly "
                "increasing in a row)", bits);
  }
  (void)hipFree(status);
  return st;
}

}  // namespace spmm

struct spmm_tile_s {
  int64_t rows = 0;
  int num_k = 0;
  spmm_csr t[kMaxK] = {};
  Plan plan;
  spmm_tile_stats stats = {};
  bool has_t = false;
  int32_t* rowid = nullptr;
  int32_t* rowptrT = nullptr;
  int32_t* colindT = nullptr;
  int32_t* perm = nullptr;
  Plan planT;
  int device = 0;
  struct VarEntry {
    int64_t N;
    int dtype;
    spmm_variant v;
  };
  VarEntry vt[16];          // forward variants
  int nvt = 0;
  VarEntry vtT[16];         // variants of the backward's dB pass (forward kernels on the transpose)
  int nvtT = 0;
  int64_t bwd_slice = 0;   // SDDMM column slice (0 = all columns in one launch)
  struct SddmmEntry {
    int64_t N;
    int G, U;
  };
  SddmmEntry sd[8];
  int nsd = 0;
  // Hot-row staging: per k-tile a tagged copy of colind (null: the k-tile stages no
  // rows and the caller's colind is read), the B row of every slot, slots of k-tile k
  // at [hot_off[k], hot_off[k + 1]).
  int32_t* hcol[kMaxK] = {};
  int32_t* hot_src = nullptr;
  int64_t hot_off[kMaxK + 1] = {};

  int64_t hot_total() const { return hot_off[num_k]; }

  ~spmm_tile_s() {
    free_plan(plan);
    free_plan(planT);
    if (rowid) (void)hipFree(rowid);
    if (rowptrT) (void)hipFree(rowptrT);
    if (colindT) (void)hipFree(colindT);
    if (perm) (void)hipFree(perm);
    for (int k = 0; k < kMaxK; ++k)
      if (hcol[k]) (void)hipFree(hcol[k]);
    if (hot_src) (void)hipFree(hot_src);
  }
};

namespace {

using VarEntry = spmm_tile_s::VarEntry;

// The variant for one call: the table's entry for (N, dtype) when it fits the call's
// alignment, otherwise the fixed rule (for a pass over `rows` rows).
spmm::Variant resolve_variant_in(const VarEntry* vt, int nvt, int64_t rows, int64_t empty, int64_t N, DT dt,
                                 uintptr_t align_or) {
  const spmm::Variant base = pick_variant(N, dt, align_or, rows, empty);
  const int esize = dt == DT::F32 ? 4 : 2;
  const int want = dt == DT::F32 ? SPMM_F32 : SPMM_BF16;
  for (int i = 0; i < nvt; ++i) {
    const auto& e = vt[i];
    if (e.N != N || e.dtype != want || e.v.kind == SPMM_KERNEL_AUTO || e.v.kind == SPMM_KERNEL_FUSED) continue;
    const int V = e.v.vec ? e.v.vec : base.V;
    if ((N % V) != 0 || (align_or % (uintptr_t)(V * esize)) != 0) return base;
    if (e.v.kind == SPMM_KERNEL_STREAM) return spmm::Variant{64, V, true, e.v.lanes ? e.v.lanes : stream_rows_for(rows)};
    int G = e.v.lanes;
    if (G == 0) {
      G = 4;
      while (G < 64 && G < (N + V - 1) / V) G *= 2;
    }
    if (!fits_grid(N, spmm::Variant{G, V, false})) return base;
    return spmm::Variant{G, V, false};
  }
  return base;
}

spmm::Variant resolve_variant(const spmm_tile_s* A, int64_t N, DT dt, uintptr_t align_or) {
  return resolve_variant_in(A->vt, A->nvt, A->rows, (int64_t)A->plan.stats[1], N, dt, align_or);
}

// Shape of the fused backward (one pass over the transposed structure for dA and dB)
// at width N, or false when the two-pass backward applies: an entry of the backward's
// table for (N, dtype) that names a dB-pass kernel, or a vector width so narrow (the
// operands' alignment) that 64-lane windows would be more than fused_windows_max(N).
// A fused entry's lanes / vec (0 = library choice) must fit the call's alignment and
// need at most that many windows, else the library's shape is used: the widest aligned
// vector (16 bytes a lane) and the smallest power-of-two group covering N, 64 lanes and
// ceil(N / (64 V)) column windows when none does.  U = the entry's
// depth, else 4 (FP32) or 2 (BF16) entries in flight per group (at most the group's
// lanes): on the heavy-tailed 2M x 2M matrix at N = 128, U = 4 ran the FP32 backward in
// 5.68 ms against 5.97 ms with U = 8 (7.8 with 16, 7.8 with 1); BF16 3.79 ms with U = 2
// against 3.89 with U = 4 and 4.25 with U = 8 (the autotuner also picks U = 2 at N = 512).
struct FusedShape {
  int G, V, U, n_win;
};
// The most column windows the fused backward may use at width N (its workspace holds
// that many arrays of partial dot products): windows of at least 256 columns, at most
// kMaxFusedWindows of them (wider N takes the two-pass form, whose workspace does not
// grow with N).
constexpr int64_t kMaxFusedWindows = 8;
int64_t fused_windows_max(int64_t N) { return std::min<int64_t>(kMaxFusedWindows, std::max<int64_t>(1, (N + 255) / 256)); }
bool fused_shape(const spmm_tile_s* A, int64_t N, DT dt, uintptr_t align_or, FusedShape* out) {
  const int esize = dt == DT::F32 ? 4 : 2;
  const int want = dt == DT::F32 ? SPMM_F32 : SPMM_BF16;
  const spmm_variant* ent = nullptr;
  for (int i = 0; i < A->nvtT; ++i)
    if (A->vtT[i].N == N && A->vtT[i].dtype == want && A->vtT[i].v.kind != SPMM_KERNEL_AUTO) ent = &A->vtT[i].v;
  if (ent && ent->kind != SPMM_KERNEL_FUSED) return false;
  auto covering = [&](int V) {
    int G = 4;
    while (G < 64 && (int64_t)G * V < N) G *= 2;
    return G;
  };
  auto aligned = [&](int V) { return (N % V) == 0 && (align_or % (uintptr_t)(V * esize)) == 0; };
  int V = 16 / esize;
  while (V > 1 && !aligned(V)) V /= 2;
  int G = covering(V);
  int U = dt == DT::F32 ? 4 : 2;
  auto windows = [&](int g, int v) { return (N + (int64_t)g * v - 1) / ((int64_t)g * v); };
  if (ent) {
    const int Ve = ent->vec ? ent->vec : V;
    const int Ge = ent->lanes ? ent->lanes : covering(Ve);
    if (aligned(Ve) && windows(Ge, Ve) <= fused_windows_max(N)) {
      V = Ve;
      G = Ge;
    }
    if (ent->depth) U = ent->depth;
  }
  const int64_t nw = windows(G, V);
  if (nw > fused_windows_max(N)) return false;
  *out = FusedShape{G, V, std::min(U, G), (int)nw};
  return true;
}

// Set (v != null) or clear (v == null) a table's entry for (N, dtype).
spmm_status set_variant_in(VarEntry* vt, int* nvt, int64_t N, spmm_dtype dtype, const spmm_variant* v) {
  int slot = -1;
  for (int i = 0; i < *nvt; ++i)
    if (vt[i].N == N && vt[i].dtype == dtype) slot = i;
  if (!v) {
    if (slot >= 0) {
      vt[slot] = vt[*nvt - 1];
      --*nvt;
    }
    return SPMM_OK;
  }
  if (slot < 0) {
    if (*nvt >= 16) return fail(SPMM_ERR_INVALID_ARG, "variant table is full");
    slot = (*nvt)++;
  }
  vt[slot].N = N;
  vt[slot].dtype = dtype;
  vt[slot].v = *v;
  return SPMM_OK;
}

// Autotuner candidates for width N: the two widest aligned vector widths, for each the
// covering group size, half of it and a full wave, a full-wave group at a quarter of
// the widest width, and the stream kernel (64, 16 and 4 rows per wave).
std::vector<spmm::Variant> candidate_variants(int64_t N, DT dt, uintptr_t align_or, int64_t rows, int64_t empty) {
  const int esize = dt == DT::F32 ? 4 : 2;
  std::vector<spmm::Variant> kv;
  auto add = [&](spmm::Variant v) {
    if (!fits_grid(N, v)) return;
    for (auto& u : kv)
      if (u.G == v.G && u.V == v.V && u.stream == v.stream && (!v.stream || u.rows == v.rows)) return;
    kv.push_back(v);
  };
  add(pick_variant(N, dt, align_or, rows, empty));
  int vmax = 16 / esize;
  while (vmax > 1 && ((N % vmax) != 0 || (align_or % (uintptr_t)(vmax * esize)) != 0)) vmax /= 2;
  for (int V = vmax; V >= 1 && V >= vmax / 4; V /= 2) {
    if ((N % V) != 0) continue;
    for (int R : {64, 16, 4}) add(spmm::Variant{64, V, true, R});
    add(spmm::Variant{64, V, false});
    if (V < vmax / 2) continue;
    int G = 4;
    while (G < 64 && G < (N + V - 1) / V) G *= 2;
    if (G >= 8) add(spmm::Variant{G / 2, V, false});
    add(spmm::Variant{G, V, false});
  }
  return kv;
}

// Forward workspace: FP32 partial rows of the plan's split-row units, then (at a
// 256-byte boundary) the staged hot rows, ceil8(N) elements apart (sized for FP32).
size_t fwd_partial_bytes(const Plan& plan, int64_t N) { return sizeof(float) * partial_ld(N) * (size_t)plan.n_seg; }
size_t fwd_workspace(const spmm_tile_s* A, const Plan& plan, int64_t N) {
  const size_t part = fwd_partial_bytes(plan, N);
  if (A->hot_total() == 0) return part;
  return align256(part) + sizeof(float) * partial_ld(N) * (size_t)A->hot_total();
}

// Fill the forward parameters for a handle and launch (arguments already checked):
// first the copy of the staged hot rows (when the handle has any), then the forward.
hipError_t launch_forward(const spmm_tile_s* A, const Plan& plan, int k_offset, const void* const* B,
                          const int64_t* ldb, DT dt, void* C, int64_t ldc, int64_t N, int accumulate,
                          void* workspace, const spmm::Variant& v, hipStream_t s) {
  const int K = A->num_k;
  const int64_t esize = dt == DT::F32 ? 4 : 2;
  const int64_t ldh = (int64_t)partial_ld(N);
  char* hot = A->hot_total() > 0 ? static_cast<char*>(workspace) + align256(fwd_partial_bytes(plan, N)) : nullptr;
  spmm::FwdParams P{};
  for (int k = 0; k < K; ++k) {
    P.t[k].rowptr = A->t[k].rowptr;
    P.t[k].colind = A->hcol[k] ? A->hcol[k] : A->t[k].colind;
    P.t[k].values = A->t[k].values;
    P.t[k].B = B[k];
    P.t[k].ldb = ldb[k];
    if (A->hcol[k]) {
      P.t[k].hot = hot + A->hot_off[k] * ldh * esize;
      P.t[k].ldh = ldh;
      P.hot = 1;
    } else {  // no tagged entries: the staged-row address is never taken
      P.t[k].hot = B[k];
      P.t[k].ldh = ldb[k];
    }
  }
  if (hot) {
    spmm::HotStageParams H{};
    uintptr_t align_or = (uintptr_t)(N * esize);
    for (int k = 0; k < K; ++k) {
      H.B[k] = B[k];
      H.ldb_bytes[k] = ldb[k] * esize;
      if (A->hot_off[k + 1] > A->hot_off[k]) align_or |= reinterpret_cast<uintptr_t>(B[k]) | (uintptr_t)(ldb[k] * esize);
    }
    for (int k = 0; k <= K; ++k) H.off[k] = A->hot_off[k];
    H.num_k = K;
    H.src = A->hot_src;
    H.dst = hot;
    H.ldh_bytes = ldh * esize;
    H.row_bytes = N * esize;
    const int width = (align_or % 16) == 0 ? 16 : ((align_or % 4) == 0 ? 4 : 2);
    hipError_t e = spmm::launch_hot_stage(H, width, s);
    if (e != hipSuccess) return e;
  }
  P.num_k = K;
  P.k_offset = (int)(((k_offset % K) + K) % K);
  P.rows = A->rows;
  P.N = N;
  P.C = C;
  P.ldc = ldc;
  P.accumulate = accumulate ? 1 : 0;
  P.long_row = plan.long_row;
  P.seg = plan.seg;
  P.n_seg = plan.n_seg;
  P.lrow = plan.lrow;
  P.n_long = plan.n_long;
  P.partial = static_cast<float*>(workspace);
  P.ldp = (int64_t)partial_ld(N);
  return spmm::launch_fwd(P, v, dt, s);
}

// Choose each k-tile's staged hot rows and build its tagged colind (synchronous).
// want < 0: none; want = 0: the library rule (kDefaultHotRows to kHotRowsCap per k-tile
// by its width, subject to the use, size and skew tests); want > 0: up to `want` of each k-tile's most used
// columns (used at least once), no further test.  Columns are ranked by use count,
// ties by index.
spmm_status select_hot(spmm_tile_s* h, const spmm_csr* tiles, int K, int32_t want, hipStream_t s,
                       int64_t* hot_nnz) {
  *hot_nnz = 0;
  if (want < 0) return SPMM_OK;
  const bool forced = want > 0;
  const int32_t min_uses = forced ? 1 : kHotMinUses;
  int64_t nnz_total = 0, max_cols = 0;
  for (int k = 0; k < K; ++k) {
    nnz_total += tiles[k].nnz;
    if (forced || tiles[k].cols <= kHotMaxCols) max_cols = std::max<int64_t>(max_cols, tiles[k].cols);
  }
  if (nnz_total == 0 || max_cols == 0 || (!forced && nnz_total < kHotMinNnz)) return SPMM_OK;
  int32_t* dbuf = nullptr;  // column counts, then the slot of each column
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(&dbuf), sizeof(int32_t) * (size_t)max_cols));
  std::vector<std::vector<int32_t>> chosen(K);
  std::vector<int32_t> cnt, slot_of;
  auto run = [&]() -> spmm_status {
    for (int k = 0; k < K; ++k) {
      const spmm_csr& t = tiles[k];
      if (t.nnz == 0 || t.cols == 0 || (!forced && t.cols > kHotMaxCols)) continue;
      cnt.assign((size_t)t.cols, 0);
      HIP_TRY(hipMemsetAsync(dbuf, 0, sizeof(int32_t) * (size_t)t.cols, s));
      HIP_TRY(spmm::launch_count_columns(t.colind, t.nnz, dbuf, s));
      HIP_TRY(hipMemcpyAsync(cnt.data(), dbuf, sizeof(int32_t) * (size_t)t.cols, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      std::vector<int32_t>& c = chosen[k];
      const int64_t hmax =
          forced ? want : std::min<int64_t>(kHotRowsCap, std::max<int64_t>(kDefaultHotRows, t.cols / kHotColsPerRow));
      for (int64_t j = 0; j < t.cols; ++j)
        if (cnt[j] >= min_uses) c.push_back((int32_t)j);
      auto hotter = [&](int32_t a, int32_t b) { return cnt[a] != cnt[b] ? cnt[a] > cnt[b] : a < b; };
      if ((int64_t)c.size() > hmax) {
        std::nth_element(c.begin(), c.begin() + hmax, c.end(), hotter);
        c.resize((size_t)hmax);
      }
      std::sort(c.begin(), c.end(), hotter);
      int64_t cov = 0;
      for (int32_t j : c) cov += cnt[j];
      const int64_t H = (int64_t)c.size();
      if (!forced && (8 * cov < t.nnz || cov * t.cols < kHotConcentration * H * t.nnz)) c.clear();
      if (!c.empty()) *hot_nnz += cov;
    }
    int64_t total = 0;
    for (int k = 0; k < K; ++k) {
      h->hot_off[k] = total;
      total += (int64_t)chosen[k].size();
    }
    h->hot_off[K] = total;
    if (total == 0) return SPMM_OK;
    if (dalloc(&h->hot_src, total) != hipSuccess) return fail(SPMM_ERR_ALLOC, "device allocation of the hot-row list failed");
    for (int k = 0; k < K; ++k) {
      const std::vector<int32_t>& c = chosen[k];
      if (c.empty()) continue;
      const spmm_csr& t = tiles[k];
      slot_of.assign((size_t)t.cols, -1);
      for (size_t i = 0; i < c.size(); ++i) slot_of[(size_t)c[i]] = (int32_t)i;
      if (dalloc(&h->hcol[k], t.nnz) != hipSuccess) return fail(SPMM_ERR_ALLOC, "device allocation of the tagged colind failed");
      HIP_TRY(hipMemcpyAsync(dbuf, slot_of.data(), sizeof(int32_t) * (size_t)t.cols, hipMemcpyHostToDevice, s));
      HIP_TRY(spmm::launch_tag_hot(t.colind, t.nnz, dbuf, h->hcol[k], s));
      HIP_TRY(hipMemcpyAsync(h->hot_src + h->hot_off[k], c.data(), sizeof(int32_t) * c.size(), hipMemcpyHostToDevice, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    return SPMM_OK;
  };
  spmm_status st = spmm::guarded(run);
  (void)hipFree(dbuf);
  return st;
}

// Fields of a variant entry; the fused backward kind belongs to the backward's table only.
bool valid_variant(const spmm_variant& v, spmm_dtype dtype, bool bwd) {
  if (v.kind < SPMM_KERNEL_AUTO || v.kind > (bwd ? SPMM_KERNEL_FUSED : SPMM_KERNEL_STREAM)) return false;
  if (v.lanes != 0 && !pow2_lanes(v.lanes)) return false;
  if (v.vec != 0 && v.vec != 1 && v.vec != 2 && v.vec != 4 && !(v.vec == 8 && dtype == SPMM_BF16)) return false;
  if (v.kind == SPMM_KERNEL_FUSED) {
    if (v.depth != 0 && v.depth != 1 && v.depth != 2 && v.depth != 4 && v.depth != 8) return false;
    if (v.depth != 0 && v.lanes != 0 && v.depth > v.lanes) return false;
  } else if (v.depth != 0) {
    return false;
  }
  return true;
}

}  // namespace

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
  spmm::TraceRange trace_range("spmm_tile_create");
  if (!out) return fail(SPMM_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (rows < 0 || rows >= ((int64_t)1 << 31)) return fail(SPMM_ERR_INVALID_ARG, "rows=%lld out of range", (long long)rows);
  if (num_k < 1 || num_k > kMaxK) return fail(SPMM_ERR_INVALID_ARG, "num_k=%d outside [1, %d]", num_k, kMaxK);
  if (!tiles) return fail(SPMM_ERR_INVALID_ARG, "tiles is null");
  const unsigned flags = opts ? opts->flags : 0u;
  if (flags & ~(SPMM_TILE_VALIDATE | SPMM_TILE_TRANSPOSE)) return fail(SPMM_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
  int32_t long_row = (opts && opts->long_row > 0) ? opts->long_row : kDefaultLongRow;
  int32_t segment = (opts && opts->segment > 0) ? opts->segment : kDefaultSegment;
  if (opts && (opts->long_row < 0 || opts->segment < 0 || opts->bwd_slice < 0))
    return fail(SPMM_ERR_INVALID_ARG, "negative long_row/segment/bwd_slice");
  // The stream kernels sum the lengths of 64 unsplit rows in 32 bits.
  if (long_row > kMaxLongRow)
    return fail(SPMM_ERR_INVALID_ARG, "long_row=%d above %d ((2^31 - 1) / 64)", long_row, kMaxLongRow);
  const int32_t hot_rows = opts ? opts->hot_rows : 0;
  if (hot_rows < -1 || hot_rows > kMaxHotRows)
    return fail(SPMM_ERR_INVALID_ARG, "hot_rows=%d outside [-1, %d]", hot_rows, kMaxHotRows);
  int64_t units_bound = 0;
  for (int k = 0; k < num_k; ++k) {
    const spmm_csr& t = tiles[k];
    if (t.cols < 0 || t.cols >= ((int64_t)1 << 31)) return fail(SPMM_ERR_INVALID_ARG, "tile %d: cols out of range", k);
    if (t.nnz < 0) return fail(SPMM_ERR_INVALID_ARG, "tile %d: negative nnz", k);
    if (t.nnz > spmm::kMaxNnz) return fail(SPMM_ERR_UNSUPPORTED, "tile %d: nnz > 2^31 - 2^16 needs 64-bit indices", k);
    if (!t.rowptr) return fail(SPMM_ERR_INVALID_ARG, "tile %d: rowptr is null", k);
    if (t.nnz > 0 && (!t.colind || !t.values)) return fail(SPMM_ERR_INVALID_ARG, "tile %d: colind/values null", k);
    units_bound += t.nnz / segment + rows;
  }
  if (units_bound >= ((int64_t)1 << 31)) return fail(SPMM_ERR_UNSUPPORTED, "split-row plan would exceed 2^31 units");
  if (!(opts && opts->long_row > 0) && rows > 0) {
    // Default split threshold: 128, doubled while below twice the mean combined row
    // length, so that tiles of near-uniform rows are not split into units.
    int64_t nnz_total = 0;
    for (int k = 0; k < num_k; ++k) nnz_total += tiles[k].nnz;
    while ((int64_t)long_row * rows < 2 * nnz_total && long_row < (1 << 20)) long_row *= 2;
  }
  if ((flags & SPMM_TILE_TRANSPOSE) && num_k != 1)
    return fail(SPMM_ERR_UNSUPPORTED, "SPMM_TILE_TRANSPOSE needs a single tile (num_k = 1)");

  hipStream_t s = static_cast<hipStream_t>(stream);
  spmm_tile_s* h = new (std::nothrow) spmm_tile_s();
  if (!h) return fail(SPMM_ERR_ALLOC, "host allocation failed");
  h->rows = rows;
  h->num_k = num_k;
  for (int k = 0; k < num_k; ++k) h->t[k] = tiles[k];
  h->bwd_slice = opts ? opts->bwd_slice : 0;
  (void)hipGetDevice(&h->device);

  int64_t hot_nnz = 0;
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
    st = select_hot(h, tiles, num_k, hot_rows, s, &hot_nnz);
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
  spmm_status st = spmm::guarded(body);
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
  S.long_row = h->plan.long_row;
  S.segment = h->plan.segment;
  S.hot_rows = h->hot_total();
  S.hot_nnz = hot_nnz;
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
  *bytes = fwd_workspace(A, A->plan, N);
  return SPMM_OK;
}

// Backward workspace: FP32 partial rows of the transposed plan's split rows, then
// (16-byte aligned) either A's values gathered into the transposed order (the two-pass
// form) or the fused form's partial dot products, one array of nnz per column window
// when G * V < N (at most fused_windows_max(N) windows: at least 256 columns each, at
// most 8).
static size_t bwd_partial_bytes(const spmm_tile_s* A, int64_t N) {
  return (sizeof(float) * partial_ld(N) * (size_t)A->planT.n_seg + 15) & ~(size_t)15;
}
static size_t bwd_workspace(const spmm_tile_s* A, int64_t N) {
  return bwd_partial_bytes(A, N) + sizeof(float) * (size_t)A->t[0].nnz * (size_t)fused_windows_max(N);
}

spmm_status spmm_bwd_workspace_bytes(spmm_tile_t A, int64_t N, size_t* bytes) {
  if (!A || !bytes) return fail(SPMM_ERR_INVALID_ARG, "null argument");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  *bytes = bwd_workspace(A, N);
  return SPMM_OK;
}

spmm_status spmm_fwd(spmm_tile_t A, int k_offset, const void* const* B, const int64_t* ldb, spmm_dtype b_dtype,
                     void* C, int64_t ldc, spmm_dtype c_dtype, int64_t N, int accumulate, void* workspace,
                     size_t ws_bytes, void* stream) {
  spmm::TraceRange trace_range("spmm_fwd");
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
  const size_t need = fwd_workspace(A, A->plan, N);
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

  const spmm::Variant v = resolve_variant(A, N, dt, align_or);
  HIP_TRY(launch_forward(A, A->plan, k_offset, B, ldb, dt, C, ldc, N, accumulate, workspace, v,
                         static_cast<hipStream_t>(stream)));
  return SPMM_OK;
}

spmm_status spmm_tile_set_variant(spmm_tile_t A, int64_t N, spmm_dtype dtype, const spmm_variant* v) {
  if (!A) return fail(SPMM_ERR_INVALID_ARG, "tile is null");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  if (dtype != SPMM_F32 && dtype != SPMM_BF16) return fail(SPMM_ERR_INVALID_ARG, "unknown dtype");
  if (v && !valid_variant(*v, dtype, false)) return fail(SPMM_ERR_INVALID_ARG, "invalid variant fields");
  return set_variant_in(A->vt, &A->nvt, N, dtype, v);
}

spmm_status spmm_tile_set_bwd_variant(spmm_tile_t A, int64_t N, spmm_dtype dtype, const spmm_variant* v) {
  if (!A) return fail(SPMM_ERR_INVALID_ARG, "tile is null");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  if (dtype != SPMM_F32 && dtype != SPMM_BF16) return fail(SPMM_ERR_INVALID_ARG, "unknown dtype");
  if (v && !valid_variant(*v, dtype, true)) return fail(SPMM_ERR_INVALID_ARG, "invalid variant fields");
  return set_variant_in(A->vtT, &A->nvtT, N, dtype, v);
}

spmm_status spmm_tile_get_variant(spmm_tile_t A, int64_t N, spmm_dtype dtype, int32_t bwd, spmm_variant* out) {
  if (!A) return fail(SPMM_ERR_INVALID_ARG, "tile is null");
  if (!out) return fail(SPMM_ERR_INVALID_ARG, "out is null");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  if (dtype != SPMM_F32 && dtype != SPMM_BF16) return fail(SPMM_ERR_INVALID_ARG, "unknown dtype");
  if (bwd != 0 && bwd != 1) return fail(SPMM_ERR_INVALID_ARG, "bwd=%d is not 0 or 1", (int)bwd);
  const spmm_tile_s::VarEntry* vt = bwd ? A->vtT : A->vt;
  const int n = bwd ? A->nvtT : A->nvt;
  *out = spmm_variant{SPMM_KERNEL_AUTO, 0, 0, 0};
  for (int i = 0; i < n; ++i)
    if (vt[i].N == N && vt[i].dtype == (int)dtype) *out = vt[i].v;
  return SPMM_OK;
}

spmm_status spmm_tile_set_sddmm_variant(spmm_tile_t A, int64_t N, int32_t lanes, int32_t nnz_per_group) {
  if (!A) return fail(SPMM_ERR_INVALID_ARG, "tile is null");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  int slot = -1;
  for (int i = 0; i < A->nsd; ++i)
    if (A->sd[i].N == N) slot = i;
  if (lanes == 0) {
    if (slot >= 0) A->sd[slot] = A->sd[--A->nsd];
    return SPMM_OK;
  }
  if (!pow2_lanes(lanes)) return fail(SPMM_ERR_INVALID_ARG, "lanes=%d is not 4, 8, 16, 32 or 64", lanes);
  if (nnz_per_group != 1 && nnz_per_group != 2 && nnz_per_group != 4 && nnz_per_group != 8)
    return fail(SPMM_ERR_INVALID_ARG, "nnz_per_group=%d is not 1, 2, 4 or 8", nnz_per_group);
  if (nnz_per_group > lanes) return fail(SPMM_ERR_INVALID_ARG, "nnz_per_group > lanes");
  if (slot < 0) {
    if (A->nsd >= 8) return fail(SPMM_ERR_INVALID_ARG, "SDDMM variant table is full");
    slot = A->nsd++;
  }
  A->sd[slot] = {N, lanes, nnz_per_group};
  return SPMM_OK;
}

static spmm_status autotune_impl(spmm_tile_t A, int64_t N, spmm_dtype dtype, const void* const* B,
                                 const int64_t* ldb, void* C, int64_t ldc, int tune_plan, void* stream,
                                 spmm_variant* chosen);

spmm_status spmm_tile_autotune(spmm_tile_t A, int64_t N, spmm_dtype dtype, const void* const* B,
                               const int64_t* ldb, void* C, int64_t ldc, int tune_plan, void* stream,
                               spmm_variant* chosen) {
  return spmm::guarded([&]() { return autotune_impl(A, N, dtype, B, ldb, C, ldc, tune_plan, stream, chosen); });
}

static spmm_status autotune_impl(spmm_tile_t A, int64_t N, spmm_dtype dtype, const void* const* B,
                                 const int64_t* ldb, void* C, int64_t ldc, int tune_plan, void* stream,
                                 spmm_variant* chosen) {
  if (!A) return fail(SPMM_ERR_INVALID_ARG, "tile is null");
  if (!B || !ldb) return fail(SPMM_ERR_INVALID_ARG, "B/ldb array is null");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  if (dtype != SPMM_F32 && dtype != SPMM_BF16) return fail(SPMM_ERR_INVALID_ARG, "unknown dtype");
  if (ldc < N) return fail(SPMM_ERR_INVALID_ARG, "ldc < N");
  if (!C && A->rows > 0) return fail(SPMM_ERR_INVALID_ARG, "C is null");
  const DT dt = dtype == SPMM_F32 ? DT::F32 : DT::BF16;
  const int esize = dt == DT::F32 ? 4 : 2;
  uintptr_t align_or = reinterpret_cast<uintptr_t>(C) | (uintptr_t)(ldc * esize);
  for (int k = 0; k < A->num_k; ++k) {
    if (!B[k] && A->t[k].cols > 0) return fail(SPMM_ERR_INVALID_ARG, "B[%d] is null", k);
    if (ldb[k] < N) return fail(SPMM_ERR_INVALID_ARG, "ldb[%d] < N", k);
    if (ldb[k] * esize >= ((int64_t)1 << 32)) return fail(SPMM_ERR_UNSUPPORTED, "ldb[%d] too large", k);
    align_or |= reinterpret_cast<uintptr_t>(B[k]) | (uintptr_t)(ldb[k] * esize);
  }
  if ((N + 63) / 64 > 65535) return fail(SPMM_ERR_UNSUPPORTED, "N too large for one launch");
  if (A->rows == 0) return SPMM_OK;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != A->device) return fail(SPMM_ERR_INVALID_ARG, "current device differs from the handle's");
  hipStream_t s = static_cast<hipStream_t>(stream);

  const spmm::Variant base = pick_variant(N, dt, align_or, A->rows, (int64_t)A->plan.stats[1]);
  const std::vector<spmm::Variant> kv = candidate_variants(N, dt, align_or, A->rows, (int64_t)A->plan.stats[1]);
  // Split-plan candidates (threshold, unit length).
  std::vector<std::pair<int32_t, int32_t>> pc;
  pc.push_back({A->plan.long_row, A->plan.segment});
  if (tune_plan) {
    const std::pair<int32_t, int32_t> extra[] = {{128, 64}, {256, 128}, {512, 256}, {1024, 512}};
    for (auto& p : extra)
      if (p.first != A->plan.long_row || p.second != A->plan.segment) pc.push_back(p);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  void* ws = nullptr;
  size_t ws_cap = 0;
  float best = 1e30f;
  int best_p = 0;
  spmm::Variant best_v = base;
  std::vector<Plan> plans(pc.size());
  spmm_status st = SPMM_OK;
  for (size_t pi = 0; pi < pc.size() && st == SPMM_OK; ++pi) {
    const Plan* plan = &A->plan;
    if (pi > 0) {
      const int32_t* rps[kMaxK];
      for (int k = 0; k < A->num_k; ++k) rps[k] = A->t[k].rowptr;
      st = build_plan(rps, A->num_k, A->rows, pc[pi].first, pc[pi].second, s, &plans[pi]);
      if (st != SPMM_OK) break;
      plan = &plans[pi];
    }
    const size_t need = fwd_workspace(A, *plan, N);
    if (need > ws_cap) {
      if (ws) (void)hipFree(ws);
      ws = nullptr;
      if (hipMalloc(&ws, need) != hipSuccess) {
        st = fail(SPMM_ERR_ALLOC, "autotune scratch allocation failed");
        break;
      }
      ws_cap = need;
    }
    for (const auto& v : kv) {
      hipError_t e = launch_forward(A, *plan, 0, B, ldb, dt, C, ldc, N, 0, ws, v, s);
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_forward(A, *plan, 0, B, ldb, dt, C, ldc, N, 0, ws, v, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        st = fail(SPMM_ERR_HIP, "autotune launch: %s", hipGetErrorString(e));
        break;
      }
      if (ms < best) {
        best = ms;
        best_p = (int)pi;
        best_v = v;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ws) (void)hipFree(ws);
  if (st == SPMM_OK && best_p > 0) {
    free_plan(A->plan);
    A->plan = plans[best_p];
    plans[best_p] = Plan();
    A->stats.long_rows = A->plan.n_long;
    A->stats.segments = A->plan.n_seg;
    A->stats.long_row = A->plan.long_row;
    A->stats.segment = A->plan.segment;
  }
  for (auto& p : plans) free_plan(p);
  if (st != SPMM_OK) return st;
  spmm_variant out{best_v.stream ? SPMM_KERNEL_STREAM : SPMM_KERNEL_ROWSPLIT, best_v.stream ? best_v.rows : best_v.G,
                   best_v.V, 0};
  st = spmm_tile_set_variant(A, N, dtype, &out);
  if (st == SPMM_OK && chosen) *chosen = out;
  return st;
}

spmm_status spmm_tile_accumulate(void* C, int64_t ldc, const void* Ptile, int64_t ldp, int64_t rows, int64_t N,
                                 spmm_dtype dtype, void* stream) {
  spmm::TraceRange trace_range("spmm_tile_accumulate");
  if (rows < 0 || N < 1) return fail(SPMM_ERR_INVALID_ARG, "rows=%lld N=%lld", (long long)rows, (long long)N);
  if (dtype != SPMM_F32 && dtype != SPMM_BF16) return fail(SPMM_ERR_INVALID_ARG, "unknown dtype");
  if (ldc < N || ldp < N) return fail(SPMM_ERR_INVALID_ARG, "leading dimension < N");
  if (rows > 0 && (!C || !Ptile)) return fail(SPMM_ERR_INVALID_ARG, "C/Ptile is null");
  if (rows == 0) return SPMM_OK;
  const DT dt = dtype == SPMM_F32 ? DT::F32 : DT::BF16;
  const int esize = dt == DT::F32 ? 4 : 2;
  const uintptr_t a = reinterpret_cast<uintptr_t>(C) | reinterpret_cast<uintptr_t>(Ptile) |
                      (uintptr_t)(ldc * esize) | (uintptr_t)(ldp * esize);
  int V = 16 / esize;
  while (V > 1 && ((N % V) != 0 || (a % (uintptr_t)(V * esize)) != 0)) V /= 2;
  if (rows * (N / V) / spmm::kBlock >= ((int64_t)1 << 31)) return fail(SPMM_ERR_UNSUPPORTED, "tile too large");
  HIP_TRY(spmm::launch_accumulate(C, ldc, Ptile, ldp, rows, N, dt, V, static_cast<hipStream_t>(stream)));
  return SPMM_OK;
}

// The fused backward (dA and dB in one pass over the transposed structure), then the
// fix-up of the transposed plan's split rows (arguments already checked).
static hipError_t launch_backward_fused(const spmm_tile_s* A, const FusedShape& fs, const void* dC, int64_t lddc,
                                        const void* B, int64_t ldb, float* dA, void* dB, int64_t lddb, int64_t N,
                                        DT dt, void* workspace, hipStream_t s) {
  const spmm_csr& t = A->t[0];
  spmm::BwdFusedParams F{};
  F.rowptrT = A->rowptrT;
  F.colindT = A->colindT;
  F.perm = A->perm;
  F.values = t.values;
  F.dC = dC;
  F.lddc = lddc;
  F.B = B;
  F.ldb = ldb;
  F.dA = dA;
  F.dB = dB;
  F.lddb = lddb;
  F.cols = t.cols;
  F.N = N;
  F.long_row = A->planT.long_row;
  F.seg = A->planT.seg;
  F.n_seg = A->planT.n_seg;
  F.partial = static_cast<float*>(workspace);
  F.ldp = (int64_t)partial_ld(N);
  F.n_win = fs.n_win;
  F.nnz = t.nnz;
  F.dA_part = fs.n_win > 1 ? reinterpret_cast<float*>(static_cast<char*>(workspace) + bwd_partial_bytes(A, N))
                           : nullptr;
  hipError_t e = spmm::launch_bwd_fused(F, fs.G, fs.V, fs.U, dt, s);
  if (e != hipSuccess || A->planT.n_long == 0) return e;
  spmm::FwdParams P{};
  P.num_k = 1;
  P.rows = t.cols;
  P.N = N;
  P.C = dB;
  P.ldc = lddb;
  P.seg = A->planT.seg;
  P.n_seg = A->planT.n_seg;
  P.lrow = A->planT.lrow;
  P.n_long = A->planT.n_long;
  P.partial = F.partial;
  P.ldp = F.ldp;
  return spmm::launch_fixup(P, fs.G, fs.V, dt, s);
}

spmm_status spmm_tile_accumulate_n(void* C, int64_t ldc, const void* const* Pt, const int64_t* ldp, int n,
                                   int64_t rows, int64_t N, spmm_dtype dtype, void* stream) {
  spmm::TraceRange trace_range("spmm_tile_accumulate_n");
  if (rows < 0 || N < 1 || n < 0) return fail(SPMM_ERR_INVALID_ARG, "rows=%lld N=%lld n=%d", (long long)rows,
                                               (long long)N, n);
  if (dtype != SPMM_F32 && dtype != SPMM_BF16) return fail(SPMM_ERR_INVALID_ARG, "unknown dtype");
  if (n > 0 && (!Pt || !ldp)) return fail(SPMM_ERR_INVALID_ARG, "P/ldp is null");
  if (ldc < N) return fail(SPMM_ERR_INVALID_ARG, "ldc < N");
  if (rows > 0 && !C) return fail(SPMM_ERR_INVALID_ARG, "C is null");
  const DT dt = dtype == SPMM_F32 ? DT::F32 : DT::BF16;
  const int esize = dt == DT::F32 ? 4 : 2;
  uintptr_t a = reinterpret_cast<uintptr_t>(C) | (uintptr_t)(ldc * esize);
  for (int t = 0; t < n; ++t) {
    if (ldp[t] < N) return fail(SPMM_ERR_INVALID_ARG, "ldp[%d] < N", t);
    if (rows > 0 && !Pt[t]) return fail(SPMM_ERR_INVALID_ARG, "P[%d] is null", t);
    a |= reinterpret_cast<uintptr_t>(Pt[t]) | (uintptr_t)(ldp[t] * esize);
  }
  if (rows == 0 || n == 0) return SPMM_OK;
  int V = 16 / esize;
  while (V > 1 && ((N % V) != 0 || (a % (uintptr_t)(V * esize)) != 0)) V /= 2;
  HIP_TRY(spmm::launch_accumulate_n(C, ldc, Pt, ldp, n, rows, N, dt, V, static_cast<hipStream_t>(stream)));
  return SPMM_OK;
}

spmm_status spmm_bwd(spmm_tile_t A, const void* dC, int64_t lddc, const void* B, int64_t ldb, int64_t N,
                     spmm_dtype dtype, float* dA_values, void* dB, int64_t lddb, void* workspace, size_t ws_bytes,
                     void* stream) {
  spmm::TraceRange trace_range("spmm_bwd");
  if (!A) return fail(SPMM_ERR_INVALID_ARG, "A is null");
  if (dtype != SPMM_F32 && dtype != SPMM_BF16) return fail(SPMM_ERR_INVALID_ARG, "unknown dtype");
  const DT dt = dtype == SPMM_F32 ? DT::F32 : DT::BF16;
  const int64_t esize = dt == DT::F32 ? 4 : 2;
  if (A->num_k != 1) return fail(SPMM_ERR_UNSUPPORTED, "spmm_bwd needs a single-tile handle");
  if (!A->has_t) return fail(SPMM_ERR_UNSUPPORTED, "handle was created without SPMM_TILE_TRANSPOSE");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  if (!dC && A->rows > 0) return fail(SPMM_ERR_INVALID_ARG, "dC is null");
  if (lddc < N) return fail(SPMM_ERR_INVALID_ARG, "lddc < N");
  if (dA_values && !B && A->t[0].cols > 0) return fail(SPMM_ERR_INVALID_ARG, "B is null");
  if (dA_values && ldb < N) return fail(SPMM_ERR_INVALID_ARG, "ldb < N");
  if (dB && lddb < N) return fail(SPMM_ERR_INVALID_ARG, "lddb < N");
  if (lddc * esize >= ((int64_t)1 << 32)) return fail(SPMM_ERR_UNSUPPORTED, "lddc too large");
  const spmm_csr& t = A->t[0];
  const size_t need = dB ? bwd_workspace(A, N) : 0;
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

  // Both gradients, no column slices requested: one fused pass when a group covers N.
  FusedShape fs{};
  if (dA_values && dB && t.cols > 0 && !(A->bwd_slice > 0 && A->bwd_slice < N) &&
      fused_shape(A, N, dt,
                  reinterpret_cast<uintptr_t>(dC) | reinterpret_cast<uintptr_t>(B) | reinterpret_cast<uintptr_t>(dB) |
                      (uintptr_t)(lddc * esize) | (uintptr_t)(ldb * esize) | (uintptr_t)(lddb * esize),
                  &fs)) {
    HIP_TRY(launch_backward_fused(A, fs, dC, lddc, B, ldb, dA_values, dB, lddb, N, dt, workspace, s));
    return SPMM_OK;
  }

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
    const uintptr_t a = reinterpret_cast<uintptr_t>(dC) | reinterpret_cast<uintptr_t>(B) |
                        (uintptr_t)(lddc * esize) | (uintptr_t)(ldb * esize);
    int V = (int)(16 / esize);
    while (V > 1 && ((N % V) != 0 || (a % (uintptr_t)(V * esize)) != 0)) V /= 2;
    // Column slices: one launch per slice of `slice` columns (all of N when 0).
    const int64_t slice = (A->bwd_slice > 0 && A->bwd_slice < N && (A->bwd_slice % V) == 0) ? A->bwd_slice : N;
    const int64_t need_lanes = (slice + V - 1) / V;
    // 8 lanes x U non-zeros per group measured best on the heavy-tailed 2M x 2M matrix at
    // N = 128: U = 4 (32 B rows in flight per wave) for FP32, U = 2 for BF16, whose
    // 16-element loads make each row fetch twice as wide (narrower slices use fewer lanes).
    int G = 4;
    while (G < 8 && G < need_lanes) G *= 2;
    int U = dt == DT::F32 ? 4 : 2;
    for (int i = 0; i < A->nsd; ++i)
      if (A->sd[i].N == N) {
        G = A->sd[i].G;
        U = A->sd[i].U;
      }
    if (U > G) U = G;
    for (int64_t c = 0; c < N; c += slice) {
      P.c_begin = c;
      P.c_end = c + slice < N ? c + slice : N;
      P.accumulate = c > 0 ? 1 : 0;
      HIP_TRY(spmm::launch_sddmm(P, G, V, U, dt, s));
    }
  }
  if (dB && t.cols > 0) {
    float* valuesT = reinterpret_cast<float*>(static_cast<char*>(workspace) + bwd_partial_bytes(A, N));
    HIP_TRY(spmm::launch_gather_values(A->perm, t.values, valuesT, t.nnz, s));
    spmm::FwdParams P{};
    P.t[0].rowptr = A->rowptrT;
    P.t[0].colind = A->colindT;
    P.t[0].values = valuesT;
    P.t[0].B = dC;
    P.t[0].ldb = lddc;
    P.t[0].hot = dC;  // the transposed structure has no tagged entries
    P.t[0].ldh = lddc;
    P.num_k = 1;
    P.k_offset = 0;
    P.rows = t.cols;
    P.N = N;
    P.C = dB;
    P.ldc = lddb;
    P.accumulate = 0;
    P.long_row = A->planT.long_row;
    P.seg = A->planT.seg;
    P.n_seg = A->planT.n_seg;
    P.lrow = A->planT.lrow;
    P.n_long = A->planT.n_long;
    P.partial = static_cast<float*>(workspace);
    P.ldp = (int64_t)partial_ld(N);
    const uintptr_t a = reinterpret_cast<uintptr_t>(dC) | reinterpret_cast<uintptr_t>(dB) |
                        (uintptr_t)(lddc * esize) | (uintptr_t)(lddb * esize);
    HIP_TRY(spmm::launch_fwd(P, resolve_variant_in(A->vtT, A->nvtT, t.cols, (int64_t)A->planT.stats[1], N, dt, a), dt,
                             s));
  }
  return SPMM_OK;
}

static spmm_status autotune_bwd_impl(spmm_tile_t A, int64_t N, spmm_dtype dtype, const void* dC, int64_t lddc,
                                     const void* B, int64_t ldb, float* dA, void* dB, int64_t lddb, void* stream,
                                     spmm_variant* chosen) {
  if (!A) return fail(SPMM_ERR_INVALID_ARG, "tile is null");
  if (A->num_k != 1) return fail(SPMM_ERR_UNSUPPORTED, "the dB pass needs a single-tile handle");
  if (!A->has_t) return fail(SPMM_ERR_UNSUPPORTED, "handle was created without SPMM_TILE_TRANSPOSE");
  if (N < 1) return fail(SPMM_ERR_INVALID_ARG, "N=%lld < 1", (long long)N);
  if (dtype != SPMM_F32 && dtype != SPMM_BF16) return fail(SPMM_ERR_INVALID_ARG, "unknown dtype");
  const DT dt = dtype == SPMM_F32 ? DT::F32 : DT::BF16;
  const int64_t esize = dt == DT::F32 ? 4 : 2;
  const spmm_csr& t = A->t[0];
  if (!dC && A->rows > 0) return fail(SPMM_ERR_INVALID_ARG, "dC is null");
  if (!dB && t.cols > 0) return fail(SPMM_ERR_INVALID_ARG, "dB is null");
  if (lddc < N || lddb < N) return fail(SPMM_ERR_INVALID_ARG, "leading dimension < N");
  const bool full = B != nullptr && dA != nullptr;  // time whole backward passes, fused shapes included
  if (full && ldb < N) return fail(SPMM_ERR_INVALID_ARG, "ldb < N");
  if (lddc * esize >= ((int64_t)1 << 32)) return fail(SPMM_ERR_UNSUPPORTED, "lddc too large");
  if ((N + 63) / 64 > 65535) return fail(SPMM_ERR_UNSUPPORTED, "N too large for one launch");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != A->device) return fail(SPMM_ERR_INVALID_ARG, "current device differs from the handle's");
  uintptr_t a = reinterpret_cast<uintptr_t>(dC) | reinterpret_cast<uintptr_t>(dB) | (uintptr_t)(lddc * esize) |
                (uintptr_t)(lddb * esize);
  // Candidates: the dB pass's kernel variants (two-pass backward) and, when B and dA are
  // given, fused shapes at the widest aligned vector width and at half and a quarter of it,
  // each with 2, 4 and 8 entries in flight per group.
  std::vector<spmm_variant> cand;
  for (const auto& v : candidate_variants(N, dt, a, t.cols, (int64_t)A->planT.stats[1]))
    cand.push_back(spmm_variant{v.stream ? SPMM_KERNEL_STREAM : SPMM_KERNEL_ROWSPLIT, v.stream ? v.rows : v.G, v.V, 0});
  if (full) {
    a |= reinterpret_cast<uintptr_t>(B) | (uintptr_t)(ldb * esize);
    int vmax = (int)(16 / esize);
    while (vmax > 1 && ((N % vmax) != 0 || (a % (uintptr_t)(vmax * esize)) != 0)) vmax /= 2;
    for (int V = vmax; V >= 1 && V >= vmax / 4; V /= 2) {
      if ((N % V) != 0) continue;
      int G = 4;
      while (G < 64 && (int64_t)G * V < N) G *= 2;
      if ((N + (int64_t)G * V - 1) / ((int64_t)G * V) <= fused_windows_max(N))
        for (int U : {2, 4, 8})
          if (U <= G) cand.push_back(spmm_variant{SPMM_KERNEL_FUSED, G, V, U});
    }
  }
  // Each candidate is timed through spmm_bwd itself with the candidate as the table's
  // entry (3 calls after a warm-up call), so the choice measures exactly what later
  // calls run; the entry found before tuning is restored if a call fails.
  spmm_variant prev{SPMM_KERNEL_AUTO, 0, 0, 0};
  (void)spmm_tile_get_variant(A, N, dtype, 1, &prev);
  spmm_variant best = cand.empty() ? spmm_variant{SPMM_KERNEL_AUTO, 0, 0, 0} : cand[0];
  if (t.cols > 0 && !cand.empty()) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t wsb = bwd_workspace(A, N);
    void* ws = nullptr;
    HIP_TRY(hipMalloc(&ws, wsb > 0 ? wsb : 16));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best_ms = 1e30f;
    auto run = [&]() -> spmm_status {
      HIP_TRY(hipEventCreate(&e0));
      HIP_TRY(hipEventCreate(&e1));
      for (const auto& v : cand) {
        spmm_status st = set_variant_in(A->vtT, &A->nvtT, N, dtype, &v);
        if (st != SPMM_OK) return st;
        auto call = [&]() {
          return spmm_bwd(A, dC, lddc, full ? B : nullptr, ldb, N, dtype, full ? dA : nullptr, dB, lddb, ws, wsb,
                          stream);
        };
        if ((st = call()) != SPMM_OK) return st;
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r)
          if ((st = call()) != SPMM_OK) return st;
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
          best_ms = ms;
          best = v;
        }
      }
      return SPMM_OK;
    };
    spmm_status st = run();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(ws);
    if (st != SPMM_OK) {
      (void)set_variant_in(A->vtT, &A->nvtT, N, dtype, prev.kind == SPMM_KERNEL_AUTO ? nullptr : &prev);
      return st;
    }
  }
  spmm_status st = set_variant_in(A->vtT, &A->nvtT, N, dtype, best.kind == SPMM_KERNEL_AUTO ? nullptr : &best);
  if (st == SPMM_OK && chosen) *chosen = best;
  return st;
}

spmm_status spmm_tile_autotune_bwd(spmm_tile_t A, int64_t N, spmm_dtype dtype, const void* dC, int64_t lddc,
                                   const void* B, int64_t ldb, float* dA, void* dB, int64_t lddb, void* stream,
                                   spmm_variant* chosen) {
  return spmm::guarded(
      [&]() { return autotune_bwd_impl(A, N, dtype, dC, lddc, B, ldb, dA, dB, lddb, stream, chosen); });
}

}  // extern "C"

struct spmm_batch_s {
  int count = 0;
  DT dt = DT::F32;
  int device = 0;
  spmm::BatchTileDev* d_tiles = nullptr;
  spmm::BatchItem* d_items = nullptr;
  int64_t n_items = 0;
  spmm::BatchItem* d_fix = nullptr;
  int64_t n_fix = 0;
  unsigned* d_counter = nullptr;  // persistent mode: kClaimSlices claim counters per item class
  bool persistent = false;
  // Single-launch form: 64-bit claim counters (kClaimSlices, kCounter64Stride apart) then
  // one arrival counter per fix-up item; never reset.
  bool single = false;
  unsigned long long* d_c64 = nullptr;
  int single_grid = 0;
  // Reservation-grid form: mode (0 = none), entries, their item offsets and coordinates,
  // one claim counter per entry.
  int grid_mode = 0;
  int n_entries = 0;
  unsigned class_mask = 0;  // single-launch forms: the kernel instance covering the batch's classes
  int32_t* d_entry_off = nullptr;
  int32_t* d_entry_ijk = nullptr;
  unsigned* d_counterE = nullptr;
  size_t ws_bytes = 0;
  int64_t class_off[spmm::kBatchClasses] = {};
  int64_t class_cnt[spmm::kBatchClasses] = {};
  int class_grid[spmm::kBatchClasses] = {};
  std::vector<spmm_variant> variants;
  ~spmm_batch_s() {
    if (d_tiles) (void)hipFree(d_tiles);
    if (d_items) (void)hipFree(d_items);
    if (d_fix) (void)hipFree(d_fix);
    if (d_counter) (void)hipFree(d_counter);
    if (d_c64) (void)hipFree(d_c64);
    if (d_entry_off) (void)hipFree(d_entry_off);
    if (d_entry_ijk) (void)hipFree(d_entry_ijk);
    if (d_counterE) (void)hipFree(d_counterE);
  }
};

namespace {

// Batched variant of one tile: the handle's table entry for (N, dtype), else the rule
// below; vectors assume 16-byte aligned rows (a documented requirement of spmm_batched).
void batch_variant(const spmm_tile_s* A, int64_t N, DT dt, spmm::BatchTileDev* bt, spmm_variant* out) {
  int Vs = 4;  // stream / unit vector (at most 4 elements per lane): widest dividing N, not wider than needed
  while (Vs > 1 && ((N % Vs) != 0 || 64 * (Vs / 2) >= N)) Vs /= 2;
  const spmm_variant* e = nullptr;
  for (int i = 0; i < A->nvt; ++i)
    if (A->vt[i].N == N && A->vt[i].dtype == (dt == DT::F32 ? SPMM_F32 : SPMM_BF16) &&
        A->vt[i].v.kind != SPMM_KERNEL_AUTO)
      e = &A->vt[i].v;
  // without an entry: the stream kernel for N >= 64 on tiles with more than 1/8 empty rows,
  // else row-split items over 256-byte windows (64 FP32 / 128 BF16 columns); the batch
  // kernels' row-split items always load 4-element vectors, so their windows differ
  // from the single-tile rule's at BF16
  bool stream = N >= 64 && (int64_t)A->plan.stats[1] * 8 > A->rows;
  int G = 8;
  if (e) {
    stream = e->kind == SPMM_KERNEL_STREAM;
    if (stream && e->vec && (N % e->vec) == 0) Vs = e->vec;
    if (!stream && e->lanes >= 4 && e->vec >= 1) {
      // keep the tuned column window (lanes x vec) with the batch's 4-element vectors
      G = std::max(8, std::min(64, e->lanes * e->vec / 4));
    }
  }
  if (!stream) {
    if ((N % 4) != 0) {  // row-split items load 4 elements per lane; otherwise stream
      stream = true;
    } else if (!e || e->lanes < 4) {
      const int g_max = dt == DT::F32 ? 16 : 32;
      G = 8;
      while (G < g_max && G * 4 < N) G *= 2;
    }
  }
  bt->kind = stream ? 0 : 1;
  bt->G = stream ? 64 : G;
  bt->V = Vs;
  *out = spmm_variant{stream ? SPMM_KERNEL_STREAM : SPMM_KERNEL_ROWSPLIT, bt->G, stream ? Vs : 4, 0};
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// Batch creation; coords (3 per tile) and grid_mode select the reservation-grid form.
spmm_status batch_create_impl(int count, const spmm_tile_t* tiles, const int64_t* N, spmm_dtype dtype,
                              int64_t item_nnz, unsigned flags, const int32_t* coords, int grid_mode, void* stream,
                              spmm_batch_t* out) {
  if (!out) return fail(SPMM_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (count < 1) return fail(SPMM_ERR_INVALID_ARG, "count=%d < 1", count);
  if (!tiles || !N) return fail(SPMM_ERR_INVALID_ARG, "tiles/N is null");
  if (dtype != SPMM_F32 && dtype != SPMM_BF16) return fail(SPMM_ERR_INVALID_ARG, "unknown dtype");
  if (item_nnz != 0 && (item_nnz < 64 || item_nnz > ((int64_t)1 << 20)))
    return fail(SPMM_ERR_INVALID_ARG, "item_nnz=%lld out of range", (long long)item_nnz);
  if (flags & ~(unsigned)(SPMM_BATCH_PERSISTENT | SPMM_BATCH_SINGLE))
    return fail(SPMM_ERR_INVALID_ARG, "unknown batch flags 0x%x", flags);
  const double item_target = item_nnz ? (double)item_nnz : 256.0;
  for (int t = 0; t < count; ++t) {
    if (!tiles[t]) return fail(SPMM_ERR_INVALID_ARG, "tile %d is null", t);
    if (tiles[t]->num_k != 1) return fail(SPMM_ERR_UNSUPPORTED, "tile %d has %d k-tiles; batches take single tiles", t,
                                          tiles[t]->num_k);
    if (N[t] < 1 || N[t] > (int64_t)1 << 20) return fail(SPMM_ERR_INVALID_ARG, "N[%d]=%lld out of range", t, (long long)N[t]);
  }
  const DT dt = dtype == SPMM_F32 ? DT::F32 : DT::BF16;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  for (int t = 0; t < count; ++t)
    if (tiles[t]->device != dev) return fail(SPMM_ERR_INVALID_ARG, "tile %d lives on another device", t);
  spmm_batch_s* b = new (std::nothrow) spmm_batch_s();
  if (!b) return fail(SPMM_ERR_ALLOC, "host allocation failed");
  b->count = count;
  b->dt = dt;
  b->device = dev;
  b->persistent = (flags & SPMM_BATCH_PERSISTENT) != 0;
  b->single = (flags & SPMM_BATCH_SINGLE) != 0 || grid_mode != 0;
  b->grid_mode = grid_mode;
  b->variants.resize(count);
  // Reservation grid: entry of each tile, (i, k) or (i, j, k), entries in lexicographic order.
  std::vector<int32_t> entry_of;
  std::vector<int32_t> entry_ijk;
  if (grid_mode) {
    std::vector<std::array<int32_t, 3>> keys(count);
    for (int t = 0; t < count; ++t)
      keys[t] = grid_mode == SPMM_RESERVE_3D ? std::array<int32_t, 3>{coords[3 * t], coords[3 * t + 1], coords[3 * t + 2]}
                                             : std::array<int32_t, 3>{coords[3 * t], 0, coords[3 * t + 2]};
    std::vector<std::array<int32_t, 3>> uniq(keys);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    entry_of.resize(count);
    for (int t = 0; t < count; ++t)
      entry_of[t] = (int32_t)(std::lower_bound(uniq.begin(), uniq.end(), keys[t]) - uniq.begin());
    b->n_entries = (int)uniq.size();
    // an entry's coordinates: those of its first tile (for 2D, j of that tile; unused)
    entry_ijk.assign(3 * uniq.size(), 0);
    for (int t = count - 1; t >= 0; --t)
      for (int c = 0; c < 3; ++c) entry_ijk[3 * entry_of[t] + c] = coords[3 * t + c];
  }
  auto body = [&]() -> spmm_status {
    std::vector<spmm::BatchTileDev> bt(count);
    struct Costed {
      double cost;
      spmm::BatchItem it;
    };
    std::vector<Costed> items;
    std::vector<spmm::BatchItem> fix;
    int64_t part = 0;
    std::vector<int32_t> rp;
    std::vector<spmm::Seg> segs;
    for (int t = 0; t < count; ++t) {
      const spmm_tile_s* A = tiles[t];
      spmm::BatchTileDev& d = bt[t];
      d.rowptr = A->t[0].rowptr;
      d.colind = A->t[0].colind;
      d.values = A->t[0].values;
      d.seg = A->plan.seg;
      d.lrow = A->plan.lrow;
      d.rows = A->rows;
      d.N = N[t];
      d.long_row = A->plan.long_row;
      d.ldp = (int32_t)partial_ld(N[t]);
      d.part_off = part;
      part += (int64_t)d.ldp * A->plan.n_seg;
      batch_variant(A, N[t], dt, &d, &b->variants[t]);
      const int64_t wrow = d.kind == 0 ? 64 * d.V : (int64_t)d.G * 4;  // row-split items: 4 elements per lane
      const int64_t wunit = 64 * d.V;
      const int nw_rows = (int)((N[t] + wrow - 1) / wrow);
      const int nw_unit = (int)((N[t] + wunit - 1) / wunit);
      // Costs from the row pointer (host copy) and the unit list.
      rp.resize((size_t)A->rows + 1);
      HIP_TRY(hipMemcpyAsync(rp.data(), A->t[0].rowptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost, s));
      segs.resize((size_t)A->plan.n_seg);
      if (A->plan.n_seg > 0)
        HIP_TRY(hipMemcpyAsync(segs.data(), A->plan.seg, sizeof(spmm::Seg) * segs.size(), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      // Rows per item: about item_target non-zeros of work (so that the waves of the
      // GPU share few tiles at a time), a whole number of row groups, at most 64 rows.
      int64_t nz_short = 0, rows_short = 0;
      for (int64_t r = 0; r < A->rows; ++r) {
        const int64_t l = (int64_t)rp[r + 1] - rp[r];
        if (l <= d.long_row) {
          nz_short += l;
          ++rows_short;
        }
      }
      const double avg = rows_short ? (double)nz_short / (double)rows_short : 1.0;
      const int unit_rows = d.kind == 0 ? 1 : 64 / d.G;
      int rpi = 64;
      while (rpi > unit_rows && rpi * std::max(avg, 1.0) > item_target) rpi /= 2;
      for (int64_t r0 = 0; r0 < A->rows; r0 += rpi) {
        const int64_t r1 = std::min<int64_t>(A->rows, r0 + rpi);
        int64_t nz = 0;
        for (int64_t r = r0; r < r1; ++r) {
          const int64_t l = (int64_t)rp[r + 1] - rp[r];
          if (l <= d.long_row) nz += l;
        }
        for (int w = 0; w < nw_rows; ++w) {
          const double width = (double)std::min<int64_t>(wrow, N[t] - w * wrow);
          items.push_back({(double)(nz + (r1 - r0)) * width, spmm::BatchItem{t, (int32_t)r0, w, (int32_t)((r1 - r0) << 8)}});
        }
      }
      for (int64_t si = 0; si < A->plan.n_seg; ++si)
        for (int w = 0; w < nw_unit; ++w) {
          const double width = (double)std::min<int64_t>(wunit, N[t] - w * wunit);
          items.push_back({(double)(segs[si].p1 - segs[si].p0) * width, spmm::BatchItem{t, (int32_t)si, w, 1}});
        }
      for (int64_t r = 0; r < A->plan.n_long; ++r)
        for (int w = 0; w < nw_unit; ++w) fix.push_back(spmm::BatchItem{t, (int32_t)r, w, 2});
    }
    if ((int64_t)items.size() >= ((int64_t)1 << 32)) return fail(SPMM_ERR_UNSUPPORTED, "work list too long");
    // Order: tiles by descending total cost; inside a tile, column window by column
    // window, split-row units first (longest first), then the row items in row order.  Keeping a tile's items
    // together keeps its B resident in the caches while the waves work on it;
    // big tiles first leave the small ones to fill the end of the launch.
    std::vector<double> tile_cost(count, 0.0);
    for (const auto& c : items) tile_cost[c.it.tile] += c.cost;
    std::vector<int> rank(count);
    {
      std::vector<int> order(count);
      for (int t = 0; t < count; ++t) order[t] = t;
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tile_cost[x] > tile_cost[y]; });
      for (int i = 0; i < count; ++i) rank[order[i]] = i;
    }
    // item class: stream V -> log2 V; row-split G -> 3 + log2(G / 8); unit V -> 7 + log2 V
    auto log2i = [](int v) { int l = 0; while ((1 << l) < v) ++l; return l; };
    auto cls = [&](const spmm::BatchItem& it) {
      const spmm::BatchTileDev& d = bt[it.tile];
      if ((it.type & 255) == 1) return spmm::kClassUnit + log2i(d.V);
      if (d.kind == 0) return log2i(d.V);
      return spmm::kClassRowsplit + log2i(d.G / 8);
    };
    std::stable_sort(items.begin(), items.end(), [&](const Costed& x, const Costed& y) {
      const int cx = cls(x.it), cy = cls(y.it);
      if (cx != cy && !b->single) return cx < cy;  // one launch per class: class by class
      if (grid_mode) {  // entry by entry; inside an entry, its products in j order
        const int ex = entry_of[x.it.tile], ey = entry_of[y.it.tile];
        if (ex != ey) return ex < ey;
        const int jx = coords[3 * x.it.tile + 1], jy = coords[3 * y.it.tile + 1];
        if (jx != jy) return jx < jy;
        if (x.it.tile != y.it.tile) return x.it.tile < y.it.tile;
      }
      if (x.it.tile != y.it.tile) return rank[x.it.tile] < rank[y.it.tile];
      // one column window at a time: the waves then share that window's slice of B
      if (x.it.window != y.it.window) return x.it.window < y.it.window;
      if ((x.it.type & 255) != (y.it.type & 255)) return (x.it.type & 255) > (y.it.type & 255);  // units first
      if ((x.it.type & 255) == 1) return x.cost > y.cost;
      return false;                                               // rows keep their order
    });
    std::vector<spmm::BatchItem> list(items.size());
    unsigned present = 0u;
    for (size_t i = 0; i < items.size(); ++i) {
      list[i] = items[i].it;
      b->class_cnt[cls(list[i])] += 1;
      present |= 1u << cls(list[i]);
    }
    b->class_mask = spmm::single_mask_for(present);
    for (int c = 1; c < spmm::kBatchClasses; ++c) b->class_off[c] = b->class_off[c - 1] + b->class_cnt[c - 1];
    b->n_items = (int64_t)list.size();
    b->n_fix = (int64_t)fix.size();
    b->ws_bytes = sizeof(float) * (size_t)part;
    if (dalloc(&b->d_tiles, count) != hipSuccess || dalloc(&b->d_items, b->n_items) != hipSuccess ||
        dalloc(&b->d_fix, b->n_fix) != hipSuccess ||
        (b->persistent && !b->single && dalloc(&b->d_counter, spmm::kBatchCounters) != hipSuccess) ||
        (b->single && dalloc(&b->d_c64, (int64_t)spmm::kClaimSlices * spmm::kCounter64Stride) != hipSuccess))
      return fail(SPMM_ERR_ALLOC, "device allocation of the batch failed");
    if (b->single && b->n_items >= ((int64_t)1 << 31))
      return fail(SPMM_ERR_UNSUPPORTED, "work list too long for the single-launch form");
    HIP_TRY(hipMemcpyAsync(b->d_tiles, bt.data(), sizeof(spmm::BatchTileDev) * bt.size(), hipMemcpyHostToDevice, s));
    if (b->n_items)
      HIP_TRY(hipMemcpyAsync(b->d_items, list.data(), sizeof(spmm::BatchItem) * list.size(), hipMemcpyHostToDevice, s));
    if (b->n_fix)
      HIP_TRY(hipMemcpyAsync(b->d_fix, fix.data(), sizeof(spmm::BatchItem) * fix.size(), hipMemcpyHostToDevice, s));
    if (b->d_counter) HIP_TRY(hipMemsetAsync(b->d_counter, 0, sizeof(unsigned) * spmm::kBatchCounters, s));
    if (b->d_c64)
      HIP_TRY(hipMemsetAsync(b->d_c64, 0, sizeof(unsigned long long) * (size_t)spmm::kClaimSlices * spmm::kCounter64Stride,
                             s));
    HIP_TRY(hipStreamSynchronize(s));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (grid_mode) {
      std::vector<int32_t> eoff(b->n_entries + 1, 0);
      for (const auto& it : list) eoff[entry_of[it.tile] + 1] += 1;
      for (int e = 0; e < b->n_entries; ++e) eoff[e + 1] += eoff[e];
      if (dalloc(&b->d_entry_off, b->n_entries + 1) != hipSuccess ||
          dalloc(&b->d_entry_ijk, 3 * (int64_t)b->n_entries) != hipSuccess ||
          dalloc(&b->d_counterE, (int64_t)b->n_entries * spmm::kCounterStride) != hipSuccess)
        return fail(SPMM_ERR_ALLOC, "device allocation of the reservation grid failed");
      HIP_TRY(hipMemcpyAsync(b->d_entry_off, eoff.data(), sizeof(int32_t) * eoff.size(), hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(b->d_entry_ijk, entry_ijk.data(), sizeof(int32_t) * entry_ijk.size(), hipMemcpyHostToDevice,
                             s));
      HIP_TRY(hipStreamSynchronize(s));
      // resident workgroups, a multiple of the XCD count so every XCD has workers
      const int64_t full = (int64_t)cus * spmm::batch_reserve_blocks_per_cu(dt, b->class_mask);
      b->single_grid = (int)std::max<int64_t>(spmm::kXcds, full - full % spmm::kXcds);
      return SPMM_OK;
    }
    if (b->single) {
      // resident workgroups of the union kernel (persistent), at most one wave per item
      const int64_t full = (int64_t)cus * spmm::batch_single_blocks_per_cu(dt, b->class_mask);
      const int64_t need = (b->n_items + spmm::kBlock / 64 - 1) / (spmm::kBlock / 64);
      b->single_grid = (int)std::max<int64_t>(1, std::min(full, need));
      return SPMM_OK;
    }
    int occ[spmm::kBatchClasses] = {};
    if (b->persistent) spmm::batch_blocks_per_cu(dt, occ);
    for (int c = 0; c < spmm::kBatchClasses; ++c) {
      const int64_t waves = (int64_t)(spmm::kBlock / 64);
      if (b->persistent) {
        if (b->class_cnt[c] >= ((int64_t)1 << 31))
          return fail(SPMM_ERR_UNSUPPORTED, "work list too long for 32-bit claim counters");
        // resident workgroups, at most one wave per claim chunk: small classes launch small grids
        const int64_t full = (int64_t)cus * std::max(1, occ[c]);
        const int64_t need = (b->class_cnt[c] + waves * spmm::kClaimChunk - 1) / (waves * spmm::kClaimChunk);
        b->class_grid[c] = (int)std::max<int64_t>(1, std::min(full, need));
      } else {
        const int64_t need = (b->class_cnt[c] + waves - 1) / waves;  // one wave per item
        if (need * spmm::kBlock >= ((int64_t)1 << 32))
          return fail(SPMM_ERR_UNSUPPORTED, "work list too long for one launch per class");
        b->class_grid[c] = (int)std::max<int64_t>(1, need);
      }
    }
    return SPMM_OK;
  };
  spmm_status st = spmm::guarded(body);
  if (st != SPMM_OK) {
    delete b;
    return st;
  }
  *out = b;
  return SPMM_OK;
}

}  // namespace

extern "C" {

spmm_status spmm_batch_create(int count, const spmm_tile_t* tiles, const int64_t* N, spmm_dtype dtype,
                              int64_t item_nnz, unsigned flags, void* stream, spmm_batch_t* out) {
  spmm::TraceRange trace_range("spmm_batch_create");
  return batch_create_impl(count, tiles, N, dtype, item_nnz, flags, nullptr, 0, stream, out);
}

spmm_status spmm_batch_create_grid(int count, const spmm_tile_t* tiles, const int64_t* N, spmm_dtype dtype,
                                   const int32_t* coords, int mode, int64_t item_nnz, void* stream, spmm_batch_t* out) {
  spmm::TraceRange trace_range("spmm_batch_create_grid");
  if (!out) return fail(SPMM_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (mode != SPMM_RESERVE_2D && mode != SPMM_RESERVE_3D && mode != SPMM_RESERVE_OWN)
    return fail(SPMM_ERR_INVALID_ARG, "unknown reservation mode %d", mode);
  if (!coords) return fail(SPMM_ERR_INVALID_ARG, "coords is null");
  for (int t = 0; t < count; ++t)
    for (int c = 0; c < 3; ++c)
      if (coords[3 * t + c] < 0) return fail(SPMM_ERR_INVALID_ARG, "tile %d: negative grid coordinate", t);
  return batch_create_impl(count, tiles, N, dtype, item_nnz, SPMM_BATCH_SINGLE | SPMM_BATCH_PERSISTENT, coords, mode,
                           stream, out);
}

spmm_status spmm_batch_destroy(spmm_batch_t batch) {
  if (!batch) return fail(SPMM_ERR_INVALID_ARG, "batch is null");
  delete batch;
  return SPMM_OK;
}

spmm_status spmm_batch_workspace_bytes(spmm_batch_t batch, size_t* bytes) {
  if (!batch || !bytes) return fail(SPMM_ERR_INVALID_ARG, "null argument");
  *bytes = batch->ws_bytes;
  return SPMM_OK;
}

spmm_status spmm_batch_get_variant(spmm_batch_t batch, int t, spmm_variant* out) {
  if (!batch || !out) return fail(SPMM_ERR_INVALID_ARG, "null argument");
  if (t < 0 || t >= batch->count) return fail(SPMM_ERR_INVALID_ARG, "tile index %d out of range", t);
  *out = batch->variants[t];
  return SPMM_OK;
}

spmm_status spmm_batched(spmm_batch_t batch, const void* const* B, const int64_t* ldb, void* const* C,
                         const int64_t* ldc, int accumulate, void* workspace, size_t ws_bytes, void* stream) {
  spmm::TraceRange trace_range("spmm_batched");
  if (!batch) return fail(SPMM_ERR_INVALID_ARG, "batch is null");
  if (!B || !ldb || !C || !ldc) return fail(SPMM_ERR_INVALID_ARG, "operand arrays must be device arrays, not null");
  if (batch->ws_bytes > 0) {
    if (!workspace || ws_bytes < batch->ws_bytes)
      return fail(SPMM_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", batch->ws_bytes,
                  workspace ? ws_bytes : 0);
    if (reinterpret_cast<uintptr_t>(workspace) % 16) return fail(SPMM_ERR_WORKSPACE, "workspace must be 16-byte aligned");
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != batch->device) return fail(SPMM_ERR_INVALID_ARG, "current device differs from the batch's");
  spmm::BatchParams P{};
  P.tiles = batch->d_tiles;
  P.items = batch->d_items;
  P.n_items = batch->n_items;
  P.fix = batch->d_fix;
  P.n_fix = batch->n_fix;
  P.B = B;
  P.ldb = ldb;
  P.C = C;
  P.ldc = ldc;
  P.partial = static_cast<float*>(workspace);
  P.counter = batch->d_counter;
  P.accumulate = accumulate ? 1 : 0;
  if (batch->grid_mode) {
    P.entry_off = batch->d_entry_off;
    P.entry_ijk = batch->d_entry_ijk;
    P.n_entries = batch->n_entries;
    P.grid_mode = batch->grid_mode;
    P.counterE = batch->d_counterE;
    HIP_TRY(spmm::launch_batch_reserve(P, batch->single_grid, batch->class_mask, batch->dt,
                                       static_cast<hipStream_t>(stream)));
    return SPMM_OK;
  }
  if (batch->single) {
    P.counter64 = batch->d_c64;
    HIP_TRY(spmm::launch_batch_single(P, batch->single_grid, batch->class_mask, batch->dt, batch->persistent,
                                      static_cast<hipStream_t>(stream)));
    return SPMM_OK;
  }
  HIP_TRY(spmm::launch_batch(P, batch->class_off, batch->class_cnt, batch->class_grid, batch->dt, batch->persistent,
                             static_cast<hipStream_t>(stream)));
  return SPMM_OK;
}

}  // extern "C"
