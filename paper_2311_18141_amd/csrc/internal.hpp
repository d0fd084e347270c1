// Internal declarations shared by the HIP translation units of libspmm.
// Nothing here is part of the public ABI (include/spmm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <exception>
#include <new>

#include "spmm.h"

namespace spmm {

constexpr int kMaxK = 16;      // k-tiles per tile row in one fused launch
// Largest non-zero count of a sparse operand: positions are int32, and the kernels step
// them by up to 1024 (a group, wave or workgroup width) while below the count, so the
// count keeps 2^16 of headroom under 2^31.
constexpr int64_t kMaxNnz = ((int64_t)1 << 31) - ((int64_t)1 << 16);
constexpr int kBlock = 256;    // threads per workgroup for every kernel here
// Grid cap for grid-stride kernels: a launch must stay below 2^32 threads.
constexpr int64_t kMaxGridBlocks = (int64_t)1 << 20;

enum class DT : int { F32 = 0, BF16 = 1 };

// Record the thread-local message spmm_last_error() returns; returns st.
spmm_status set_error(spmm_status st, const char* fmt, ...);

// A named roctx range around an entry point, for timelines from rocprofv3's marker
// trace: on only when the environment sets SPMM_TRACE (to anything but 0) and the
// roctx library can be opened; otherwise a range costs one predictable branch.
struct TraceRange {
  explicit TraceRange(const char* name);
  ~TraceRange();
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
  bool on;
};

// Runs f() and turns a C++ exception (a failed host allocation, in practice) into a
// status, so that no exception leaves an entry point of the C ABI.
template <typename F>
spmm_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return set_error(SPMM_ERR_ALLOC, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(SPMM_ERR_HIP, "unexpected error: %s", e.what());
  }
}
// Row-pointer and column-index checks of one CSR matrix (synchronous on s).
spmm_status validate_csr(const int32_t* rowptr, const int32_t* colind, int64_t rows, int64_t cols, int64_t nnz,
                         hipStream_t s);

// One k-tile as the forward kernels see it.
struct TileDev {
  const int32_t* rowptr;
  const int32_t* colind;  // column indices; an entry with bit 31 set names staged row (bit 31 cleared) of `hot`
  const float* values;
  const void* B;         // dense operand rows for this tile's columns
  int64_t ldb;
  const void* hot;       // staged copies of this tile's most used B rows (forward only; else unused)
  int64_t ldh;           // row pitch of `hot` in elements
};

// Column indices at or above this bit pattern name a staged B row (the handle's tagged
// copy of colind; the caller's arrays never have it: indices are below 2^31).
constexpr uint32_t kHotTag = 0x80000000u;

// A split work unit: row, k-tile, [p0, p1) in that tile's CSR positions.
struct Seg {
  int32_t row, k, p0, p1;
};

// A split row: row, and its units [s0, s1) in the unit list.
struct LongRow {
  int32_t row, s0, s1, pad;
};

struct FwdParams {
  TileDev t[kMaxK];
  int num_k;
  int k_offset;          // normalised to [0, num_k)
  int64_t rows;
  int64_t N;
  void* C;
  int64_t ldc;
  int accumulate;
  int32_t long_row;      // rows with combined length > long_row are done by units + fix-up
  const Seg* seg;
  int64_t n_seg;
  const LongRow* lrow;
  int64_t n_long;
  float* partial;        // n_seg x ldp FP32 partial sums
  int64_t ldp;
  int64_t row_blocks;    // workgroups of the row-split part (units come after)
  int32_t stream_rows;   // stream variant: rows per wave (1..64)
  int32_t hot;           // some k-tile reads staged hot rows (tagged colind)
};

// Kernel variant: G lanes per row (group), V elements per lane per load;
// stream = one wave streams the non-zeros of 64 consecutive rows (G = 64).
struct Variant {
  int G;
  int V;
  bool stream = false;
  int rows = 64;  // stream: rows per wave
};

// ---- launchers (defined in the .hip files) --------------------------------
hipError_t launch_fwd(const FwdParams& P, Variant v, DT dt, hipStream_t s);

// ---- hot-row staging (hot.hip) ----------------------------------------------
// Per call: copy the staged B rows of every k-tile into the workspace block
// `dst` (slots of k-tile k at [off[k], off[k+1]), row pitch ldh_bytes), so that the
// forward reads them from contiguous, evenly spread addresses.
struct HotStageParams {
  const void* B[kMaxK];
  int64_t ldb_bytes[kMaxK];
  int64_t off[kMaxK + 1];
  int num_k;
  const int32_t* src;      // B row of each slot
  char* dst;
  int64_t ldh_bytes;
  int64_t row_bytes;       // N * element size
};
hipError_t launch_hot_stage(const HotStageParams& P, int width_bytes, hipStream_t s);
// cnt[c] += occurrences of column c in colind[0, nnz) (cnt zeroed by the caller;
// structure.hip).
hipError_t launch_count_columns(const int32_t* colind, int64_t nnz, int32_t* cnt, hipStream_t s);
// out[p] = slot_of[colind[p]] >= 0 ? kHotTag | slot_of[colind[p]] : colind[p].
hipError_t launch_tag_hot(const int32_t* colind, int64_t nnz, const int32_t* slot_of, int32_t* out, hipStream_t s);

// ---- batched persistent launch (batch.hip) --------------------------------
struct BatchTileDev {
  const int32_t* rowptr;
  const int32_t* colind;
  const float* values;
  const Seg* seg;          // the tile's split-row units
  const LongRow* lrow;     // the tile's split rows
  int64_t rows;
  int64_t N;
  int64_t part_off;        // FP32 offset of this tile's partial rows in the workspace
  int32_t long_row;
  int32_t kind;            // 0 stream, 1 row-split
  int32_t G;               // row-split lanes per row
  int32_t V;               // stream / unit / fix-up vector width
  int32_t ldp;             // partial row pitch (floats)
  int32_t pad;
};

// type & 255 = 0: rows [a, a + (type >> 8)) of `tile` (at most 64), column window `window`;
// 1: split-row unit a; 2: split row a (fix-up).
struct BatchItem {
  int32_t tile, a, window, type;
};

struct BatchParams {
  const BatchTileDev* tiles;
  const BatchItem* items;
  int64_t n_items;
  const BatchItem* fix;
  int64_t n_fix;
  const void* const* B;    // device array: B[t]
  const int64_t* ldb;      // device array
  void* const* C;          // device array: C[t]
  const int64_t* ldc;      // device array
  float* partial;
  unsigned* counter;       // persistent mode: the class's kClaimSlices claim counters
  int accumulate;
  // Single-launch form (every class in one kernel): per-XCD claim counters, 64-bit and
  // never reset (see batch_union).
  unsigned long long* counter64;
  // Reservation-grid hand-out (the single-GPU form of Algorithm 3's work grids): the list is
  // grouped into n_entries entries (items [entry_off[e], entry_off[e + 1])), entry e with
  // grid coordinates entry_ijk[3e..3e+2] and a claim counter counterE[e * kCounterStride],
  // zeroed by a reset kernel before each call.
  const int32_t* entry_off;
  const int32_t* entry_ijk;
  int32_t n_entries;
  int32_t grid_mode;       // SPMM_RESERVE_*
  unsigned* counterE;
};
// 64-bit claim counters of the single-launch form, 32 apart (one 256-byte line each).
constexpr int kCounter64Stride = 32;
// The single-launch form: every item of the list (tile by tile) by one kernel that
// switches on the item's class, then, when some tile has split rows, the fix-up launch.
// persistent = false: one wave per item (grid = ceil(n_items / 4)); true: `grid`
// resident workgroups claiming from per-XCD slices.
// `mask` (one of the kMask* below) selects the kernel instance that holds just the item
// classes of the batch.
hipError_t launch_batch_single(const BatchParams& P, int grid, unsigned mask, DT dt, bool persistent, hipStream_t s);
int batch_single_blocks_per_cu(DT dt, unsigned mask);
// Reservation-grid hand-out: a reset kernel zeroes the entry counters, then `grid`
// resident workgroups claim items entry by entry in each worker's visiting order.
hipError_t launch_batch_reserve(const BatchParams& P, int grid, unsigned mask, DT dt, hipStream_t s);
int batch_reserve_blocks_per_cu(DT dt, unsigned mask);
// C = C + P_0 + ... + P_{n-1} (in that order, FP32 sums, one rounding for BF16); the
// partials go to the kernel kAccMax at a time.
constexpr int kAccMax = 16;
struct AccList {
  const void* p[kAccMax];
  int64_t ld[kAccMax];
  int n;
};
hipError_t launch_accumulate_n(void* C, int64_t ldc, const void* const* Pt, const int64_t* ldp, int n, int64_t rows,
                               int64_t N, DT dt, int V, hipStream_t s);
// Items a persistent wave claims with one fetch-and-add.
constexpr int kClaimChunk = 1;
// The chip's XCDs (each with its own L2); workgroups are dealt to them round-robin
// in workgroup-id order.
constexpr int kXcds = 8;
// Persistent mode splits each class's item list into kClaimSlices contiguous slices
// with a counter each (one per XCD), kCounterStride unsigned apart (one 256-byte
// line per counter); a batch holds kBatchClasses x kClaimSlices counters.
constexpr int kClaimSlices = kXcds;
constexpr int kCounterStride = 64;
// Item classes: stream V = 1, 2, 4 (0..2); row-split G = 8, 16, 32, 64 with V = 4 (3..6);
// split-row units with V = 1, 2, 4 (7..9).
constexpr int kClassRowsplit = 3;
constexpr int kClassUnit = 7;
constexpr int kBatchClasses = 10;
constexpr int kBatchCounters = kBatchClasses * kClaimSlices * kCounterStride;
// Class sets of the precompiled single-launch instances (bit c = item class c): stream
// V = 1, 2 or 4 with the units of the same V; every row-split class with every unit; all.
constexpr unsigned kMaskStream1 = (1u << 0) | (1u << kClassUnit);
constexpr unsigned kMaskStream2 = (1u << 1) | (1u << (kClassUnit + 1));
constexpr unsigned kMaskStream4 = (1u << 2) | (1u << (kClassUnit + 2));
constexpr unsigned kMaskRowsplit = (0xFu << kClassRowsplit) | (0x7u << kClassUnit);
constexpr unsigned kMaskAll = (1u << kBatchClasses) - 1u;
// The narrowest of those sets that contains `present`.
inline unsigned single_mask_for(unsigned present) {
  for (unsigned m : {kMaskStream1, kMaskStream2, kMaskStream4, kMaskRowsplit})
    if ((present & ~m) == 0u) return m;
  return kMaskAll;
}
// One launch per item class present (off/cnt: the class's slice of the item list;
// grid: its workgroups), then the fix-up.  persistent = false: one wave per item;
// true: `grid` resident workgroups claim kClaimChunk items at a time from the
// class's counters (reset by a kernel first, so graph replays start clean).
hipError_t launch_batch(const BatchParams& P, const int64_t* off, const int64_t* cnt, const int* grid, DT dt,
                        bool persistent, hipStream_t s);
void batch_blocks_per_cu(DT dt, int* out);

struct SddmmParams {
  const int32_t* rowid;
  const int32_t* colind;
  int64_t nnz;
  const void* dC;          // FP32 or BF16, as the launch's dtype
  int64_t lddc;
  const void* B;
  int64_t ldb;
  int64_t N;
  float* dA;
  int64_t c_begin, c_end;  // column range of this launch
  int accumulate;          // add to dA (later slices)
};
// Fused backward over the transposed structure (one pass gathers each dC row once for
// both gradients): for every row j of A^T (column j of A), with B[j, :] held in
// registers, each entry q (original row i = colindT[q], position p = perm[q]) gives
//   dA[p] = <dC[i, :], B[j, :]>   and   dB[j, :] += values[p] * dC[i, :].
// Rows of A^T longer than long_row are cut into the transposed plan's units, whose dB
// partial rows go to `partial` and are summed by the forward's fix-up.
struct BwdFusedParams {
  const int32_t* rowptrT;
  const int32_t* colindT;
  const int32_t* perm;
  const float* values;     // A's values in A's CSR order (read through perm)
  const void* dC;          // rows x N, FP32 or BF16 as the launch's dtype
  int64_t lddc;
  const void* B;           // cols x N
  int64_t ldb;
  float* dA;               // nnz, A's CSR order
  void* dB;                // cols x N
  int64_t lddb;
  int64_t cols;            // rows of A^T
  int64_t N;
  int32_t long_row;
  const Seg* seg;          // transposed plan's split units
  int64_t n_seg;
  float* partial;          // n_seg x ldp
  int64_t ldp;
  int32_t n_win;           // column windows of G * V columns (blockIdx.y); 1: dA stored directly
  int64_t nnz;
  float* dA_part;          // n_win > 1: n_win x nnz partial dot products, transposed order
};
// G lanes per row of A^T, V columns per lane and load, n_win windows of G * V columns,
// U entries in flight; with n_win > 1 the partial dot products are then summed into dA.

hipError_t launch_bwd_fused(const BwdFusedParams& P, int G, int V, int U, DT dt, hipStream_t s);
// The forward's split-row fix-up alone (sums each split row's unit partials into C),
// with G * V columns per group.
hipError_t launch_fixup(const FwdParams& P, int G, int V, DT dt, hipStream_t s);

// out[q] = values[perm[q]] for q < nnz.
hipError_t launch_gather_values(const int32_t* perm, const float* values, float* out, int64_t nnz, hipStream_t s);
// G lanes per group, V columns per lane and load, U non-zeros per group.
hipError_t launch_sddmm(const SddmmParams& P, int G, int V, int U, DT dt, hipStream_t s);
hipError_t launch_accumulate(void* C, int64_t ldc, const void* Pt, int64_t ldp, int64_t rows, int64_t N, DT dt,
                             int V, hipStream_t s);

// Structure utilities (utils.hip).
hipError_t launch_validate_rowptr(const int32_t* rowptr, int64_t rows, int64_t nnz, uint32_t* status,
                                  hipStream_t s);
hipError_t launch_validate_colind(const int32_t* rowptr, const int32_t* colind, int64_t rows,
                                  int64_t cols, uint32_t* status, hipStream_t s);

struct PlanCountParams {
  const int32_t* rowptr[kMaxK];
  int num_k;
  int64_t rows;
  int32_t long_row;
  int32_t segment;
  int32_t* nseg;          // per row
  int32_t* islong;        // per row
  unsigned long long* stats;  // [0] max row, [1] empty rows, [2..34] log2 histogram
};
hipError_t launch_plan_count(const PlanCountParams& P, hipStream_t s);

struct PlanEmitParams {
  const int32_t* rowptr[kMaxK];
  int num_k;
  int64_t rows;
  int32_t segment;
  const int32_t* nseg;
  const int32_t* seg_off;
  const int32_t* islong;
  const int32_t* long_off;
  Seg* seg;
  LongRow* lrow;
};
hipError_t launch_plan_emit(const PlanEmitParams& P, hipStream_t s);

// Exclusive scan of n int32 values; total (nullable, device) receives the sum.
// temp must hold scan_temp_elems(n) int32 values.
int64_t scan_temp_elems(int64_t n);
hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* total, int32_t* temp,
                          hipStream_t s);

// Transposed structure by a stable LSD radix sort of (colind, position).
int64_t transpose_temp_bytes(int64_t rows, int64_t cols, int64_t nnz);
hipError_t build_transpose(const int32_t* rowptr, const int32_t* colind, int64_t rows, int64_t cols,
                           int64_t nnz, int32_t* rowid, int32_t* rowptrT, int32_t* colindT, int32_t* perm,
                           void* temp, hipStream_t s);

}  // namespace spmm
