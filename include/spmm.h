/*
 * spmm.h -- C ABI of the MI355X (gfx950) local sparse-times-dense multiply.
 *
 * The operation is the local tile product that every GPU runs inside the
 * stationary-C algorithm of Brock, Buluc and Yelick, "RDMA-Based Algorithms
 * for Sparse Matrix Multiplication on GPUs" (ICS'24):
 *
 *     C_ij  =  C_ij  +  sum over k of  A_ik * B_kj          (Section 2.1)
 *
 * with the owner of C(i,j) walking k' = 0..K-1 and multiplying tile
 * k = (k' + offset) mod K (Section 3.3, Algorithm 2), A's tiles in CSR
 * (values, row pointer, column indices; Section 3.1 and Section 5.2) with FP32
 * values and 32-bit indices (Section 6).  The gradient pass, BF16 storage of
 * the dense operands and the batched launch are additions of this library.
 *
 * Conventions shared by every entry point:
 *   - Pointers documented "device" point to GPU memory of the current HIP
 *     device; "host" pointers to CPU memory.  The caller owns every buffer it
 *     passes in; buffers handed to spmm_tile_create must outlive the handle.
 *   - Dense matrices are row-major with a leading dimension (in elements)
 *     >= their width.  A B_k row is one contiguous run of N elements.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     spmm_fwd, spmm_bwd and spmm_batched only enqueue work: no host
 *     synchronisation, no device allocation, so they can be captured in a
 *     HIP graph.  Creation and destruction calls are synchronous.
 *   - With SPMM_TRACE set (to anything but 0) in the environment, the main entry
 *     points (tile and batch creation, spmm_fwd, spmm_bwd, spmm_batched,
 *     spmm_tile_accumulate, spgemm_create, spgemm_compute) each open a roctx range
 *     named after themselves, for rocprofv3's marker trace; the roctx library is
 *     loaded on the first range, and without it tracing stays off.
 *   - Every function returns an spmm_status; nothing is thrown across the ABI.
 *     Argument checks finish before any HIP call.  spmm_last_error() returns a
 *     thread-local message describing the most recent failure.
 *   - Values are read live on every call: a handle caches structure only
 *     (pattern, transposed pattern, work plans), never values, so changes to
 *     `values` between calls take effect without re-creating the handle.
 */
#ifndef SPMM_H
#define SPMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPMM_OK = 0,
  SPMM_ERR_INVALID_ARG = 1,  /* null pointer, negative size, ld < width, bad enum ... */
  SPMM_ERR_BAD_CSR = 2,      /* validation found a malformed CSR tile */
  SPMM_ERR_UNSUPPORTED = 3,  /* valid request the library does not implement */
  SPMM_ERR_WORKSPACE = 4,    /* workspace pointer null or smaller than required */
  SPMM_ERR_HIP = 5,          /* a HIP runtime call failed; see spmm_last_error() */
  SPMM_ERR_ALLOC = 6         /* host or device allocation failed (creation calls only) */
} spmm_status;

typedef enum { SPMM_F32 = 0, SPMM_BF16 = 1 } spmm_dtype;

/* One CSR tile A_ik of a tile row. */
typedef struct {
  int64_t cols;            /* columns of the tile = rows of its dense operand B_k */
  int64_t nnz;             /* stored entries; at most 2^31 - 2^16 (int32 positions, with headroom
                              for the kernels' strides) */
  const int32_t* rowptr;   /* device, rows+1 entries, rowptr[0] = 0, rowptr[rows] = nnz */
  const int32_t* colind;   /* device, nnz entries, tile-local, strictly increasing per row */
  const float* values;     /* device, nnz entries, FP32; read on every call */
} spmm_csr;

/* Flags for spmm_tile_opts.flags. */
#define SPMM_TILE_VALIDATE 1u   /* check the CSR invariants on the device; SPMM_ERR_BAD_CSR on failure */
#define SPMM_TILE_TRANSPOSE 2u  /* also build the transposed structure needed by spmm_bwd (needs num_k = 1) */

typedef struct {
  unsigned flags;
  int32_t long_row;        /* rows whose length over all k-tiles exceeds this are split across
                              work units with a deterministic fix-up; 0 = library default
                              (128, doubled while below twice the mean row length); at most
                              33,554,431 ((2^31 - 1) / 64), else INVALID_ARG */
  int32_t segment;         /* minimum non-zeros per split work unit (a row of length L gets units
                              of max(segment, ceil(sqrt(L)))); 0 = library default (64) */
  int32_t bwd_slice;       /* spmm_bwd computes dA in column slices of this width, one launch
                              per slice, so a slice of B can stay cache-resident (the two-pass
                              backward: no fused pass while a slice narrower than N is set);
                              0 = one launch */
  int32_t hot_rows;        /* hot-row staging of the forward: the B rows of each k-tile's most used
                              columns are copied on every spmm_fwd call into one contiguous block of
                              the workspace and read there (the handle keeps a copy of colind with
                              those entries tagged; results are bit-identical).  -1 = off; 0 =
                              library rule (up to one row per 128 columns of a k-tile of <= 2^27
                              columns, at least 16384 and at most 65536 rows, each
                              used >= 16 times, for tiles of >= 2^20 non-zeros, where they serve
                              >= 1/8 of the k-tile's non-zeros and >= 8x their share of its
                              columns); n > 0 = up to n most used columns of every k-tile
                              (n <= 2^24), no further test.  Staging rows needs workspace (see
                              spmm_fwd_workspace_bytes); the handle's staging choice holds for
                              every N and dtype. */
} spmm_tile_opts;

/* Opaque handle to one tile row (A_i0 ... A_i,K-1): the sparse operand of one C
   tile's stationary-C loop.  A single tile is the case K = 1. */
typedef struct spmm_tile_s* spmm_tile_t;

/* Structural statistics gathered at creation (Section 6 defines load
   imbalance as max/avg non-zeros; these are the per-row analogues). */
typedef struct {
  int64_t rows, num_k, nnz_total;
  int64_t max_row;           /* longest row, non-zeros summed over the k-tiles */
  int64_t empty_rows;        /* rows with no non-zero in any k-tile */
  int64_t long_rows;         /* rows handled by the split path */
  int64_t segments;          /* split work units */
  int64_t hist_log2[33];     /* rows by bit length of their combined length (0 = empty) */
  int64_t nnz_per_k[16];
  int64_t has_transpose;
  int64_t long_rows_t, segments_t;   /* the same for the transposed structure */
  int64_t long_row, segment;         /* split threshold and unit length of the current plan */
  int64_t hot_rows;                  /* staged B rows over all k-tiles (0: staging off) */
  int64_t hot_nnz;                   /* non-zeros that read a staged row */
} spmm_tile_stats;

/*
 * Create a tile-row handle from num_k (1..16) CSR tiles that share `rows`.
 * Builds, on `stream`, the work plan for the row-split and split-row paths
 * and, with SPMM_TILE_TRANSPOSE, the transposed structure (rowptrT, colindT,
 * perm) by a stable sort on column index.  Synchronous.  The library allocates
 * the handle's own device memory here (released by spmm_tile_destroy); the
 * tile arrays stay owned by the caller and must outlive the handle.
 * Errors: INVALID_ARG (null/negative/num_k out of range), BAD_CSR (with VALIDATE),
 * UNSUPPORTED (TRANSPOSE with num_k > 1, nnz > 2^31 - 2^16), ALLOC, HIP.
 */
spmm_status spmm_tile_create(int64_t rows, int num_k, const spmm_csr* tiles /* host, num_k */,
                             const spmm_tile_opts* opts /* host, nullable */, void* stream,
                             spmm_tile_t* out /* host */);
spmm_status spmm_tile_destroy(spmm_tile_t tile);
spmm_status spmm_tile_get_stats(spmm_tile_t tile, spmm_tile_stats* out /* host */);

/*
 * Copy the transposed structure of a K = 1 handle into caller buffers (device):
 * rowptrT[cols+1], colindT[nnz] (original row of each entry), perm[nnz]
 * (original CSR position).  Entries of one output row are ordered by
 * increasing original row.  Asynchronous on `stream`.  Errors: INVALID_ARG,
 * UNSUPPORTED (handle built without SPMM_TILE_TRANSPOSE), HIP.
 */
spmm_status spmm_tile_export_transpose(spmm_tile_t tile, int32_t* rowptrT, int32_t* colindT,
                                       int32_t* perm, void* stream);

/* Forward kernel variants.  A handle keeps one variant per (N, dtype); without an
   entry the library picks by a fixed rule.  FP32: column windows of 64 columns (256
   bytes of each B row), of 128 for N >= 256 and, on tiles with more than 1/8 empty
   rows, for N a multiple of 128; the stream kernel on tiles with more than 1/8 empty
   rows and a full-wave row-split group otherwise.  BF16: full-wave row-split groups
   over the fewest windows of at most 256 columns, each on the narrowest vector that
   gives that count (at N = 64, the stream kernel on tiles with more than 1/8 empty
   rows).  Below N = 64: the row-split group that covers N with the widest aligned
   vector.  These entry points exist for tuning and
   tests; results of every variant agree within the tolerance of the operation (and
   bit-for-bit on integer-valued inputs). */
#define SPMM_KERNEL_AUTO 0
#define SPMM_KERNEL_ROWSPLIT 1   /* a group of `lanes` lanes owns one row and a column window */
#define SPMM_KERNEL_STREAM 2     /* a wave streams the non-zeros of `lanes` (4..64) consecutive rows */
#define SPMM_KERNEL_FUSED 3      /* backward only: dA and dB in one pass over the transposed structure,
                                    `lanes` lanes per row of A^T and column window of lanes x vec columns */
typedef struct {
  int32_t kind;    /* SPMM_KERNEL_* */
  int32_t lanes;   /* ROWSPLIT: lanes per row; STREAM: rows per wave; 4..64, power of two;
                      0 = library choice */
  int32_t vec;     /* elements per lane per load: 1, 2, 4 (and 8 for BF16); 0 = widest aligned */
  int32_t depth;   /* FUSED only: entries of a row of A^T in flight per group, 1, 2, 4 or 8 (at
                      most `lanes`); 0 = library choice (4 FP32, 2 BF16); must be 0 for the other kinds */
} spmm_variant;

/* Set (v != NULL) or clear (v == NULL) the variant used for width N and `dtype`.
   A variant whose vector width does not fit a call's alignment, or whose column
   windows (lanes x vec columns each) would number more than 65535, falls back to the
   library's choice for that call.  Errors: INVALID_ARG (bad field values, table of
   16 entries full). */
spmm_status spmm_tile_set_variant(spmm_tile_t tile, int64_t N, spmm_dtype dtype, const spmm_variant* v);

/* Read back the entry for width N and `dtype` of the forward's variant table (bwd = 0)
   or of the backward's dB-pass table (bwd = 1): the variant set by spmm_tile_set_variant,
   spmm_tile_set_bwd_variant or an autotuner, or kind SPMM_KERNEL_AUTO when there is
   none.  With the setters it lets a caller keep autotuned choices (for instance in a
   file) and apply them to a later handle of the same structure.  Errors: INVALID_ARG. */
spmm_status spmm_tile_get_variant(spmm_tile_t tile, int64_t N, spmm_dtype dtype, int32_t bwd,
                                  spmm_variant* out /* host */);

/* Shape of the backward's sampled dense-dense kernel (dA on A's pattern; a gradient
   pass this library adds, not a kernel of the paper) at width N: groups of
   `lanes` lanes (4, 8, 16, 32, 64), each owning `nnz_per_group` consecutive non-zeros
   (1, 2, 4, 8; at most `lanes`).  lanes = 0 clears the entry (library choice).  Results
   do not depend on the shape beyond FP32 summation order within a dot product.
   Errors: INVALID_ARG (bad values, table of 8 entries full). */
spmm_status spmm_tile_set_sddmm_variant(spmm_tile_t tile, int64_t N, int32_t lanes, int32_t nnz_per_group);

/* Time the forward variants (and, with tune_plan != 0, split thresholds, which
   rebuilds the handle's split-row plan) on the caller's real operands and keep the
   fastest for (N, dtype).  Synchronous; allocates its own scratch; overwrites C.
   After it returns, query spmm_fwd_workspace_bytes again (the plan may have
   changed).  `chosen` (nullable) receives the winner.  Errors: as spmm_fwd, ALLOC. */
spmm_status spmm_tile_autotune(spmm_tile_t tile, int64_t N, spmm_dtype dtype, const void* const* B,
                               const int64_t* ldb, void* C, int64_t ldc, int tune_plan, void* stream,
                               spmm_variant* chosen /* host */);

/* Workspace (device bytes) spmm_fwd needs for this handle at width N: FP32 partial
   rows of the split-row units, plus, with hot-row staging, 4 * ceil8(N) bytes per
   staged row (after a 256-byte boundary).  Calls that share a workspace must not
   overlap. */
spmm_status spmm_fwd_workspace_bytes(spmm_tile_t A, int64_t N, size_t* bytes /* host */);

/*
 * Forward local SpMM over a tile row (Section 2.1; k order of Algorithm 2):
 *   C = [accumulate ? C : 0] + sum_{k'=0}^{K-1} A_k B_k,   k = (k' + k_offset) mod K.
 * B: host array of K device pointers; B[k] is cols_k x N row-major with leading
 * dimension ldb[k] (host array).  C: device, rows x N, leading dimension ldc.
 * dtype: (F32, F32) or (BF16, BF16) for (B, C); products and sums are FP32 and
 * a BF16 C is rounded once (nearest-even) at the store.  1 <= N <= 64 x 65535
 * (4,194,240: one launch walks the column windows of 64 or more columns in its grid's
 * second dimension).  Asynchronous.
 * Errors: INVALID_ARG, UNSUPPORTED (mixed dtypes, N > 4,194,240), WORKSPACE, HIP.
 */
spmm_status spmm_fwd(spmm_tile_t A, int k_offset, const void* const* B, const int64_t* ldb,
                     spmm_dtype b_dtype, void* C, int64_t ldc, spmm_dtype c_dtype, int64_t N,
                     int accumulate, void* workspace, size_t ws_bytes, void* stream);

/*
 * The forward without a workspace, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results as spmm_fwd (bit for bit); the scratch spmm_fwd
 * takes as `workspace` (split-row partial rows, staged hot rows) is instead a fixed
 * device array of spmm_noalloc_scratch_bytes() bytes (64 MiB) per GPU, which the
 * library holds from its load until the process ends; its address on each device is
 * looked up on the first call made there.  The call allocates nothing and makes no
 * allocating library call.  Every call on one GPU shares that GPU's array, so calls
 * that overlap on one GPU (other streams, other threads) race and must not be made;
 * the array keeps the last call's contents, none of which a later call reads before
 * writing.  Errors: as spmm_fwd, and WORKSPACE when spmm_fwd_workspace_bytes(A, N)
 * exceeds the array (use spmm_fwd with a workspace then).
 */
spmm_status spmm_fwd_noalloc(spmm_tile_t A, int k_offset, const void* const* B, const int64_t* ldb,
                             spmm_dtype b_dtype, void* C, int64_t ldc, spmm_dtype c_dtype, int64_t N, int accumulate,
                             void* stream);
size_t spmm_noalloc_scratch_bytes(void);

/* The backward keeps its own variant per (N, dtype), set here (v != NULL) or cleared
   (v == NULL; the library rule then applies).  Kind SPMM_KERNEL_FUSED selects the fused
   backward (when spmm_bwd is asked for both dA and dB): a group of `lanes` lanes owns one
   row of A^T with `vec` columns per lane, in column windows of lanes x vec columns when
   that is less than N (at most min(8, ceil(N / 256)) windows; 0 = library choice; a
   shape that does not fit a call's alignment or needs more windows falls back to the
   library's).
   Kinds ROWSPLIT and STREAM select the two-pass backward (SDDMM for dA, then the forward
   kernels over the transposed structure for dB) and name the dB pass's kernel.  Without
   an entry the fused backward runs whenever the operands' alignment allows at most 8
   windows of at least 256 columns (or one group covers N).
   Results of every variant agree as the forward's do (dB bit-identical between the fused
   and two-pass forms at the same vector width and split plan; dA within FP32 summation
   order).  Errors: INVALID_ARG (bad field values, table of 16 entries full). */
spmm_status spmm_tile_set_bwd_variant(spmm_tile_t tile, int64_t N, spmm_dtype dtype, const spmm_variant* v);

/* Time the backward's variants on the caller's operands for a K = 1 handle built with
   SPMM_TILE_TRANSPOSE and keep the fastest for (N, dtype): dC (rows x N, ld lddc), dB
   (cols x N, ld lddb) and, when B (cols x N, ld ldb) and dA (nnz FP32) are both given, the
   whole backward (fused shapes and the two-pass form with each dB-pass kernel) through
   spmm_bwd; with B or dA NULL only the dB pass's kernels (dB alone).  Synchronous;
   allocates its own scratch; overwrites dB (and dA).  `chosen` (nullable) receives the
   winner.  Errors: INVALID_ARG, UNSUPPORTED (no transpose, num_k > 1, ld too large),
   ALLOC, HIP. */
spmm_status spmm_tile_autotune_bwd(spmm_tile_t tile, int64_t N, spmm_dtype dtype, const void* dC, int64_t lddc,
                                   const void* B /* nullable */, int64_t ldb, float* dA /* nullable */, void* dB,
                                   int64_t lddb, void* stream, spmm_variant* chosen /* host */);

/* Workspace (device bytes) spmm_bwd needs for this handle at width N when dB is
   wanted: FP32 partial rows of the transposed plan's split rows plus 4 x min(8, max(1,
   ceil(N / 256))) bytes per non-zero (A's values gathered into the transposed order by
   the two-pass form, or the fused form's partial dot products, one per column window). */
spmm_status spmm_bwd_workspace_bytes(spmm_tile_t A, int64_t N, size_t* bytes /* host */);

/*
 * Backward of C = A B for a K = 1 handle built with SPMM_TILE_TRANSPOSE, given
 * dC = dL/dC (device, rows x N, ld lddc) and B (device, cols x N, ld ldb), both in
 * `dtype` (FP32, or BF16 for the backward of a BF16 forward):
 *   dA_values[p] = sum_n dC[i, n] * B[colind[p], n]   for p in row i   (FP32; nullable: skipped)
 *   dB = A^T dC   (device, cols x N, ld lddb, in `dtype`; nullable: skipped)
 * Products and sums are FP32; a BF16 dB is rounded once (RNE) at the store.  dA is
 * on A's pattern, in A's CSR order; no gradient flows to the pattern.  The gradient
 * pass is not in the paper: it is this library's addition (the forward's adjoint).
 * With both outputs wanted (and no column slices set), one pass over the transposed
 * structure gathers each dC row once for both (see SPMM_KERNEL_FUSED; wider than one
 * group, in column windows whose partial dot products a small kernel sums
 * into dA in window order); otherwise dA is a sampled dense-dense product in A's order
 * and dB a pass of the forward kernels.
 * 1 <= N <= 4,194,240, as for spmm_fwd.  Asynchronous; no allocation and no host
 * synchronisation, so a call can be captured in a HIP graph.  Errors: INVALID_ARG,
 * UNSUPPORTED (no transpose, num_k > 1, ld too large, N too large), WORKSPACE, HIP.
 */
spmm_status spmm_bwd(spmm_tile_t A, const void* dC, int64_t lddc, const void* B, int64_t ldb, int64_t N,
                     spmm_dtype dtype, float* dA_values, void* dB, int64_t lddb, void* workspace,
                     size_t ws_bytes, void* stream);

/*
 * Batched launch: many independent single-tile products C_t = [C_t] + A_t B_t in
 * one launch per kernel class present in the batch (a class is one kernel shape:
 * stream V, row-split G, or split-row unit V), plus, when some tile has split rows,
 * a fix-up launch.  The batch form and its load balancing are additions of this
 * library; they stand in, on one GPU, for the work claiming of Section 3.4 (a remote
 * fetch-and-add per work item, Algorithm 3).
 *
 * spmm_batch_create builds, synchronously, the work list: items of up to 64 rows
 * of one tile and one column window, holding about `item_nnz` non-zeros (0: 256;
 * else 64..1048576), and the split-row units of each tile's plan, with each tile's
 * kernel variant taken from its handle's entry for (N_t, dtype) (set by
 * spmm_tile_autotune or spmm_tile_set_variant) or from a fixed rule.  Items are
 * ordered tile by tile (largest first) and column window by column window.
 * `flags`: 0 = one wave per item, handed out by the hardware dispatcher in list
 * order; SPMM_BATCH_PERSISTENT = resident workgroups (#CU x occupancy) whose waves
 * claim one item at a time with a fetch-and-add on device counters (each class's
 * list cut into one contiguous slice per XCD with its own counter; a wave drains its
 * XCD's slice, then the others; a reset kernel runs first).  SPMM_BATCH_SINGLE (alone
 * or with SPMM_BATCH_PERSISTENT) = one launch for every item of the batch: one kernel
 * runs every class, switching per item, over a work list ordered tile by tile regardless
 * of class (followed by the fix-up launch when some tile has split rows); with
 * SPMM_BATCH_PERSISTENT its resident workgroups claim items from one contiguous slice
 * of the whole list per XCD, stealing from the others when theirs is drained, with
 * 64-bit claim counters that are never reset (each call advances them by a known
 * amount), so no reset launch is needed, graph replays included.  All forms give
 * identical results.  Every tile must be a single-tile handle
 * (num_k = 1) on the current device, and must outlive the batch.  The batch
 * allocates its own device memory (work list; claim counters when persistent).
 * Errors: INVALID_ARG, UNSUPPORTED (num_k > 1, work list too long; single launch: 2^31
 * items or more), ALLOC, HIP.
 */
#define SPMM_BATCH_PERSISTENT 1u
#define SPMM_BATCH_SINGLE 2u
typedef struct spmm_batch_s* spmm_batch_t;
spmm_status spmm_batch_create(int count, const spmm_tile_t* tiles /* host, count */,
                              const int64_t* N /* host, count */, spmm_dtype dtype, int64_t item_nnz,
                              unsigned flags, void* stream, spmm_batch_t* out /* host */);
spmm_status spmm_batch_destroy(spmm_batch_t batch);
/* Workspace (device bytes) spmm_batched needs: FP32 partial rows of split rows. */
spmm_status spmm_batch_workspace_bytes(spmm_batch_t batch, size_t* bytes /* host */);
/* The variant the batch uses for tile t (kind STREAM or ROWSPLIT; lanes, vec). */
spmm_status spmm_batch_get_variant(spmm_batch_t batch, int t, spmm_variant* out /* host */);

/*
 * A batch whose items are handed out through a reservation grid, the single-GPU form
 * of the work-stealing algorithms' work grids (Section 3.4, Algorithm 3).  Tile t of
 * the batch is one component product C(i,j) (+)= A(i,k) B(k,j); coords[3t..3t+2]
 * (host) = (i, j, k).  `mode`:
 *   SPMM_RESERVE_2D  grid over (i, k): the entry of a stationary tile A(i,k) hands out,
 *                    one fetch-and-add per item, the items of its products in j order
 *                    ("the next piece of work of that tile"); workers take their own
 *                    entries, then steal from every other entry in cyclic order
 *                    (random work stealing);
 *   SPMM_RESERVE_3D  grid over (i, j, k), one entry per product: workers take the
 *                    entries of their C tile, then those sharing their A tile, then
 *                    their B tile, then the rest (locality-aware work stealing);
 *   SPMM_RESERVE_OWN grid over (i, k), own entries only (no stealing).
 * Workers are the waves of #CU x occupancy resident workgroups; their own entries
 * follow their XCD (with E entries, E >= 8: XCD x owns the x-th eighth; fewer: entry
 * x E / 8).  Each call zeroes the grid's counters with a reset kernel, then runs one
 * kernel for every item class (and the fix-up launch when some tile has split rows, as
 * with SPMM_BATCH_SINGLE).  Results are bit-identical to the other batch forms.  A tile
 * handle may appear several times (the same A(i,k) against each B(k,j)).  item_nnz as
 * for spmm_batch_create (items of at most 64 rows; larger items suit large tiles).
 * Errors: as spmm_batch_create, INVALID_ARG (bad coords or mode).
 */
#define SPMM_RESERVE_2D 1
#define SPMM_RESERVE_3D 2
#define SPMM_RESERVE_OWN 3
spmm_status spmm_batch_create_grid(int count, const spmm_tile_t* tiles /* host, count */,
                                   const int64_t* N /* host, count */, spmm_dtype dtype,
                                   const int32_t* coords /* host, 3 x count */, int mode, int64_t item_nnz,
                                   void* stream, spmm_batch_t* out /* host */);

/*
 * Run the batch: B, ldb, C, ldc are DEVICE arrays of `count` entries (pointers to
 * each tile's B_t (cols_t x N_t) and C_t (rows_t x N_t), row-major, in the batch's
 * dtype, and their leading dimensions).  Every row of every B_t and C_t must start
 * on a 16-byte boundary (base pointer and ld * element size multiples of 16); the
 * library cannot check device-resident arguments.  Asynchronous; no host
 * synchronisation, no allocation: capturable in a HIP graph (a persistent batch
 * resets its claim counters by a kernel on every replay; a single-launch batch needs
 * no reset).  Calls on one batch must not overlap (they share the claim counters and
 * the workspace; a persistent single-launch batch's counters also assume that every
 * earlier call ran to completion).  Errors: INVALID_ARG, WORKSPACE, HIP.
 */
spmm_status spmm_batched(spmm_batch_t batch, const void* const* B, const int64_t* ldb, void* const* C,
                         const int64_t* ldc, int accumulate, void* workspace, size_t ws_bytes, void* stream);

/*
 * Dense partial-tile accumulate of the stationary-A algorithm (Section 3.2,
 * Algorithm 1): the owner of C(i,j) adds a partial product tile computed by the
 * owner of A(i,k):  C = C + Ptile.  C (device, rows x N, ld ldc) and Ptile (device,
 * rows x N, ld ldp) share `dtype`; the sum is formed in FP32 and a BF16 C is
 * rounded once.  Asynchronous.  Errors: INVALID_ARG, HIP.
 */
spmm_status spmm_tile_accumulate(void* C, int64_t ldc, const void* Ptile, int64_t ldp, int64_t rows, int64_t N,
                                 spmm_dtype dtype, void* stream);

/*
 * The owner's accumulate of several partial tiles (Algorithm 3's queue of partial
 * products, drained in order):  C = C + P_0 + ... + P_{n-1}, summed in FP32 in that
 * order; a BF16 C is rounded once per 16 partials.  P (host array of n device
 * pointers) and ldp (host, n) describe the partials, rows x N each, in `dtype`.
 * Asynchronous.  Errors: INVALID_ARG, HIP.
 */
spmm_status spmm_tile_accumulate_n(void* C, int64_t ldc, const void* const* P, const int64_t* ldp, int n,
                                   int64_t rows, int64_t N, spmm_dtype dtype, void* stream);

/*
 * Local sparse-times-sparse product C = A B (CSR x CSR -> CSR): the local step of
 * the paper's SpGEMM experiments (Section 6.2 computes C = A A with the same
 * distributed algorithms, each GPU multiplying pairs of sparse tiles; Section 4
 * bounds the local product's arithmetic intensity by its compression factor).
 *
 * A is M x A->cols, B is A->cols x B->cols; both canonical CSR (int32 indices,
 * FP32 values, strictly increasing columns per row; SPMM_TILE_VALIDATE checks it),
 * device arrays owned by the caller that must outlive the plan; their row pointers and
 * column indices must not change while it lives (the plan is built from them), their
 * values may.
 *
 * spgemm_create analyses the structure and runs the symbolic product,
 * synchronously: products per row, C's entries per row and C's row pointer
 * (kept in the plan), and allocates the plan's own device memory (row lists;
 * dense accumulators for long rows, zeroed).  C's pattern is structural: (i, j) is
 * present when some product a_ip * b_pj exists, even if the sum is zero.
 * spgemm_info returns nnz(C) and the number of products (2 x products = flops).
 * spgemm_rowptr copies C's row pointer (M + 1 int32) to a device buffer.
 * spgemm_compute writes C's column indices (sorted within each row) and values
 * (FP32 sums; their order of summation inside a row is not fixed, so the last bits
 * may differ between calls) into device buffers of nnz(C) entries, reading A's
 * and B's values live; asynchronous, no allocation, no host synchronisation.
 * Calls on one plan must not overlap (they share the dense accumulators).
 *
 * The plan keeps C's column indices (4 bytes per entry of C, indexed like C, allocated
 * at creation) when the rows they cover hold at least a quarter of C and the array
 * takes at most a quarter of the free device memory; flag SPGEMM_BITMAP_ONLY keeps
 * none.  They cover every row except the long rows (more entries than the largest
 * workgroup table holds: 4,096 or 8,192, by the LDS left beside a bitmap over C's
 * columns) that go without a split table of B (binary-searched windows, or dense rows
 * for a very wide B).  The first compute call finds the columns with hash tables,
 * sorts and bitmaps, as every call does without a kept pattern, and copies them into
 * the plan at its end; later calls add each product of a covered row into its sum
 * with one LDS atomic (found by binary search over the row's kept columns, or at its
 * column in the window's sums) and write the entries in the kept order.  A call made
 * while its stream is being captured into a graph keeps nothing (its copy would run
 * only at replay), so the first call outside capture does.  The results are the same
 * either way.  spgemm_pattern_entries returns how many entries of C the plan keeps
 * (0: none).
 * Errors: INVALID_ARG, BAD_CSR (with SPMM_TILE_VALIDATE), UNSUPPORTED (nnz > 2^31 - 2^16,
 * C with >= 2^31 entries), ALLOC, HIP.
 */
#define SPGEMM_BITMAP_ONLY 16u  /* spgemm_create: keep no column pattern; every compute call finds the columns */
typedef struct spgemm_s* spgemm_t;
spmm_status spgemm_create(int64_t M, const spmm_csr* A /* host */, const spmm_csr* B /* host */, unsigned flags,
                          void* stream, spgemm_t* out /* host */);
spmm_status spgemm_destroy(spgemm_t plan);
spmm_status spgemm_info(spgemm_t plan, int64_t* nnz_c /* host, nullable */, int64_t* products /* host, nullable */);
spmm_status spgemm_pattern_entries(spgemm_t plan, int64_t* entries /* host */);
spmm_status spgemm_rowptr(spgemm_t plan, int32_t* rowptrC /* device, M + 1 */, void* stream);
spmm_status spgemm_compute(spgemm_t plan, int32_t* colindC /* device, nnz(C) */, float* valuesC /* device */,
                           void* stream);

/*
 * Gather micro-benchmark (a measurement aid beside the method, not a step of it):
 * the forward's memory access without its arithmetic.  For i in [0, n), the row
 * idx[i] of `table` (device, rows x row_bytes bytes, 16-byte aligned) is read whole
 * with 16-byte vector loads, several rows in flight per wave; indices outside
 * [0, rows) are skipped.  *out (device, one word) receives the XOR of every 32-bit
 * word read (order-free, so a CPU can check it).  Timing a call over a table that
 * fits a cache level gives that level's ceiling for such gathers.  row_bytes: a
 * multiple of 16 up to 1024, or of 1024 up to 4096.  Asynchronous.
 * Errors: INVALID_ARG, HIP.
 */
spmm_status spmm_gather_probe(const void* table, int64_t rows, int64_t row_bytes, const int32_t* idx /* device */,
                              int64_t n, uint32_t* out /* device */, void* stream);

const char* spmm_status_string(spmm_status status);
const char* spmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPMM_H */
