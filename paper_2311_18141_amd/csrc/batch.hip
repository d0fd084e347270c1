// Batched local SpMM: many independent single-tile products C_t = A_t B_t in a
// handful of launches, one per kernel class present in the batch (so that every
// class runs with its own register allocation).  The host builds a work list of
// items (up to 64 rows of one tile and one column window, or one split-row unit),
// tile by tile (largest tiles first) and window by window, so that the waves share
// one slice of one tile's B in the caches at a time.
//
// Two ways to hand items to waves:
//  * flat (default): one wave per item; the hardware dispatcher hands out
//    workgroups as CUs free up, which is the dynamic load balancing.
//  * persistent: #CU x occupancy resident workgroups; each wave claims kClaimChunk
//    consecutive items with one fetch-and-add on a device counter (the single-GPU
//    form of claiming work with a remote fetch-and-add) until the list is drained.
//    The list is cut into one contiguous slice per XCD, each with its own counter:
//    a wave claims from its XCD's slice, then from the others in turn, and asks for
//    its next chunk before it works through the current one.  On the 512-tile
//    uneven batch, contiguous per-XCD slices ran 1.26x faster than chunks dealt to
//    the counters in turn, and one item per claim 1.34x faster than eight.
// Workgroups are dealt to the XCDs round-robin, so in the flat mode every XCD takes
// every eighth item and all of them work on the same few tiles at any time.
// Items write disjoint output rows (split rows: disjoint partial rows) and every
// row is summed in CSR order by one wave, so the result does not depend on which
// wave runs which item; split rows are finished by a second, fix-up launch.
#include <algorithm>

#include "elem.hpp"
#include "fwd_common.hpp"
#include "internal.hpp"

namespace spmm {
namespace {

template <typename E>
struct Ops {
  using T = typename E::T;
  const T* B;
  int64_t ldb;
  T* C;
  int64_t ldc;
};

template <typename E>
__device__ __forceinline__ Ops<E> item_ops(const BatchParams& P, int t) {
  Ops<E> o;
  o.B = static_cast<const typename E::T*>(P.B[t]);
  o.ldb = P.ldb[t];
  o.C = static_cast<typename E::T*>(P.C[t]);
  o.ldc = P.ldc[t];
  return o;
}

template <int V, typename E, bool ACC>
__device__ __forceinline__ void store_c(typename E::T* c, float (&acc)[V]) {
  if constexpr (ACC) {
    float old[V];
    load_vec<E, V>(c, old);
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] += old[e];
  }
  store_vec<E, V>(c, acc);
}

// Rows [r0, r0+nrows) (nrows <= 64) of one tile, streamed by the whole wave (see fwd_stream).
template <int V, typename E, bool ACC>
__device__ __forceinline__ void item_stream(const BatchTileDev& bt, const Ops<E>& op, int64_t r0, int nrows, int window,
                                            int32_t* s_pref, int32_t* s_beg) {
  using T = typename E::T;
  constexpr int U = V >= 8 ? 4 : 8;
  const int lane = threadIdx.x & 63;
  const int64_t c0 = (int64_t)window * (64 * V) + (int64_t)lane * V;
  const bool active = c0 < bt.N;
  const int64_t cl = active ? c0 : 0;
  const int64_t row = r0 + lane;
  const bool inrow = lane < nrows && row < bt.rows;
  int32_t b = 0, L = 0;
  if (inrow) {
    b = bt.rowptr[row];
    L = bt.rowptr[row + 1] - b;
  }
  const int32_t Ls = (L > bt.long_row) ? 0 : L;
  int32_t incl = Ls;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  s_pref[lane] = incl - Ls;
  if (lane == 63) s_pref[64] = incl;
  s_beg[lane] = b;
  const int32_t total = __builtin_amdgcn_readlane(incl, 63);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  float acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = 0.0f;
  if constexpr (!ACC) {
    uint64_t em = __ballot(inrow && L == 0);
    while (em) {
      const int i = __ffsll((long long)em) - 1;
      em &= em - 1;
      if (active) store_vec<E, V>(op.C + (r0 + i) * op.ldc + c0, acc);
    }
  }
  const uint64_t ldbb = (uint64_t)(op.ldb * (int64_t)sizeof(T));
  const uint64_t base = reinterpret_cast<uint64_t>(op.B);
  const uint64_t coff = (uint64_t)(cl * (int64_t)sizeof(T));  // this lane's columns, added after the broadcast
  for (int32_t qc = 0; qc < total; qc += 64) {
    const int n = min(64, total - qc);
    const int32_t q = qc + lane;
    int ri = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
      const int cand = ri + step;
      if (cand <= 63 && s_pref[cand] <= q) ri = cand;
    }
    uint64_t addr = 0;
    float val = 0.0f;
    int end = 0;
    if (lane < n) {
      const int32_t p = s_beg[ri] + (q - s_pref[ri]);
      const uint32_t col = (uint32_t)__builtin_nontemporal_load(bt.colind + p);
      val = __builtin_nontemporal_load(bt.values + p);
      addr = base + (uint64_t)col * ldbb;
      end = (q + 1 == s_pref[ri + 1]) ? 1 : 0;
    }
    const uint32_t alo = (uint32_t)addr, ahi = (uint32_t)(addr >> 32);
    auto issue = [&](float (&bv)[U][V], int u0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int jj = min(u0 + u, n - 1);
        const uint64_t a = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)ahi, jj) << 32) |
                           (uint32_t)__builtin_amdgcn_readlane((int)alo, jj);
        load_vec_at<E, V>(a + coff, bv[u]);
      }
    };
    auto consume = [&](const float (&bv)[U][V], int u0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int jj = min(u0 + u, n - 1);
        const bool ok = u0 + u < n;
        const float v = ok ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(val), jj)) : 0.0f;
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] = fmaf(v, ok ? bv[u][e] : 0.0f, acc[e]);
        if (ok && __builtin_amdgcn_readlane(end, jj)) {
          const int r = __builtin_amdgcn_readlane(ri, jj);
          if (active) store_c<V, E, ACC>(op.C + (r0 + r) * op.ldc + c0, acc);
#pragma unroll
          for (int e = 0; e < V; ++e) acc[e] = 0.0f;
        }
      }
    };
    float bA[U][V], bB[U][V];
    issue(bA, 0);
    for (int u0 = 0;;) {
      if (u0 + U < n) issue(bB, u0 + U);
      consume(bA, u0);
      u0 += U;
      if (u0 >= n) break;
      if (u0 + U < n) issue(bA, u0 + U);
      consume(bB, u0);
      u0 += U;
      if (u0 >= n) break;
    }
  }
}

// Rows [r0, r0+nrows) of one tile, 64/G rows at a time, G lanes per row.
template <int G, int V, typename E, bool ACC>
__device__ __forceinline__ void item_rowsplit(const BatchTileDev& bt, const Ops<E>& op, int64_t r0, int nrows,
                                              int window) {
  using T = typename E::T;
  constexpr int GPW = 64 / G;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int64_t c0 = (int64_t)window * (G * V) + (int64_t)gl * V;
  const bool active = c0 < bt.N;
  const int64_t cl = active ? c0 : 0;
  TileDev t;
  t.rowptr = bt.rowptr;
  t.colind = bt.colind;
  t.values = bt.values;
  t.B = op.B;
  t.ldb = op.ldb;
  t.hot = op.B;  // batches read the caller's colind: no tagged entries
  t.ldh = op.ldb;
  const char* brow = reinterpret_cast<const char*>(op.B) + cl * (int64_t)sizeof(T);
  const uint32_t ldbb = (uint32_t)(op.ldb * (int64_t)sizeof(T));
  // the item's row extents, loaded once: lane l holds rows r0 + l (nrows <= 64)
  int32_t my_p0 = 0, my_p1 = 0;
  if (lane < nrows && r0 + lane < bt.rows) {
    my_p0 = bt.rowptr[r0 + lane];
    my_p1 = bt.rowptr[r0 + lane + 1];
  }
  for (int rr = 0; rr < nrows; rr += GPW) {
    const int64_t row = r0 + rr + lane / G;
    const bool inrow = rr + lane / G < nrows && row < bt.rows;
    const int src = (rr + lane / G) & 63;
    int32_t p0 = __builtin_amdgcn_ds_bpermute(src << 2, my_p0);
    int32_t p1 = __builtin_amdgcn_ds_bpermute(src << 2, my_p1);
    if (!inrow) p1 = p0;
    const bool split = p1 - p0 > bt.long_row;
    if (split) p1 = p0;
    float acc[V];
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] = 0.0f;
    accumulate_range<G, V, E>(t, p0, p1, brow, ldbb, gl, acc);
    if (inrow && !split && active) store_c<V, E, ACC>(op.C + row * op.ldc + c0, acc);
  }
}

// One split-row unit: partial sum over [p0, p1) into the workspace (full wave).
template <int V, typename E>
__device__ __forceinline__ void item_unit(const BatchParams& P, const BatchTileDev& bt, const Ops<E>& op,
                                          int s, int window) {
  using T = typename E::T;
  const int lane = threadIdx.x & 63;
  const int64_t c0 = (int64_t)window * (64 * V) + (int64_t)lane * V;
  const bool active = c0 < bt.N;
  const int64_t cl = active ? c0 : 0;
  TileDev t;
  t.rowptr = bt.rowptr;
  t.colind = bt.colind;
  t.values = bt.values;
  t.B = op.B;
  t.ldb = op.ldb;
  t.hot = op.B;  // batches read the caller's colind: no tagged entries
  t.ldh = op.ldb;
  const Seg d = bt.seg[s];
  float acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = 0.0f;
  accumulate_range<64, V, E>(t, d.p0, d.p1, reinterpret_cast<const char*>(op.B) + cl * (int64_t)sizeof(T),
                             (uint32_t)(op.ldb * (int64_t)sizeof(T)), lane, acc);
  if (active) store_f32v<V>(P.partial + bt.part_off + (int64_t)s * bt.ldp + c0, acc);
}

template <typename E, bool ACC, int CLS>
__device__ __forceinline__ void run_item(const BatchParams& P, int64_t it, int32_t* s_pref, int32_t* s_beg) {
  const BatchItem item = P.items[it];
  const BatchTileDev& bt = P.tiles[item.tile];
  const Ops<E> op = item_ops<E>(P, item.tile);
  const int nrows = item.type >> 8;
  if constexpr (CLS < kClassRowsplit) {
    item_stream<1 << CLS, E, ACC>(bt, op, item.a, nrows, item.window, s_pref, s_beg);
  } else if constexpr (CLS < kClassUnit) {
    item_rowsplit<8 << (CLS - kClassRowsplit), 4, E, ACC>(bt, op, item.a, nrows, item.window);
  } else {
    item_unit<1 << (CLS - kClassUnit), E>(P, bt, op, item.a, item.window);
  }
}

// One claim of kClaimChunk items from slice s (lane 0's fetch-and-add, broadcast).
__device__ __forceinline__ unsigned claim(unsigned* counter, int s, int lane) {
  unsigned c = 0;
  if (lane == 0) c = atomicAdd(counter + (int64_t)s * kCounterStride, (unsigned)kClaimChunk);
  return (unsigned)__builtin_amdgcn_readlane((int)c, 0);
}

// One kernel per item class and hand-out mode.
template <typename E, bool ACC, int CLS, bool PERSIST>
__global__ void __launch_bounds__(kBlock) batch_class(BatchParams P) {
  __shared__ int32_t s_mem[(kBlock / 64) * 129];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  int32_t* s_pref = s_mem + w * 129;
  int32_t* s_beg = s_pref + 65;
  if constexpr (PERSIST) {
    // slice s = items [n s / S, n (s + 1) / S); start on this XCD's slice, then visit
    // the others in turn; a wave leaves after finding every slice drained
    int s = (int)(blockIdx.x % kClaimSlices);
    int visited = 1;
    unsigned got = claim(P.counter, s, lane);
    for (;;) {
      const int64_t lo = P.n_items * s / kClaimSlices;
      const int64_t hi = P.n_items * (s + 1) / kClaimSlices;
      const int64_t base = lo + got;
      if (base >= hi) {
        if (visited == kClaimSlices) break;
        ++visited;
        s = (s + 1) % kClaimSlices;
        got = claim(P.counter, s, lane);
        continue;
      }
      const int64_t end = base + kClaimChunk < hi ? base + kClaimChunk : hi;
      got = claim(P.counter, s, lane);  // the next chunk, in flight during this one
      for (int64_t it = base; it < end; ++it) run_item<E, ACC, CLS>(P, it, s_pref, s_beg);
    }
  } else {
    (void)lane;
    const int64_t it = (int64_t)blockIdx.x * (kBlock / 64) + w;
    if (it < P.n_items) run_item<E, ACC, CLS>(P, it, s_pref, s_beg);
  }
}

// Split rows: C row = [C] + sum of the row's unit partials in CSR order.
template <int V, typename E, bool ACC>
__device__ __forceinline__ void fix_row(const BatchParams& P, const BatchTileDev& bt, const Ops<E>& op, int r,
                                        int window) {
  const int lane = threadIdx.x & 63;
  const int64_t c0 = (int64_t)window * (64 * V) + (int64_t)lane * V;
  if (c0 >= bt.N) return;
  const LongRow lr = bt.lrow[r];
  float acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = 0.0f;
  for (int s = lr.s0; s < lr.s1; ++s) {
    float x[V];
    load_f32v<V>(P.partial + bt.part_off + (int64_t)s * bt.ldp + c0, x);
#pragma unroll
    for (int e = 0; e < V; ++e) acc[e] += x[e];
  }
  store_c<V, E, ACC>(op.C + (int64_t)lr.row * op.ldc + c0, acc);
}

template <typename E, bool ACC>
__global__ void __launch_bounds__(kBlock) batch_fixup(BatchParams P) {
  const int64_t f = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (f >= P.n_fix) return;
  const BatchItem it = P.fix[f];
  const BatchTileDev& bt = P.tiles[it.tile];
  const Ops<E> op = item_ops<E>(P, it.tile);
  switch (bt.V) {
    case 1: fix_row<1, E, ACC>(P, bt, op, it.a, it.window); return;
    case 2: fix_row<2, E, ACC>(P, bt, op, it.a, it.window); return;
    default: fix_row<4, E, ACC>(P, bt, op, it.a, it.window); return;
  }
}

// Reset the claim counters inside the stream (a kernel, so that a captured graph
// resets them on every replay).
__global__ void __launch_bounds__(kBlock) batch_reset(unsigned* counter, int n) {
  for (int i = (int)threadIdx.x; i < n; i += kBlock) counter[i] = 0u;
}

// ---- Single-launch form ---------------------------------------------------------
// Every item class in one kernel: each item (one wave) switches, uniformly, to its
// class's code, so the whole batch is one launch, followed by the fix-up launch when
// some tile has split rows.  (Summing a split row in the same launch, by the unit that
// arrives last, needs an agent-scope release per unit, and on this GPU that writes back
// the XCD's L2 each time: on the R-MAT row block's 16 products, 1.29M units per call,
// it made the launch 5x slower than a separate fix-up launch.)
//
// The claim counters of the persistent hand-out are 64-bit and never reset, which keeps
// the items to one launch (graph replays included): every wave makes exactly one failed
// claim on each slice it visits (all of them), so every call adds exactly items + waves
// to a slice's counter and a claim's place in this call is its value modulo that.
// Calls on one batch must not overlap (they never could: they share the workspace).

__device__ __forceinline__ uint64_t claim64(unsigned long long* counter, int s, int lane) {
  unsigned long long c = 0;
  if (lane == 0) c = atomicAdd(counter + (int64_t)s * kCounter64Stride, 1ull);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)c, 0);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(c >> 32), 0);
  return ((uint64_t)hi << 32) | lo;
}

// MASK: the item classes a kernel instance contains (bit c = class c); the host picks the
// narrowest precompiled mask that covers the classes of its batch, since one kernel for
// every class holds the registers of the widest one.
template <typename E, bool ACC, unsigned MASK>
__device__ __forceinline__ void union_item(const BatchParams& P, int64_t it, int32_t* s_pref, int32_t* s_beg) {
  const BatchItem item = P.items[it];
  const BatchTileDev& bt = P.tiles[item.tile];
  const int type = item.type & 255;
  const int lv = bt.V == 4 ? 2 : (bt.V == 2 ? 1 : 0);
  int cls;
  if (type == 1)
    cls = kClassUnit + lv;
  else if (bt.kind == 0)
    cls = lv;
  else
    cls = kClassRowsplit + (bt.G == 8 ? 0 : (bt.G == 16 ? 1 : (bt.G == 32 ? 2 : 3)));
  switch (cls) {
    case 0: if constexpr ((MASK >> 0) & 1u) run_item<E, ACC, 0>(P, it, s_pref, s_beg); break;
    case 1: if constexpr ((MASK >> 1) & 1u) run_item<E, ACC, 1>(P, it, s_pref, s_beg); break;
    case 2: if constexpr ((MASK >> 2) & 1u) run_item<E, ACC, 2>(P, it, s_pref, s_beg); break;
    case 3: if constexpr ((MASK >> 3) & 1u) run_item<E, ACC, 3>(P, it, s_pref, s_beg); break;
    case 4: if constexpr ((MASK >> 4) & 1u) run_item<E, ACC, 4>(P, it, s_pref, s_beg); break;
    case 5: if constexpr ((MASK >> 5) & 1u) run_item<E, ACC, 5>(P, it, s_pref, s_beg); break;
    case 6: if constexpr ((MASK >> 6) & 1u) run_item<E, ACC, 6>(P, it, s_pref, s_beg); break;
    case 7: if constexpr ((MASK >> 7) & 1u) run_item<E, ACC, 7>(P, it, s_pref, s_beg); break;
    case 8: if constexpr ((MASK >> 8) & 1u) run_item<E, ACC, 8>(P, it, s_pref, s_beg); break;
    default: if constexpr ((MASK >> 9) & 1u) run_item<E, ACC, 9>(P, it, s_pref, s_beg); break;
  }
}

template <typename E, bool ACC, bool PERSIST, unsigned MASK>
__global__ void __launch_bounds__(kBlock) batch_union(BatchParams P) {
  __shared__ int32_t s_mem[(kBlock / 64) * 129];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  int32_t* s_pref = s_mem + w * 129;
  int32_t* s_beg = s_pref + 65;
  if constexpr (PERSIST) {
    const uint64_t waves = (uint64_t)gridDim.x * (kBlock / 64);
    int s = (int)(blockIdx.x % kClaimSlices);
    int visited = 1;
    uint64_t got = claim64(P.counter64, s, lane);
    for (;;) {
      const int64_t lo = P.n_items * s / kClaimSlices;
      const int64_t hi = P.n_items * (s + 1) / kClaimSlices;
      const int64_t it = lo + (int64_t)(got % ((uint64_t)(hi - lo) + waves));
      if (it >= hi) {
        if (visited == kClaimSlices) break;
        ++visited;
        s = (s + 1) % kClaimSlices;
        got = claim64(P.counter64, s, lane);
        continue;
      }
      got = claim64(P.counter64, s, lane);  // the next item, in flight during this one
      union_item<E, ACC, MASK>(P, (int64_t)__builtin_amdgcn_readfirstlane((int)it), s_pref, s_beg);
    }
  } else {
    const int64_t it = (int64_t)blockIdx.x * (kBlock / 64) + w;
    if (it < P.n_items) union_item<E, ACC, MASK>(P, (int64_t)__builtin_amdgcn_readfirstlane((int)it), s_pref, s_beg);
  }
}

// ---- Reservation-grid hand-out -------------------------------------------------
// The work-stealing algorithms of Section 3.4 (Algorithm 3) reserve work with a
// fetch-and-add on an element of a work grid: a 2-D grid over the stationary operand's
// tiles (i, k), whose counter hands out the next piece of work of that tile (here the
// next item: a row range and window of the next column block j, in j order), or, for
// locality-aware stealing, a 3-D grid over the products (i, j, k).  Workers (the waves
// of resident workgroups) do their own work first and then steal.  Ownership follows
// the XCD (workgroup b runs on XCD b mod 8): with E >= 8 entries XCD x owns the x-th
// eighth of them, with fewer, entry x E / 8, so an entry's workers share an L2.
//  * SPMM_RESERVE_2D: own entries, then every other entry in cyclic order (random stealing).
//  * SPMM_RESERVE_3D: entries sharing the first own entry's C tile (i, j), then its A tile
//    (i, k), then its B tile (k, j), then the rest, each pass in cyclic order.
//  * SPMM_RESERVE_OWN: own entries only (no stealing), the static assignment that
//    stealing is measured against.
__device__ __forceinline__ bool reserve_in_pass(const int32_t* ijk, int e, int e0, int pass) {
  const int i = ijk[3 * e], j = ijk[3 * e + 1], k = ijk[3 * e + 2];
  const int i0 = ijk[3 * e0], j0 = ijk[3 * e0 + 1], k0 = ijk[3 * e0 + 2];
  const bool c = i == i0 && j == j0, a = i == i0 && k == k0, b = k == k0 && j == j0;
  switch (pass) {
    case 0: return c;
    case 1: return a && !c;
    case 2: return b && !c && !a;
    default: return !c && !a && !b;
  }
}

template <typename E, bool ACC, unsigned MASK>
__global__ void __launch_bounds__(kBlock) batch_reserve(BatchParams P) {
  __shared__ int32_t s_mem[(kBlock / 64) * 129];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  int32_t* s_pref = s_mem + w * 129;
  int32_t* s_beg = s_pref + 65;
  const int ne = P.n_entries;
  const int x = (int)(blockIdx.x % kXcds);
  int own_lo, own_n;
  if (ne >= kXcds) {
    own_lo = (x * ne + kXcds - 1) / kXcds;
    own_n = ((x + 1) * ne + kXcds - 1) / kXcds - own_lo;
  } else {
    own_lo = x * ne / kXcds;
    own_n = 1;
  }
  const bool three_d = P.grid_mode == SPMM_RESERVE_3D;
  const int visit = P.grid_mode == SPMM_RESERVE_OWN ? own_n : ne;
  for (int pass = 0; pass < (three_d ? 4 : 1); ++pass) {
    for (int idx = 0; idx < visit; ++idx) {
      const int e = (own_lo + idx) % ne;
      if (three_d && !reserve_in_pass(P.entry_ijk, e, own_lo, pass)) continue;
      const int64_t lo = P.entry_off[e];
      const int64_t n = (int64_t)P.entry_off[e + 1] - lo;
      unsigned got = claim(P.counterE, e, lane);
      while ((int64_t)got < n) {
        const unsigned next = claim(P.counterE, e, lane);  // the next item, in flight during this one
        union_item<E, ACC, MASK>(P, (int64_t)__builtin_amdgcn_readfirstlane((int)(lo + got)), s_pref, s_beg);
        got = next;
      }
    }
  }
}

template <typename E, bool ACC, unsigned MASK>
hipError_t launch_reserve_m(const BatchParams& P, int grid, hipStream_t s) {
  const int nc = P.n_entries * kCounterStride;
  hipLaunchKernelGGL(batch_reset, dim3((unsigned)((nc + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, P.counterE, nc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((batch_reserve<E, ACC, MASK>), dim3((unsigned)grid), dim3(kBlock), 0, s, P);
  e = hipGetLastError();
  if (e != hipSuccess || P.n_fix == 0) return e;
  hipLaunchKernelGGL((batch_fixup<E, ACC>), dim3((unsigned)((P.n_fix + 3) / 4)), dim3(kBlock), 0, s, P);
  return hipGetLastError();
}

template <typename E, bool ACC>
hipError_t launch_reserve_t(const BatchParams& P, int grid, unsigned mask, hipStream_t s) {
  if (P.n_items == 0) return hipSuccess;
  switch (mask) {
    case kMaskStream1: return launch_reserve_m<E, ACC, kMaskStream1>(P, grid, s);
    case kMaskStream2: return launch_reserve_m<E, ACC, kMaskStream2>(P, grid, s);
    case kMaskStream4: return launch_reserve_m<E, ACC, kMaskStream4>(P, grid, s);
    case kMaskRowsplit: return launch_reserve_m<E, ACC, kMaskRowsplit>(P, grid, s);
    default: return launch_reserve_m<E, ACC, kMaskAll>(P, grid, s);
  }
}

// C += P_0 + ... + P_{n-1} over a rows x N block, in that order; one thread per V elements.
template <int V, typename E>
__global__ void __launch_bounds__(kBlock) accumulate_n_kernel(typename E::T* C, int64_t ldc, AccList L, int64_t rows,
                                                              int64_t N) {
  const int64_t per_row = N / V;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < rows * per_row; i += (int64_t)gridDim.x * kBlock) {
    const int64_t r = i / per_row, c = (i - r * per_row) * V;
    float x[V];
    load_vec<E, V>(C + r * ldc + c, x);
    for (int t = 0; t < L.n; ++t) {
      float y[V];
      load_vec<E, V>(static_cast<const typename E::T*>(L.p[t]) + r * L.ld[t] + c, y);
#pragma unroll
      for (int e = 0; e < V; ++e) x[e] += y[e];
    }
    store_vec<E, V>(C + r * ldc + c, x);
  }
}

template <typename E, bool ACC, unsigned MASK>
hipError_t launch_single_m(const BatchParams& P, int grid, bool persistent, hipStream_t s) {
  if (persistent)
    hipLaunchKernelGGL((batch_union<E, ACC, true, MASK>), dim3((unsigned)grid), dim3(kBlock), 0, s, P);
  else
    hipLaunchKernelGGL((batch_union<E, ACC, false, MASK>), dim3((unsigned)((P.n_items + 3) / 4)), dim3(kBlock), 0, s,
                       P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || P.n_fix == 0) return e;
  hipLaunchKernelGGL((batch_fixup<E, ACC>), dim3((unsigned)((P.n_fix + 3) / 4)), dim3(kBlock), 0, s, P);
  return hipGetLastError();
}

template <typename E, bool ACC>
hipError_t launch_single_t(const BatchParams& P, int grid, bool persistent, unsigned mask, hipStream_t s) {
  if (P.n_items == 0) return hipSuccess;
  switch (mask) {
    case kMaskStream1: return launch_single_m<E, ACC, kMaskStream1>(P, grid, persistent, s);
    case kMaskStream2: return launch_single_m<E, ACC, kMaskStream2>(P, grid, persistent, s);
    case kMaskStream4: return launch_single_m<E, ACC, kMaskStream4>(P, grid, persistent, s);
    case kMaskRowsplit: return launch_single_m<E, ACC, kMaskRowsplit>(P, grid, persistent, s);
    default: return launch_single_m<E, ACC, kMaskAll>(P, grid, persistent, s);
  }
}

template <typename E, unsigned MASK>
int occ_of(bool reserve) {
  int n = 0;
  const hipError_t e =
      reserve ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_reserve<E, false, MASK>, kBlock, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_union<E, false, true, MASK>, kBlock, 0);
  return (e == hipSuccess && n > 0) ? n : 2;
}

template <typename E>
int occ_mask(unsigned mask, bool reserve) {
  switch (mask) {
    case kMaskStream1: return occ_of<E, kMaskStream1>(reserve);
    case kMaskStream2: return occ_of<E, kMaskStream2>(reserve);
    case kMaskStream4: return occ_of<E, kMaskStream4>(reserve);
    case kMaskRowsplit: return occ_of<E, kMaskRowsplit>(reserve);
    default: return occ_of<E, kMaskAll>(reserve);
  }
}

template <typename E, bool ACC, int CLS>
hipError_t launch_class(const BatchParams& P, int grid, bool persistent, hipStream_t s) {
  if (persistent)
    hipLaunchKernelGGL((batch_class<E, ACC, CLS, true>), dim3((unsigned)grid), dim3(kBlock), 0, s, P);
  else
    hipLaunchKernelGGL((batch_class<E, ACC, CLS, false>), dim3((unsigned)grid), dim3(kBlock), 0, s, P);
  return hipGetLastError();
}

template <typename E, bool ACC>
hipError_t launch_batch_t(const BatchParams& P0, const int64_t* off, const int64_t* cnt, const int* grid,
                          bool persistent, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (persistent) {
    hipLaunchKernelGGL(batch_reset, dim3(1), dim3(kBlock), 0, s, P0.counter, kBatchCounters);
    e = hipGetLastError();
  }
  // units first (their partials feed the fix-up), then the row classes
  static constexpr int order[kBatchClasses] = {7, 8, 9, 0, 1, 2, 3, 4, 5, 6};
  for (int oi = 0; oi < kBatchClasses && e == hipSuccess; ++oi) {
    const int c = order[oi];
    if (cnt[c] == 0) continue;
    BatchParams P = P0;
    P.items = P0.items + off[c];
    P.n_items = cnt[c];
    P.counter = P0.counter ? P0.counter + (int64_t)c * kClaimSlices * kCounterStride : nullptr;
    switch (c) {
      case 0: e = launch_class<E, ACC, 0>(P, grid[c], persistent, s); break;
      case 1: e = launch_class<E, ACC, 1>(P, grid[c], persistent, s); break;
      case 2: e = launch_class<E, ACC, 2>(P, grid[c], persistent, s); break;
      case 3: e = launch_class<E, ACC, 3>(P, grid[c], persistent, s); break;
      case 4: e = launch_class<E, ACC, 4>(P, grid[c], persistent, s); break;
      case 5: e = launch_class<E, ACC, 5>(P, grid[c], persistent, s); break;
      case 6: e = launch_class<E, ACC, 6>(P, grid[c], persistent, s); break;
      case 7: e = launch_class<E, ACC, 7>(P, grid[c], persistent, s); break;
      case 8: e = launch_class<E, ACC, 8>(P, grid[c], persistent, s); break;
      default: e = launch_class<E, ACC, 9>(P, grid[c], persistent, s); break;
    }
  }
  if (e == hipSuccess && P0.n_fix > 0) {
    hipLaunchKernelGGL((batch_fixup<E, ACC>), dim3((unsigned)((P0.n_fix + 3) / 4)), dim3(kBlock), 0, s, P0);
    e = hipGetLastError();
  }
  return e;
}

template <typename E, int CLS>
int occupancy_of() {
  int n = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_class<E, false, CLS, true>, kBlock, 0);
  return (e == hipSuccess && n > 0) ? n : 2;
}

template <typename E>
void occupancy_all(int* out) {
  out[0] = occupancy_of<E, 0>();
  out[1] = occupancy_of<E, 1>();
  out[2] = occupancy_of<E, 2>();
  out[3] = occupancy_of<E, 3>();
  out[4] = occupancy_of<E, 4>();
  out[5] = occupancy_of<E, 5>();
  out[6] = occupancy_of<E, 6>();
  out[7] = occupancy_of<E, 7>();
  out[8] = occupancy_of<E, 8>();
  out[9] = occupancy_of<E, 9>();
}

}  // namespace

hipError_t launch_batch(const BatchParams& P, const int64_t* off, const int64_t* cnt, const int* grid, DT dt,
                        bool persistent, hipStream_t s) {
  if (dt == DT::F32)
    return P.accumulate ? launch_batch_t<F32E, true>(P, off, cnt, grid, persistent, s)
                        : launch_batch_t<F32E, false>(P, off, cnt, grid, persistent, s);
  return P.accumulate ? launch_batch_t<BF16E, true>(P, off, cnt, grid, persistent, s)
                      : launch_batch_t<BF16E, false>(P, off, cnt, grid, persistent, s);
}

hipError_t launch_batch_single(const BatchParams& P, int grid, unsigned mask, DT dt, bool persistent, hipStream_t s) {
  if (dt == DT::F32)
    return P.accumulate ? launch_single_t<F32E, true>(P, grid, persistent, mask, s)
                        : launch_single_t<F32E, false>(P, grid, persistent, mask, s);
  return P.accumulate ? launch_single_t<BF16E, true>(P, grid, persistent, mask, s)
                      : launch_single_t<BF16E, false>(P, grid, persistent, mask, s);
}

hipError_t launch_batch_reserve(const BatchParams& P, int grid, unsigned mask, DT dt, hipStream_t s) {
  if (dt == DT::F32)
    return P.accumulate ? launch_reserve_t<F32E, true>(P, grid, mask, s)
                        : launch_reserve_t<F32E, false>(P, grid, mask, s);
  return P.accumulate ? launch_reserve_t<BF16E, true>(P, grid, mask, s)
                      : launch_reserve_t<BF16E, false>(P, grid, mask, s);
}

int batch_reserve_blocks_per_cu(DT dt, unsigned mask) {
  return dt == DT::F32 ? occ_mask<F32E>(mask, true) : occ_mask<BF16E>(mask, true);
}

template <typename E, int V>
hipError_t launch_acc_n(void* C, int64_t ldc, const AccList& L, int64_t rows, int64_t N, hipStream_t s) {
  const int64_t n = rows * (N / V);
  if (n == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, kMaxGridBlocks);
  hipLaunchKernelGGL((accumulate_n_kernel<V, E>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                     static_cast<typename E::T*>(C), ldc, L, rows, N);
  return hipGetLastError();
}

hipError_t launch_accumulate_n(void* C, int64_t ldc, const void* const* Pt, const int64_t* ldp, int n, int64_t rows,
                               int64_t N, DT dt, int V, hipStream_t s) {
  // partials in launches of up to kAccMax each, in order
  for (int t0 = 0; t0 < n; t0 += kAccMax) {
    AccList L{};
    L.n = std::min(kAccMax, n - t0);
    for (int t = 0; t < L.n; ++t) {
      L.p[t] = Pt[t0 + t];
      L.ld[t] = ldp[t0 + t];
    }
    hipError_t e;
    if (dt == DT::F32) {
      e = V == 4 ? launch_acc_n<F32E, 4>(C, ldc, L, rows, N, s)
                 : (V == 2 ? launch_acc_n<F32E, 2>(C, ldc, L, rows, N, s) : launch_acc_n<F32E, 1>(C, ldc, L, rows, N, s));
    } else {
      e = V == 8 ? launch_acc_n<BF16E, 8>(C, ldc, L, rows, N, s)
                 : (V == 4 ? launch_acc_n<BF16E, 4>(C, ldc, L, rows, N, s)
                           : (V == 2 ? launch_acc_n<BF16E, 2>(C, ldc, L, rows, N, s)
                                     : launch_acc_n<BF16E, 1>(C, ldc, L, rows, N, s)));
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int batch_single_blocks_per_cu(DT dt, unsigned mask) {
  return dt == DT::F32 ? occ_mask<F32E>(mask, false) : occ_mask<BF16E>(mask, false);
}

void batch_blocks_per_cu(DT dt, int* out) {
  if (dt == DT::F32)
    occupancy_all<F32E>(out);
  else
    occupancy_all<BF16E>(out);
}

}  // namespace spmm
