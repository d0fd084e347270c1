/*
 * FP64 CPU oracle for the local sparse-times-dense multiply.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: only the tests, the package's smoke check and the bench's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP library; the two meet only at the seeded inputs.
 *
 * Every routine is the plain definition written out, in double precision,
 * with no blocking or reordering beyond what the definition states.  FP32 and
 * BF16 inputs widen to double exactly, and the product of two FP32 numbers is
 * exact in double, so the only rounding is the double-precision summation.
 *
 * Passages followed (Brock, Bulu\c{c}, Yelick, "RDMA-Based Algorithms for
 * Sparse Matrix Multiplication on GPUs", ICS'24):
 *   - Section 2.1: a C tile is C_ij = C_ij + sum over k of A_ik B_kj.
 *   - Section 3.3, Algorithm 2: the owner of C(i,j) walks k' = 0..K-1 and
 *     multiplies tile k = (k' + i + j) mod K, accumulating into its C tile.
 *   - Section 3.1 / Section 5.2: sparse tiles are CSR (values, row pointer,
 *     column indices); Section 6: FP32 values, 32-bit indices.
 * The backward routines (SDDMM, A^T dC, transposed structure) and the BF16
 * rounding are not in the paper; they are the textbook definitions.
 * The sparse-times-sparse product (Section 6.2 multiplies C = A A with a local
 * SpGEMM inside the same distributed algorithms) is its textbook definition too:
 * a structural product pattern with the products summed in Gustavson order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

/* Row of CSR position p: the i with rowptr[i] <= p < rowptr[i+1] (binary search). */
static int64_t row_of(const int32_t* rowptr, int64_t M, int64_t p) {
  int64_t lo = 0, hi = M; /* invariant: rowptr[lo] <= p < rowptr[hi] */
  while (hi - lo > 1) {
    int64_t mid = lo + (hi - lo) / 2;
    if ((int64_t)rowptr[mid] <= p) lo = mid; else hi = mid;
  }
  return lo;
}

/*
 * SpMM over one tile row (Section 2.1, Algorithm 2):
 *   C[r, n] = acc * C0[i, n] + sum_{k'=0}^{K-1} sum_{p in row i of tile k} val_k[p] * B_k[col_k[p], n]
 * with k = (k' + k_offset) mod K and i = rows[r] (or r when rows is NULL).
 * S[r, n] (nullable) is the same sum over absolute values: sum |val| * |B|, the
 * scale against which rounding errors of any summation order are bounded.
 * B_k is row-major with leading dimension ldb[k]; C0 row-major (ldc0); outputs
 * row-major with leading dimension ldo.
 */
EXPORT void oracle_spmm(int64_t n_out, const int64_t* rows, int num_k, int k_offset,
                        const int32_t* const* rowptr, const int32_t* const* colind,
                        const float* const* values, const float* const* B, const int64_t* ldb,
                        int64_t N, int accumulate, const float* C0, int64_t ldc0,
                        double* C, double* S, int64_t ldo) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t r = 0; r < n_out; ++r) {
    int64_t i = rows ? rows[r] : r;
    double* c = C + r * ldo;
    double* s = S ? S + r * ldo : NULL;
    for (int64_t n = 0; n < N; ++n) {
      c[n] = accumulate ? (double)C0[i * ldc0 + n] : 0.0;
      if (s) s[n] = 0.0;
    }
    for (int kk = 0; kk < num_k; ++kk) {
      int k = (int)(((int64_t)kk + k_offset) % num_k);
      if (k < 0) k += num_k;
      for (int64_t p = rowptr[k][i]; p < rowptr[k][i + 1]; ++p) {
        double a = (double)values[k][p];
        const float* b = B[k] + (int64_t)colind[k][p] * ldb[k];
        for (int64_t n = 0; n < N; ++n) {
          c[n] += a * (double)b[n];
          if (s) s[n] += fabs(a) * fabs((double)b[n]);
        }
      }
    }
  }
}

/*
 * Sampled dense-dense product on A's pattern (the gradient of a loss with
 * respect to A's stored values when dL/dC = dC):
 *   dA[e] = sum_n dC[i, n] * B[colind[p], n],  p = entries[e] (or e), i = row of p.
 * S[e] (nullable) = sum_n |dC[i,n]| * |B[colind[p], n]|.
 */
EXPORT void oracle_sddmm(int64_t M, const int32_t* rowptr, const int32_t* colind,
                         int64_t n_entries, const int64_t* entries,
                         const float* dC, int64_t lddc, const float* B, int64_t ldb, int64_t N,
                         double* dA, double* S) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t e = 0; e < n_entries; ++e) {
    int64_t p = entries ? entries[e] : e;
    int64_t i = row_of(rowptr, M, p);
    const float* g = dC + i * lddc;
    const float* b = B + (int64_t)colind[p] * ldb;
    double acc = 0.0, sc = 0.0;
    for (int64_t n = 0; n < N; ++n) {
      acc += (double)g[n] * (double)b[n];
      sc += fabs((double)g[n]) * fabs((double)b[n]);
    }
    dA[e] = acc;
    if (S) S[e] = sc;
  }
}

/*
 * dB = A^T dC by direct scatter over A's non-zeros (deliberately not through a
 * transposed structure):  for every p in row i:  dB[colind[p], :] += val[p] * dC[i, :].
 * Only output rows listed in out_rows (or all K rows when NULL) are formed;
 * output slot r holds row out_rows[r].  Serial on purpose: the scatter has no
 * races and its summation order is A's CSR order.
 */
EXPORT int oracle_spmm_t(int64_t M, int64_t K, const int32_t* rowptr, const int32_t* colind,
                         const float* values, const float* dC, int64_t lddc, int64_t N,
                         int64_t n_out, const int64_t* out_rows, double* dB, double* S, int64_t ldo) {
  int64_t* slot = (int64_t*)malloc((size_t)(K > 0 ? K : 1) * sizeof(int64_t));
  if (!slot) return -1;
  for (int64_t j = 0; j < K; ++j) slot[j] = out_rows ? -1 : j;
  if (out_rows)
    for (int64_t r = 0; r < n_out; ++r) slot[out_rows[r]] = r;
  for (int64_t r = 0; r < n_out; ++r)
    for (int64_t n = 0; n < N; ++n) {
      dB[r * ldo + n] = 0.0;
      if (S) S[r * ldo + n] = 0.0;
    }
  for (int64_t i = 0; i < M; ++i) {
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      int64_t r = slot[colind[p]];
      if (r < 0) continue;
      double a = (double)values[p];
      const float* g = dC + i * lddc;
      for (int64_t n = 0; n < N; ++n) {
        dB[r * ldo + n] += a * (double)g[n];
        if (S) S[r * ldo + n] += fabs(a) * fabs((double)g[n]);
      }
    }
  }
  free(slot);
  return 0;
}

/*
 * Transposed structure of a CSR tile by counting sort:
 *   cnt[j] = number of p with colind[p] == j;  rowptrT = exclusive prefix sum of cnt;
 *   then each p, visited in increasing order, goes to the next free slot q of its
 *   column:  colindT[q] = row of p,  perm[q] = p.
 * Visiting p in increasing order makes every output row list its entries by
 * increasing original row (a stable sort by column).
 */
EXPORT void oracle_transpose(int64_t M, int64_t K, const int32_t* rowptr, const int32_t* colind,
                             int32_t* rowptrT, int32_t* colindT, int32_t* perm) {
  int64_t* next = (int64_t*)calloc((size_t)K + 1, sizeof(int64_t));
  int64_t nnz = rowptr[M];
  for (int64_t p = 0; p < nnz; ++p) next[colind[p] + 1] += 1;
  for (int64_t j = 0; j < K; ++j) next[j + 1] += next[j];
  for (int64_t j = 0; j <= K; ++j) rowptrT[j] = (int32_t)next[j];
  for (int64_t i = 0; i < M; ++i)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      int64_t q = next[colind[p]]++;
      colindT[q] = (int32_t)i;
      perm[q] = (int32_t)p;
    }
  free(next);
}

/*
 * FP32 -> BF16 (the upper 16 bits of an FP32 pattern), round to nearest, ties to
 * even, from the definition: keep the upper half; if the discarded lower half is
 * more than half an upper-half ulp, or exactly half and the kept half is odd,
 * step the kept half up by one (a carry into the exponent gives the next binade
 * or infinity, as it should).  Infinities and zeros keep their sign.  Any NaN
 * becomes the canonical quiet NaN 0x7FC0.
 */
EXPORT void oracle_f32_to_bf16(int64_t n, const float* x, uint16_t* y) {
  for (int64_t t = 0; t < n; ++t) {
    uint32_t bits;
    memcpy(&bits, &x[t], sizeof bits);
    uint32_t exponent = (bits >> 23) & 0xFFu, mantissa = bits & 0x7FFFFFu;
    if (exponent == 0xFFu && mantissa != 0u) {
      y[t] = 0x7FC0u;
      continue;
    }
    uint32_t upper = bits >> 16, lower = bits & 0xFFFFu;
    if (lower > 0x8000u || (lower == 0x8000u && (upper & 1u))) upper += 1u;
    y[t] = (uint16_t)upper;
  }
}

/*
 * Sparse times sparse, C = A B, for output rows i = rows[r] (or r when rows is
 * NULL), A M x K and B K x N in CSR.  The pattern of C is structural: (i, j) is
 * present when some p in row i of A has j in row colA[p] of B (whatever the values,
 * so cancellation to zero keeps the entry).  Pass 1 counts the distinct columns of
 * every output row: counts[r].
 */
EXPORT int oracle_spgemm_count(int64_t n_out, const int64_t* rows, const int32_t* rowptrA, const int32_t* colA,
                               const int32_t* rowptrB, const int32_t* colB, int64_t N, int64_t* counts) {
  int failed = 0;
#pragma omp parallel
  {
    int64_t* mark = (int64_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(int64_t));
    if (!mark) {
#pragma omp atomic write
      failed = 1;
    } else {
      for (int64_t j = 0; j < N; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 256)
      for (int64_t r = 0; r < n_out; ++r) {
        int64_t i = rows ? rows[r] : r, cnt = 0;
        for (int64_t p = rowptrA[i]; p < rowptrA[i + 1]; ++p) {
          int64_t k = colA[p];
          for (int64_t q = rowptrB[k]; q < rowptrB[k + 1]; ++q) {
            int64_t j = colB[q];
            if (mark[j] != r) {
              mark[j] = r;
              ++cnt;
            }
          }
        }
        counts[r] = cnt;
      }
      free(mark);
    }
  }
  return failed ? -1 : 0;
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/*
 * Pass 2 of C = A B: for every output row r (offset[r] = its start in the output),
 *   C[i, j] = sum over p in row i of A, q in row colA[p] of B with colB[q] = j of valA[p] * valB[q]
 * accumulated in that (Gustavson) order in double, written with the row's columns in
 * increasing order; S[i, j] (nullable) is the same sum over |valA[p]| * |valB[q]|.
 */
EXPORT int oracle_spgemm_fill(int64_t n_out, const int64_t* rows, const int32_t* rowptrA, const int32_t* colA,
                              const float* valA, const int32_t* rowptrB, const int32_t* colB, const float* valB,
                              int64_t N, const int64_t* offset, int64_t* colC, double* valC, double* S) {
  int failed = 0;
#pragma omp parallel
  {
    double* acc = (double*)malloc((size_t)(N > 0 ? N : 1) * sizeof(double));
    double* sc = (double*)malloc((size_t)(N > 0 ? N : 1) * sizeof(double));
    int64_t* mark = (int64_t*)malloc((size_t)(N > 0 ? N : 1) * sizeof(int64_t));
    if (!acc || !sc || !mark) {
#pragma omp atomic write
      failed = 1;
    } else {
      for (int64_t j = 0; j < N; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 256)
      for (int64_t r = 0; r < n_out; ++r) {
        int64_t i = rows ? rows[r] : r;
        int64_t* cols = colC + offset[r];
        int64_t cnt = 0;
        for (int64_t p = rowptrA[i]; p < rowptrA[i + 1]; ++p) {
          int64_t k = colA[p];
          double a = (double)valA[p];
          for (int64_t q = rowptrB[k]; q < rowptrB[k + 1]; ++q) {
            int64_t j = colB[q];
            if (mark[j] != r) {
              mark[j] = r;
              acc[j] = 0.0;
              sc[j] = 0.0;
              cols[cnt++] = j;
            }
            acc[j] += a * (double)valB[q];
            sc[j] += fabs(a) * fabs((double)valB[q]);
          }
        }
        qsort(cols, (size_t)cnt, sizeof(int64_t), cmp_i64);
        for (int64_t t = 0; t < cnt; ++t) {
          valC[offset[r] + t] = acc[cols[t]];
          if (S) S[offset[r] + t] = sc[cols[t]];
        }
      }
    }
    free(acc);
    free(sc);
    free(mark);
  }
  return failed ? -1 : 0;
}
