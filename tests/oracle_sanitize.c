/*
 * Memory-safety driver for the CPU oracle: built together with oracle/oracle.c under
 * gcc's AddressSanitizer and UndefinedBehaviorSanitizer, it calls every exported
 * oracle routine on small inputs held in exactly sized heap blocks (so that any read
 * or write one element past a buffer is reported), covering the edge cases the
 * routines must handle: empty rows and tiles, N = 0, a row subset, a negative tile
 * offset, nullable scale outputs, structural zeros from cancellation, and the BF16
 * rounding of zeros, infinities, NaNs and subnormals.  A few results are checked
 * against hand-computed values; the exit status is 0 when every check holds.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_spmm(int64_t n_out, const int64_t* rows, int num_k, int k_offset, const int32_t* const* rowptr,
                 const int32_t* const* colind, const float* const* values, const float* const* B,
                 const int64_t* ldb, int64_t N, int accumulate, const float* C0, int64_t ldc0, double* C,
                 double* S, int64_t ldo);
void oracle_sddmm(int64_t M, const int32_t* rowptr, const int32_t* colind, int64_t n_entries,
                  const int64_t* entries, const float* dC, int64_t lddc, const float* B, int64_t ldb,
                  int64_t N, double* dA, double* S);
int oracle_spmm_t(int64_t M, int64_t K, const int32_t* rowptr, const int32_t* colind, const float* values,
                  const float* dC, int64_t lddc, int64_t N, int64_t n_out, const int64_t* out_rows, double* dB,
                  double* S, int64_t ldo);
void oracle_transpose(int64_t M, int64_t K, const int32_t* rowptr, const int32_t* colind, int32_t* rowptrT,
                      int32_t* colindT, int32_t* perm);
void oracle_f32_to_bf16(int64_t n, const float* x, uint16_t* y);
int oracle_spgemm_count(int64_t n_out, const int64_t* rows, const int32_t* rowptrA, const int32_t* colA,
                        const int32_t* rowptrB, const int32_t* colB, int64_t N, int64_t* counts);
int oracle_spgemm_fill(int64_t n_out, const int64_t* rows, const int32_t* rowptrA, const int32_t* colA,
                       const float* valA, const int32_t* rowptrB, const int32_t* colB, const float* valB,
                       int64_t N, const int64_t* offset, int64_t* colC, double* valC, double* S);

static int failures = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

/* Exactly sized heap copies (an empty array gets a one-byte block, so that it is still
 * a valid pointer that nothing may read). */
static void* dup_block(const void* src, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(2);
  }
  if (bytes) memcpy(p, src, bytes);
  return p;
}
#define DUP(arr, n) dup_block((arr), sizeof((arr)[0]) * (size_t)(n))

/* Tile k of a 3 x 4 tile row; rows of different lengths, one empty row, one empty tile. */
static void check_spmm(void) {
  /* tile 0 (3 x 2): row 0 = {0:1, 1:2}, row 1 = {}, row 2 = {1:-1} */
  const int32_t rp0[] = {0, 2, 2, 3}, ci0[] = {0, 1, 1};
  const float v0[] = {1.f, 2.f, -1.f};
  /* tile 1 (3 x 3): empty */
  const int32_t rp1[] = {0, 0, 0, 0}, ci1[] = {0};
  const float v1[] = {0.f};
  /* tile 2 (3 x 1): row 1 = {0:3} */
  const int32_t rp2[] = {0, 0, 1, 1}, ci2[] = {0};
  const float v2[] = {3.f};
  const int64_t N = 2;
  const float B0[] = {1.f, 10.f, 100.f, 1000.f};             /* 2 x 2, ld 2 */
  const float B1[] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}; /* 3 x 3, ld 3 */
  const float B2[] = {7.f, -7.f};                            /* 1 x 2, ld 3: only N read */
  const float C0[] = {1.f, 1.f, 0.f, 2.f, 2.f, 0.f, 3.f, 3.f};  /* 3 x 2, ld 3 */
  int32_t* rp[3] = {DUP(rp0, 4), DUP(rp1, 4), DUP(rp2, 4)};
  int32_t* ci[3] = {DUP(ci0, 3), dup_block(ci1, 0), DUP(ci2, 1)};
  float* vv[3] = {DUP(v0, 3), dup_block(v1, 0), DUP(v2, 1)};
  float* Bk[3] = {DUP(B0, 4), DUP(B1, 9), DUP(B2, 2)};
  const int64_t ldb[3] = {2, 3, 3};
  float* c0 = DUP(C0, 8);
  for (int k_offset = -4; k_offset <= 4; k_offset += 4) {
    double* C = malloc(sizeof(double) * 3 * 2);
    double* S = malloc(sizeof(double) * 3 * 2);
    oracle_spmm(3, NULL, 3, k_offset, (const int32_t* const*)rp, (const int32_t* const*)ci,
                (const float* const*)vv, (const float* const*)Bk, ldb, N, 1, c0, 3, C, S, 2);
    /* row 0: 1 + (1*1 + 2*100), 1 + (1*10 + 2*1000); row 1: 2 + 3*7, 2 + 3*(-7);
       row 2: 3 + (-1)*100, 3 + (-1)*1000 */
    CHECK(C[0] == 202.0 && C[1] == 2011.0);
    CHECK(C[2] == 23.0 && C[3] == -19.0);
    CHECK(C[4] == -97.0 && C[5] == -997.0);
    CHECK(S[0] == 201.0 && S[3] == 21.0 && S[5] == 1000.0);
    free(C);
    free(S);
  }
  /* a row subset, no scale output, no accumulation, N = 0 and N = 1 */
  const int64_t rows[] = {2, 0};
  int64_t* rs = DUP(rows, 2);
  double* C = malloc(sizeof(double) * 2 * 1);
  oracle_spmm(2, rs, 3, 1, (const int32_t* const*)rp, (const int32_t* const*)ci, (const float* const*)vv,
              (const float* const*)Bk, ldb, 1, 0, NULL, 0, C, NULL, 1);
  CHECK(C[0] == -100.0 && C[1] == 201.0);
  oracle_spmm(2, rs, 3, 0, (const int32_t* const*)rp, (const int32_t* const*)ci, (const float* const*)vv,
              (const float* const*)Bk, ldb, 0, 0, NULL, 0, C, NULL, 0);
  oracle_spmm(0, NULL, 3, 0, (const int32_t* const*)rp, (const int32_t* const*)ci, (const float* const*)vv,
              (const float* const*)Bk, ldb, 1, 0, NULL, 0, C, NULL, 1);
  free(C);
  free(rs);
  free(c0);
  for (int k = 0; k < 3; ++k) {
    free(rp[k]);
    free(ci[k]);
    free(vv[k]);
    free(Bk[k]);
  }
}

static void check_sddmm_and_transpose(void) {
  /* A (4 x 3): row 0 = {0, 2}, row 1 = {}, row 2 = {1}, row 3 = {0, 1, 2} */
  const int32_t rp_[] = {0, 2, 2, 3, 6}, ci_[] = {0, 2, 1, 0, 1, 2};
  const float va_[] = {1.f, -2.f, 3.f, 4.f, -5.f, 6.f};
  int32_t* rp = DUP(rp_, 5);
  int32_t* ci = DUP(ci_, 6);
  float* va = DUP(va_, 6);
  const int64_t N = 3;
  /* dC (4 x 3) with leading dimension 4: the block ends with the last row's third
     element, so reading a padding slot past it would be reported */
  const float dC_[] = {1, 2, 3, 9, 0, 0, 0, 9, 0, 5, 0, 9, -1, 4, 2};
  const float B_[] = {1, 0, 0, 0, 1, 0, 0, 0, 1}; /* 3 x 3 identity, ld 3 */
  float* dC = DUP(dC_, 15);
  float* B = DUP(B_, 9);
  double* dA = malloc(sizeof(double) * 6);
  double* S = malloc(sizeof(double) * 6);
  oracle_sddmm(4, rp, ci, 6, NULL, dC, 4, B, 3, N, dA, S);
  CHECK(dA[0] == 1.0 && dA[1] == 3.0);        /* row 0 . e0, row 0 . e2 */
  CHECK(dA[2] == 5.0);                        /* row 2 of dC . e1 */
  CHECK(dA[3] == dC_[12] && dA[4] == dC_[13] && dA[5] == dC_[14]);
  const int64_t ent_[] = {5, 0};
  int64_t* ent = DUP(ent_, 2);
  oracle_sddmm(4, rp, ci, 2, ent, dC, 4, B, 3, N, dA, NULL);
  CHECK(dA[0] == dC_[14] && dA[1] == 1.0);
  oracle_sddmm(4, rp, ci, 0, NULL, dC, 4, B, 3, N, dA, S);

  /* transpose: column j of A becomes row j, entries by increasing original row */
  int32_t* rpT = malloc(sizeof(int32_t) * 4);
  int32_t* ciT = malloc(sizeof(int32_t) * 6);
  int32_t* perm = malloc(sizeof(int32_t) * 6);
  oracle_transpose(4, 3, rp, ci, rpT, ciT, perm);
  const int32_t wrp[] = {0, 2, 4, 6}, wci[] = {0, 3, 2, 3, 0, 3}, wperm[] = {0, 3, 2, 4, 1, 5};
  CHECK(memcmp(rpT, wrp, sizeof wrp) == 0 && memcmp(ciT, wci, sizeof wci) == 0 &&
        memcmp(perm, wperm, sizeof wperm) == 0);

  /* dB = A^T dC: all rows, then the subset {2, 0}, then no rows */
  double* dB = malloc(sizeof(double) * 3 * 3);
  double* Sb = malloc(sizeof(double) * 3 * 3);
  CHECK(oracle_spmm_t(4, 3, rp, ci, va, dC, 4, N, 3, NULL, dB, Sb, 3) == 0);
  /* dB[0] = 1 * dC[0] + 4 * dC[3]; dB[2] = -2 * dC[0] + 6 * dC[3] */
  for (int n = 0; n < 3; ++n) {
    CHECK(dB[0 * 3 + n] == 1.0 * dC_[n] + 4.0 * dC_[12 + n]);
    CHECK(dB[2 * 3 + n] == -2.0 * dC_[n] + 6.0 * dC_[12 + n]);
  }
  const int64_t orows_[] = {2, 0};
  int64_t* orows = DUP(orows_, 2);
  double* dB2 = malloc(sizeof(double) * 2 * 3);
  CHECK(oracle_spmm_t(4, 3, rp, ci, va, dC, 4, N, 2, orows, dB2, NULL, 3) == 0);
  CHECK(memcmp(dB2, dB + 6, 3 * sizeof(double)) == 0 && memcmp(dB2 + 3, dB, 3 * sizeof(double)) == 0);
  CHECK(oracle_spmm_t(4, 3, rp, ci, va, dC, 4, N, 0, orows, dB2, NULL, 3) == 0);

  /* an empty tile: no rows at all, and rows but no entries */
  const int32_t zrp_[] = {0, 0, 0};
  int32_t* zrp = DUP(zrp_, 3);
  int32_t* zci = dup_block(ci_, 0);
  int32_t* zrpT = malloc(sizeof(int32_t) * 6);
  oracle_transpose(2, 5, zrp, zci, zrpT, zci, zci);
  CHECK(zrpT[0] == 0 && zrpT[5] == 0);
  oracle_transpose(0, 0, zrp, zci, zrpT, zci, zci);
  CHECK(zrpT[0] == 0);
  free(zrp);
  free(zci);
  free(zrpT);
  free(orows);
  free(dB2);
  free(dB);
  free(Sb);
  free(rpT);
  free(ciT);
  free(perm);
  free(ent);
  free(dA);
  free(S);
  free(dC);
  free(B);
  free(rp);
  free(ci);
  free(va);
}

static void check_bf16(void) {
  const uint32_t in_[] = {
      0x00000000u, 0x80000000u, 0x7F800000u, 0xFF800000u, /* zeros, infinities */
      0x7FC00001u, 0xFFFFFFFFu, 0x7F800001u,              /* NaNs */
      0x00000001u, 0x80008000u, 0x00018000u,              /* subnormals, ties */
      0x3F808000u, 0x3F818000u, 0x3F808001u,              /* tie to even (down, up), above half */
      0x7F7FFFFFu,                                        /* largest finite: rounds to infinity */
  };
  const uint16_t want[] = {0x0000u, 0x8000u, 0x7F80u, 0xFF80u, 0x7FC0u, 0x7FC0u, 0x7FC0u,
                           0x0000u, 0x8000u, 0x0002u, 0x3F80u, 0x3F82u, 0x3F81u, 0x7F80u};
  const int64_t n = (int64_t)(sizeof in_ / sizeof in_[0]);
  float* x = dup_block(in_, sizeof in_);
  uint16_t* y = malloc(sizeof(uint16_t) * (size_t)n);
  oracle_f32_to_bf16(n, x, y);
  for (int64_t t = 0; t < n; ++t) CHECK(y[t] == want[t]);
  oracle_f32_to_bf16(0, x, y);
  free(x);
  free(y);
}

static void check_spgemm(void) {
  /* A (3 x 2): row 0 = {0:1, 1:1}, row 1 = {}, row 2 = {1:2};
     B (2 x 4): row 0 = {1:1, 3:5}, row 1 = {1:-1, 2:7}.
     C row 0 = {1: 0 (cancelled, kept), 2: 7, 3: 5}; row 2 = {1: -2, 2: 14} */
  const int32_t rpA_[] = {0, 2, 2, 3}, cA_[] = {0, 1, 1};
  const float vA_[] = {1.f, 1.f, 2.f};
  const int32_t rpB_[] = {0, 2, 4}, cB_[] = {1, 3, 1, 2};
  const float vB_[] = {1.f, 5.f, -1.f, 7.f};
  int32_t* rpA = DUP(rpA_, 4);
  int32_t* cA = DUP(cA_, 3);
  float* vA = DUP(vA_, 3);
  int32_t* rpB = DUP(rpB_, 3);
  int32_t* cB = DUP(cB_, 4);
  float* vB = DUP(vB_, 4);
  int64_t* counts = malloc(sizeof(int64_t) * 3);
  CHECK(oracle_spgemm_count(3, NULL, rpA, cA, rpB, cB, 4, counts) == 0);
  CHECK(counts[0] == 3 && counts[1] == 0 && counts[2] == 2);
  const int64_t off_[] = {0, 3, 3};
  int64_t* off = DUP(off_, 3);
  int64_t* colC = malloc(sizeof(int64_t) * 5);
  double* valC = malloc(sizeof(double) * 5);
  double* S = malloc(sizeof(double) * 5);
  CHECK(oracle_spgemm_fill(3, NULL, rpA, cA, vA, rpB, cB, vB, 4, off, colC, valC, S) == 0);
  const int64_t wcol[] = {1, 2, 3, 1, 2};
  const double wval[] = {0.0, 7.0, 5.0, -2.0, 14.0}, wS[] = {2.0, 7.0, 5.0, 2.0, 14.0};
  CHECK(memcmp(colC, wcol, sizeof wcol) == 0 && memcmp(valC, wval, sizeof wval) == 0 &&
        memcmp(S, wS, sizeof wS) == 0);
  /* a row subset (row 2 only) without scale output; then no rows; then N = 0 */
  const int64_t rows_[] = {2};
  int64_t* rows = DUP(rows_, 1);
  int64_t* off0 = calloc(1, sizeof(int64_t));
  CHECK(oracle_spgemm_count(1, rows, rpA, cA, rpB, cB, 4, counts) == 0 && counts[0] == 2);
  CHECK(oracle_spgemm_fill(1, rows, rpA, cA, vA, rpB, cB, vB, 4, off0, colC, valC, NULL) == 0);
  CHECK(colC[0] == 1 && colC[1] == 2 && valC[0] == -2.0 && valC[1] == 14.0);
  CHECK(oracle_spgemm_count(0, NULL, rpA, cA, rpB, cB, 4, counts) == 0);
  CHECK(oracle_spgemm_fill(0, NULL, rpA, cA, vA, rpB, cB, vB, 4, off0, colC, valC, S) == 0);
  const int32_t erpB_[] = {0, 0, 0};
  int32_t* erpB = DUP(erpB_, 3);
  int32_t* ecB = dup_block(cB_, 0);
  float* evB = dup_block(vB_, 0);
  CHECK(oracle_spgemm_count(3, NULL, rpA, cA, erpB, ecB, 0, counts) == 0);
  CHECK(counts[0] == 0 && counts[1] == 0 && counts[2] == 0);
  CHECK(oracle_spgemm_fill(3, NULL, rpA, cA, vA, erpB, ecB, evB, 0, off, colC, valC, S) == 0);
  free(erpB);
  free(ecB);
  free(evB);
  free(off0);
  free(rows);
  free(S);
  free(valC);
  free(colC);
  free(off);
  free(counts);
  free(rpA);
  free(cA);
  free(vA);
  free(rpB);
  free(cB);
  free(vB);
}

int main(void) {
  check_spmm();
  check_sddmm_and_transpose();
  check_bf16();
  check_spgemm();
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("oracle sanitizer driver: all checks passed\n");
  return 0;
}
