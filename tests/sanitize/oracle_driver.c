/* Runs the CPU oracle's entry points on seeded random pairs, including the
 * edge cases (empty and one-symbol sequences, o = e, o = 0, e = 0, wide
 * alphabets), so that an AddressSanitizer / UndefinedBehaviorSanitizer
 * build of sw_oracle.c reports any out-of-bounds access, leak or undefined
 * operation.  Test infrastructure only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/sw_oracle.h"

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32(void) {   /* xorshift64* */
  rng ^= rng >> 12;
  rng ^= rng << 25;
  rng ^= rng >> 27;
  return (uint32_t)((rng * 0x2545F4914F6CDD1Dull) >> 32);
}
static int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u32() % (uint32_t)(hi - lo + 1)); }

int main(void) {
  const int32_t gaps[][2] = {{3, 1}, {1, 1}, {0, 0}, {5, 0}, {11, 1}, {2, 2}};
  int failures = 0;
  for (int trial = 0; trial < 400; ++trial) {
    const int32_t n = (trial % 3 == 0) ? 24 : 4;
    int8_t *mat = malloc((size_t)n * n);
    for (int32_t a = 0; a < n; ++a)
      for (int32_t b = 0; b < n; ++b) mat[a * n + b] = (int8_t)(a == b ? uniform(1, 6) : -uniform(0, 4));
    const int32_t o = gaps[trial % 6][0], e = gaps[trial % 6][1];
    const int64_t lq = (trial % 17 == 0) ? 0 : uniform(1, 60);
    const int64_t lr = (trial % 19 == 0) ? 0 : uniform(1, 90);
    int8_t *q = malloc((size_t)(lq > 0 ? lq : 1)), *r = malloc((size_t)(lr > 0 ? lr : 1));
    for (int64_t i = 0; i < lq; ++i) q[i] = (int8_t)uniform(0, n - 1);
    for (int64_t j = 0; j < lr; ++j) r[j] = (int8_t)(j > 5 && next_u32() % 4 ? r[j - 5] : uniform(0, n - 1));
    const int64_t cap = lq + lr + 2;
    uint32_t *cig = malloc(sizeof(uint32_t) * (size_t)cap);
    int64_t *maxcol = malloc(sizeof(int64_t) * (size_t)(lr > 0 ? lr : 1));
    orc_result res;
    const int64_t mask = (trial % 5 == 0) ? 0 : -1;
    if (orc_align(q, lq, r, lr, mat, n, o, e, 7u, mask, &res, cig, cap, maxcol) != 0) ++failures;
    if (res.score2 > 0) {
      orc_sub sub;
      uint32_t *cig2 = malloc(sizeof(uint32_t) * (size_t)cap);
      if (orc_suboptimal(q, lq, r, lr, mat, n, o, e, res.score2, res.ref_end2, &sub, cig2, cap) != 0)
        ++failures;
      free(cig2);
    }
    if (lr > 0 && lq > 0) (void)orc_column_row(q, lq, r, lr, mat, n, o, e, lr - 1, res.score1);
    free(q); free(r); free(cig); free(maxcol); free(mat);
  }
  /* many pairs over threads */
  {
    const int32_t n = 4;
    int8_t mat[16];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) mat[a * 4 + b] = (int8_t)(a == b ? 2 : -2);
    enum { NP = 64 };
    int64_t qoff[NP + 1], roff[NP + 1], pq[NP], pr[NP], coff[NP + 1];
    qoff[0] = roff[0] = coff[0] = 0;
    for (int p = 0; p < NP; ++p) {
      qoff[p + 1] = qoff[p] + uniform(0, 40);
      roff[p + 1] = roff[p] + uniform(0, 80);
      pq[p] = pr[p] = p;
      coff[p + 1] = coff[p] + (qoff[p + 1] - qoff[p]) + (roff[p + 1] - roff[p]) + 2;
    }
    int8_t *qc = malloc((size_t)qoff[NP] + 1), *rc = malloc((size_t)roff[NP] + 1);
    for (int64_t i = 0; i < qoff[NP]; ++i) qc[i] = (int8_t)uniform(0, 3);
    for (int64_t j = 0; j < roff[NP]; ++j) rc[j] = (int8_t)uniform(0, 3);
    orc_result *res = malloc(sizeof(orc_result) * NP);
    uint32_t *cig = malloc(sizeof(uint32_t) * (size_t)coff[NP]);
    if (orc_align_many(qc, qoff, rc, roff, pq, pr, NP, mat, n, 3, 1, 7u, -1, res, cig, coff, 4) != 0)
      ++failures;
    free(qc); free(rc); free(res); free(cig);
  }
  printf("oracle driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
