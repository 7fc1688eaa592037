/*
 * sw_oracle.h -- plain CPU reference for the SSW alignment path.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists so that tests, the smoke check
 * and the CPU-baseline leg of the benchmark can check the GPU library.  The
 * product path never links, loads or calls it, and it shares no code, header
 * or table with the GPU library.
 *
 * Everything here is the plain definition, written out with 64-bit integer
 * scores and no blocking, vectorisation or reordering:
 *
 *   Smith-Waterman-Gotoh local alignment with affine gaps (paper, Introduction;
 *   method section "Algorithm and implementation"):
 *     H(i,j) = max(0, H(i-1,j-1) + S(q_i, r_j), E(i,j), F(i,j))
 *     E(i,j) = max(E(i,j-1) - e, H(i,j-1) - o)      (gap consuming reference)
 *     F(i,j) = max(F(i-1,j) - e, H(i-1,j) - o)      (gap consuming query)
 *   with H = 0 and E = F = -inf outside the matrix.  A gap of length k costs
 *   o + (k-1)*e.  S(a,b) = matrix[a*n + b] (a: query symbol, b: reference
 *   symbol).
 *
 *   The "max" array of the method section: maxcol[j] = max_i H(i,j).
 *
 * Tie-break rules (the paper leaves ties open; these are the stated readings):
 *   T1 end    : among cells with H = score1, smallest j, then smallest i.
 *   T2 begin  : among begins from which an alignment reaches the T1 end with
 *               score exactly score1, largest jb, then largest ib.
 *   T3 CIGAR  : traceback of the 3-state global DP on [ib..ie] x [jb..je],
 *               preferring M, then D (state E), then I (state F); inside a gap
 *               state, "open" before "extend".
 *   T4 score2 : mask columns [ref_begin1 - m, ref_end1 + m]; score2 is the
 *               largest maxcol value outside, ref_end2 its smallest column.
 *   T5        : score1 == 0 -> no alignment, every coordinate -1.
 *
 * Pins (tests/test_oracle_pins.py): exhaustive enumeration of all local
 * alignments on short sequences fixes score1, the max array, T1, T2, T4 and
 * T3 at every gap setting o >= e >= 0 (the enumeration walks gap state paths,
 * re-opened runs included, so the T3 choice digits are defined at o == e and
 * o == 0 as well); Kadane's maximum subarray (no gap can pay) and a one-matrix
 * linear-gap SW (o == e) fix score1 and the max array at larger sizes.
 *
 * All coordinates are 0-based and inclusive.  CIGAR entries are
 * (length << 4) | op with op M=0, I=1 (consumes query), D=2 (consumes
 * reference), as in SAM.
 */
#ifndef SW_ORACLE_H
#define SW_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_FLAG_BEGIN  1u
#define ORC_FLAG_CIGAR  2u
#define ORC_FLAG_SCORE2 4u

typedef struct {
  int64_t score1, score2;
  int64_t read_begin1, read_end1;
  int64_t ref_begin1, ref_end1;
  int64_t ref_end2;
  int64_t cigar_len;   /* number of runs written (or needed, if cap was short) */
} orc_result;

/* Forward full-matrix pass (linear space).  Writes maxcol[0..lr) when maxcol
 * is not NULL.  Returns score1 and the T1 end (-1, -1 when score1 == 0). */
void orc_fill(const int8_t *q, int64_t lq, const int8_t *r, int64_t lr,
              const int8_t *mat, int32_t n, int32_t o, int32_t e,
              int64_t *maxcol, int64_t *score1, int64_t *qend, int64_t *rend);

/* T2 by the paper's reversed pass: T1 applied to the local DP on the reversed
 * prefixes q[0..qend] and r[0..rend].  Returns 0, or -1 when the reversed
 * pass does not reach score1 (which would be an internal inconsistency). */
int orc_begin_reverse(const int8_t *q, const int8_t *r,
                      const int8_t *mat, int32_t n, int32_t o, int32_t e,
                      int64_t qend, int64_t rend, int64_t score1,
                      int64_t *qbeg, int64_t *rbeg);

/* T2 by a second, independent route: a forward DP whose states carry the
 * start of the best alignment, compared as (score, jb, ib).  Returns 0, or -1
 * when the carried score at the end cell is not score1. */
int orc_begin_startprop(const int8_t *q, int64_t lq, const int8_t *r, int64_t lr,
                        const int8_t *mat, int32_t n, int32_t o, int32_t e,
                        int64_t qend, int64_t rend, int64_t score1,
                        int64_t *qbeg, int64_t *rbeg);

/* T3: full-rectangle global DP on q[qbeg..qend] x r[rbeg..rend] and its
 * traceback.  Writes up to cap runs into cigar and returns the number of runs
 * (which may exceed cap: then only the first cap are written), or -1 on
 * allocation failure.  *score_out receives the global optimum. */
int64_t orc_traceback(const int8_t *q, const int8_t *r,
                      const int8_t *mat, int32_t n, int32_t o, int32_t e,
                      int64_t qbeg, int64_t qend, int64_t rbeg, int64_t rend,
                      uint32_t *cigar, int64_t cap, int64_t *score_out);

/* T4 on a max array. */
void orc_score2(const int64_t *maxcol, int64_t lr, int64_t ref_begin1,
                int64_t ref_end1, int64_t mask_len,
                int64_t *score2, int64_t *ref_end2);

/* The whole path for one pair.  mask_len < 0 selects max(lq/2, 15).
 * CIGAR and SCORE2 imply BEGIN.  cigar may be NULL when cap is 0.
 * maxcol_out, when not NULL, receives the max array [lr].
 * Returns 0, or -1 on an internal inconsistency or allocation failure. */
int orc_align(const int8_t *q, int64_t lq, const int8_t *r, int64_t lr,
              const int8_t *mat, int32_t n, int32_t o, int32_t e,
              uint32_t flags, int64_t mask_len,
              orc_result *res, uint32_t *cigar, int64_t cap, int64_t *maxcol_out);

/* Many pairs, spread over nthreads POSIX threads (one pair per task; the
 * per-pair work is orc_align unchanged).  Queries and references are
 * concatenated code arrays with offsets [count+1].  CIGARs go to
 * cigar + cigar_off[p] with capacity cigar_off[p+1]-cigar_off[p].  Returns 0
 * or the number of pairs whose orc_align failed. */
int64_t orc_align_many(const int8_t *qcat, const int64_t *qoff,
                       const int8_t *rcat, const int64_t *roff,
                       const int64_t *pair_q, const int64_t *pair_r, int64_t npairs,
                       const int8_t *mat, int32_t n, int32_t o, int32_t e,
                       uint32_t flags, int64_t mask_len,
                       orc_result *res, uint32_t *cigar, const int64_t *cigar_off,
                       int32_t nthreads);

/* The suboptimal alignment behind score2 (method section; Fig. 1 caption,
 * whose dashed arrows trace it).  Reading: it ends in column ref_end2 at the
 * smallest row i with H(i, ref_end2) = score2; its begin is T2 relative to
 * that end (the start-propagation DP); its CIGAR is T3 on the rectangle.
 * score2 <= 0: every coordinate -1, no CIGAR. */
typedef struct {
  int64_t read_begin2, read_end2, ref_begin2;
  int64_t cigar_len;
} orc_sub;

/* Smallest row i with H(i, col) == target (the forward recurrence up to
 * column col), or -1. */
int64_t orc_column_row(const int8_t *q, int64_t lq, const int8_t *r, int64_t lr,
                       const int8_t *mat, int32_t n, int32_t o, int32_t e,
                       int64_t col, int64_t target);

/* Returns 0, or -1 on an internal inconsistency or allocation failure. */
int orc_suboptimal(const int8_t *q, int64_t lq, const int8_t *r, int64_t lr,
                   const int8_t *mat, int32_t n, int32_t o, int32_t e,
                   int64_t score2, int64_t ref_end2,
                   orc_sub *res, uint32_t *cigar, int64_t cap);

/* Many pairs (score2 and ref_end2 per pair, from the primary results) over
 * nthreads threads; CIGARs as in orc_align_many.  Returns 0 or the number of
 * failed pairs. */
int64_t orc_suboptimal_many(const int8_t *qcat, const int64_t *qoff,
                            const int8_t *rcat, const int64_t *roff,
                            const int64_t *pair_q, const int64_t *pair_r, int64_t npairs,
                            const int8_t *mat, int32_t n, int32_t o, int32_t e,
                            const int64_t *score2, const int64_t *ref_end2,
                            orc_sub *res, uint32_t *cigar, const int64_t *cigar_off,
                            int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
