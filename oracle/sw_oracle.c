/*
 * sw_oracle.c -- plain CPU reference for the SSW alignment path.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the
 * CPU-baseline leg of the benchmark.  Never linked into the GPU library.
 * Built with -O2 -fno-tree-vectorize; scores are int64 throughout.
 *
 * Method section "Algorithm and implementation" of the paper, in order:
 *   1. fill the SW matrix, keeping the per-column max array and the column of
 *      the overall maximum                                  -> orc_fill
 *   2. end position from the max array and that column      -> orc_fill (T1)
 *   3. reversed SW from the end finds the beginning         -> orc_begin_reverse
 *   4. banded SW between begin and end gives the alignment  -> orc_traceback
 *      (the oracle uses the whole rectangle, no band)
 *   5. second-best score from the max array with the primary
 *      alignment's region masked (Figure 1 caption)         -> orc_score2
 * orc_begin_startprop computes step 3's result a second way for cross-checks.
 */
#include "sw_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define NEG_INF (INT64_MIN / 4)

static int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

static int64_t score_of(const int8_t *mat, int32_t n, int8_t a, int8_t b) {
  return (int64_t)mat[(int64_t)a * n + b];
}

/* ---- step 1/2: forward fill, max array, T1 end ------------------------- */
void orc_fill(const int8_t *q, int64_t lq, const int8_t *r, int64_t lr,
              const int8_t *mat, int32_t n, int32_t o, int32_t e,
              int64_t *maxcol, int64_t *score1, int64_t *qend, int64_t *rend) {
  int64_t best = 0, bi = -1, bj = -1;
  if (lq <= 0 || lr <= 0) {
    for (int64_t j = 0; j < lr; ++j)
      if (maxcol) maxcol[j] = 0;
    *score1 = 0; *qend = -1; *rend = -1;
    return;
  }
  /* hprev[i] = H(i, j-1); hcur[i] = H(i, j); erow[i] = E(i, j-1) */
  int64_t *hprev = (int64_t *)malloc(sizeof(int64_t) * lq);
  int64_t *hcur = (int64_t *)malloc(sizeof(int64_t) * lq);
  int64_t *erow = (int64_t *)malloc(sizeof(int64_t) * lq);
  for (int64_t i = 0; i < lq; ++i) { hprev[i] = 0; erow[i] = NEG_INF; }
  for (int64_t j = 0; j < lr; ++j) {
    int64_t colmax = 0;
    int64_t f = NEG_INF;          /* F(i-1, j) */
    for (int64_t i = 0; i < lq; ++i) {
      int64_t hdiag = (i > 0) ? hprev[i - 1] : 0;   /* H(i-1, j-1) */
      int64_t hleft = hprev[i];                     /* H(i, j-1)   */
      int64_t hup = (i > 0) ? hcur[i - 1] : 0;      /* H(i-1, j)   */
      int64_t eij = max2(erow[i] - e, hleft - o);
      int64_t fij = max2(f - e, hup - o);
      int64_t h = hdiag + score_of(mat, n, q[i], r[j]);
      h = max2(h, eij);
      h = max2(h, fij);
      h = max2(h, 0);
      hcur[i] = h;
      erow[i] = eij;
      f = fij;
      if (h > colmax) colmax = h;
      if (h > best) { best = h; bi = i; bj = j; }  /* strict: first j, then first i */
    }
    if (maxcol) maxcol[j] = colmax;
    int64_t *t = hprev; hprev = hcur; hcur = t;
  }
  free(hprev); free(hcur); free(erow);
  *score1 = best;
  *qend = best > 0 ? bi : -1;
  *rend = best > 0 ? bj : -1;
}

/* ---- step 3: reversed pass (T2 = T1 in reversed coordinates) ----------- */
int orc_begin_reverse(const int8_t *q, const int8_t *r,
                      const int8_t *mat, int32_t n, int32_t o, int32_t e,
                      int64_t qend, int64_t rend, int64_t score1,
                      int64_t *qbeg, int64_t *rbeg) {
  int64_t lq = qend + 1, lr = rend + 1;
  int8_t *qr = (int8_t *)malloc(lq > 0 ? lq : 1);
  int8_t *rr = (int8_t *)malloc(lr > 0 ? lr : 1);
  for (int64_t i = 0; i < lq; ++i) qr[i] = q[qend - i];
  for (int64_t j = 0; j < lr; ++j) rr[j] = r[rend - j];
  int64_t s, ei, ej;
  orc_fill(qr, lq, rr, lr, mat, n, o, e, NULL, &s, &ei, &ej);
  free(qr); free(rr);
  if (s != score1 || s <= 0) return -1;
  *qbeg = qend - ei;
  *rbeg = rend - ej;
  return 0;
}

/* ---- step 3, second route: start propagation --------------------------- */
typedef struct { int64_t s, jb, ib; } cand;

/* lexicographic max of (score, jb, ib) */
static cand cbetter(cand a, cand b) {
  if (a.s != b.s) return a.s > b.s ? a : b;
  if (a.jb != b.jb) return a.jb > b.jb ? a : b;
  return a.ib >= b.ib ? a : b;
}
static cand cadd(cand a, int64_t d) {
  if (a.s <= NEG_INF / 2) return a;
  a.s += d;
  return a;
}

int orc_begin_startprop(const int8_t *q, int64_t lq, const int8_t *r, int64_t lr,
                        const int8_t *mat, int32_t n, int32_t o, int32_t e,
                        int64_t qend, int64_t rend, int64_t score1,
                        int64_t *qbeg, int64_t *rbeg) {
  (void)lq; (void)lr;   /* only the prefix rectangle up to the end cell matters */
  const cand none = {NEG_INF, -1, -1};
  int64_t rows = qend + 1;
  if (rows <= 0) return -1;
  cand *hprev = (cand *)malloc(sizeof(cand) * rows);
  cand *hcur = (cand *)malloc(sizeof(cand) * rows);
  cand *erow = (cand *)malloc(sizeof(cand) * rows);
  for (int64_t i = 0; i < rows; ++i) { hprev[i] = none; erow[i] = none; }
  cand result = none;
  for (int64_t j = 0; j <= rend; ++j) {
    cand f = none;
    for (int64_t i = 0; i < rows; ++i) {
      int64_t sij = score_of(mat, n, q[i], r[j]);
      /* every alignment, no zero floor: fresh start here, or continue */
      cand fresh = {sij, j, i};
      cand diag = (i > 0) ? cadd(hprev[i - 1], sij) : none;
      cand eij = cbetter(cadd(erow[i], -e), cadd(hprev[i], -o));
      cand fij = cbetter(cadd(f, -e), (i > 0) ? cadd(hcur[i - 1], -o) : none);
      cand h = cbetter(cbetter(fresh, diag), cbetter(eij, fij));
      hcur[i] = h;
      erow[i] = eij;
      f = fij;
    }
    if (j == rend) result = hcur[qend];
    cand *t = hprev; hprev = hcur; hcur = t;
  }
  free(hprev); free(hcur); free(erow);
  if (result.s != score1) return -1;
  *qbeg = result.ib;
  *rbeg = result.jb;
  return 0;
}

/* ---- step 4: global DP on the begin..end rectangle and traceback -------- */
/* per-cell choice byte: bits 0-1 = H source (0 diag, 1 E, 2 F),
 * bit 2 = E opened here (from H), bit 3 = F opened here (from H) */
int64_t orc_traceback(const int8_t *q, const int8_t *r,
                      const int8_t *mat, int32_t n, int32_t o, int32_t e,
                      int64_t qbeg, int64_t qend, int64_t rbeg, int64_t rend,
                      uint32_t *cigar, int64_t cap, int64_t *score_out) {
  int64_t m = qend - qbeg + 1, w = rend - rbeg + 1;
  if (m <= 0 || w <= 0) { if (score_out) *score_out = 0; return 0; }
  int64_t W = w + 1;
  uint8_t *ch = (uint8_t *)malloc((size_t)((m + 1) * W));
  int64_t *hp = (int64_t *)malloc(sizeof(int64_t) * W);  /* H row i-1 */
  int64_t *hc = (int64_t *)malloc(sizeof(int64_t) * W);  /* H row i   */
  int64_t *fp = (int64_t *)malloc(sizeof(int64_t) * W);  /* F row i-1 */
  int64_t *fc = (int64_t *)malloc(sizeof(int64_t) * W);  /* F row i   */
  if (!ch || !hp || !hc || !fp || !fc) {
    free(ch); free(hp); free(hc); free(fp); free(fc);
    return -1;
  }
  /* row 0: H(0,0) = 0; H(0,j) = E(0,j) = -(o + (j-1)e) */
  hp[0] = 0; fp[0] = NEG_INF; ch[0] = 0;
  {
    int64_t ev = NEG_INF;
    for (int64_t j = 1; j <= w; ++j) {
      int64_t open = hp[j - 1] - o, ext = ev - e;
      ev = max2(ext, open);
      hp[j] = ev; fp[j] = NEG_INF;
      ch[j] = (uint8_t)(1 | ((open >= ext) ? 4 : 0));
    }
  }
  for (int64_t i = 1; i <= m; ++i) {
    /* column 0: H(i,0) = F(i,0) = -(o + (i-1)e) */
    int64_t fopen0 = hp[0] - o, fext0 = fp[0] - e;
    fc[0] = max2(fext0, fopen0);
    hc[0] = fc[0];
    ch[i * W] = (uint8_t)(2 | ((fopen0 >= fext0) ? 8 : 0));
    int64_t ev = NEG_INF;   /* E(i, j-1) */
    for (int64_t j = 1; j <= w; ++j) {
      int64_t eopen = hc[j - 1] - o, eext = ev - e;
      int64_t eij = max2(eext, eopen);
      int64_t fopen = hp[j] - o, fext = fp[j] - e;
      int64_t fij = max2(fext, fopen);
      int64_t diag = hp[j - 1] + score_of(mat, n, q[qbeg + i - 1], r[rbeg + j - 1]);
      int64_t h = max2(diag, max2(eij, fij));
      uint8_t c;
      if (h == diag) c = 0;
      else if (h == eij) c = 1;
      else c = 2;
      if (eopen >= eext) c |= 4;
      if (fopen >= fext) c |= 8;
      ch[i * W + j] = c;
      hc[j] = h; fc[j] = fij; ev = eij;
    }
    int64_t *t = hp; hp = hc; hc = t;
    t = fp; fp = fc; fc = t;
  }
  if (score_out) *score_out = hp[w];
  /* traceback from (m, w) in state H; ops collected end -> begin */
  int64_t cap_ops = m + w + 2;
  uint8_t *ops = (uint8_t *)malloc((size_t)cap_ops);
  int64_t nops = 0;
  int64_t i = m, j = w;
  int state = 0; /* 0 = H, 1 = E, 2 = F */
  while (i > 0 || j > 0) {
    uint8_t c = ch[i * W + j];
    if (state == 0) {
      int src = c & 3;
      if (src == 0 && i > 0 && j > 0) { ops[nops++] = 0; --i; --j; }
      else if (src == 1) state = 1;
      else state = 2;
    } else if (state == 1) {      /* D: consumes reference */
      ops[nops++] = 2;
      state = (c & 4) ? 0 : 1;
      --j;
    } else {                      /* I: consumes query */
      ops[nops++] = 1;
      state = (c & 8) ? 0 : 2;
      --i;
    }
  }
  free(ch); free(hp); free(hc); free(fp); free(fc);
  /* reverse and run-length encode */
  int64_t runs = 0;
  int64_t k = nops - 1;
  while (k >= 0) {
    uint8_t op = ops[k];
    int64_t len = 0;
    while (k >= 0 && ops[k] == op) { ++len; --k; }
    if (runs < cap) cigar[runs] = (uint32_t)((len << 4) | op);
    ++runs;
  }
  free(ops);
  return runs;
}

/* ---- step 5: second-best score from the masked max array --------------- */
void orc_score2(const int64_t *maxcol, int64_t lr, int64_t ref_begin1,
                int64_t ref_end1, int64_t mask_len,
                int64_t *score2, int64_t *ref_end2) {
  int64_t lo = ref_begin1 - mask_len, hi = ref_end1 + mask_len;
  int64_t best = 0, at = -1;
  for (int64_t j = 0; j < lr; ++j) {
    if (j >= lo && j <= hi) continue;
    if (maxcol[j] > best) { best = maxcol[j]; at = j; }
  }
  *score2 = best;
  *ref_end2 = best > 0 ? at : -1;
}

/* ---- the whole path ----------------------------------------------------- */
int orc_align(const int8_t *q, int64_t lq, const int8_t *r, int64_t lr,
              const int8_t *mat, int32_t n, int32_t o, int32_t e,
              uint32_t flags, int64_t mask_len,
              orc_result *res, uint32_t *cigar, int64_t cap, int64_t *maxcol_out) {
  if (flags & (ORC_FLAG_CIGAR | ORC_FLAG_SCORE2)) flags |= ORC_FLAG_BEGIN;
  if (mask_len < 0) mask_len = (lq / 2 > 15) ? lq / 2 : 15;
  res->score1 = 0; res->score2 = 0;
  res->read_begin1 = res->read_end1 = -1;
  res->ref_begin1 = res->ref_end1 = -1;
  res->ref_end2 = -1;
  res->cigar_len = 0;
  int64_t *maxcol = (int64_t *)malloc(sizeof(int64_t) * (lr > 0 ? lr : 1));
  if (!maxcol) return -1;
  int64_t s1, ie, je;
  orc_fill(q, lq, r, lr, mat, n, o, e, maxcol, &s1, &ie, &je);
  if (maxcol_out) memcpy(maxcol_out, maxcol, sizeof(int64_t) * (size_t)(lr > 0 ? lr : 0));
  res->score1 = s1;
  if (s1 <= 0) { free(maxcol); return 0; }       /* T5 */
  res->read_end1 = ie;
  res->ref_end1 = je;
  int rc = 0;
  if (flags & ORC_FLAG_BEGIN) {
    int64_t ib, jb;
    if (orc_begin_reverse(q, r, mat, n, o, e, ie, je, s1, &ib, &jb) != 0) rc = -1;
    else { res->read_begin1 = ib; res->ref_begin1 = jb; }
  }
  if (rc == 0 && (flags & ORC_FLAG_CIGAR)) {
    int64_t gs;
    int64_t runs = orc_traceback(q, r, mat, n, o, e, res->read_begin1, ie,
                                 res->ref_begin1, je, cigar, cap, &gs);
    if (runs < 0 || gs != s1) rc = -1;
    else res->cigar_len = runs;
  }
  if (rc == 0 && (flags & ORC_FLAG_SCORE2)) {
    orc_score2(maxcol, lr, res->ref_begin1, je, mask_len, &res->score2, &res->ref_end2);
  }
  free(maxcol);
  return rc;
}

/* ---- the suboptimal alignment (method section, Fig. 1 caption) ---------- */
/* The alignment behind score2: it ends in column ref_end2 at the smallest row
 * whose H equals score2; its begin is T2 relative to that end (largest jb,
 * then largest ib, among begins of alignments reaching the end with score
 * exactly score2 -- the start-propagation DP, which carries that begin for
 * every cell); its CIGAR is T3 on the begin..end rectangle. */
int64_t orc_column_row(const int8_t *q, int64_t lq, const int8_t *r, int64_t lr,
                       const int8_t *mat, int32_t n, int32_t o, int32_t e,
                       int64_t col, int64_t target) {
  if (lq <= 0 || col < 0 || col >= lr) return -1;
  /* the forward recurrence of orc_fill, columns 0..col, keeping column col */
  int64_t *hprev = (int64_t *)malloc(sizeof(int64_t) * lq);
  int64_t *hcur = (int64_t *)malloc(sizeof(int64_t) * lq);
  int64_t *erow = (int64_t *)malloc(sizeof(int64_t) * lq);
  for (int64_t i = 0; i < lq; ++i) { hprev[i] = 0; erow[i] = NEG_INF; }
  int64_t row = -1;
  for (int64_t j = 0; j <= col; ++j) {
    int64_t f = NEG_INF;
    for (int64_t i = 0; i < lq; ++i) {
      int64_t hdiag = (i > 0) ? hprev[i - 1] : 0;
      int64_t hup = (i > 0) ? hcur[i - 1] : 0;
      int64_t eij = max2(erow[i] - e, hprev[i] - o);
      int64_t fij = max2(f - e, hup - o);
      int64_t h = max2(max2(hdiag + score_of(mat, n, q[i], r[j]), eij), max2(fij, 0));
      hcur[i] = h;
      erow[i] = eij;
      f = fij;
      if (j == col && row < 0 && h == target) row = i;
    }
    int64_t *t = hprev; hprev = hcur; hcur = t;
  }
  free(hprev); free(hcur); free(erow);
  return row;
}

int orc_suboptimal(const int8_t *q, int64_t lq, const int8_t *r, int64_t lr,
                   const int8_t *mat, int32_t n, int32_t o, int32_t e,
                   int64_t score2, int64_t ref_end2,
                   orc_sub *res, uint32_t *cigar, int64_t cap) {
  res->read_begin2 = res->read_end2 = res->ref_begin2 = -1;
  res->cigar_len = 0;
  if (score2 <= 0) return 0;
  int64_t ie = orc_column_row(q, lq, r, lr, mat, n, o, e, ref_end2, score2);
  if (ie < 0) return -1;
  int64_t ib, jb;
  if (orc_begin_startprop(q, lq, r, lr, mat, n, o, e, ie, ref_end2, score2, &ib, &jb) != 0)
    return -1;
  int64_t gs;
  int64_t runs = orc_traceback(q, r, mat, n, o, e, ib, ie, jb, ref_end2, cigar, cap, &gs);
  if (runs < 0 || gs != score2) return -1;
  res->read_begin2 = ib;
  res->read_end2 = ie;
  res->ref_begin2 = jb;
  res->cigar_len = runs;
  return 0;
}

typedef struct {
  const int8_t *qcat; const int64_t *qoff;
  const int8_t *rcat; const int64_t *roff;
  const int64_t *pq, *pr; int64_t npairs;
  const int8_t *mat; int32_t n, o, e;
  const int64_t *score2, *ref_end2;
  orc_sub *res; uint32_t *cigar; const int64_t *coff;
  int64_t next, failures;
  pthread_mutex_t mu;
} sub_ctx;

static void *sub_worker(void *arg) {
  sub_ctx *c = (sub_ctx *)arg;
  for (;;) {
    pthread_mutex_lock(&c->mu);
    int64_t p = c->next++;
    pthread_mutex_unlock(&c->mu);
    if (p >= c->npairs) break;
    int64_t qi = c->pq[p], ri = c->pr[p];
    uint32_t *cg = NULL; int64_t cap = 0;
    if (c->cigar && c->coff) { cg = c->cigar + c->coff[p]; cap = c->coff[p + 1] - c->coff[p]; }
    if (orc_suboptimal(c->qcat + c->qoff[qi], c->qoff[qi + 1] - c->qoff[qi],
                       c->rcat + c->roff[ri], c->roff[ri + 1] - c->roff[ri],
                       c->mat, c->n, c->o, c->e, c->score2[p], c->ref_end2[p],
                       &c->res[p], cg, cap) != 0) {
      pthread_mutex_lock(&c->mu);
      c->failures++;
      pthread_mutex_unlock(&c->mu);
    }
  }
  return NULL;
}

int64_t orc_suboptimal_many(const int8_t *qcat, const int64_t *qoff,
                            const int8_t *rcat, const int64_t *roff,
                            const int64_t *pair_q, const int64_t *pair_r, int64_t npairs,
                            const int8_t *mat, int32_t n, int32_t o, int32_t e,
                            const int64_t *score2, const int64_t *ref_end2,
                            orc_sub *res, uint32_t *cigar, const int64_t *cigar_off,
                            int32_t nthreads) {
  sub_ctx c;
  c.qcat = qcat; c.qoff = qoff; c.rcat = rcat; c.roff = roff;
  c.pq = pair_q; c.pr = pair_r; c.npairs = npairs;
  c.mat = mat; c.n = n; c.o = o; c.e = e;
  c.score2 = score2; c.ref_end2 = ref_end2;
  c.res = res; c.cigar = cigar; c.coff = cigar_off;
  c.next = 0; c.failures = 0;
  pthread_mutex_init(&c.mu, NULL);
  if (nthreads < 1) nthreads = 1;
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  for (int32_t t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, sub_worker, &c);
  for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&c.mu);
  return c.failures;
}

/* ---- many pairs over threads ------------------------------------------- */
typedef struct {
  const int8_t *qcat; const int64_t *qoff;
  const int8_t *rcat; const int64_t *roff;
  const int64_t *pq, *pr; int64_t npairs;
  const int8_t *mat; int32_t n, o, e;
  uint32_t flags; int64_t mask_len;
  orc_result *res; uint32_t *cigar; const int64_t *coff;
  int64_t next;             /* shared task counter */
  int64_t failures;
  pthread_mutex_t mu;
} many_ctx;

static void *many_worker(void *arg) {
  many_ctx *c = (many_ctx *)arg;
  for (;;) {
    pthread_mutex_lock(&c->mu);
    int64_t p = c->next++;
    pthread_mutex_unlock(&c->mu);
    if (p >= c->npairs) break;
    int64_t qi = c->pq[p], ri = c->pr[p];
    const int8_t *q = c->qcat + c->qoff[qi];
    const int8_t *r = c->rcat + c->roff[ri];
    int64_t lq = c->qoff[qi + 1] - c->qoff[qi];
    int64_t lr = c->roff[ri + 1] - c->roff[ri];
    uint32_t *cg = NULL; int64_t cap = 0;
    if (c->cigar && c->coff) { cg = c->cigar + c->coff[p]; cap = c->coff[p + 1] - c->coff[p]; }
    if (orc_align(q, lq, r, lr, c->mat, c->n, c->o, c->e, c->flags, c->mask_len,
                  &c->res[p], cg, cap, NULL) != 0) {
      pthread_mutex_lock(&c->mu);
      c->failures++;
      pthread_mutex_unlock(&c->mu);
    }
  }
  return NULL;
}

int64_t orc_align_many(const int8_t *qcat, const int64_t *qoff,
                       const int8_t *rcat, const int64_t *roff,
                       const int64_t *pair_q, const int64_t *pair_r, int64_t npairs,
                       const int8_t *mat, int32_t n, int32_t o, int32_t e,
                       uint32_t flags, int64_t mask_len,
                       orc_result *res, uint32_t *cigar, const int64_t *cigar_off,
                       int32_t nthreads) {
  many_ctx c;
  c.qcat = qcat; c.qoff = qoff; c.rcat = rcat; c.roff = roff;
  c.pq = pair_q; c.pr = pair_r; c.npairs = npairs;
  c.mat = mat; c.n = n; c.o = o; c.e = e;
  c.flags = flags; c.mask_len = mask_len;
  c.res = res; c.cigar = cigar; c.coff = cigar_off;
  c.next = 0; c.failures = 0;
  pthread_mutex_init(&c.mu, NULL);
  if (nthreads < 1) nthreads = 1;
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  for (int32_t t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, many_worker, &c);
  for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&c.mu);
  return c.failures;
}
