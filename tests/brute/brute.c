/*
 * brute.c -- exhaustive enumeration of local alignments, used only by the
 * tests to pin the oracle.  It uses no dynamic programming: it walks every
 * op string (M, I, D) from every start cell by depth-first search and scores
 * each one directly with the affine model (a gap of length k costs o+(k-1)e).
 * It shares no code with the oracle or with the GPU library.
 *
 * Every prefix of a walk is itself an alignment; its "cell" is
 * (last query index consumed, last reference index consumed).  A walk always
 * starts with an M at its begin cell.
 *
 * Outputs for one pair:
 *   score1           largest score over all alignments (0 if none positive)
 *   maxcol[j]        max(0, best score of an alignment whose cell has column j)
 *   (ie, je)         among cells of score1 alignments: smallest j, then i
 *   (ib, jb)         among begins of score1 alignments whose cell is (ie, je):
 *                    largest jb, then largest ib
 *   ops              among score1 state paths from (ib, jb) to (ie, je): the
 *                    op string of the path whose backward choice digits are
 *                    smallest (state H: M=0 < D=1 < I=2; each gap symbol:
 *                    opening = 0, extending the gap state = 1).
 *
 * A state path is an op string plus, for every gap symbol that follows a gap
 * symbol of the same kind, whether it extends the gap (cost e) or opens a new
 * one straight after it (cost o: the gap state is left for H and entered
 * again, which the three-state recurrence allows).  For o > e a re-opened
 * run scores less than the extended one, so the op string alone fixes the
 * best path; for o == e both score the same and the digits decide between
 * them.  Pass 3 enumerates both choices; passes 1 and 2 need only the
 * extending one, since re-opening never raises a score (o >= e).
 */
#include <stdint.h>
#include <string.h>

#define MAXL 16
#define MAXOPS (2 * MAXL + 2)

typedef struct {
  const int8_t *q, *r, *mat;
  int lq, lr, n, o, e;
  int pass;
  /* pass 1 */
  int64_t best;
  int64_t maxcol[MAXL];
  int ie, je;
  /* pass 2 */
  int ib, jb, have_begin;
  /* pass 3 */
  uint8_t ops[MAXOPS];
  uint8_t opn[MAXOPS];   /* per op: 1 when a gap symbol opens its gap (or op is M) */
  int nops;
  uint8_t best_dig[4 * MAXOPS];
  int best_ndig, have_path;
  uint8_t best_ops[MAXOPS];
  int best_nops;
} bctx;

static int sc(const bctx *c, int i, int j) { return c->mat[c->q[i] * c->n + c->r[j]]; }

/* backward choice digits of a state path (forward order ops[0..nops), with
 * opn[k] = 1 when gap symbol k opens its gap) */
static int digits(const uint8_t *ops, const uint8_t *opn, int nops, uint8_t *dig) {
  int nd = 0;
  int k = nops - 1;
  while (k >= 0) {
    uint8_t op = ops[k];
    if (op == 0) { dig[nd++] = 0; --k; continue; }
    dig[nd++] = (op == 2) ? 1 : 2;   /* H picks D (state E) or I (state F) */
    /* inside the gap state: emit the symbol, then leave it (open) or stay
     * (extend: the previous symbol is the same gap kind) */
    for (;;) {
      const int open = opn[k];
      dig[nd++] = open ? 0 : 1;
      --k;
      if (open) break;
    }
  }
  return nd;
}

static int dig_less(const uint8_t *a, int na, const uint8_t *b, int nb) {
  int m = na < nb ? na : nb;
  for (int k = 0; k < m; ++k)
    if (a[k] != b[k]) return a[k] < b[k];
  return na < nb;
}

static void visit(bctx *c, int i, int j, int64_t s, int i0, int j0) {
  if (c->pass == 4) {   /* smallest row of a cell in column je with score best */
    if (j == c->je && s == c->best && (c->ie < 0 || i < c->ie)) c->ie = i;
    return;
  }
  if (c->pass == 1) {
    if (s > c->maxcol[j]) c->maxcol[j] = s;
    if (s > c->best) {
      c->best = s; c->ie = i; c->je = j;
    } else if (s == c->best && s > 0 && (j < c->je || (j == c->je && i < c->ie))) {
      c->ie = i; c->je = j;
    }
  } else if (c->pass == 2) {
    if (s == c->best && i == c->ie && j == c->je) {
      if (!c->have_begin || j0 > c->jb || (j0 == c->jb && i0 > c->ib)) {
        c->have_begin = 1; c->ib = i0; c->jb = j0;
      }
    }
  } else {
    if (s == c->best && i == c->ie && j == c->je) {
      uint8_t dig[4 * MAXOPS];
      int nd = digits(c->ops, c->opn, c->nops, dig);
      if (!c->have_path || dig_less(dig, nd, c->best_dig, c->best_ndig)) {
        c->have_path = 1;
        memcpy(c->best_dig, dig, (size_t)nd); c->best_ndig = nd;
        memcpy(c->best_ops, c->ops, (size_t)c->nops); c->best_nops = c->nops;
      }
    }
  }
}

static void walk(bctx *c, int i, int j, int64_t s, uint8_t last, int i0, int j0) {
  visit(c, i, j, s, i0, j0);
  if (i + 1 < c->lq && j + 1 < c->lr) {
    c->opn[c->nops] = 1;
    c->ops[c->nops++] = 0;
    walk(c, i + 1, j + 1, s + sc(c, i + 1, j + 1), 0, i0, j0);
    c->nops--;
  }
  for (int g = 0; g < 2; ++g) {   /* g = 0: D consumes the reference; g = 1: I the query */
    const uint8_t op = g == 0 ? 2 : 1;
    const int ni = g == 0 ? i : i + 1, nj = g == 0 ? j + 1 : j;
    if (ni >= c->lq || nj >= c->lr) continue;
    /* after a symbol of the same gap: extend; in pass 3 also re-open */
    for (int open = (last == op) ? 0 : 1; open <= 1; ++open) {
      if (open && last == op && c->pass != 3) break;
      c->opn[c->nops] = (uint8_t)open;
      c->ops[c->nops++] = op;
      walk(c, ni, nj, s - (open ? c->o : c->e), op, i0, j0);
      c->nops--;
    }
  }
}

static void run_from(bctx *c, int i0, int j0) {
  c->nops = 0;
  c->opn[c->nops] = 1;
  c->ops[c->nops++] = 0;
  walk(c, i0, j0, sc(c, i0, j0), 0, i0, j0);
}

/* returns 0, or -1 when the inputs exceed MAXL */
int brute_align(const int8_t *q, int lq, const int8_t *r, int lr,
                const int8_t *mat, int n, int o, int e,
                int64_t *score1, int64_t *maxcol, int *ends, int *begins,
                uint8_t *ops_out, int *nops_out) {
  if (lq > MAXL || lr > MAXL || lq < 0 || lr < 0) return -1;
  bctx c;
  memset(&c, 0, sizeof c);
  c.q = q; c.r = r; c.mat = mat; c.lq = lq; c.lr = lr; c.n = n; c.o = o; c.e = e;
  c.ie = c.je = -1;
  c.pass = 1;
  for (int i0 = 0; i0 < lq; ++i0)
    for (int j0 = 0; j0 < lr; ++j0) run_from(&c, i0, j0);
  *score1 = c.best;
  for (int j = 0; j < lr; ++j) maxcol[j] = c.maxcol[j];
  ends[0] = ends[1] = begins[0] = begins[1] = -1;
  *nops_out = 0;
  if (c.best <= 0) return 0;
  ends[0] = c.ie; ends[1] = c.je;
  c.pass = 2;
  for (int i0 = 0; i0 < lq; ++i0)
    for (int j0 = 0; j0 < lr; ++j0) run_from(&c, i0, j0);
  begins[0] = c.ib; begins[1] = c.jb;
  c.pass = 3;
  run_from(&c, c.ib, c.jb);
  memcpy(ops_out, c.best_ops, (size_t)c.best_nops);
  *nops_out = c.best_nops;
  return 0;
}

/* The alignment behind a given (score s, column je), found the same way:
 * the smallest row ie of a cell in column je reached by an alignment of
 * score s; then, among alignments of score s whose cell is (ie, je), the
 * begin with the largest jb, then the largest ib; then the op string with the
 * smallest backward choice digits.  Returns 0 (ends/begins -1 when no
 * alignment of score s ends in column je), or -1 when inputs exceed MAXL. */
int brute_sub(const int8_t *q, int lq, const int8_t *r, int lr,
              const int8_t *mat, int n, int o, int e, int je, int64_t s,
              int *ends, int *begins, uint8_t *ops_out, int *nops_out) {
  if (lq > MAXL || lr > MAXL || lq < 0 || lr < 0) return -1;
  bctx c;
  memset(&c, 0, sizeof c);
  c.q = q; c.r = r; c.mat = mat; c.lq = lq; c.lr = lr; c.n = n; c.o = o; c.e = e;
  c.best = s; c.ie = -1; c.je = je;
  ends[0] = ends[1] = begins[0] = begins[1] = -1;
  *nops_out = 0;
  c.pass = 4;
  for (int i0 = 0; i0 < lq; ++i0)
    for (int j0 = 0; j0 < lr; ++j0) run_from(&c, i0, j0);
  if (c.ie < 0) return 0;
  ends[0] = c.ie; ends[1] = je;
  c.pass = 2;
  for (int i0 = 0; i0 < lq; ++i0)
    for (int j0 = 0; j0 < lr; ++j0) run_from(&c, i0, j0);
  begins[0] = c.ib; begins[1] = c.jb;
  c.pass = 3;
  run_from(&c, c.ib, c.jb);
  memcpy(ops_out, c.best_ops, (size_t)c.best_nops);
  *nops_out = c.best_nops;
  return 0;
}
