"""The reversed pass's drift band is exact (Method: reversed SW from the end).

The GPU reversed pass evaluates only the cells of reverse(q[0..ie]) x
reverse(r[0..je]) with  i - j <= Gq  and  j - i <= Gr  (reversed row i,
column j; cells outside hold values no higher than the true ones), where

    G' = (smax*min(ie+1, je+1) - o + e - score1) / e
    Gq = min(G', (smax*(ie+1) - o + e - score1) / (smax + e))
    Gr = min(G', (smax*(je+1) - o + e - score1) / (smax + e))

(floors, clamped at 0).  Here the band is checked by brute force: the
reversed local DP with every cell outside the band at its lowest value (H 0,
no gap state) must find the same begin (T2: first reversed column reaching
score1, smallest reversed row there) as the oracle's unbanded one.  The DP is
written out in this file; it shares nothing with the oracle or the library.
"""
from __future__ import annotations

import numpy as np

import oracle
from workloads import dna_matrix, mutate_many, protein_matrix_standin

NEG = -(10 ** 9)


def _bands(smax, o, e, ie, je, s1):
    base = -o + e - s1
    gp = max(0, (smax * min(ie + 1, je + 1) + base) // e)
    gq = min(gp, max(0, (smax * (ie + 1) + base) // (smax + e)))
    gr = min(gp, max(0, (smax * (je + 1) + base) // (smax + e)))
    return gq, gr


def _banded_reverse_begin(q, r, mat, o, e, ie, je, s1, lo, hi):
    """Begin by the reversed local DP with cells where i - j > lo or j - i > hi
    held out.  Returns (qbeg, rbeg, best) with best the banded maximum."""
    m, n = ie + 1, je + 1
    hprev = [0] * (n + 1)
    fprev = [NEG] * (n + 1)
    hit = None          # (reversed column, reversed row) of the first cell at s1
    best = 0
    for i in range(m):
        h = [0] * (n + 1)
        f = [NEG] * (n + 1)
        ev = NEG
        qi = int(q[ie - i])
        for j in range(n):
            if i - j > lo or j - i > hi:
                ev = NEG
                continue
            ev = max(ev - e, h[j] - o)
            f[j + 1] = max(fprev[j + 1] - e, hprev[j + 1] - o)
            v = max(0, hprev[j] + int(mat[qi, r[je - j]]), ev, f[j + 1])
            h[j + 1] = v
            best = max(best, v)
            if v == s1 and (hit is None or (j, i) < hit):
                hit = (j, i)
        hprev, fprev = h, f
    if hit is None:
        return None, None, best
    return ie - hit[1], je - hit[0], best


def _cases():
    g = np.random.Generator(np.random.PCG64(1208_6350))
    dna = dna_matrix()
    for k in range(90):
        lr = int(g.integers(20, 90))
        lq = int(g.integers(8, min(lr, 45)))
        r = g.integers(0, 4, size=lr).astype(np.int8)
        p = int(g.integers(0, lr - lq + 1))
        sub = [0.0, 0.03, 0.1][k % 3]
        indel = [0.0, 0.05, 0.15][(k // 3) % 3]
        q, _ = mutate_many(g, r[p:p + lq], np.array([0, lq]), sub, indel / 2, indel / 2, 3)
        if k % 9 == 0:
            q = g.integers(0, 4, size=lq).astype(np.int8)     # no true hit
        if len(q) == 0:
            continue
        o, e = [(3, 1), (2, 2), (5, 1), (1, 1)][k % 4]
        yield q, r, dna, o, e
    prot = protein_matrix_standin()
    for k in range(20):
        lr = int(g.integers(20, 60))
        lq = int(g.integers(8, 30))
        r = g.integers(0, prot.shape[0], size=lr).astype(np.int8)
        p = int(g.integers(0, max(1, lr - lq + 1)))
        q = r[p:p + lq].copy()
        for _ in range(int(g.integers(0, 4))):
            q[int(g.integers(0, len(q)))] = int(g.integers(0, prot.shape[0]))
        yield q, r, prot, 11, 1


def test_reverse_drift_band_keeps_the_begin():
    active = 0
    for q, r, mat, o, e in _cases():
        a = oracle.align(q, r, mat, o, e, flags=oracle.FLAG_ALL)
        if a.score1 <= 0:
            continue
        ie, je, s1 = a.read_end1, a.ref_end1, a.score1
        smax = int(np.max(mat))
        gq, gr = _bands(smax, o, e, ie, je, s1)
        if gq < ie or gr < je:
            active += 1
        qb, rb, best = _banded_reverse_begin(q, r, mat, o, e, ie, je, s1, gq, gr)
        assert best == s1, (o, e, ie, je, s1, gq, gr)
        assert (qb, rb) == (a.read_begin1, a.ref_begin1), (o, e, ie, je, s1, gq, gr)
    assert active >= 40   # the band leaves cells out in most cases


def test_query_side_is_tighter_than_the_symmetric_band():
    # a 100-row reversed region against 300 columns at score 180, +2/-2/3/1:
    # G' = 200 - 2 - 180 = 18 on both sides, the query side (insertions also
    # use up rows) 18 // 3 = 6
    assert _bands(2, 3, 1, 99, 299, 180) == (6, 18)
