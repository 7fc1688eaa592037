"""Pins of the CPU oracle against facts fixed outside the oracle itself.

* P1: exhaustive enumeration of all local alignments (tests/brute) on short
  sequences fixes score1, the max array, the T1 end, the T2 begin and the T3
  CIGAR (the state path with the smallest backward choice-digit string; the
  enumeration covers re-opened gap runs, so o == e is pinned too), at every
  gap setting o >= e >= 0 including o == e and o == 0.
* P2: closed forms (self-alignment, exact substring, one substitution, one
  deletion, one-symbol query).
* P3: special cases that reduce to textbook routines (Kadane's maximum
  subarray when no gap can pay; one-matrix linear-gap SW when o == e).
* P4: the begin from the reversed pass equals the begin from start
  propagation.
* P5: invariants (score bounds, reversal, CIGAR re-scoring, first/last op,
  max-array consistency, monotonicity, the deletion-tail bound on score2).

The paper prints no worked example with sequences (its Figure 1 is an image
that is not available), so no value here comes from the paper's text.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
from tests import brute
from tests.helpers import kadane_local, rescore, score2_from_maxcol, textbook_linear_sw
from workloads import dna_matrix, mutate_many, protein_matrix_standin

GAPS = [(3, 1), (2, 1), (5, 2), (11, 1), (1, 1), (4, 4), (3, 0), (0, 0), (2, 2), (3, 3)]


def _check_against_brute(q, r, mat, o, e):
    b = brute.enumerate_align(q, r, mat, o, e)
    a, maxcol = oracle.align(q, r, mat, o, e, with_maxcol=True)
    s1, ie, je, mc = oracle.fill(q, r, mat, o, e)
    assert s1 == b["score1"] == a.score1
    assert list(mc) == list(b["maxcol"])
    assert list(maxcol) == list(b["maxcol"])
    if b["score1"] <= 0:
        assert (a.read_end1, a.ref_end1, a.read_begin1, a.ref_begin1) == (-1, -1, -1, -1)
        assert a.cigar == [] and a.score2 == 0 and a.ref_end2 == -1
        return
    assert (ie, je) == b["end"] == (a.read_end1, a.ref_end1)
    assert (a.read_begin1, a.ref_begin1) == b["begin"]
    sp = oracle.begin_startprop(q, r, mat, o, e, ie, je, s1)
    assert sp == b["begin"]
    sc, cq, cr = rescore(q, r, mat, o, e, a.read_begin1, a.ref_begin1, a.cigar)
    assert sc == a.score1
    assert cq == a.read_end1 - a.read_begin1 + 1 and cr == a.ref_end1 - a.ref_begin1 + 1
    assert a.cigar == b["cigar"]
    m = max(len(q) // 2, 15)
    assert (a.score2, a.ref_end2) == score2_from_maxcol(b["maxcol"], a.ref_begin1, a.ref_end1, m)


@pytest.mark.parametrize("o,e", [(3, 1), (2, 1), (1, 1), (5, 2), (2, 2), (0, 0), (3, 0)])
def test_brute_all_ternary_pairs_len3(o, e):
    """Every pair of length-3 sequences over 3 symbols (729 pairs)."""
    mat = np.array([[2, -1, -2], [-1, 2, -1], [-2, -1, 3]], dtype=np.int8)
    seqs = [np.array(s, dtype=np.int8) for s in itertools.product(range(3), repeat=3)]
    for q in seqs:
        for r in seqs:
            _check_against_brute(q, r, mat, o, e)


@pytest.mark.parametrize("o,e", GAPS)
def test_brute_random_dna(o, e):
    g = np.random.Generator(np.random.PCG64(1000 + 7 * o + e))
    for _ in range(60):
        lq, lr = int(g.integers(1, 9)), int(g.integers(1, 9))
        mm = -int(g.integers(1, 4))
        mat = dna_matrix(2, mm)
        q = g.integers(0, 4, size=lq).astype(np.int8)
        r = g.integers(0, 4, size=lr).astype(np.int8)
        _check_against_brute(q, r, mat, o, e)


def test_brute_random_matrix_and_protein():
    g = np.random.Generator(np.random.PCG64(4242))
    prot = protein_matrix_standin()
    for k in range(120):
        lq, lr = int(g.integers(1, 8)), int(g.integers(1, 8))
        if k % 2 == 0:
            n = 5
            mat = g.integers(-4, 5, size=(n, n)).astype(np.int8)   # asymmetric on purpose
        else:
            n, mat = 24, prot
        o, e = GAPS[k % len(GAPS)]
        q = g.integers(0, n, size=lq).astype(np.int8)
        r = g.integers(0, n, size=lr).astype(np.int8)
        _check_against_brute(q, r, mat, o, e)


def test_brute_planted_len8():
    """Mutated copies, so that gaps actually occur in optimal alignments."""
    g = np.random.Generator(np.random.PCG64(77))
    mat = dna_matrix()
    for k in range(80):
        lr = int(g.integers(5, 9))
        r = g.integers(0, 4, size=lr).astype(np.int8)
        q, _ = mutate_many(g, r, np.array([0, lr]), 0.1, 0.15, 0.15, 2)
        q = q[:8]
        if len(q) == 0:
            continue
        o, e = [(3, 1), (2, 1), (1, 1), (4, 1), (2, 2), (3, 3), (0, 0)][k % 7]
        _check_against_brute(q, r, mat, o, e)


# ---------------------------------------------------------------- P2
def test_self_alignment_closed_form():
    g = np.random.Generator(np.random.PCG64(5))
    for L in (1, 7, 50, 300):
        s = g.integers(0, 4, size=L).astype(np.int8)
        a = oracle.align(s, s, dna_matrix(2, -3), 3, 1)
        assert a.score1 == 2 * L
        assert (a.read_begin1, a.ref_begin1, a.read_end1, a.ref_end1) == (0, 0, L - 1, L - 1)
        assert a.cigar == [(L, "M")]


def test_exact_substring_and_single_edits():
    g = np.random.Generator(np.random.PCG64(6))
    mat = dna_matrix()
    ref = g.integers(0, 4, size=3000).astype(np.int8)
    L, p = 60, 1234
    q = ref[p:p + L].copy()
    a = oracle.align(q, ref, mat, 3, 1)
    assert a.score1 == 2 * L and a.ref_begin1 == p and a.ref_end1 == p + L - 1
    assert a.cigar == [(L, "M")]
    # one interior substitution
    q2 = q.copy()
    q2[30] = (q2[30] + 1) % 4
    a = oracle.align(q2, ref, mat, 3, 1)
    assert a.score1 == 2 * L - 4 and a.ref_begin1 == p and a.cigar == [(L, "M")]
    # one interior deletion of k reference symbols
    for k in (1, 2, 3):
        qd = np.concatenate([ref[p:p + 30], ref[p + 30 + k:p + L + k]])
        a = oracle.align(qd, ref, mat, 3, 1)
        assert a.score1 == 2 * L - 3 - (k - 1) * 1
        ops = [op for _, op in a.cigar]
        assert ops == ["M", "D", "M"] and a.cigar[1][0] == k
        assert a.cigar[0][0] + a.cigar[2][0] == L


def test_one_symbol_query():
    g = np.random.Generator(np.random.PCG64(8))
    mat = protein_matrix_standin()
    for _ in range(50):
        r = g.integers(0, 24, size=int(g.integers(1, 40))).astype(np.int8)
        q = g.integers(0, 24, size=1).astype(np.int8)
        vals = mat[q[0], r].astype(int)
        a = oracle.align(q, r, mat, 11, 1)
        best = max(0, vals.max())
        assert a.score1 == best
        if best > 0:
            assert a.ref_end1 == int(np.nonzero(vals == best)[0][0]) == a.ref_begin1
            assert a.cigar == [(1, "M")]


# ---------------------------------------------------------------- P3
def test_no_gap_pays_reduces_to_kadane():
    g = np.random.Generator(np.random.PCG64(9))
    for k in range(40):
        n = 4 if k % 2 else 24
        mat = dna_matrix(3, -2) if n == 4 else protein_matrix_standin()
        lq, lr = int(g.integers(1, 40)), int(g.integers(1, 60))
        q = g.integers(0, n, size=lq).astype(np.int8)
        r = g.integers(0, n, size=lr).astype(np.int8)
        if k % 3 == 0 and lr > 5:        # plant a copy so the best segment is long
            ln = min(lq, lr)
            q[:ln] = r[:ln]
        smax = int(mat.max())
        o = 2 * smax * min(lq, lr) + 1
        s1, mc, end, begin = kadane_local(q, r, mat)
        a, maxcol = oracle.align(q, r, mat, o, 1, with_maxcol=True)
        assert a.score1 == s1
        assert list(maxcol) == list(mc)
        if s1 > 0:
            assert (a.read_end1, a.ref_end1) == end
            assert (a.read_begin1, a.ref_begin1) == begin
            assert a.cigar == [(a.read_end1 - a.read_begin1 + 1, "M")]


def test_linear_gaps_match_textbook():
    g = np.random.Generator(np.random.PCG64(10))
    for k in range(30):
        mat = dna_matrix(2, -1 - (k % 3))
        lq, lr = int(g.integers(1, 30)), int(g.integers(1, 40))
        r = g.integers(0, 4, size=lr).astype(np.int8)
        q, _ = mutate_many(g, r[:lq], np.array([0, min(lq, lr)]), 0.1, 0.1, 0.1, 3)
        if len(q) == 0:
            q = np.array([1], dtype=np.int8)
        gpen = 1 + (k % 3)
        s1, mc = textbook_linear_sw(q, r, mat, gpen)
        a, maxcol = oracle.align(q, r, mat, gpen, gpen, with_maxcol=True)
        assert a.score1 == s1
        assert list(maxcol) == list(mc)


# ---------------------------------------------------------------- P4 / P5
def _planted_pair(g, lr, lq, sub=0.03, indel=0.01):
    r = g.integers(0, 4, size=lr).astype(np.int8)
    p = int(g.integers(0, lr - lq + 1))
    q, _ = mutate_many(g, r[p:p + lq], np.array([0, lq]), sub, indel / 2, indel / 2, 3)
    return q, r


def test_begin_two_routes_agree_medium():
    g = np.random.Generator(np.random.PCG64(11))
    mat = dna_matrix()
    for k in range(60):
        q, r = _planted_pair(g, int(g.integers(150, 400)), int(g.integers(20, 150)))
        if k % 5 == 0:
            q = g.integers(0, 4, size=len(q)).astype(np.int8)   # random read
        s1, ie, je, _ = oracle.fill(q, r, mat, 3, 1)
        if s1 == 0:
            continue
        assert oracle.begin_reverse(q, r, mat, 3, 1, ie, je, s1) == \
            oracle.begin_startprop(q, r, mat, 3, 1, ie, je, s1)


def test_invariants_random_medium():
    g = np.random.Generator(np.random.PCG64(12))
    for k in range(60):
        n = 4 if k % 3 else 24
        mat = dna_matrix() if n == 4 else protein_matrix_standin()
        o, e = ((3, 1), (5, 2), (11, 1), (2, 2))[k % 4]
        if n == 4:
            q, r = _planted_pair(g, int(g.integers(60, 300)), int(g.integers(10, 60)))
        else:
            r = g.integers(0, n, size=int(g.integers(30, 200))).astype(np.int8)
            q = g.integers(0, n, size=int(g.integers(10, 80))).astype(np.int8)
        a, maxcol = oracle.align(q, r, mat, o, e, with_maxcol=True)
        m = max(len(q) // 2, 15)
        # I1
        assert a.score1 >= a.score2 >= 0
        # I2: reversing both sequences keeps score1
        ar = oracle.align(q[::-1], r[::-1], mat, o, e)
        assert ar.score1 == a.score1
        if a.score1 == 0:
            continue
        # I3
        sc, cq, cr = rescore(q, r, mat, o, e, a.read_begin1, a.ref_begin1, a.cigar)
        assert sc == a.score1
        assert cq == a.read_end1 - a.read_begin1 + 1 and cr == a.ref_end1 - a.ref_begin1 + 1
        # I4
        assert a.cigar[0][1] == "M" and a.cigar[-1][1] == "M"
        assert mat[q[a.read_begin1], r[a.ref_begin1]] > 0
        assert mat[q[a.read_end1], r[a.ref_end1]] > 0
        # I5
        assert maxcol[a.ref_end1] == a.score1 and maxcol.max() == a.score1
        assert not (maxcol[:a.ref_end1] == a.score1).any()
        # I8: the primary's deletion tail bounds score2 from below
        if a.ref_end1 + m + 1 < len(r):
            assert a.score2 >= a.score1 - o - m * e
        # score2 by its definition
        assert (a.score2, a.ref_end2) == score2_from_maxcol(maxcol, a.ref_begin1, a.ref_end1, m)


def test_monotonicity():
    g = np.random.Generator(np.random.PCG64(13))
    for _ in range(20):
        q, r = _planted_pair(g, 120, 40, sub=0.08, indel=0.05)
        base = oracle.align(q, r, dna_matrix(2, -2), 3, 1).score1
        assert oracle.align(q, r, dna_matrix(3, -2), 3, 1).score1 >= base
        assert oracle.align(q, r, dna_matrix(2, -2), 4, 1).score1 <= base
        assert oracle.align(q, r, dna_matrix(2, -2), 3, 2).score1 <= base


def test_no_alignment_cases():
    mat = dna_matrix()
    a = oracle.align(np.array([0, 1], np.int8), np.zeros(0, np.int8), mat, 3, 1)
    assert a.score1 == 0 and a.ref_end1 == -1 and a.cigar == [] and a.ref_end2 == -1
    neg = np.full((4, 4), -1, dtype=np.int8)
    a = oracle.align(np.array([0, 1, 2], np.int8), np.array([0, 1, 2], np.int8), neg, 3, 1)
    assert a.score1 == 0 and a.read_begin1 == -1 and a.score2 == 0


def test_flags_and_mask_len():
    g = np.random.Generator(np.random.PCG64(14))
    q, r = _planted_pair(g, 400, 100)
    mat = dna_matrix()
    full, maxcol = oracle.align(q, r, mat, 3, 1, with_maxcol=True)
    only = oracle.align(q, r, mat, 3, 1, flags=0)
    assert only.score1 == full.score1 and only.ref_end1 == full.ref_end1
    assert only.ref_begin1 == -1 and only.cigar == [] and only.score2 == 0
    for m in (0, 5, 40):
        a = oracle.align(q, r, mat, 3, 1, flags=oracle.FLAG_SCORE2, mask_len=m)
        assert (a.score2, a.ref_end2) == score2_from_maxcol(maxcol, full.ref_begin1,
                                                            full.ref_end1, m)


def test_align_many_matches_single():
    from workloads import random_pairs
    b = random_pairs(99, 50, (5, 80), (5, 200))
    rec, cig, coff = oracle.align_many(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r,
                                       b.matrix, b.gap_open, b.gap_extend, nthreads=4)
    for p in range(b.npairs):
        a = oracle.align(b.query(p), b.ref(p), b.matrix, b.gap_open, b.gap_extend)
        assert list(rec[p][:7]) == [a.score1, a.score2, a.read_begin1, a.read_end1,
                                    a.ref_begin1, a.ref_end1, a.ref_end2]
        assert oracle.decode_cigar(cig[coff[p]:coff[p] + rec[p][7]]) == a.cigar


def test_brute_open_extend_tie():
    """A case where opening and extending a deletion tie on an optimal path
    (o - e small); the stated rule takes "open" first in the backward walk."""
    q = np.array([3, 3, 2, 1, 3, 2, 2], dtype=np.int8)
    r = np.array([3, 3, 2, 0, 1, 1, 0, 3, 2, 2], dtype=np.int8)
    _check_against_brute(q, r, dna_matrix(3, -3), 4, 3)
    assert oracle.align(q, r, dna_matrix(3, -3), 4, 3).cigar == \
        [(3, "M"), (2, "D"), (1, "M"), (1, "D"), (3, "M")]


@pytest.mark.parametrize("o,e", [(4, 3), (3, 2), (5, 4), (2, 1)])
def test_brute_close_gap_costs(o, e):
    """Longer planted pairs (up to 10) with o - e = 1, where co-optimal
    placements of gaps are common."""
    g = np.random.Generator(np.random.PCG64(3000 + o))
    for _ in range(25):
        lr = int(g.integers(6, 11))
        r = g.integers(0, 4, size=lr).astype(np.int8)
        q, _ = mutate_many(g, r, np.array([0, lr]), 0.15, 0.15, 0.2, 3)
        q = q[:10]
        if len(q) == 0:
            continue
        _check_against_brute(q, r, dna_matrix(3, -int(g.integers(1, 4))), o, e)


# ---------------------------------------------------------------------------
# the suboptimal alignment behind score2
# ---------------------------------------------------------------------------
def _score2_from_brute(b, mask_len):
    """T4 on the brute-force max array (independent of the oracle)."""
    if b["score1"] <= 0:
        return 0, -1
    lo, hi = b["begin"][1] - mask_len, b["end"][1] + mask_len
    best, at = 0, -1
    for j, v in enumerate(b["maxcol"]):
        if lo <= j <= hi:
            continue
        if v > best:
            best, at = int(v), j
    return best, at


@pytest.mark.parametrize("o,e", [(3, 1), (2, 1), (5, 2), (4, 1), (2, 2), (0, 0)])
def test_suboptimal_matches_brute_force(o, e):
    """End row (smallest row of column ref_end2 at score2), T2 begin relative to
    that end, and the T3 CIGAR of the alignment behind score2, against
    exhaustive enumeration, with narrow masks so that score2 is often set."""
    g = np.random.Generator(np.random.PCG64(41 + o * 10 + e))
    mat = dna_matrix()
    checked = 0
    for _ in range(400):
        lq = int(g.integers(2, 8))
        lr = int(g.integers(3, 11))
        q = g.integers(0, 4, size=lq).astype(np.int8)
        r = g.integers(0, 4, size=lr).astype(np.int8)
        if g.random() < 0.5:   # plant a second copy of part of the query
            k = int(g.integers(1, min(lq, lr) + 1))
            p0 = int(g.integers(0, lr - k + 1))
            r[p0:p0 + k] = q[:k]
        mask = int(g.integers(0, 3))
        b = brute.enumerate_align(q, r, mat, o, e)
        s2, e2 = _score2_from_brute(b, mask)
        a = oracle.align(q, r, mat, o, e, mask_len=mask)
        assert (a.score2, a.ref_end2) == (s2, e2)
        rb2, re2, jb2, cig2 = oracle.suboptimal(q, r, mat, o, e, s2, e2)
        if s2 <= 0:
            assert (rb2, re2, jb2, cig2) == (-1, -1, -1, [])
            continue
        bs = brute.enumerate_sub(q, r, mat, o, e, e2, s2)
        assert bs["end"] == (re2, e2), (q, r, o, e, mask)
        assert bs["begin"] == (rb2, jb2), (q, r, o, e, mask)
        assert bs["cigar"] == cig2, (q, r, o, e, mask)
        assert rescore(q, r, mat, o, e, rb2, jb2, cig2)[0] == s2
        checked += 1
    assert checked > 100


def test_suboptimal_column_row_and_crossing_primary():
    """A second copy right of a long primary with a narrow mask: the
    suboptimal alignment may reach back into the masked columns; its score is
    score2 and it ends in column ref_end2 at the first row of that score."""
    g = np.random.Generator(np.random.PCG64(77))
    mat = dna_matrix()
    for _ in range(50):
        q = g.integers(0, 4, size=40).astype(np.int8)
        r = np.concatenate([g.integers(0, 4, size=20), q, g.integers(0, 4, size=5), q[:25],
                            g.integers(0, 4, size=20)]).astype(np.int8)
        a = oracle.align(q, r, mat, 3, 1, mask_len=2)
        rb2, re2, jb2, cig2 = oracle.suboptimal(q, r, mat, 3, 1, a.score2, a.ref_end2)
        assert a.score2 > 0
        assert rescore(q, r, mat, 3, 1, rb2, jb2, cig2)[0] == a.score2
        span_r = sum(n for n, op in cig2 if op in "MD")
        assert jb2 + span_r - 1 == a.ref_end2
        assert oracle.column_row(q, r, mat, 3, 1, a.ref_end2, a.score2) == re2
        for i in range(re2):   # no smaller row of that column reaches score2
            assert oracle.column_row(q[:i + 1], r, mat, 3, 1, a.ref_end2, a.score2) in (-1, re2)
