"""GPU parity: the HIP path against the CPU oracle, bit-exact in every field
(score1, score2, begins, ends, ref_end2) and in the CIGAR, on seeded inputs.

Every test here calls the library through the C ABI (ctypes)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import paper_1208_6350_amd as swx
import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# Every parity test runs with the default routing, with every pair forced
# onto the batched (one pair per lane half) path with 32- and with 24-row
# strips, one wave per task and (cooperative) a workgroup's four waves per
# task, in grid order and from the device queue, and with every pair forced
# onto the intra-sequence (one pair per wave) path, on packed 16-bit lanes
# where the scores fit and on 32-bit lanes throughout.
PATHS = {"auto": {"long_cells": -1},
         "rows24": {"long_cells": 1 << 62, "long_rlen": 1 << 62, "fill_rows": 24},
         "batched": {"long_cells": 1 << 62, "long_rlen": 1 << 62, "fill_coop": 1},
         "coop": {"long_cells": 1 << 62, "long_rlen": 1 << 62, "fill_coop": 2},
         "coop_queue": {"long_cells": 1 << 62, "long_rlen": 1 << 62, "fill_coop": 2,
                        "fill_sched": 2, "fill_rows": 16},
         "intra": {"long_cells": 0, "long_rlen": 0, "intra_jobs": 256, "intra_bits": 16},
         "intra32": {"long_cells": 0, "long_rlen": 0, "intra_jobs": 256, "intra_bits": 32}}


@pytest.fixture(scope="module", params=list(PATHS))
def ctx(request):
    c = swx.Context(0)
    c.set_tuning(**PATHS[request.param])
    c.path = request.param
    yield c
    c.close()


def run_both(ctx, b: W.Batch, flags=swx.SWX_ALL, mask_len=-1, nthreads=8):
    _say(f"[parity] {b.name}: {b.npairs} pairs, flags={flags}, mask_len={mask_len}")
    recs, cig = ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat,
                                b.roff, b.pair_q, b.pair_r, flags, mask_len)
    ref, rcig, rcoff = oracle.align_many(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r,
                                         b.matrix, b.gap_open, b.gap_extend, flags, mask_len,
                                         nthreads=nthreads)
    return recs, cig, ref, rcig, rcoff


FIELDS = ["score1", "score2", "read_begin1", "read_end1", "ref_begin1", "ref_end1", "ref_end2"]


def assert_parity(ctx, b, flags=swx.SWX_ALL, mask_len=-1):
    recs, cig, ref, rcig, rcoff = run_both(ctx, b, flags, mask_len)
    bad = []
    for k, f in enumerate(FIELDS):
        got = recs[f].astype(np.int64)
        exp = ref[:, k]
        if f == "score2" and not (flags & swx.SWX_SCORE2):
            exp = np.zeros_like(exp)
        if f == "ref_end2" and not (flags & swx.SWX_SCORE2):
            exp = np.full_like(exp, -1)
        if f in ("read_begin1", "ref_begin1") and not (flags & 7):
            exp = np.where(ref[:, 0] > 0, -1, exp)
        mism = np.nonzero(got != exp)[0]
        if len(mism):
            p = int(mism[0])
            bad.append(f"{f}: {len(mism)} mismatches, first pair {p}: gpu {got[p]} oracle {exp[p]}")
    assert not bad, "; ".join(bad)
    if flags & swx.SWX_CIGAR:
        for p in range(b.npairs):
            g = cig[recs["cigar_off"][p]:recs["cigar_off"][p] + recs["cigar_len"][p]]
            e = rcig[rcoff[p]:rcoff[p] + ref[p, 7]]
            if not np.array_equal(g, e):
                raise AssertionError(f"CIGAR mismatch at pair {p}: gpu {swx.decode_cigar(g)} "
                                     f"oracle {swx.decode_cigar(e)}")
    else:
        assert (recs["cigar_len"] == 0).all()
    return recs


def test_random_dna_small(ctx):
    b = W.random_pairs(101, 300, (1, 90), (0, 260))
    recs = assert_parity(ctx, b)
    assert (recs["score1"] > 0).sum() > 200


def test_random_dna_gap_settings(ctx):
    for seed, (o, e) in enumerate([(2, 1), (5, 2), (1, 1), (4, 3), (6, 0), (0, 0)]):
        b = W.random_pairs(200 + seed, 150, (1, 70), (1, 200), o=o, e=e)
        assert_parity(ctx, b)


def test_random_protein_general_profile(ctx):
    b = W.random_pairs(301, 200, (1, 100), (1, 300), alphabet=24, o=11, e=1)
    assert_parity(ctx, b)


def test_asymmetric_matrix_five_symbols(ctx):
    g = np.random.Generator(np.random.PCG64(7))
    mat = g.integers(-5, 6, size=(5, 5)).astype(np.int8)
    b = W.random_pairs(302, 150, (1, 60), (1, 150), alphabet=5, matrix=mat, o=3, e=1)
    assert_parity(ctx, b)


def test_flags_and_mask(ctx):
    b = W.random_pairs(303, 120, (5, 80), (20, 300))
    for flags in (0, swx.SWX_BEGIN, swx.SWX_CIGAR, swx.SWX_SCORE2):
        assert_parity(ctx, b, flags=flags)
    for m in (0, 3, 40):
        assert_parity(ctx, b, mask_len=m)


def test_edge_cases(ctx):
    mat = W.dna_matrix()
    qs = [np.array([0], np.int8), np.array([1, 2, 3], np.int8), np.array([2] * 40, np.int8),
          np.array([0, 1], np.int8), np.arange(64, dtype=np.int8) % 4]
    rs = [np.array([0], np.int8), np.zeros(0, np.int8), np.array([2] * 70, np.int8),
          np.array([3, 3, 3], np.int8), np.arange(64, dtype=np.int8) % 4]
    b = W.from_lists("edges", mat, 3, 1, qs, rs)
    assert_parity(ctx, b)
    neg = np.full((4, 4), -1, np.int8)
    b2 = W.from_lists("no-positive", neg, 3, 1, qs, rs)
    recs = assert_parity(ctx, b2)
    assert (recs["score1"] == 0).all() and (recs["ref_end1"] == -1).all()


def test_lane_width_threshold(ctx):
    """Scores around the 16-bit limit (2047): the saturated pairs are re-run
    on 32-bit lanes and every result must equal the oracle's."""
    g = np.random.Generator(np.random.PCG64(11))
    mat = W.dna_matrix(8, -8)
    qs, rs = [], []
    for L in (250, 255, 256, 257, 258, 300, 40):
        ref = g.integers(0, 4, size=L + 100).astype(np.int8)
        qs.append(ref[50:50 + L].copy())
        rs.append(ref)
    b = W.from_lists("threshold", mat, 10, 2, qs, rs)
    recs = assert_parity(ctx, b)
    if ctx.path in ("batched", "rows24", "coop", "coop_queue"):
        assert set(recs["lane_bits"]) == {16, 32}


@pytest.mark.parametrize("match,o,e,L", [
    (1, 2, 1, 991),    # bias = o; a-priori bound 991: column max over row pairs, at its limit
    (1, 2, 1, 992),    # bias = o; bound 992: one max per row
    (2, 1, 1, 495),    # o below the worst mismatch (bias = 2, not o); paired rows
    (2, 1, 1, 600),    # neither
])
def test_column_max_forms(ctx, match, o, e, L):
    """The 16-bit fill's forms on either side of their conditions: the column
    maximum over pairs of rows (only when every score of the batch is at most
    991, so that value * 32 + row code stays below 0x7C00) and H - o taken as
    H itself (only when the bias can be the gap open penalty).  Planted exact
    copies reach the a-priori bound (smax times the longest query) itself,
    mutated copies and random pairs give ends and begins in every row of a
    strip."""
    g = np.random.Generator(np.random.PCG64(1000 + L + 7 * o))
    mat = W.dna_matrix(match, -match)
    qs, rs = [], []
    for k in range(10):
        ref = g.integers(0, 4, size=L + 120).astype(np.int8)
        q = ref[40 + k:40 + k + L].copy()
        if k >= 2:   # mutated copies
            flip = g.random(L) < 0.02 * k
            q[flip] = (q[flip] + g.integers(1, 4, size=int(flip.sum()))) % 4
        qs.append(q)
        rs.append(ref)
    for k in range(20):   # short random pairs beside them
        qs.append(g.integers(0, 4, size=int(g.integers(1, 80))).astype(np.int8))
        rs.append(g.integers(0, 4, size=int(g.integers(1, 300))).astype(np.int8))
    b = W.from_lists(f"forms-{match}-{o}-{L}", mat, o, e, qs, rs)
    recs = assert_parity(ctx, b)
    assert int(recs["score1"].max()) == match * L


@pytest.mark.parametrize("o", [253, 254])
def test_bias_byte_limit(ctx, o):
    """The fills' bias becomes the gap open penalty when every biased score
    S + o still fits a byte: with +2/-2 scores, o = 253 takes bias = o (the
    largest biased score is exactly 255), o = 254 keeps bias = 2.  Either way
    every result equals the oracle's."""
    b = W.random_pairs(1300 + o, 200, (1, 90), (1, 260), o=o, e=1)
    recs = assert_parity(ctx, b)
    assert (recs["score1"] > 0).sum() > 100


def test_many_tasks_ragged(ctx):
    b = W.random_pairs(404, 700, (1, 200), (1, 500))
    assert_parity(ctx, b)


def test_config1_single_pair(ctx):
    b = W.config1()
    assert_parity(ctx, b)
    # the single-pair entry point gives the same record
    rec, cig = ctx.align_pair(b.query(0), b.ref(0), b.matrix, b.gap_open, b.gap_extend)
    a = oracle.align(b.query(0), b.ref(0), b.matrix, b.gap_open, b.gap_extend)
    assert (rec["score1"], rec["score2"], rec["read_begin1"], rec["read_end1"], rec["ref_begin1"],
            rec["ref_end1"], rec["ref_end2"]) == (a.score1, a.score2, a.read_begin1,
                                                  a.read_end1, a.ref_begin1, a.ref_end1,
                                                  a.ref_end2)
    assert cig == a.cigar


def test_config4_sample(ctx):
    b = W.config4(npairs=3000)
    assert_parity(ctx, b)


def test_all_vs_all_short_reads(ctx):
    """Every pair of 90 overlapping 70-nt reads (4,005 pairs, one shared
    code array for queries and references)."""
    b = W.all_vs_all(n_reads=90)
    assert_parity(ctx, b)


def test_config3_sample(ctx):
    full = W.config3(ntargets=600)
    assert_parity(ctx, full)


def test_batch_equals_single(ctx):
    """Each pair aligned inside a batch equals the same pair aligned alone."""
    b = W.random_pairs(505, 40, (5, 120), (10, 300))
    recs, cig = ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat,
                                b.roff, b.pair_q, b.pair_r)
    for p in range(b.npairs):
        rec, c1 = ctx.align_pair(b.query(p), b.ref(p), b.matrix, b.gap_open, b.gap_extend)
        for f in FIELDS:
            assert rec[f] == recs[f][p], (p, f)
        assert c1 == swx.decode_cigar(cig[recs["cigar_off"][p]:recs["cigar_off"][p] +
                                          recs["cigar_len"][p]])


def test_single_pair_calls_equal_batch(ctx):
    """The one-pair entry point (captured graphs per size class, reused across
    calls; the batch path beyond them): edge shapes, protein, every flag set
    and mask width, and a bad symbol, each equal to the batch result."""
    g = np.random.Generator(np.random.PCG64(44))
    qs = [np.array([1], np.int8), np.array([0, 1, 2, 3] * 20, np.int8),
          g.integers(0, 4, 300).astype(np.int8), g.integers(0, 4, 70).astype(np.int8)]
    rs = [np.array([1, 2, 1], np.int8), np.zeros(0, np.int8),
          g.integers(0, 4, 1500).astype(np.int8), g.integers(0, 4, 5000).astype(np.int8)]
    dna = W.from_lists("single-dna", W.dna_matrix(), 3, 1, qs, rs)
    prot = W.random_pairs(515, 6, (20, 200), (50, 700), alphabet=24,
                          matrix=W.protein_matrix_standin(), o=11, e=1)
    for b in (dna, prot):
        for flags, mask in ((swx.SWX_ALL, -1), (0, -1), (swx.SWX_BEGIN, -1),
                            (swx.SWX_SCORE2 | swx.SWX_BEGIN, 7)):
            recs, cig = ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff,
                                        b.rcat, b.roff, b.pair_q, b.pair_r, flags, mask)
            for p in range(b.npairs):
                for rep in range(2):   # the second call replays the cached graph
                    rec, c1 = ctx.align_pair(b.query(p), b.ref(p), b.matrix, b.gap_open,
                                             b.gap_extend, flags, mask)
                    for f in FIELDS:
                        assert rec[f] == recs[f][p], (b.name, flags, p, f)
                    assert c1 == swx.decode_cigar(cig[recs["cigar_off"][p]:recs["cigar_off"][p] +
                                                      recs["cigar_len"][p]])
    bad = dna.ref(2).copy()
    bad[10] = 7
    with pytest.raises(swx.SwxError) as ei:
        ctx.align_pair(dna.query(2), bad, dna.matrix, dna.gap_open, dna.gap_extend)
    assert ei.value.status == -1


def test_rejected_single_pair_leaves_no_trace(ctx):
    """A one-pair call rejected for a bad reference symbol leaves nothing
    behind in the cached one-pair graph: a later, shorter reference of the
    same size class (the bad byte's position lies past its end) aligns and
    equals the batch result."""
    g = np.random.Generator(np.random.PCG64(4400))
    q = g.integers(0, 4, 120).astype(np.int8)
    bad = g.integers(0, 4, 1500).astype(np.int8)
    bad[1400] = 7
    good = g.integers(0, 4, 1100).astype(np.int8)
    good[300:420] = q
    m = W.dna_matrix()
    rec, c1 = ctx.align_pair(q, good, m, 3, 1)          # caches the size class's graph
    with pytest.raises(swx.SwxError) as ei:
        ctx.align_pair(q, bad, m, 3, 1)
    assert ei.value.status == -1
    b = W.from_lists("after-reject", m, 3, 1, [q], [good])
    recs, cig = ctx.align_batch(b.matrix, 3, 1, b.qcat, b.qoff, b.rcat, b.roff, b.pair_q,
                                b.pair_r)
    for rep in range(2):
        rec, c1 = ctx.align_pair(q, good, m, 3, 1)
        for f in FIELDS:
            assert rec[f] == recs[f][0], f
        assert c1 == swx.decode_cigar(cig[:recs["cigar_len"][0]])
    assert rec["score1"] >= 200


def test_invalid_symbols_rejected(ctx):
    b = W.random_pairs(606, 5, (3, 10), (3, 10))
    b.rcat[2] = 9
    with pytest.raises(swx.SwxError) as ei:
        ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat, b.roff,
                        b.pair_q, b.pair_r)
    assert ei.value.status == -1


@pytest.mark.parametrize("which", ["q", "r"])
def test_invalid_symbol_anywhere_is_found(ctx, which):
    # symbols are checked 16 bytes at a time after an unaligned head: a bad
    # byte at every position of the first words, of the last words and in
    # the middle, with each kind of bad value (n, the top of the range, and
    # negative ones), is found; the untouched batch passes
    b = W.random_pairs(607, 40, (30, 90), (30, 90))
    ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat, b.roff,
                    b.pair_q, b.pair_r)
    cat = b.qcat if which == "q" else b.rcat
    n = b.matrix.shape[0]
    L = len(cat)
    spots = list(range(0, 40)) + list(range(L // 2 - 20, L // 2 + 20)) + list(range(L - 40, L))
    for k, pos in enumerate(spots):
        bad = [n, 31, 32, 127, -1, -128][k % 6]
        keep = int(cat[pos])
        cat[pos] = bad
        with pytest.raises(swx.SwxError) as ei:
            ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat, b.roff,
                            b.pair_q, b.pair_r)
        assert ei.value.status == -1, (which, pos, bad)
        cat[pos] = keep


@pytest.mark.parametrize("shift", [0, 1, 7, 15])
def test_invalid_symbol_in_unaligned_device_input(ctx, shift):
    # device-resident codes starting at every alignment class: the unaligned
    # head, the 16-byte body and the tail are each checked
    import torch
    b = W.random_pairs(608, 30, (20, 60), (20, 60))
    dev = torch.device("cuda:0")
    to = lambda x: torch.as_tensor(np.ascontiguousarray(x)).to(dev)
    L = len(b.rcat)
    buf = torch.zeros(L + 32, dtype=torch.int8, device=dev)
    rc = buf[shift:shift + L]
    dq, dqo, dro, dpq, dpr = to(b.qcat), to(b.qoff), to(b.roff), to(b.pair_q), to(b.pair_r)
    recs = torch.empty(b.npairs * swx.REC_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    cig = torch.empty(int(b.qlen().sum() + b.rlen().sum() + b.npairs), dtype=torch.int32,
                      device=dev)

    def run(cat):
        rc.copy_(torch.as_tensor(cat).to(dev))
        torch.cuda.synchronize()
        st, _ = swx.swx_align_batch(ctx.handle, b.matrix, b.gap_open, b.gap_extend, dq, dqo, rc,
                                    dro, dpq, dpr, swx.SWX_ALL, -1, swx.SWX_MEM_DEVICE, recs, cig,
                                    swx.SWX_MEM_DEVICE)
        torch.cuda.synchronize()
        return st

    assert run(b.rcat) == 0
    n = b.matrix.shape[0]
    for pos in (0, 1, 14, 15, 16, 17, L // 2, L - 17, L - 16, L - 2, L - 1):
        for bad in (n, -1):
            cat = b.rcat.copy()
            cat[pos] = bad
            assert run(cat) == -1, (shift, pos, bad)


def _two_copy_pairs(seed, npairs, alphabet=4, o=3, e=1):
    """References holding two mutated copies of the query (the second often
    partial), so that score2 comes from a real second hit."""
    g = np.random.Generator(np.random.PCG64(seed))
    qs, rs = [], []
    for _ in range(npairs):
        lq = int(g.integers(8, 120))
        q = g.integers(0, alphabet, size=lq).astype(np.int8)
        parts = [g.integers(0, alphabet, size=int(g.integers(0, 60)))]
        for k in range(2):
            c = q[:int(g.integers(max(4, lq // 3), lq + 1))] if k else q
            c = c.copy()
            sub = g.random(len(c)) < 0.05
            c[sub] = (c[sub] + g.integers(1, alphabet, size=int(sub.sum()))) % alphabet
            parts += [c, g.integers(0, alphabet, size=int(g.integers(0, 40)))]
        if g.random() < 0.5:
            parts = parts[::-1]
        qs.append(q)
        rs.append(np.concatenate(parts).astype(np.int8))
    mat = W.dna_matrix(n=alphabet) if alphabet <= 8 else W.protein_matrix_standin()
    return W.from_lists(f"two-copies-{seed}", mat, o, e, qs, rs)


@pytest.mark.parametrize("mask_len", [2, -1])
def test_suboptimal_alignment(ctx, mask_len):
    """SWX_SUBOPT: the alignment behind score2 (end row, begin, CIGAR) equals
    the oracle's, and the primary records are unchanged."""
    for b in (_two_copy_pairs(71, 120), W.random_pairs(72, 150, (1, 90), (0, 300), planted=0.8),
              _two_copy_pairs(73, 60, alphabet=24, o=11, e=1)):
        _say(f"[parity] {b.name}: suboptimal, mask_len={mask_len}")
        recs, cig, sub = ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff,
                                         b.rcat, b.roff, b.pair_q, b.pair_r,
                                         swx.SWX_ALL | swx.SWX_SUBOPT, mask_len)
        ref, rcig, rcoff = oracle.align_many(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r,
                                             b.matrix, b.gap_open, b.gap_extend, swx.SWX_ALL,
                                             mask_len)
        for k, f in enumerate(FIELDS):
            assert np.array_equal(recs[f].astype(np.int64), ref[:, k]), f
        sref, scig, scoff = oracle.suboptimal_many(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q,
                                                   b.pair_r, b.matrix, b.gap_open, b.gap_extend,
                                                   ref[:, 1], ref[:, 6])
        s2 = ref[:, 1]
        assert np.array_equal(sub["score1"].astype(np.int64), s2)
        for f, col in (("read_begin1", 0), ("read_end1", 1), ("ref_begin1", 2)):
            got = sub[f].astype(np.int64)
            bad = np.nonzero(got != sref[:, col])[0]
            assert len(bad) == 0, f"{f}: pair {bad[0]} gpu {got[bad[0]]} oracle {sref[bad[0], col]}"
        assert np.array_equal(sub["ref_end1"].astype(np.int64), ref[:, 6])
        assert (sub["score2"] == 0).all() and (sub["ref_end2"] == -1).all()
        for p in range(b.npairs):
            g = cig[sub["cigar_off"][p]:sub["cigar_off"][p] + sub["cigar_len"][p]]
            e = scig[scoff[p]:scoff[p] + sref[p, 3]]
            assert np.array_equal(g, e), (p, swx.decode_cigar(g), swx.decode_cigar(e))
            pg = cig[recs["cigar_off"][p]:recs["cigar_off"][p] + recs["cigar_len"][p]]
            assert np.array_equal(pg, rcig[rcoff[p]:rcoff[p] + ref[p, 7]]), p
        assert (s2 > 0).sum() > b.npairs // 3


def test_single_pair_suboptimal(ctx):
    """SWX_SUBOPT through the one-pair call (swx_align): the primary record and
    CIGAR, and the suboptimal alignment's begins, end and CIGAR, equal the
    oracle's, pair by pair."""
    for b in (_two_copy_pairs(74, 24), _two_copy_pairs(75, 12, alphabet=24, o=11, e=1)):
        _say(f"[parity] {b.name}: one-pair calls with the suboptimal alignment")
        ref, rcig, rcoff = oracle.align_many(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r,
                                             b.matrix, b.gap_open, b.gap_extend)
        seen2 = 0
        for p in range(b.npairs):
            q, r = b.query(p), b.ref(p)
            rec, cig, sub, scig = ctx.align_pair(q, r, b.matrix, b.gap_open, b.gap_extend,
                                                 flags=swx.SWX_ALL | swx.SWX_SUBOPT)
            for k, f in enumerate(FIELDS):
                assert rec[f] == ref[p, k], (p, f)
            assert cig == swx.decode_cigar(rcig[rcoff[p]:rcoff[p] + ref[p, 7]]), p
            rb2, re2, fb2, ocig = oracle.suboptimal(q, r, b.matrix, b.gap_open, b.gap_extend,
                                                    int(ref[p, 1]), int(ref[p, 6]))
            assert sub["score1"] == ref[p, 1], p
            assert (sub["read_begin1"], sub["read_end1"], sub["ref_begin1"]) == (rb2, re2, fb2), p
            assert sub["ref_end1"] == ref[p, 6], p
            assert scig == ocig, (p, scig, ocig)
            seen2 += ref[p, 1] > 0
        assert seen2 > b.npairs // 3
