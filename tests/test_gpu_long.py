"""GPU parity of the intra-sequence path (long pairs: one pair spread over a
wave, the reference cut into column chunks with a warm-up overlap), of the
routing between the two paths, and of the invariance of every result under
the launch configuration (rule I9: results never depend on lane width,
batching, chunking or strip height).  Bit-exact against the CPU oracle."""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1208_6350_amd as swx
import workloads as W
from tests.test_gpu_parity import FIELDS, assert_parity

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture()
def ctx():
    c = swx.Context(0)
    yield c
    c.close()


def test_all_long_chunked(ctx):
    """Every pair through the intra path, references cut into many chunks, on
    packed 16-bit lanes (two chunks per wave) and on 32-bit lanes."""
    b = W.random_pairs(701, 40, (1, 900), (0, 6000))
    for bits in (16, 32, 0):
        ctx.set_tuning(long_cells=0, long_rlen=0, intra_jobs=400, intra_bits=bits)
        recs = assert_parity(ctx, b)
        if bits:
            assert (recs["lane_bits"][recs["score1"] > 0] == bits).all()


def test_intra_lane_width_limit(ctx):
    """Long pairs whose a-priori score bound lies just inside and just outside
    the 16-bit lanes (smax * min(qlen, rlen) + bias <= 32766, rule T6): the
    first take packed 16-bit lanes, the second 32-bit ones, and both reach
    scores near the limit exactly."""
    ctx.set_tuning(long_cells=0, long_rlen=0, intra_jobs=64, intra_bits=16)
    g = np.random.Generator(np.random.PCG64(4094))
    mat = W.dna_matrix(8, -8)   # smax 8, bias 8: the bound is 8 * L + 8
    qs, rs = [], []
    for L in (4094, 4095):
        ref = g.integers(0, 4, size=L + 300).astype(np.int8)
        qs.append(ref[100:100 + L].copy())
        rs.append(ref)
    b = W.from_lists("intra-16-limit", mat, 10, 2, qs, rs)
    recs = assert_parity(ctx, b)
    assert list(recs["score1"]) == [8 * 4094, 8 * 4095]
    assert list(recs["lane_bits"]) == [16, 32]


def test_long_gap_settings(ctx):
    """o = e (linear gaps), e = 0 (no chunking possible) and wide gaps."""
    ctx.set_tuning(long_cells=0, long_rlen=0, intra_jobs=200)
    for seed, (o, e) in enumerate([(1, 1), (6, 0), (5, 2), (11, 1)]):
        b = W.random_pairs(720 + seed, 12, (20, 700), (100, 3000), o=o, e=e)
        assert_parity(ctx, b)


def test_long_multi_strip(ctx):
    """Queries taller than one strip (hand-over rows between strips), planted
    so that the reversed pass and the traceback walk long paths."""
    ctx.set_tuning(long_cells=0, long_rlen=0, intra_jobs=64)
    b = W.random_pairs(731, 6, (1100, 2600), (2600, 5000), planted=1.0)
    recs = assert_parity(ctx, b)
    assert (recs["score1"] > 1000).all()


def test_long_protein(ctx):
    ctx.set_tuning(long_cells=0, long_rlen=0, intra_jobs=64)
    b = W.random_pairs(741, 8, (200, 1300), (500, 3000), alphabet=24, o=11, e=1)
    assert_parity(ctx, b)


def test_mixed_routing(ctx):
    """Short and long pairs in one call: each takes its own path."""
    ctx.set_tuning(long_cells=150_000, long_rlen=4000)
    b = W.random_pairs(751, 120, (1, 600), (0, 5000))
    cells = b.qlen().astype(np.int64) * b.rlen()
    assert ((cells > 150_000) | (b.rlen() > 4000)).any() and (cells <= 150_000).any()
    assert_parity(ctx, b)


def test_tuning_invariance(ctx):
    """The same pairs under several launch configurations give identical
    records and CIGARs."""
    b = W.random_pairs(761, 150, (1, 700), (0, 3000))
    base = None
    for tune in ({}, {"long_cells": -1}, {"fill_rows": 16}, {"fill_rows": 24},
                 {"long_cells": 0, "long_rlen": 0, "intra_jobs": 1},
                 {"long_cells": 0, "long_rlen": 0, "intra_jobs": 5000},
                 {"long_cells": 100_000, "long_rlen": 1000, "fill_rows": 16},
                 {"long_cells": 100_000, "side_streams": 0},
                 {"fill_sched": 0}, {"fill_sched": 2}, {"fill_sched": 2, "fill_rows": 16},
                 {"fill_coop": 1}, {"fill_coop": 2}, {"fill_coop": 2, "fill_sched": 2},
                 {"fill_coop": 2, "fill_sched": 0, "fill_rows": 24},
                 {"fill_coop": 2, "long_cells": 1 << 62, "long_rlen": 1 << 62},
                 {"long_cells": 0, "long_rlen": 0, "intra_bits": 32},
                 {"long_cells": 0, "long_rlen": 0, "intra_bits": 16},
                 {"long_cells": 0, "long_rlen": 0, "intra_jobs": 4000}):
        ctx.set_tuning(**{"long_cells": 1 << 22, "long_rlen": 1 << 16, "intra_jobs": 2048,
                          "fill_rows": 32, "side_streams": 1, "fill_sched": 1, "fill_coop": 0,
                          "intra_bits": 0, **tune})
        _say(f"[tuning] {tune}")
        recs, cig = ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat,
                                    b.roff, b.pair_q, b.pair_r)
        got = [tuple(int(recs[f][p]) for f in FIELDS) +
               tuple(int(w) for w in cig[recs["cigar_off"][p]:recs["cigar_off"][p] +
                                         recs["cigar_len"][p]]) for p in range(b.npairs)]
        if base is None:
            base = got
        else:
            assert got == base, f"results differ under tuning {tune}"


def test_tuning_rejects_bad_values(ctx):
    for bad in ({"fill_rows": 20}, {"intra_jobs": 0}, {"long_cells": -2}, {"long_rlen": -1},
                {"side_streams": 2}, {"fill_sched": 3}, {"fill_sched": -1}, {"fill_coop": 3},
                {"fill_coop": -1}, {"intra_bits": 8}, {"intra_bits": -1}):
        with pytest.raises(swx.SwxError) as ei:
            ctx.set_tuning(**bad)
        assert ei.value.status == -1


def test_config2_full_size(ctx):
    """The single long-reference workload at full size (1,000 x 5,000,000),
    default launch configuration, against the oracle's stored result."""
    with open(os.path.join(GOLDEN, "config2.json")) as f:
        gold = json.load(f)
    b = W.config2()
    _say(f"[long] config2: qlen {b.qlen()[0]} rlen {b.rlen()[0]}")
    rec, cig = ctx.align_pair(b.query(0), b.ref(0), b.matrix, b.gap_open, b.gap_extend)
    for f in FIELDS:
        assert rec[f] == gold[f], (f, rec[f], gold[f])
    assert [[n, op] for n, op in cig] == gold["cigar"]
    # the planted near-copies make score2 a real second hit
    assert gold["score2"] > gold["score1"] // 2


def test_config5_long_requests(ctx):
    """Long serving requests (10-kb read vs 20-kb window at 10% error) through
    the default routing, against the oracle."""
    pool = W.config5_pool(n_short=4, n_long=3)
    sel = np.nonzero(pool.qlen() >= 5000)[0][:3]
    b = pool.subset(sel)
    _say(f"[long] config5 long requests: {b.npairs}")
    assert_parity(ctx, b)


def test_autotune_keeps_results_and_caches(ctx, tmp_path):
    """The autotuner only changes speed: results after tuning equal those
    before, and a second call with the same kind of work reads the cache."""
    b = W.random_pairs(771, 300, (1, 500), (0, 2500))
    recs0, cig0 = ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat,
                                  b.roff, b.pair_q, b.pair_r)
    cache = str(tmp_path / "tune.jsonl")
    t1, fc1 = ctx.autotune(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat, b.roff,
                           b.pair_q, b.pair_r, max_pairs=200, cache_path=cache)
    _say(f"[tune] {t1}")
    assert not fc1 and t1["fill_rows"] in (16, 24, 32) and t1 == ctx.tuning()
    recs1, cig1 = ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat,
                                  b.roff, b.pair_q, b.pair_r)
    for f in FIELDS + ["cigar_off", "cigar_len"]:   # lane_bits is diagnostic only
        assert np.array_equal(recs0[f], recs1[f]), f
    assert np.array_equal(cig0, cig1)
    ctx.set_tuning(fill_rows=16 if t1["fill_rows"] == 32 else 32)
    t2, fc2 = ctx.autotune(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat, b.roff,
                           b.pair_q, b.pair_r, max_pairs=200, cache_path=cache)
    assert fc2 and t2 == t1 and ctx.tuning() == t1


def test_single_pair_protein_beyond_graph_capacity(ctx):
    """One protein pair above the one-pair graph's capacity (reference over
    65,536 residues): swx_align takes the batch path and reads the profile's
    resident device tables; equal to the oracle."""
    g = np.random.Generator(np.random.PCG64(8123))
    mat = W.protein_matrix_standin()
    q = g.integers(0, 24, 150).astype(np.int8)
    r = g.integers(0, 24, 70_000).astype(np.int8)
    r[31_000:31_150] = q
    r[50_000:50_120] = q[10:130]
    for o, e in ((11, 1), (5, 5)):
        rec, cig = ctx.align_pair(q, r, mat, o, e)
        a = oracle.align(q, r, mat, o, e)
        for f in FIELDS:
            assert rec[f] == getattr(a, f), (o, e, f)
        assert cig == a.cigar
