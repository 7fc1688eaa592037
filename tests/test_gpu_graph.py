"""GPU tests of graph mode: the batched path captured once as a hipGraph and
replayed.  Every replay (with other eager work of the program and
synchronisations between replays) must equal the same chain issued eagerly
and the oracle, bit for bit, and new batch contents loaded into the graph's
buffers must give new, correct results."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import paper_1208_6350_amd as swx
import workloads as W
from tests.test_gpu_parity import FIELDS

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _graph_for(ctx, b, max_pairs, max_qlen, max_rlen, extra=1.2, route=0):
    return swx.Graph(ctx, b.matrix, b.gap_open, b.gap_extend, max_pairs=max_pairs,
                     max_qlen=max_qlen, max_rlen=max_rlen, qcat_cap=int(len(b.qcat) * extra) + 64,
                     rcat_cap=int(len(b.rcat) * extra) + 64, nq_cap=max_pairs + 1,
                     nr_cap=max_pairs + 2, route=route)


ROUTES = [0, 1]   # batched (one pair per lane half), intra (one pair per wave)


def _check_oracle(b, recs, cig):
    ref, rcig, rcoff = oracle.align_many(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r,
                                         b.matrix, b.gap_open, b.gap_extend)
    for k, f in enumerate(FIELDS):
        bad = np.nonzero(recs[f].astype(np.int64) != ref[:, k])[0]
        assert len(bad) == 0, f"{f}: pair {bad[0]} gpu {recs[f][bad[0]]} oracle {ref[bad[0], k]}"
    for p in range(b.npairs):
        g = cig[recs["cigar_off"][p]:recs["cigar_off"][p] + recs["cigar_len"][p]]
        assert np.array_equal(g, rcig[rcoff[p]:rcoff[p] + ref[p, 7]]), p


@pytest.fixture()
def ctx():
    c = swx.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("route", ROUTES)
def test_graph_replays_equal_eager_and_oracle(ctx, route):
    a = W.random_pairs(901, 300, (1, 150), (0, 500))
    other = W.random_pairs(902, 80, (1, 60), (0, 200))
    g = _graph_for(ctx, a, max_pairs=384, max_qlen=160, max_rlen=520, route=route)
    try:
        g.load(a.qcat, a.qoff, a.rcat, a.roff, a.pair_q, a.pair_r)
        g.run(eager=True)
        recs_e, cig_e = g.read()
        _check_oracle(a, recs_e, cig_e)
        for k in range(3):
            # the program's own eager work between replays
            ctx.align_batch(other.matrix, other.gap_open, other.gap_extend, other.qcat, other.qoff,
                            other.rcat, other.roff, other.pair_q, other.pair_r)
            g.run()
            recs_g, cig_g = g.read()
            _say(f"[graph] replay {k}: {len(recs_g)} records")
            assert recs_g.tobytes() == recs_e.tobytes(), f"replay {k} differs from eager"
            assert np.array_equal(cig_g, cig_e), f"replay {k} CIGARs differ"
        # new contents in the same buffers
        b = W.random_pairs(903, 250, (1, 160), (0, 520))
        g.load(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r)
        g.run()
        recs_b, cig_b = g.read()
        _check_oracle(b, recs_b, cig_b)
        # the same pairs through the ordinary batch call
        recs_c, cig_c = ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat,
                                        b.roff, b.pair_q, b.pair_r)
        for f in FIELDS:
            assert np.array_equal(recs_b[f], recs_c[f]), f
    finally:
        g.close()


@pytest.mark.parametrize("route", ROUTES)
def test_graph_wide_lanes_and_protein(ctx, route):
    """Scores past the 16-bit field (re-run on 32-bit lanes inside the graph)
    and the general-alphabet profile."""
    gen = np.random.Generator(np.random.PCG64(13))
    mat = W.dna_matrix(8, -8)
    qs, rs = [], []
    for L in (250, 256, 258, 300, 40, 120):
        ref = gen.integers(0, 4, size=L + 100).astype(np.int8)
        qs.append(ref[50:50 + L].copy())
        rs.append(ref)
    b = W.from_lists("graph-threshold", mat, 10, 2, qs, rs)
    g = _graph_for(ctx, b, max_pairs=8, max_qlen=300, max_rlen=400, route=route)
    try:
        g.load(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r)
        for k in range(2):
            g.run()
            recs, cig = g.read()
            _check_oracle(b, recs, cig)
        assert set(recs["lane_bits"]) == ({16, 32} if route == 0 else {32})
    finally:
        g.close()
    p = W.random_pairs(904, 120, (1, 120), (1, 300), alphabet=24, o=11, e=1)
    g = _graph_for(ctx, p, max_pairs=128, max_qlen=120, max_rlen=300, route=route)
    try:
        g.load(p.qcat, p.qoff, p.rcat, p.roff, p.pair_q, p.pair_r)
        g.run()
        recs, cig = g.read()
        _check_oracle(p, recs, cig)
    finally:
        g.close()


def test_graph_long_queries_intra_route(ctx):
    """The intra route with queries taller than one strip (hand-over rows)."""
    b = W.random_pairs(906, 12, (600, 2500), (800, 3000), planted=0.7)
    g = _graph_for(ctx, b, max_pairs=16, max_qlen=2600, max_rlen=3100, route=1)
    try:
        g.load(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r)
        for k in range(2):
            g.run()
            recs, cig = g.read()
            _check_oracle(b, recs, cig)
    finally:
        g.close()


def test_graph_load_checks_indices_offsets_and_lengths(ctx):
    # the host rejects a batch whose indices, offsets or lengths would take a
    # kernel outside the graph's buffers; a valid batch then runs as usual
    a = W.random_pairs(906, 20, (3, 30), (3, 60))
    g = _graph_for(ctx, a, max_pairs=32, max_qlen=40, max_rlen=80)
    try:
        cases = []
        pq = a.pair_q.copy(); pq[5] = a.pair_q.max() + 100
        cases.append((a.qoff, a.roff, pq, a.pair_r))
        pr = a.pair_r.copy(); pr[7] = -1
        cases.append((a.qoff, a.roff, a.pair_q, pr))
        qo = a.qoff.copy(); qo[3], qo[4] = qo[4], qo[3]
        if qo[3] != qo[4]:
            cases.append((qo, a.roff, a.pair_q, a.pair_r))
        ro = a.roff.copy(); ro[-1] = len(a.rcat) + 5
        cases.append((a.qoff, ro, a.pair_q, a.pair_r))
        for qoff, roff, pair_q, pair_r in cases:
            with pytest.raises(swx.SwxError) as ei:
                g.load(a.qcat, qoff, a.rcat, roff, pair_q, pair_r)
            assert ei.value.status == -1
        long_q = np.concatenate([a.qcat, np.zeros(50, dtype=np.int8)])
        long_off = np.concatenate([a.qoff, [a.qoff[-1] + 50]]).astype(np.int64)
        pq = a.pair_q.copy(); pq[0] = len(a.qoff) - 1   # a 50-symbol query: above max_qlen
        with pytest.raises(swx.SwxError) as ei:
            g.load(long_q, long_off, a.rcat, a.roff, pq, a.pair_r)
        assert ei.value.status == -1
        g.load(a.qcat, a.qoff, a.rcat, a.roff, a.pair_q, a.pair_r)
        g.run()
        recs, cig = g.read()
        _check_oracle(a, recs, cig)
    finally:
        g.close()


def test_graph_rejects_bad_contents(ctx):
    a = W.random_pairs(905, 20, (3, 30), (3, 60))
    g = _graph_for(ctx, a, max_pairs=32, max_qlen=40, max_rlen=80)
    try:
        bad = a.rcat.copy()
        bad[3] = 9
        # a load checks the symbols on the host and leaves the buffers alone
        with pytest.raises(swx.SwxError) as ei:
            g.load(a.qcat, a.qoff, bad, a.roff, a.pair_q, a.pair_r)
        assert ei.value.status == -1
        g.load(a.qcat, a.qoff, a.rcat, a.roff, a.pair_q, a.pair_r)
        g.run()
        # a bad code written straight into the device buffer is found by the run
        import ctypes
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        nine = (ctypes.c_int8 * 1)(9)
        assert hip.hipMemcpy(ctypes.c_void_p(g.io.rcat + 3), ctypes.addressof(nine), 1, 1) == 0
        with pytest.raises(swx.SwxError) as ei:
            g.run()
        assert ei.value.status == -1
        g.load(a.qcat, a.qoff, a.rcat, a.roff, a.pair_q, a.pair_r)
        g.run()
        recs, cig = g.read()
        _check_oracle(a, recs, cig)
    finally:
        g.close()


@pytest.mark.parametrize("route", ROUTES)
def test_one_pair_graph_replays(ctx, route):
    """A graph of capacity one (its traceback planned on the device for the
    wave kernel): single pairs of every kind loaded and replayed in turn --
    planted hits, random pairs, an empty reference, a one-symbol query -- each
    equal to the oracle, and every replay equal to the graph's eager run."""
    g0 = np.random.Generator(np.random.PCG64(917))
    dna = W.dna_matrix()
    cases = []
    for k in range(10):
        lq = int(g0.integers(1, 160))
        lr = int(g0.integers(0, 500))
        r = g0.integers(0, 4, lr).astype(np.int8)
        q = g0.integers(0, 4, lq).astype(np.int8)
        if k % 2 == 0 and lr >= lq:   # a planted copy with a few substitutions
            p0 = int(g0.integers(0, lr - lq + 1))
            q = r[p0:p0 + lq].copy()
            flip = g0.random(lq) < 0.05
            q[flip] = (q[flip] + 1) % 4
        cases.append((q, r))
    cases.append((np.array([2], np.int8), np.zeros(0, np.int8)))
    cases.append((np.array([1], np.int8), np.array([1, 1, 3], np.int8)))
    b = W.from_lists("one-pair-graph", dna, 3, 1, [c[0] for c in cases], [c[1] for c in cases])
    g = swx.Graph(ctx, b.matrix, b.gap_open, b.gap_extend, max_pairs=1, max_qlen=160,
                  max_rlen=512, qcat_cap=256, rcat_cap=640, nq_cap=2, nr_cap=3, route=route)
    try:
        for p in range(b.npairs):
            pb = b.subset(np.array([p]))
            g.load(pb.qcat, pb.qoff, pb.rcat, pb.roff, pb.pair_q, pb.pair_r)
            g.run(eager=True)
            recs_e, cig_e = g.read()
            _check_oracle(pb, recs_e, cig_e)
            for k in range(2):
                g.run()
                recs_g, cig_g = g.read()
                assert recs_g.tobytes() == recs_e.tobytes(), (p, k)
                assert np.array_equal(cig_g, cig_e), (p, k)
        _say(f"[graph] one-pair route {route}: {b.npairs} pairs")
    finally:
        g.close()


@pytest.mark.parametrize("route", ROUTES)
def test_one_pair_graph_multi_strip(ctx, route):
    """A one-pair graph whose pairs are taller than one strip of the wave
    traceback (hand-over rows between strips inside the graph): planted
    near-copies with indels and a random pair, equal to the oracle."""
    g0 = np.random.Generator(np.random.PCG64(929))
    qs, rs = [], []
    for k in range(4):
        r = g0.integers(0, 4, 1600).astype(np.int8)
        lq = int(g0.integers(600, 900))
        p0 = int(g0.integers(0, 1600 - lq))
        src = r[p0:p0 + lq]
        q, _ = W.mutate_many(g0, src, np.array([0, lq]), 0.03, 0.01, 0.01, 3)
        qs.append(q if k < 3 else g0.integers(0, 4, lq).astype(np.int8))
        rs.append(r)
    b = W.from_lists("one-pair-graph-tall", W.dna_matrix(), 3, 1, qs, rs)
    g = swx.Graph(ctx, b.matrix, b.gap_open, b.gap_extend, max_pairs=1, max_qlen=1024,
                  max_rlen=1600, qcat_cap=1100, rcat_cap=1700, nq_cap=2, nr_cap=3, route=route)
    try:
        for p in range(b.npairs):
            pb = b.subset(np.array([p]))
            g.load(pb.qcat, pb.qoff, pb.rcat, pb.roff, pb.pair_q, pb.pair_r)
            g.run()
            recs, cig = g.read()
            _check_oracle(pb, recs, cig)
            _say(f"[graph] tall one-pair route {route} pair {p}: score {recs['score1'][0]}")
    finally:
        g.close()
