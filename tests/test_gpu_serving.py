"""GPU tests of the serving loop: each request's result is the same when it is
served in a mix of concurrent, continuously formed batches as when it is
aligned alone, and equals the oracle; admission by memory footprint and the
pending-queue limit behave as documented."""
from __future__ import annotations

import sys
import time

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


def _collect(srv, n, timeout_s=120.0):
    outs, cigs = [], []
    t_end = time.monotonic() + timeout_s
    while sum(len(o) for o in outs) < n:
        assert time.monotonic() < t_end, "completions did not arrive"
        o, c = srv.poll(4096, timeout_us=20_000, keep_cigar=True)
        outs.append(o)
        cigs.extend(c)
    out = np.concatenate(outs)
    return out, cigs


def _mix(n_short=240, n_long=3):
    pool = W.config5_pool(n_short=n_short, n_long=n_long)
    return pool


def test_serving_mix_equals_alone_and_oracle():
    pool = _mix()
    n = pool.npairs
    srv = swx.Server(pool.matrix, pool.gap_open, pool.gap_extend, workers=3, max_batch=40)
    try:
        reqs = swx.make_requests(pool.qcat, pool.qoff, pool.rcat, pool.roff, pool.pair_q,
                                 pool.pair_r)
        # staggered arrivals: later requests arrive while earlier batches run
        order = np.random.Generator(np.random.PCG64(3)).permutation(n)
        _say(f"[serve] submitting {n} requests in 8 waves")
        for chunk in np.array_split(order, 8):
            st, tk = srv.submit(reqs[chunk])
            assert st == 0 and len(tk) == len(chunk)
            time.sleep(0.002)
        out, cigs = _collect(srv, n)
        stats = srv.stats()
    finally:
        srv.close()
    assert (out["status"] == 0).all()
    assert stats["completed"] == n and stats["batches"] >= 4, stats
    # batches really ran side by side on the GPU
    spans = sorted({(int(a), int(b)) for a, b in zip(out["t_start_ns"], out["t_done_ns"])})
    overlap = any(spans[k + 1][0] < spans[k][1] for k in range(len(spans) - 1))
    _say(f"[serve] {len(spans)} batches, sizes up to {stats['max_batch_seen']}, overlap {overlap}")
    assert overlap
    # against the oracle
    ref, rcig, rcoff = oracle.align_many(pool.qcat, pool.qoff, pool.rcat, pool.roff, pool.pair_q,
                                         pool.pair_r, pool.matrix, pool.gap_open, pool.gap_extend)
    by_tag = {int(t): k for k, t in enumerate(out["tag"])}
    ctx = swx.Context(0)
    try:
        for p in range(n):
            k = by_tag[p]
            rec = out["rec"][k]
            exp = ref[p]
            for f_i, f in enumerate(FIELDS):
                assert int(rec[f]) == int(exp[f_i]), (p, f)
            assert np.array_equal(cigs[k], rcig[rcoff[p]:rcoff[p] + exp[7]]), p
        # and alone, one request per call, for a sample (including the long ones)
        for p in list(range(0, n, 37)) + list(range(n - 3, n)):
            k = by_tag[p]
            rec1, c1 = ctx.align_pair(pool.query(p), pool.ref(p), pool.matrix, pool.gap_open,
                                      pool.gap_extend)
            for f in FIELDS:
                assert rec1[f] == int(out["rec"][k][f]), (p, f)
            assert c1 == swx.decode_cigar(cigs[k]), p
    finally:
        ctx.close()


def test_registered_query_equals_inline():
    b = W.config3(ntargets=150)
    srv = swx.Server(b.matrix, b.gap_open, b.gap_extend, workers=2, max_batch=64)
    try:
        qid = srv.register_query(b.query(0))
        inline = swx.make_requests(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r)
        resident = inline.copy()
        resident["query_id"] = qid
        resident["tag"] += 1000
        assert srv.submit(inline)[0] == 0
        assert srv.submit(resident)[0] == 0
        out, cigs = _collect(srv, 2 * b.npairs)
    finally:
        srv.close()
    by_tag = {int(t): k for k, t in enumerate(out["tag"])}
    for p in range(b.npairs):
        a, r = by_tag[p], by_tag[p + 1000]
        assert out["rec"][a].tobytes() == out["rec"][r].tobytes(), p
        assert np.array_equal(cigs[a], cigs[r]), p


def test_admission_budget_and_queue_limit():
    b = W.random_pairs(811, 60, (20, 200), (50, 600))
    reqs = swx.make_requests(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r)
    # a budget below one request's footprint: every request runs alone
    srv = swx.Server(b.matrix, b.gap_open, b.gap_extend, workers=2, mem_budget=1)
    try:
        assert srv.submit(reqs)[0] == 0
        out, _ = _collect(srv, b.npairs)
        assert (out["batch_size"] == 1).all()
        assert srv.stats()["peak_inflight_bytes"] > 1
    finally:
        srv.close()
    ref, _, _ = oracle.align_many(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r, b.matrix,
                                  b.gap_open, b.gap_extend)
    by_tag = {int(t): k for k, t in enumerate(out["tag"])}
    for p in range(b.npairs):
        for f_i, f in enumerate(FIELDS):
            assert int(out["rec"][by_tag[p]][f]) == int(ref[p][f_i])
    # a short pending queue: the accepted prefix is reported with SWX_EBUSY
    srv = swx.Server(b.matrix, b.gap_open, b.gap_extend, workers=1, max_pending=5,
                     mem_budget=1)
    try:
        st, tk = srv.submit(reqs)
        assert st == swx.SWX_EBUSY and 5 <= len(tk) < b.npairs
        out, _ = _collect(srv, len(tk))
        assert srv.stats()["deferred"] == b.npairs - len(tk)
    finally:
        srv.close()


def test_size_classes_have_their_own_queue_limit():
    # long requests fill their queue and are refused; short ones submitted
    # next are still queued, and every accepted request equals the oracle
    lb = W.random_pairs(815, 8, (30, 40), (30, 40))   # at least 900 cells: long below
    sb = W.random_pairs(816, 4, (5, 10), (5, 10))     # at most 100 cells: short
    srv = swx.Server(lb.matrix, lb.gap_open, lb.gap_extend, workers=1, max_pending=2,
                     mem_budget=1, long_cells=500)
    try:
        lr = swx.make_requests(lb.qcat, lb.qoff, lb.rcat, lb.roff, lb.pair_q, lb.pair_r,
                               tags=np.arange(lb.npairs))
        st, tk = srv.submit(lr)
        assert st == swx.SWX_EBUSY and 2 <= len(tk) < lb.npairs
        sr = swx.make_requests(sb.qcat, sb.qoff, sb.rcat, sb.roff, sb.pair_q[:2], sb.pair_r[:2],
                               tags=100 + np.arange(2))
        st2, tk2 = srv.submit(sr)
        assert st2 == 0 and len(tk2) == 2
        out, _ = _collect(srv, len(tk) + 2)
    finally:
        srv.close()
    assert (out["status"] == 0).all()
    for bt, base in ((lb, 0), (sb, 100)):
        ref, _, _ = oracle.align_many(bt.qcat, bt.qoff, bt.rcat, bt.roff, bt.pair_q, bt.pair_r,
                                      bt.matrix, bt.gap_open, bt.gap_extend)
        for c in out[(out["tag"] >= base) & (out["tag"] < base + 100)]:
            p = int(c["tag"]) - base
            for f_i, f in enumerate(FIELDS):
                assert int(c["rec"][f]) == int(ref[p][f_i]), (base, p, f)


def test_invalid_request_accepts_nothing():
    b = W.random_pairs(812, 4, (3, 10), (3, 10))
    b.rcat[1] = 7
    srv = swx.Server(b.matrix, b.gap_open, b.gap_extend)
    try:
        reqs = swx.make_requests(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r)
        with pytest.raises(swx.SwxError) as ei:
            srv.submit(reqs)
        assert ei.value.status == -1
        assert srv.stats()["submitted"] == 0
    finally:
        srv.close()


def test_serving_graph_worker_equals_oracle():
    """The short-request worker replays a captured graph (intra route) in
    chunks of its capacity; requests beyond its capacities, or with an empty
    query, take the eager path.  Every result equals the oracle."""
    a = W.random_pairs(813, 150, (0, 150), (0, 900))
    big = W.random_pairs(814, 6, (200, 400), (1000, 2000), planted=0.7)
    reqs = np.concatenate([
        swx.make_requests(a.qcat, a.qoff, a.rcat, a.roff, a.pair_q, a.pair_r),
        swx.make_requests(big.qcat, big.qoff, big.rcat, big.roff, big.pair_q, big.pair_r)])
    reqs["tag"] = np.arange(len(reqs))
    srv = swx.Server(a.matrix, a.gap_open, a.gap_extend, workers=2, max_batch=48,
                     graph_batch=32, graph_max_qlen=160, graph_max_rlen=1000)
    try:
        _say(f"[serve-graph] submitting {len(reqs)} requests")
        for chunk in np.array_split(np.arange(len(reqs)), 6):
            assert srv.submit(reqs[chunk])[0] == 0
            time.sleep(0.002)
        out, cigs = _collect(srv, len(reqs))
        stats = srv.stats()
    finally:
        srv.close()
    _say(f"[serve-graph] {stats['batches']} batches, {stats['graph_batches']} through the graph")
    assert (out["status"] == 0).all()
    assert stats["graph_batches"] >= 1, stats
    by_tag = {int(t): k for k, t in enumerate(out["tag"])}
    for part, off in ((a, 0), (big, a.npairs)):
        ref, rcig, rcoff = oracle.align_many(part.qcat, part.qoff, part.rcat, part.roff,
                                             part.pair_q, part.pair_r, part.matrix,
                                             part.gap_open, part.gap_extend)
        for p in range(part.npairs):
            k = by_tag[off + p]
            for f_i, f in enumerate(FIELDS):
                assert int(out["rec"][k][f]) == int(ref[p][f_i]), (off + p, f)
            assert np.array_equal(cigs[k], rcig[rcoff[p]:rcoff[p] + ref[p, 7]]), off + p
