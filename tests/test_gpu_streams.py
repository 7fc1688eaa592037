"""The caller's stream at the boundary: swx_align_batch, swx_align and
swx_graph_run queue their work on a torch stream handed to them, after the
caller's own work on it.  The inputs are written on that stream by
asynchronous copies that the test never waits for, so a call that did not
order itself after them would read stale buffers and differ from the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1208_6350_amd as swx
import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ["score1", "score2", "read_begin1", "read_end1", "ref_begin1", "ref_end1", "ref_end2"]


def _pinned(x):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x))
    return t.pin_memory()


def _check_recs(b, recs, cig):
    ref, rcig, rcoff = oracle.align_many(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r,
                                         b.matrix, b.gap_open, b.gap_extend, nthreads=8)
    for k, f in enumerate(FIELDS):
        assert np.array_equal(recs[f].astype(np.int64), ref[:, k]), f
    for p in range(b.npairs):
        got = cig[recs["cigar_off"][p]:recs["cigar_off"][p] + recs["cigar_len"][p]]
        assert np.array_equal(got, rcig[rcoff[p]:rcoff[p] + ref[p, 7]]), p


def test_batch_on_a_torch_stream_after_its_writes():
    import torch
    dev = torch.device("cuda:0")
    b = W.random_pairs(9100, 6000, (60, 250), (100, 650))
    host = [_pinned(x) for x in (b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r)]
    bufs = [torch.zeros(h.shape, dtype=h.dtype, device=dev) for h in host]
    recs = torch.zeros(b.npairs * swx.REC_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    cig = torch.zeros(int(b.qlen().sum() + b.rlen().sum() + b.npairs), dtype=torch.int32,
                      device=dev)
    torch.cuda.synchronize()
    ctx = swx.Context(0)
    s = torch.cuda.Stream()
    try:
        for rep in range(2):
            with torch.cuda.stream(s):
                for d, h in zip(bufs, host):
                    d.zero_()
                    d.copy_(h, non_blocking=True)
            # no synchronisation: the library must queue behind the copies
            st, used = swx.swx_align_batch(ctx.handle, b.matrix, b.gap_open, b.gap_extend, *bufs,
                                           swx.SWX_ALL, -1, swx.SWX_MEM_DEVICE, recs, cig,
                                           swx.SWX_MEM_DEVICE, stream=s)
            assert st == 0, swx.swx_last_error()
            # the call returned with its outputs written: read them on the
            # same stream
            with torch.cuda.stream(s):
                r_host = recs.to("cpu", non_blocking=False)
                c_host = cig[:used].to("cpu", non_blocking=False)
            r = r_host.numpy().view(swx.REC_DTYPE)
            _check_recs(b, r, c_host.numpy().view(np.uint32))
    finally:
        ctx.close()


def test_single_pair_on_a_torch_stream_with_device_reference():
    import torch
    dev = torch.device("cuda:0")
    b = W.random_pairs(9101, 12, (40, 200), (300, 3000))
    ctx = swx.Context(0)
    s = torch.cuda.Stream()
    try:
        recs, cig = ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat,
                                    b.roff, b.pair_q, b.pair_r)
        for p in range(b.npairs):
            h = _pinned(b.ref(p))
            d = torch.zeros(len(h), dtype=torch.int8, device=dev)
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                d.copy_(h, non_blocking=True)
            prof = swx.swx_profile_create(ctx.handle, b.query(p), b.matrix, b.gap_open,
                                          b.gap_extend)
            try:
                rec, c1 = swx.swx_align(prof, (d.data_ptr(), len(h)),
                                        swx.SWX_ALL | swx.SWX_REF_DEVICE, -1, stream=s)
            finally:
                swx.swx_profile_destroy(prof)
            for f in FIELDS:
                assert rec[f] == recs[f][p], (p, f)
            assert c1 == swx.decode_cigar(cig[recs["cigar_off"][p]:recs["cigar_off"][p] +
                                              recs["cigar_len"][p]])
    finally:
        ctx.close()


def test_graph_replay_on_a_torch_stream():
    import torch
    b = W.random_pairs(9102, 200, (30, 150), (50, 600))
    ctx = swx.Context(0)
    s = torch.cuda.Stream()
    g = swx.Graph(ctx, b.matrix, b.gap_open, b.gap_extend, max_pairs=256, max_qlen=160,
                  max_rlen=640, qcat_cap=256 * 160, rcat_cap=256 * 640, nq_cap=257,
                  nr_cap=258)
    try:
        recs, cig = ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat,
                                    b.roff, b.pair_q, b.pair_r)
        g.load(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r)
        for rep in range(3):
            g.run(stream=s)
            r, c = g.read()
            for f in FIELDS:
                assert np.array_equal(r[f], recs[f]), (rep, f)
            for p in range(b.npairs):
                assert np.array_equal(c[r["cigar_off"][p]:r["cigar_off"][p] + r["cigar_len"][p]],
                                      cig[recs["cigar_off"][p]:recs["cigar_off"][p] +
                                          recs["cigar_len"][p]])
    finally:
        g.close()
        ctx.close()
