"""A pair list processed in slices (Context.align_batch_chunks): every
slice's records and CIGARs against the oracle's on the same pairs, with
host and with device-resident inputs, and with a CIGAR arena that starts too
small (the slice is run again with one that fits)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1208_6350_amd as swx
import workloads as W
from tests.fullsize import mismatches

pytestmark = pytest.mark.gpu


def _check_slices(ctx, b, slices):
    seen = 0
    for k0, k1, recs, cig in slices:
        if hasattr(recs, "cpu"):
            recs = recs.cpu().numpy().view(swx.REC_DTYPE)
            cig = cig.cpu().numpy().view(np.uint32)
        s = b.subset(np.arange(k0, k1))
        ref, rcig, rcoff = oracle.align_many(s.qcat, s.qoff, s.rcat, s.roff, s.pair_q, s.pair_r,
                                             s.matrix, s.gap_open, s.gap_extend, nthreads=8)
        bad = mismatches(recs[:k1 - k0].copy(), cig, ref, rcig, rcoff)
        assert bad["pairs_bad"] == 0, (k0, k1, bad)
        assert k0 == seen
        seen = k1
    assert seen == b.npairs


def test_all_vs_all_in_slices_host():
    ctx = swx.Context(0)
    try:
        b = W.all_vs_all(n_reads=160)   # 12,720 pairs
        _check_slices(ctx, b, ctx.align_batch_chunks(
            b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat, b.roff, b.pair_q,
            b.pair_r, chunk_pairs=5000, cigar_words_per_pair=1))
    finally:
        ctx.close()


def test_all_vs_all_in_slices_device():
    import torch
    dev = torch.device("cuda:0")
    ctx = swx.Context(0)
    try:
        b = W.all_vs_all(n_reads=200)   # 19,900 pairs
        to = lambda x: torch.as_tensor(np.ascontiguousarray(x)).to(dev)
        _check_slices(ctx, b, ctx.align_batch_chunks(
            b.matrix, b.gap_open, b.gap_extend, to(b.qcat), to(b.qoff), to(b.rcat), to(b.roff),
            to(b.pair_q), to(b.pair_r), chunk_pairs=6000, cigar_words_per_pair=2))
    finally:
        ctx.close()
