"""The batch entry point that allocates no device memory
(swx_align_batch_noalloc, scratch in the library's static per-GPU array)
against the ordinary batch call, field by field and CIGAR word by word, on two
calls in a row (the second with a smaller input, so that stale scratch from
the first would show), host and device memory, and its size limits."""
from __future__ import annotations

import numpy as np
import pytest

import paper_1208_6350_amd as swx
import workloads as W
from tests.fullsize import FIELDS

pytestmark = pytest.mark.gpu


def _host_both(ctx, b, flags=swx.SWX_ALL):
    ref_recs, ref_cig = ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff,
                                        b.rcat, b.roff, b.pair_q, b.pair_r, flags)
    recs = np.zeros(b.npairs, dtype=swx.REC_DTYPE)
    cap = swx.swx_cigar_bound(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat,
                              b.roff, b.pair_q, b.pair_r, flags)
    cig = np.zeros(max(cap, 1), dtype=np.uint32)
    st, used = swx.swx_align_batch_noalloc(ctx.handle, b.matrix, b.gap_open, b.gap_extend,
                                           b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r,
                                           flags, -1, swx.SWX_MEM_HOST, recs, cig,
                                           swx.SWX_MEM_HOST)
    assert st == 0, swx.swx_last_error()
    return ref_recs, ref_cig, recs, cig[:used]


def _same(b, ref_recs, ref_cig, recs, cig):
    for f in FIELDS + ["cigar_len", "cigar_off", "lane_bits"]:
        assert np.array_equal(recs[f], ref_recs[f]), f
    assert np.array_equal(cig, ref_cig)


def test_noalloc_equals_batch_call_twice_host_memory():
    ctx = swx.Context(0)
    try:
        big = W.config4(npairs=3000)
        small = W.random_pairs(7301, 500, (20, 200), (40, 500))
        for b in (big, small):
            _same(b, *_host_both(ctx, b))
        # protein (general profile) and long pairs (the intra path) too
        prot = W.random_pairs(7302, 300, (20, 300), (50, 900), alphabet=24,
                              matrix=W.protein_matrix_standin(), o=11, e=1)
        _same(prot, *_host_both(ctx, prot))
        lng = W.random_pairs(7303, 3, (500, 1500), (20000, 70000), planted=0.7)
        _same(lng, *_host_both(ctx, lng))
    finally:
        ctx.close()


def test_noalloc_equals_batch_call_twice_device_memory():
    import torch
    dev = torch.device("cuda:0")
    ctx = swx.Context(0)
    try:
        for b in (W.config4(npairs=3500), W.config4(seed_k=40, npairs=900)):
            to = lambda x: torch.as_tensor(np.ascontiguousarray(x)).to(dev)
            ins = [to(x) for x in (b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r)]
            out = []
            for fn in (swx.swx_align_batch, swx.swx_align_batch_noalloc):
                recs = torch.zeros(b.npairs * swx.REC_DTYPE.itemsize, dtype=torch.uint8,
                                   device=dev)
                cig = torch.zeros(int(b.qlen().sum() + b.rlen().sum() + b.npairs),
                                  dtype=torch.int32, device=dev)
                st, used = fn(ctx.handle, b.matrix, b.gap_open, b.gap_extend, *ins, swx.SWX_ALL,
                              -1, swx.SWX_MEM_DEVICE, recs, cig, swx.SWX_MEM_DEVICE)
                assert st == 0, swx.swx_last_error()
                out.append((recs.cpu().numpy().view(swx.REC_DTYPE),
                            cig[:used].cpu().numpy().view(np.uint32)))
            _same(b, out[0][0], out[0][1], out[1][0], out[1][1])
    finally:
        ctx.close()


def test_noalloc_limits():
    ctx = swx.Context(0)
    try:
        # host inputs above half of the scratch: rejected before any device work
        g = np.random.Generator(np.random.PCG64(7304))
        q = g.integers(0, 4, 100).astype(np.int8)
        r = g.integers(0, 4, 40 << 20).astype(np.int8)
        b = W.from_lists("noalloc-too-big", W.dna_matrix(), 3, 1, [q], [r])
        recs = np.zeros(1, dtype=swx.REC_DTYPE)
        cig = np.zeros(1, dtype=np.uint32)
        st, _ = swx.swx_align_batch_noalloc(ctx.handle, b.matrix, 3, 1, b.qcat, b.qoff, b.rcat,
                                            b.roff, b.pair_q, b.pair_r, swx.SWX_ALL, -1,
                                            swx.SWX_MEM_HOST, recs, cig, swx.SWX_MEM_HOST)
        assert st == -1 and "scratch" in swx.swx_last_error()
        # too many pairs
        n = swx._binding.lib().swx_align_batch_noalloc  # noqa: F841 (symbol present)
        many = W.random_pairs(7305, 65537, (1, 2), (1, 2))
        recs = np.zeros(many.npairs, dtype=swx.REC_DTYPE)
        cig = np.zeros(many.npairs * 6, dtype=np.uint32)
        st, _ = swx.swx_align_batch_noalloc(ctx.handle, many.matrix, 3, 1, many.qcat, many.qoff,
                                            many.rcat, many.roff, many.pair_q, many.pair_r,
                                            swx.SWX_ALL, -1, swx.SWX_MEM_HOST, recs, cig,
                                            swx.SWX_MEM_HOST)
        assert st == -1
        # the entry point still works afterwards
        small = W.random_pairs(7306, 200, (20, 100), (40, 300))
        _same(small, *_host_both(ctx, small))
    finally:
        ctx.close()
