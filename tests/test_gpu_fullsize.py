"""Parity at full size, in the configuration the benchmark times: inputs and
outputs device-resident (SWX_MEM_DEVICE both ways), every output requested,
every pair of the batched-DNA workload (1,000,000 read/window pairs) and of
the protein one-against-many workload (100,000 targets) compared with the
oracle field by field and CIGAR word by word.  The oracle runs on the host's
cores (about 20 s for the DNA workload on 16 threads)."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle
import paper_1208_6350_amd as swx
import workloads as W
from tests.fullsize import mismatches

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _device_run(ctx, b, flags=swx.SWX_ALL):
    import torch
    dev = torch.device("cuda:0")
    to = lambda x: torch.as_tensor(np.ascontiguousarray(x)).to(dev)
    dq, dqo, dr, dro, dpq, dpr = (to(x) for x in (b.qcat, b.qoff, b.rcat, b.roff, b.pair_q,
                                                    b.pair_r))
    recs = torch.empty(b.npairs * swx.REC_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    cig = torch.empty(int(b.qlen().sum() + b.rlen().sum() + b.npairs), dtype=torch.int32,
                      device=dev)
    torch.cuda.synchronize()
    for rep in range(2):   # the second run reuses the context's pool, as in the benchmark
        st, used = swx.swx_align_batch(ctx.handle, b.matrix, b.gap_open, b.gap_extend, dq, dqo,
                                       dr, dro, dpq, dpr, flags, -1, swx.SWX_MEM_DEVICE, recs,
                                       cig, swx.SWX_MEM_DEVICE)
        assert st == 0, swx.swx_last_error()
    torch.cuda.synchronize()
    r = recs.cpu().numpy().view(swx.REC_DTYPE)
    c = cig[:used].cpu().numpy().view(np.uint32)
    return r, c


def _oracle(b, flags=swx.SWX_ALL):
    threads = min(os.cpu_count() or 1, 16)
    return oracle.align_many(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r, b.matrix,
                             b.gap_open, b.gap_extend, flags, -1, nthreads=threads)


@pytest.mark.parametrize("tuning", [{}, {"fill_sched": 2, "side_streams": 0}])
def test_batched_dna_full_size_device_resident(tuning):
    b = W.config4()
    _say(f"[fullsize] config4 {b.npairs} pairs, tuning {tuning}")
    ctx = swx.Context(0)
    try:
        if tuning:
            ctx.set_tuning(**tuning)
        recs, cig = _device_run(ctx, b)
    finally:
        ctx.close()
    ref, rcig, rcoff = _oracle(b)
    bad = mismatches(recs, cig, ref, rcig, rcoff)
    _say(f"[fullsize] config4 mismatches {bad}")
    assert bad["pairs_bad"] == 0, bad


def test_batched_dna_reversed_pass_split():
    """263,000 pairs of the batched-DNA workload: 2,055 tasks of 128 pairs,
    just above the 8 tasks per compute unit of a 256-CU device from which the
    reversed pass runs its largest tasks four waves each on a side launch
    beside the rest.  Every pair against the oracle."""
    b = W.config4(npairs=263_000)
    _say(f"[fullsize] config4 {b.npairs} pairs (reversed-pass split)")
    ctx = swx.Context(0)
    try:
        recs, cig = _device_run(ctx, b)
    finally:
        ctx.close()
    ref, rcig, rcoff = _oracle(b)
    bad = mismatches(recs, cig, ref, rcig, rcoff)
    _say(f"[fullsize] config4 263k mismatches {bad}")
    assert bad["pairs_bad"] == 0, bad


def test_protein_search_full_size_device_resident():
    b = W.config3()
    _say(f"[fullsize] config3 {b.npairs} targets")
    ctx = swx.Context(0)
    try:
        recs, cig = _device_run(ctx, b)
    finally:
        ctx.close()
    ref, rcig, rcoff = _oracle(b)
    bad = mismatches(recs, cig, ref, rcig, rcoff)
    _say(f"[fullsize] config3 mismatches {bad}")
    assert bad["pairs_bad"] == 0, bad
