"""GPU test of the lane-width probe: the 8-bit SWAR recurrence and the packed
16-bit one give the same best score for every synthetic pair, and sampled
pairs equal the oracle's score1."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1208_6350_amd as swx
import workloads as W

pytestmark = pytest.mark.gpu


def _mix(x):
    """The probe's published integer hash (a 32-bit finaliser), in numpy."""
    x = np.asarray(x, dtype=np.uint64) & 0xFFFFFFFF
    x ^= x >> 16
    x = (x * 0x7FEB352D) & 0xFFFFFFFF
    x ^= x >> 15
    x = (x * 0x846CA68B) & 0xFFFFFFFF
    x ^= x >> 16
    return x


def test_probe_widths_agree_and_match_oracle():
    ctx = swx.Context(0)
    try:
        cols, blocks = 64, 4
        b8, ms8, _ = ctx.lane_probe(8, columns=cols, blocks=blocks)
        b16, ms16, _ = ctx.lane_probe(16, columns=cols, blocks=blocks)
    finally:
        ctx.close()
    # the 16-bit run covers the first half of the 8-bit run's pairs
    assert np.array_equal(b8[:len(b16)], b16)
    mat = W.dna_matrix(2, -2)
    ref = (_mix(np.arange(cols) + 0x9E37) & 3).astype(np.int8)
    for p in list(range(0, len(b8), 97))[:40]:
        q = (_mix(p * 16 + np.arange(16)) & 3).astype(np.int8)
        a = oracle.align(q, ref, mat, 3, 1)
        assert int(b8[p]) == a.score1, p


def test_probe_rejects_bad_widths():
    ctx = swx.Context(0)
    try:
        for bits in (4, 32):
            with pytest.raises(swx.SwxError):
                ctx.lane_probe(bits, columns=8, blocks=1)
    finally:
        ctx.close()


def test_packed_max3_is_exact_below_0x7c00():
    """The batched fill takes H as one packed f16 three-way maximum; on every
    16-bit pattern below 0x7C00 it must equal the unsigned maximum (checked on
    the device over every pair of such values with 8 third operands, and
    2^31 pseudo-random triples)."""
    ctx = swx.Context(0)
    try:
        bad, n = ctx.check_max3()
    finally:
        ctx.close()
    assert n == 0x7C00 * 0x7C00 * 16 + (1 << 26) * 32
    assert bad == 0
