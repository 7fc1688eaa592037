"""Field-by-field comparison of a whole batch's GPU records and CIGARs with
the oracle's (vectorised, for batches of up to millions of pairs).  Test-side
only: shared by the full-size parity tests and the benchmark's check of its
own timed step."""
from __future__ import annotations

import numpy as np

FIELDS = ["score1", "score2", "read_begin1", "read_end1", "ref_begin1", "ref_end1", "ref_end2"]


def mismatches(recs, cig, ref, rcig, rcoff, flags=7):
    """recs: REC_DTYPE array of the library; cig: its CIGAR arena (uint32);
    ref, rcig, rcoff: oracle.align_many's output for the same pairs.
    Returns {field: number of pairs that differ} including "cigar" (pairs
    whose CIGAR words differ) and "pairs_bad" (pairs with any difference)."""
    n = len(recs)
    bad = np.zeros(n, dtype=bool)
    out = {}
    for k, f in enumerate(FIELDS):
        d = recs[f].astype(np.int64) != ref[:, k]
        out[f] = int(d.sum())
        bad |= d
    if flags & 2:
        glen = recs["cigar_len"].astype(np.int64)
        olen = ref[:, 7]
        dl = glen != olen
        same = ~dl
        # words of the pairs whose lengths agree, gathered from both arenas
        lens = np.where(same, glen, 0)
        tot = int(lens.sum())
        dw = np.zeros(n, dtype=bool)
        if tot:
            owner = np.repeat(np.arange(n), lens)
            first = np.repeat(np.cumsum(lens) - lens, lens)
            within = np.arange(tot) - first
            g = cig[recs["cigar_off"].astype(np.int64)[owner] + within].astype(np.uint32)
            o = rcig[rcoff[:-1][owner] + within].astype(np.uint32)
            diff = g != o
            if diff.any():
                dw[np.unique(owner[diff])] = True
        out["cigar"] = int((dl | dw).sum())
        bad |= dl | dw
    out["pairs_bad"] = int(bad.sum())
    return out
