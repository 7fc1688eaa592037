"""Writes the stored expected results under tests/golden/ by calling only the
CPU oracle on the seeded workload generators.

    python tests/golden/make_golden.py

config2.json: the single long-reference pair (1,000-nt read against a
5,000,000-nt reference with three planted near-copies), every output field of
the oracle plus its CIGAR words.  The oracle needs about a minute for it, which
is why the GPU test reads the stored values instead of recomputing them."""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def config2():
    b = W.config2()
    t = time.perf_counter()
    a = oracle.align(b.query(0), b.ref(0), b.matrix, b.gap_open, b.gap_extend)
    dt = time.perf_counter() - t
    out = {
        "workload": "config2 (seed 12086350 + 2): 1,000-nt read vs 5,000,000-nt reference, "
                    "+2/-2, gap open 3, extend 1, mask_len default",
        "oracle_seconds": round(dt, 1),
        "score1": a.score1, "score2": a.score2,
        "read_begin1": a.read_begin1, "read_end1": a.read_end1,
        "ref_begin1": a.ref_begin1, "ref_end1": a.ref_end1, "ref_end2": a.ref_end2,
        "cigar": [[int(n), op] for n, op in a.cigar],
        "generator": {"locus": b.meta["locus"], "copies": b.meta["copies"]},
    }
    with open(os.path.join(HERE, "config2.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"config2: score1 {a.score1} score2 {a.score2} in {dt:.1f}s")


if __name__ == "__main__":
    config2()
