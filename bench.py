"""Benchmark: GCUPS of the whole alignment path on one MI355X.

A step is one pass of the whole path -- forward fill with the max array and
the end, exact 32-bit re-run of saturated pairs, reversed pass (begin), banded
traceback (CIGAR), masked max array (score2) and result records -- over one
batch of synthetic read/window pairs that are already resident in HBM.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2]

Prints one JSON line.  `value` is forward-fill cells (sum of qlen*rlen over
pairs) per second of the whole path, in GCUPS.  `roofline` reports the forward
fill kernel against the packed 16-bit integer VALU peak; `cpu_baseline` times
the CPU oracle on a bounded sample of the same pairs on this host's cores;
`per_pair` times the same library called one pair at a time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Integer-VALU peak of MI355X: 256 CUs x 4 SIMD x 16 lanes = 64 lane-ops per
# clock per CU at 2.4 GHz = 39.32 T lane-ops/s; packed 16-bit instructions do
# two operations per lane-op: 78.64 T ops/s.
PEAK_PK16_TOPS = 256 * 64 * 2.4e9 * 2 / 1e12
OPS_PER_CELL = 10      # algorithmic integer operations per DP cell


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--pairs", type=int, default=1_000_000)
    ap.add_argument("--per-pair-sample", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-rate", default="2e4,1e5,5e5,2e6",
                    help="offered loads of the serving phase, requests per second (comma list): "
                         "the workload's three loads, and one below capacity")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed steps (no autotuner, output modes, graph, per-pair, "
                         "serving or CPU phases): the form the kernel profiles are taken of")
    ap.add_argument("--only-config", choices=["c1", "c2", "c3", "c5_long"], default=None,
                    help="run only this entry of the per-configuration phase (default "
                         "settings, no oracle with --no-cpu) and print it: the form the "
                         "per-configuration kernel profiles are taken of")
    ap.add_argument("--no-large-avsa", action="store_true",
                    help="skip the all-vs-all run at read-overlap-graph scale (2e8 pairs)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-configuration phase (the other four workloads)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (default: tune on a 100k-pair sample first)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the timed steps, copy a device buffer of this many MiB once "
                         "(a plain copy kernel of known size for calibrating byte counters)")
    return ap.parse_args()


# Sources whose change invalidates a recorded HBM traffic figure of the fill.
FILL_SOURCES = ["paper_1208_6350_amd/csrc/fill_inter.hip", "paper_1208_6350_amd/csrc/lanes.h",
                "paper_1208_6350_amd/csrc/swx_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_inter_fill_traffic.md")


def fill_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in FILL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


VALU_FILE = os.path.join(ROOT, "profiles", "k_inter_fill_valu_counters.md")


def recorded_fields(path, pairs=None):
    """The `- key: value` lines of a committed counter summary, or None when
    the summary is missing, for another workload size or taken on a
    different version of the fill kernel."""
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("fill_source_sha256") != fill_source_hash():
        return None
    if pairs is not None and vals.get("pairs") != str(pairs):
        return None
    return vals


def recorded_traffic(pairs):
    """HBM bytes per forward-fill launch from the committed counter summary,
    or None when the summary is missing, for another workload size, or was
    taken on a different version of the fill kernel."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            vals[k.strip()] = v.strip().strip("`")
    try:
        if vals.get("fill_source_sha256") != fill_source_hash() or int(vals["pairs"]) != pairs:
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(b, seconds, gpu_out=None):
    """The oracle, unmodified, over a bounded sample of the workload.  With
    gpu_out = (records, CIGAR arena) of the timed GPU run, the oracle's results
    for the sample (the first pairs of the batch) are compared with them field
    by field and CIGAR word by word, outside the timed region."""
    import numpy as np

    import oracle
    threads = os.cpu_count() or 1
    probe = b.subset(np.arange(min(2000, b.npairs)))
    t = time.perf_counter()
    oracle.align_many(probe.qcat, probe.qoff, probe.rcat, probe.roff, probe.pair_q, probe.pair_r,
                      probe.matrix, probe.gap_open, probe.gap_extend, nthreads=threads)
    rate = probe.cells() / max(time.perf_counter() - t, 1e-6)
    n = int(min(b.npairs, max(2000, seconds * rate / (b.cells() / b.npairs))))
    s = b.subset(np.arange(n))
    t = time.perf_counter()
    ref, rcig, rcoff = oracle.align_many(s.qcat, s.qoff, s.rcat, s.roff, s.pair_q, s.pair_r,
                                         s.matrix, s.gap_open, s.gap_extend, nthreads=threads)
    dt = time.perf_counter() - t
    out = {"value": round(s.cells() / dt / 1e9, 4), "unit": "GCUPS", "cores": threads,
           "kind": "oracle",
           "sample": f"first {n} pairs of the same workload ({s.cells()/1e9:.2f} G cells, "
                     f"{dt:.1f} s, whole path incl. begin/CIGAR/score2)"}
    parity = None
    if gpu_out is not None:
        from tests.fullsize import mismatches
        recs, cig = gpu_out
        bad = mismatches(recs[:n], cig, ref, rcig, rcoff)
        parity = {"pairs": n, "mismatches": bad["pairs_bad"], "by_field": bad,
                  "checked": "records and CIGARs of the last timed step (device-resident "
                             "outputs) against the oracle on the same pairs"}
    return out, parity


_SERVE_POOL = {}


def serving_phase(rate, seconds, warmup=0.5, pool_short=50_000, pool_long=1_000, workers=3,
                  mem_budget=32 << 30, max_pending=8192, graph_batch=0, side_streams=-1):
    """Open-loop Poisson replay of the serving workload through swx_server_*:
    90% 150-nt reads vs 1-kb windows, 10% 10-kb reads vs 20-kb windows, drawn
    from a seeded pool.  Latency = completion time - scheduled arrival (so
    queueing behind an overloaded server counts).  A request that finds the
    queue full (max_pending waiting) is refused and counted, not retried, so
    an offered load above capacity measures saturated throughput and the
    queueing delay of the admitted requests.  Requests arriving in the first
    `warmup` seconds are served but not measured."""
    import numpy as np

    import paper_1208_6350_amd as swx
    import workloads as W
    key = (pool_short, pool_long)
    if key not in _SERVE_POOL:
        _SERVE_POOL[key] = W.config5_pool(n_short=pool_short, n_long=pool_long)
    pool = _SERVE_POOL[key]
    is_long = pool.meta["is_long"]
    g = W.rng_for(105)
    t_arr, which = W.poisson_schedule(g, rate, warmup + seconds, pool.npairs, is_long, 0.10)
    n = len(which)
    reqs = swx.make_requests(pool.qcat, pool.qoff, pool.rcat, pool.roff, pool.pair_q[which],
                             pool.pair_r[which], tags=np.arange(n))
    cells = (pool.qlen()[which].astype(np.int64) * pool.rlen()[which])
    lng = is_long[which]
    srv = swx.Server(pool.matrix, pool.gap_open, pool.gap_extend, workers=workers,
                     mem_budget=mem_budget, max_pending=max_pending, graph_batch=graph_batch,
                     graph_max_qlen=200, graph_max_rlen=1100, side_streams=side_streams)
    done_ns = np.zeros(n, dtype=np.int64)
    bsize = np.zeros(n, dtype=np.int64)
    accepted = np.zeros(n, dtype=bool)
    t0 = time.monotonic_ns() + 20_000_000
    arr_ns = t0 + (t_arr * 1e9).astype(np.int64)
    sub, got, nacc = 0, 0, 0
    limit = t0 + int((warmup + seconds + 120) * 1e9)
    while (sub < n or got < nacc) and time.monotonic_ns() < limit:
        now = time.monotonic_ns()
        k = int(np.searchsorted(arr_ns, now, side="right"))
        if k > sub:
            # each size class has its own queue limit: submit the arrivals
            # class by class, so that a full long queue refuses only long ones
            for c in (False, True):
                idx = sub + np.nonzero(lng[sub:k] == c)[0]
                if len(idx):
                    st, tk = srv.submit(reqs[idx])
                    accepted[idx[:len(tk)]] = True
                    nacc += len(tk)
            sub = k   # the refused rest of this arrival group is dropped
        out = srv.poll(65536, timeout_us=200)
        if len(out):
            tags = out["tag"].astype(np.int64)
            done_ns[tags] = out["t_done_ns"]
            bsize[tags] = out["batch_size"]
            got += len(out)
            if (out["status"] != 0).any():
                raise RuntimeError("serving request failed")
    stats = srv.stats()
    srv.close()
    if got < nacc or sub < n:
        raise RuntimeError(f"serving phase did not finish: {got}/{nacc}")
    meas = (t_arr >= warmup) & accepted
    offered = t_arr >= warmup
    lat_ms = (done_ns - arr_ns) / 1e6

    def pct(mask):
        if not mask.any():
            return None
        return {"p50_ms": round(float(np.percentile(lat_ms[mask], 50)), 3),
                "p99_ms": round(float(np.percentile(lat_ms[mask], 99)), 3),
                "n": int(mask.sum())}
    wall = (done_ns[meas].max() - arr_ns[offered].min()) / 1e9 if meas.any() else float("nan")
    return {"offered_per_s": rate, "seconds": seconds, "warmup_s": warmup,
            "requests_offered": int(offered.sum()), "requests_admitted": int(meas.sum()),
            "refused_queue_full": int((offered & ~accepted).sum()),
            "offered_gcups": round(float(cells.mean()) * rate / 1e9, 1),
            "sustained_gcups": round(float(cells[meas].sum()) / wall / 1e9, 1),
            "latency_all": pct(meas), "latency_short": pct(meas & ~lng),
            "latency_long": pct(meas & lng),
            "batches": stats["batches"], "max_batch": stats["max_batch_seen"],
            "mean_batch": round(float(bsize[meas].mean()), 1) if meas.any() else None,
            "workers": workers, "mem_budget_gib": mem_budget / 2**30,
            "max_pending": max_pending,
            "graph_batch": graph_batch, "graph_batches": stats["graph_batches"],
            "pool": f"{pool_short} short + {pool_long} long requests"}


def all_vs_all_phase(ctx, n_reads=4000, reps=3):
    """Every pair of n_reads overlapping 70-nt reads of one 1.5-kb region
    (n(n-1)/2 pairs), inputs and outputs device-resident, every output."""
    import numpy as np
    import torch

    import paper_1208_6350_amd as swx
    import workloads as W
    b = W.all_vs_all(n_reads=n_reads)
    dev = torch.device("cuda:0")
    to = lambda x: torch.as_tensor(np.ascontiguousarray(x)).to(dev)
    dq, dqo, dpq, dpr = to(b.qcat), to(b.qoff), to(b.pair_q), to(b.pair_r)
    recs = torch.empty(b.npairs * swx.REC_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    cig = torch.empty(int(b.qlen().sum() + b.rlen().sum() + b.npairs), dtype=torch.int32,
                      device=dev)
    ts = []
    for k in range(reps + 1):
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, _ = swx.swx_align_batch(ctx.handle, b.matrix, b.gap_open, b.gap_extend, dq, dqo, dq,
                                    dqo, dpq, dpr, swx.SWX_ALL, -1, swx.SWX_MEM_DEVICE, recs, cig,
                                    swx.SWX_MEM_DEVICE)
        torch.cuda.synchronize()
        if st != 0:
            raise swx.SwxError(st, "swx_align_batch")
        if k:
            ts.append(time.perf_counter() - t)
    best = min(ts)
    return {"reads": n_reads, "read_len": 70, "pairs": b.npairs, "cells": b.cells(),
            "ms": round(best * 1e3, 3), "gcups": round(b.cells() / best / 1e9, 1),
            "pairs_per_s": round(b.npairs / best, 0)}


def all_vs_all_large_phase(ctx, n_reads=20000, chunk_pairs=20_000_000, check_pairs=20000,
                           with_oracle=True):
    """The all-vs-all overlap at read-overlap-graph scale (n_reads reads, every
    pair i < j: about 2e8 pairs) through the sliced batch calls
    (Context.align_batch_chunks), inputs device-resident, every output; each
    slice's outputs are dropped once its call returns (the CIGAR arena of all
    pairs at once would not fit).  The oracle checks the first check_pairs
    pairs of the first slice."""
    import numpy as np
    import torch

    import paper_1208_6350_amd as swx
    import workloads as W
    t = time.perf_counter()
    b = W.all_vs_all(n_reads=n_reads)
    gen_s = time.perf_counter() - t
    dev = torch.device("cuda:0")
    to = lambda x: torch.as_tensor(np.ascontiguousarray(x)).to(dev)
    dq, dqo, dpq, dpr = to(b.qcat), to(b.qoff), to(b.pair_q), to(b.pair_r)
    args = (b.matrix, b.gap_open, b.gap_extend, dq, dqo, dq, dqo)
    # warm-up: one small slice
    for _ in ctx.align_batch_chunks(*args, dpq[:100_000], dpr[:100_000], chunk_pairs=100_000):
        pass
    torch.cuda.synchronize()
    first = None
    t = time.perf_counter()
    nslices = 0
    for k0, k1, recs, cig in ctx.align_batch_chunks(*args, dpq, dpr, chunk_pairs=chunk_pairs):
        nslices += 1
        if first is None:
            n = min(check_pairs, k1 - k0)
            first = (recs[:n * swx.REC_DTYPE.itemsize].cpu().numpy().view(swx.REC_DTYPE).copy(),
                     cig.cpu().numpy().view(np.uint32).copy(), n)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    out = {"reads": n_reads, "read_len": 70, "pairs": b.npairs, "cells": b.cells(),
           "slices": nslices, "slice_pairs": chunk_pairs, "ms": round(dt * 1e3, 1),
           "gcups": round(b.cells() / dt / 1e9, 1), "pairs_per_s": round(b.npairs / dt, 0),
           "generate_s": round(gen_s, 1)}
    if with_oracle:   # the oracle beside the timed run, as for cpu_baseline
        import oracle
        from tests.fullsize import mismatches
        recs, cig, n = first
        s = b.subset(np.arange(n))
        ref, rcig, rcoff = oracle.align_many(s.qcat, s.qoff, s.rcat, s.roff, s.pair_q, s.pair_r,
                                             s.matrix, s.gap_open, s.gap_extend,
                                             nthreads=os.cpu_count() or 1)
        out["parity"] = {"pairs": n, "mismatches": mismatches(recs, cig, ref, rcig,
                                                              rcoff)["pairs_bad"]}
    return out


def graph_phase(ctx, batch=512, reps=20):
    """Median time of one batch of `batch` short pairs (150-nt reads vs 1-kb
    windows) through swx_align_batch and through a replayed graph of the same
    capacity; inputs are reloaded into the graph each time."""
    import numpy as np

    import paper_1208_6350_amd as swx
    import workloads as W
    pool = W.config5_pool(n_short=batch, n_long=1)
    b = pool.subset(np.arange(batch))
    graphs = {name: swx.Graph(ctx, b.matrix, b.gap_open, b.gap_extend, max_pairs=batch,
                              max_qlen=200, max_rlen=1100, qcat_cap=batch * 200,
                              rcat_cap=batch * 1100 + 8, nq_cap=batch + 1, nr_cap=batch + 2,
                              route=route)
              for name, route in (("graph_batched", 0), ("graph_intra", 1))}
    times = {"call": [], "graph_batched": [], "graph_intra": []}
    try:
        for k in range(reps):
            t = time.perf_counter()
            ctx.align_batch(b.matrix, b.gap_open, b.gap_extend, b.qcat, b.qoff, b.rcat, b.roff,
                            b.pair_q, b.pair_r)
            times["call"].append(time.perf_counter() - t)
            for name, g in graphs.items():
                t = time.perf_counter()
                g.load(b.qcat, b.qoff, b.rcat, b.roff, b.pair_q, b.pair_r)
                g.run()
                g.read()
                times[name].append(time.perf_counter() - t)
    finally:
        for g in graphs.values():
            g.close()
    out = {"pairs": batch, "note": "host inputs and outputs, copies included, median of %d" % reps}
    for name, ts in times.items():
        m = float(np.median(ts)) * 1e3
        out[name] = {"ms": round(m, 3), "gcups": round(b.cells() / m / 1e6, 2)}
    return out


PEAK_U32_TOPS = 256 * 64 * 2.4e9 / 1e12   # 32-bit lanes: one operation per lane-op


def _dev_call(ctx, b, reps):
    """Best and median of `reps` timed calls (after one untimed) of the whole
    path on b with device-resident inputs and outputs; returns the times, the
    library's per-stage times of the best call and the outputs of the last."""
    import numpy as np
    import torch

    import paper_1208_6350_amd as swx
    dev = torch.device("cuda:0")
    to = lambda x: torch.as_tensor(np.ascontiguousarray(x)).to(dev)
    dq, dqo, dr, dro, dpq, dpr = (to(b.qcat), to(b.qoff), to(b.rcat), to(b.roff), to(b.pair_q),
                                  to(b.pair_r))
    recs = torch.empty(b.npairs * swx.REC_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    cig = torch.empty(int(b.qlen().sum() + b.rlen().sum() + b.npairs), dtype=torch.int32,
                      device=dev)
    ts, stages, used = [], None, 0
    for k in range(reps + 1):
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, used = swx.swx_align_batch(ctx.handle, b.matrix, b.gap_open, b.gap_extend, dq, dqo,
                                       dr, dro, dpq, dpr, swx.SWX_ALL, -1, swx.SWX_MEM_DEVICE,
                                       recs, cig, swx.SWX_MEM_DEVICE)
        torch.cuda.synchronize()
        if st != 0:
            raise swx.SwxError(st, "swx_align_batch")
        if k:
            ts.append(time.perf_counter() - t)
            if ts[-1] == min(ts):
                stages = ctx.stage_ms()
    out = (recs.cpu().numpy().view(swx.REC_DTYPE).copy(),
           cig[:used].cpu().numpy().view(np.uint32).copy())
    return ts, stages, out


def _entry(name, workload, b, ts, stages, recs, oracle_t, parity):
    """One per-configuration record: whole-path time and rate, the forward
    fill against the integer-VALU peak of the lanes it ran on, the oracle's
    time beside it and the parity of the GPU outputs."""
    import numpy as np
    best = min(ts)
    cells = b.cells()
    bits = sorted(set(int(x) for x in recs["lane_bits"]))
    # the roofline of the lanes each pair ran on: packed 16-bit lanes at the
    # packed peak, 32-bit lanes (saturated re-runs, wide long pairs) at half
    pc = (b.qlen()[b.pair_q].astype(np.float64) * b.rlen()[b.pair_r])
    w16 = recs["lane_bits"] == 16
    c16, c32 = float(pc[w16].sum()), float(pc[~w16].sum())
    ideal_s = (c16 / PEAK_PK16_TOPS + c32 / PEAK_U32_TOPS) * OPS_PER_CELL / 1e12
    fill = stages[1]
    names = ["prepare", "fill", "rerun32", "reverse", "traceback", "score2", "records"]
    return {"workload": workload, "pairs": b.npairs, "cells": cells,
            "ms": round(best * 1e3, 3), "median_ms": round(float(np.median(ts)) * 1e3, 3),
            "gcups": round(cells / best / 1e9, 2), "lane_bits": bits,
            "stages_ms": {n: round(v, 3) for n, v in zip(names, stages)},
            "roofline": {"bound": "alu", "unit": "Tops/s",
                         "peak_16": round(PEAK_PK16_TOPS, 2), "peak_32": round(PEAK_U32_TOPS, 2),
                         "cells_16": c16, "cells_32": c32,
                         "ideal_fill_ms": round(ideal_s * 1e3, 4),
                         "fill_frac": round(ideal_s / (fill * 1e-3), 4),
                         "path_frac": round(ideal_s / best, 4)},
            "oracle": oracle_t, "parity": parity}


def config_phase(ctx, reps=3, with_oracle=True, only=None):
    """The other workloads, each timed alone through the same entry point:
    the single short pair (also one call per pair through swx_align), the
    single long-reference pair, the protein one-against-many search at full
    size and one long serving request.  Beside each, the oracle's time on a
    bounded sample of it and the parity of the GPU result (against the
    oracle's, or for the long-reference pair its stored result)."""
    import numpy as np

    import workloads as W
    if with_oracle:
        import oracle
        from tests.fullsize import mismatches
    threads = os.cpu_count() or 1
    out = {}

    def oracle_pairs(b, n):
        s = b.subset(np.arange(n))
        t = time.perf_counter()
        ref, rcig, rcoff = oracle.align_many(s.qcat, s.qoff, s.rcat, s.roff, s.pair_q, s.pair_r,
                                             s.matrix, s.gap_open, s.gap_extend,
                                             nthreads=threads)
        dt = time.perf_counter() - t
        return s, dt, (ref, rcig, rcoff)

    def check(recs, cig, n, res):
        bad = mismatches(recs[:n], cig, *res)
        return {"pairs": n, "mismatches": bad["pairs_bad"]}

    # single short pair: batch entry point, and per call through swx_align
    if only in (None, "c1"):
        _config1(ctx, reps, with_oracle, out, oracle_pairs, check)
    if only in (None, "c2"):
        _config2(ctx, reps, with_oracle, out)
    if only in (None, "c3"):
        _config3(ctx, reps, with_oracle, out, oracle_pairs, check, threads)
    if only in (None, "c5_long"):
        _config5(ctx, reps, with_oracle, out, oracle_pairs, check)
    return out


def _config1(ctx, reps, with_oracle, out, oracle_pairs, check):
    import numpy as np

    import workloads as W
    b = W.config1()
    ts, st, (recs, cig) = _dev_call(ctx, b, reps * 10)
    orc = par = None
    if with_oracle:
        s, dt, res = oracle_pairs(b, 1)
        orc = {"seconds": round(dt, 4), "gcups": round(b.cells() / dt / 1e9, 4), "cores": 1,
               "sample": "the whole pair"}
        par = check(recs, cig, 1, res)
    e = _entry("c1", "one DNA pair: 150-nt read vs 2,000-nt window", b, ts, st, recs, orc, par)
    q, r = b.query(0), b.ref(0)
    for k in range(3):
        ctx.align_pair(q, r, b.matrix, b.gap_open, b.gap_extend)
    pt = []
    for k in range(50):
        t = time.perf_counter()
        ctx.align_pair(q, r, b.matrix, b.gap_open, b.gap_extend)
        pt.append(time.perf_counter() - t)
    e["per_call"] = {"entry": "swx_align (host buffers, copies included)",
                     "median_ms": round(float(np.median(pt)) * 1e3, 3),
                     "min_ms": round(min(pt) * 1e3, 3)}
    out["c1"] = e


def _config2(ctx, reps, with_oracle, out):
    """The single long-reference pair, checked against the oracle's stored
    result."""
    import numpy as np

    import workloads as W
    if with_oracle:
        import oracle
    b = W.config2()
    ts, st, (recs, cig) = _dev_call(ctx, b, reps)
    orc = par = None
    if with_oracle:
        cols = 200_000
        s = b.subset(np.arange(1))
        t = time.perf_counter()
        oracle.align(s.query(0), s.ref(0)[:cols], s.matrix, s.gap_open, s.gap_extend)
        dt = time.perf_counter() - t
        orc = {"seconds": round(dt, 3), "gcups": round(1000 * cols / dt / 1e9, 4), "cores": 1,
               "sample": f"the read against the first {cols} reference columns"}
        with open(os.path.join(ROOT, "tests", "golden", "config2.json")) as f:
            gold = json.load(f)
        fields = ["score1", "score2", "read_begin1", "read_end1", "ref_begin1", "ref_end1",
                  "ref_end2"]
        got = {k: int(recs[k][0]) for k in fields}
        ops = "MIDNSHP=X"
        words = [(int(w) >> 4, ops[int(w) & 15]) for w in
                 cig[int(recs["cigar_off"][0]):int(recs["cigar_off"][0]) +
                     int(recs["cigar_len"][0])]]
        same = all(got[k] == gold[k] for k in fields) and \
            words == [(int(n), op) for n, op in gold["cigar"]]
        par = {"pairs": 1, "mismatches": 0 if same else 1,
               "checked": "every field and the CIGAR against the oracle's stored result"}
    out["c2"] = _entry("c2", "one 1,000-nt read vs a 5,000,000-nt reference", b, ts, st, recs,
                       orc, par)


def _config3(ctx, reps, with_oracle, out, oracle_pairs, check, threads):
    """The protein one-against-many search at full size."""
    import workloads as W
    b = W.config3()
    ts, st, (recs, cig) = _dev_call(ctx, b, reps)
    orc = par = None
    if with_oracle:
        n = 20_000
        s, dt, res = oracle_pairs(b, n)
        orc = {"seconds": round(dt, 3), "gcups": round(s.cells() / dt / 1e9, 4),
               "cores": threads, "sample": f"the first {n} targets"}
        par = check(recs, cig, n, res)
    out["c3"] = _entry("c3", "protein search: 300-aa query vs 100,000 targets (50-5,000 aa)",
                       b, ts, st, recs, orc, par)


def _config5(ctx, reps, with_oracle, out, oracle_pairs, check):
    """One long serving request alone."""
    import numpy as np

    import workloads as W
    pool = W.config5_pool(n_short=1, n_long=1)
    b = pool.subset(np.arange(1, 2))
    ts, st, (recs, cig) = _dev_call(ctx, b, reps)
    orc = par = None
    if with_oracle:
        s, dt, res = oracle_pairs(b, 1)
        orc = {"seconds": round(dt, 3), "gcups": round(b.cells() / dt / 1e9, 4), "cores": 1,
               "sample": "the whole pair"}
        par = check(recs, cig, 1, res)
    out["c5_long"] = _entry("c5_long", "one long serving request: 10,000-nt read vs "
                            "20,000-nt window, 10% error", b, ts, st, recs, orc, par)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is "
                                   "described in DESIGN.md but not built", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1208_6350_amd as swx
    import workloads as W

    if args.only_config:
        cctx = swx.Context(0)
        try:
            out = config_phase(cctx, with_oracle=not args.no_cpu, only=args.only_config)
        finally:
            cctx.close()
        print(json.dumps(out), flush=True)
        return
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    b = W.config4(npairs=args.pairs)
    print(f"[bench] generated {b.npairs} pairs in {time.perf_counter() - t0:.1f}s", flush=True,
          file=sys.stderr)
    cells = b.cells()
    to = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to(dev)
    dq, dqo, dr, dro = to(b.qcat, None), to(b.qoff, None), to(b.rcat, None), to(b.roff, None)
    dpq, dpr = to(b.pair_q, None), to(b.pair_r, None)
    recs = torch.empty(b.npairs * swx.REC_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    cap = int(b.qlen().sum() + b.rlen().sum() + b.npairs)
    cig = torch.empty(cap, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: {nbytes} bytes read and written", flush=True, file=sys.stderr)
        del src, dst
    ctx = swx.Context(0)
    tuning = None
    if not args.no_autotune and not args.headline_only:
        t = time.perf_counter()
        tuning, _ = ctx.autotune(b.matrix, b.gap_open, b.gap_extend, dq, dqo, dr, dro, dpq, dpr,
                                 max_pairs=100_000, in_mem=swx.SWX_MEM_DEVICE)
        print(f"[bench] autotuned in {time.perf_counter() - t:.1f}s: {tuning}", flush=True,
              file=sys.stderr)

    def step():
        st, used = swx.swx_align_batch(ctx.handle, b.matrix, b.gap_open, b.gap_extend, dq, dqo,
                                       dr, dro, dpq, dpr, swx.SWX_ALL, -1, swx.SWX_MEM_DEVICE,
                                       recs, cig, swx.SWX_MEM_DEVICE)
        if st != 0:
            raise swx.SwxError(st, "swx_align_batch")
        return used

    for k in range(args.warmup):
        step()
        print(f"[bench] warmup {k + 1}/{args.warmup} done", flush=True, file=sys.stderr)
    torch.cuda.synchronize()
    fill_ms = []
    stages = None
    t0 = time.perf_counter()
    step_used = []
    for k in range(args.steps):
        step_used.append(step())
        st_ms = ctx.stage_ms()
        fill_ms.append(st_ms[1])
        stages = st_ms if stages is None else [a + c for a, c in zip(stages, st_ms)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] {args.steps} timed steps in {dt:.3f}s", flush=True, file=sys.stderr)
    # the last timed step's outputs, kept for the parity check (later phases
    # reuse the buffers)
    last_used = step_used[-1]
    gpu_out = (recs.cpu().numpy().view(swx.REC_DTYPE).copy(),
               cig[:last_used].cpu().numpy().view(np.uint32).copy())
    ms_per_step = dt * 1e3 / args.steps
    value = cells * args.steps / dt / 1e9
    fill_avg = sum(fill_ms) / len(fill_ms)
    achieved = cells * OPS_PER_CELL / (fill_avg * 1e-3) / 1e12
    names = ["prepare", "fill", "rerun32", "reverse", "traceback", "score2", "records"]
    stage_avg = {n: round(v / args.steps, 3) for n, v in zip(names, stages)}

    # the paper's output modes side by side (its own comparison: score only,
    # score with begin/end, full alignment with CIGAR and score2)
    modes = {}
    for name, fl in () if args.headline_only else (
            ("score_end", 0), ("begin_end", swx.SWX_BEGIN), ("full", swx.SWX_ALL)):
        ts = []
        for k in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st, _ = swx.swx_align_batch(ctx.handle, b.matrix, b.gap_open, b.gap_extend, dq, dqo, dr,
                                        dro, dpq, dpr, fl, -1, swx.SWX_MEM_DEVICE, recs, cig,
                                        swx.SWX_MEM_DEVICE)
            torch.cuda.synchronize()
            if st != 0:
                raise swx.SwxError(st, "swx_align_batch")
            ts.append(time.perf_counter() - t)
        best = min(ts[1:])
        modes[name] = {"ms": round(best * 1e3, 3), "gcups": round(cells / best / 1e9, 1)}

    # the alignment behind score2 as well (the suboptimal alignment's passes
    # on top of the full output)
    if not args.headline_only:
        sub = torch.empty(b.npairs * swx.REC_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        cig2 = torch.empty(2 * cap, dtype=torch.int32, device=dev)
        ts = []
        for k in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st, _ = swx.swx_align_batch(ctx.handle, b.matrix, b.gap_open, b.gap_extend, dq, dqo, dr,
                                        dro, dpq, dpr, swx.SWX_ALL | swx.SWX_SUBOPT, -1,
                                        swx.SWX_MEM_DEVICE, recs, cig2, swx.SWX_MEM_DEVICE, sub)
            torch.cuda.synchronize()
            if st != 0:
                raise swx.SwxError(st, "swx_align_batch")
            ts.append(time.perf_counter() - t)
        best = min(ts[1:])
        modes["full_subopt"] = {"ms": round(best * 1e3, 3), "gcups": round(cells / best / 1e9, 1)}
        del sub, cig2

    # the recurrence's cell rate at 8-bit (SWAR) and packed 16-bit lane widths
    lanes = None
    if not args.headline_only:
        lanes = {}
        res = {}
        for bits in (16, 8):
            ctx.lane_probe(bits, columns=256, blocks=256)   # warm-up
            best, ms, gcups = ctx.lane_probe(bits, columns=4096, blocks=2048)
            res[bits] = best
            lanes[f"w{bits}"] = {"ms": round(ms, 3), "gcups": round(gcups, 1)}
        lanes["same_scores"] = bool(np.array_equal(res[8][:len(res[16])], res[16]))
        lanes["note"] = ("synthetic 16-row DNA pairs x 4096 columns, recurrence + column max; "
                         "8-bit = four SWAR byte lanes per register")

    # graph mode against the ordinary call on small batches of short pairs
    # (serving-sized: where per-call planning and launches dominate)
    graph_cmp = None if args.headline_only else graph_phase(ctx)
    configs = None
    if not args.headline_only and not args.no_configs:
        print("[bench] per-configuration phase", flush=True, file=sys.stderr)
        cctx = swx.Context(0)   # the library's default settings, not those tuned above
        try:
            configs = config_phase(cctx, with_oracle=not args.no_cpu)
        finally:
            cctx.close()
    avsa = None if args.headline_only else all_vs_all_phase(ctx)
    avsa_large = None
    if not args.headline_only and not args.no_large_avsa:
        print("[bench] all-vs-all at scale", flush=True, file=sys.stderr)
        avsa_large = all_vs_all_large_phase(ctx, with_oracle=not args.no_cpu)

    # per-pair form: the same library, one pair per call
    per_pair = None
    if args.per_pair_sample > 0 and not args.headline_only:
        pp = b.subset(np.arange(min(args.per_pair_sample, b.npairs)))
        # one untimed pass: the first call of each size class captures its graph
        for p in range(pp.npairs):
            ctx.align_pair(pp.query(p), pp.ref(p), pp.matrix, pp.gap_open, pp.gap_extend)
        t = time.perf_counter()
        for p in range(pp.npairs):
            ctx.align_pair(pp.query(p), pp.ref(p), pp.matrix, pp.gap_open, pp.gap_extend)
        pdt = time.perf_counter() - t
        per_pair = {"value": round(pp.cells() / pdt / 1e9, 4), "unit": "GCUPS",
                    "pairs": pp.npairs, "ms_per_pair": round(pdt * 1e3 / pp.npairs, 3)}
    ctx.close()

    line = {
        "metric": "GCUPS (fill+traceback) batched vs per-pair at 1 GPU",
        "value": round(value, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16",
        "data": "synthetic",
        "config": {"workload": f"batched uneven DNA: {b.npairs} read/window pairs, reads "
                               "100-250 nt, windows +0-400 nt, 1-3% subs, 0.5% indels, 10% "
                               "random reads; +2/-2, gap open 3, extend 1; score, score2, "
                               "begins, ends, CIGAR per pair",
                   "pairs": b.npairs, "cells": cells, "global_batch": b.npairs,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(PEAK_PK16_TOPS, 2), "unit": "Tops/s",
                     "frac": round(achieved / PEAK_PK16_TOPS, 4),
                     "traffic": recorded_traffic(b.npairs),
                     "valu_busy": (lambda v: float(v["valu_busy"]) if v else None)(
                         recorded_fields(VALU_FILE)),
                     "kernel": "k_inter_fill (forward fill, packed 16-bit lanes)",
                     "fill_ms": round(fill_avg, 3), "ops_per_cell": OPS_PER_CELL,
                     # the whole path (fill, saturation re-run, reverse, traceback,
                     # score2) against the same roofline: GCUPS x 10 ops / peak
                     "path_frac": round(value * OPS_PER_CELL / 1e3 / PEAK_PK16_TOPS, 4)},
        "stages_ms": stage_avg,
        "tuning": tuning,
        "modes": modes,
        "graph": graph_cmp,
        "lane_widths": lanes,
        "all_vs_all": avsa,
        "all_vs_all_large": avsa_large,
        "configs": configs,
        "per_pair": per_pair,
    }
    if not args.no_serve and not args.headline_only:
        print("[bench] serving phase", flush=True, file=sys.stderr)
        line["serving"] = [serving_phase(float(r), args.serve_seconds)
                           for r in str(args.serve_rate).split(",")]
    if not args.no_cpu and not args.headline_only:
        line["cpu_baseline"], line["parity"] = cpu_baseline(b, args.cpu_seconds, gpu_out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
