"""CPU tests of the serving policy through its virtual-clock simulator
(swx_server_simulate): the schedule equals a plain restatement of the
documented policy, and the policy's guarantees (memory budget, the long
requests' share, the short-only worker, FIFO order per class, batch and
queue limits) hold on replayed arrival schedules.  No device is needed."""
from __future__ import annotations

import numpy as np
import pytest

import paper_1208_6350_amd as swx

SWX_EINVAL = -1


def _footprint(q, r, n):
    band = min(r, q + 64)
    return 64 * (q + r) + (n + 1) * q + q * band // 2 + 4096


def _policy_schedule(arr, ql, rl, *, cells_per_us, batch_us, request_us, n, mem_budget,
                     max_pending, workers, max_batch, long_cells):
    """The serving policy as the header states it, written out plainly."""
    mem_budget = mem_budget if mem_budget > 0 else 4 << 30
    max_pending = max_pending if max_pending > 0 else 1 << 20
    workers = min(workers if workers > 0 else 3, 16)
    max_batch = max_batch if max_batch > 0 else 1 << 16
    long_cells = long_cells if long_cells > 0 else 1 << 22
    N = len(arr)
    fp = [_footprint(int(ql[k]), int(rl[k]), n) for k in range(N)]
    cls = [1 if int(ql[k]) * int(rl[k]) > long_cells else 0 for k in range(N)]
    res = [dict(start=-1.0, done=-1.0, batch=-1, worker=-1, size=0, status=0) for _ in range(N)]
    pending = [[], []]
    inflight, inflight_long = 0, 0
    busy = [None] * workers          # (done time, class, bytes, members)
    nb = 0

    def admissible(f, c, extra):
        if inflight == 0 and extra == 0:
            return True
        if inflight + extra + f > mem_budget:
            return False
        return c == 0 or inflight_long + extra + f <= mem_budget // 4 * 3

    def dispatch(t):
        nonlocal inflight, inflight_long, nb
        for w in range(workers):
            if busy[w] is not None:
                continue
            order = [0] if (w == 0 and workers > 1) else [1, 0]
            # a long head above the long share waits for an idle device, and
            # no short batch starts meanwhile
            drain = bool(pending[1]) and fp[pending[1][0]] > mem_budget // 4 * 3
            c = next((k for k in order if pending[k] and not (k == 0 and drain)
                      and admissible(fp[pending[k][0]], k, 0)), -1)
            if c < 0:
                continue
            members, extra = [], 0
            while pending[c] and len(members) < max_batch and admissible(fp[pending[c][0]], c, extra):
                extra += fp[pending[c][0]]
                members.append(pending[c].pop(0))
            inflight += extra
            if c == 1:
                inflight_long += extra
            cells = 0.0
            for k in members:
                cells += float(ql[k]) * float(rl[k])
            done = t + (batch_us + request_us * float(len(members)) + cells / cells_per_us)
            for k in members:
                res[k].update(start=t, done=done, batch=nb, worker=w, size=len(members))
            busy[w] = (done, c, extra, members)
            nb += 1

    a = 0
    while True:
        cand = [(busy[w][0], w) for w in range(workers) if busy[w] is not None]
        t_done, wd = min(cand) if cand else (np.inf, -1)
        t_arr = arr[a] if a < N else np.inf
        if wd < 0 and a >= N:
            break
        if wd >= 0 and t_done <= t_arr:
            _, c, extra, _ = busy[wd]
            inflight -= extra
            if c == 1:
                inflight_long -= extra
            busy[wd] = None
            t = t_done
        else:
            t = t_arr
            if len(pending[cls[a]]) >= max_pending:
                res[a]["status"] = swx.SWX_EBUSY
            else:
                pending[cls[a]].append(a)
            a += 1
        dispatch(t)
    return res, fp, cls


def _workload(seed, n=600, rate_per_us=0.02, long_frac=0.1):
    g = np.random.Generator(np.random.PCG64(seed))
    arr = np.cumsum(g.exponential(1.0 / rate_per_us, size=n))
    arr[g.random(n) < 0.1] = 0   # some bursts
    arr = np.maximum.accumulate(np.sort(arr))
    is_long = g.random(n) < long_frac
    ql = np.where(is_long, g.integers(5000, 10001, n), g.integers(50, 251, n))
    rl = np.where(is_long, g.integers(10000, 20001, n), g.integers(300, 1201, n))
    return arr, ql, rl


CASES = [
    dict(workers=3, mem_budget=0, max_pending=0, max_batch=0),
    dict(workers=1, mem_budget=0, max_pending=0, max_batch=16),
    dict(workers=4, mem_budget=200 << 20, max_pending=64, max_batch=32),
    dict(workers=2, mem_budget=20 << 20, max_pending=0, max_batch=0),
    dict(workers=3, mem_budget=1, max_pending=8, max_batch=0),   # everything runs alone
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_schedule_equals_policy_statement(case):
    arr, ql, rl = _workload(100 + case)
    kw = dict(cells_per_us=2e5, batch_us=50.0, request_us=0.5, n=4, long_cells=0, **CASES[case])
    out, st = swx.simulate_serving(arr, ql, rl, **kw)
    ref, fp, cls = _policy_schedule(arr, ql, rl, **kw)
    for k in range(len(arr)):
        r = ref[k]
        got = (out["start_us"][k], out["done_us"][k], out["batch_id"][k], out["worker"][k],
               out["batch_size"][k], out["status"][k], out["footprint"][k], out["cls"][k])
        exp = (r["start"], r["done"], r["batch"], r["worker"], r["size"], r["status"], fp[k], cls[k])
        assert got == exp, (case, k, got, exp)
    acc = int((out["status"] == 0).sum())
    assert st["submitted"] == acc and st["completed"] == acc and st["admitted"] == acc
    assert st["deferred"] == len(arr) - acc and st["pending"] == 0 and st["inflight_bytes"] == 0


def _intervals(out):
    ok = out["status"] == 0
    return [(float(out["start_us"][k]), float(out["done_us"][k]), k) for k in np.nonzero(ok)[0]]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_policy_guarantees(case):
    cfg = CASES[case]
    arr, ql, rl = _workload(200 + case, n=800, rate_per_us=0.05)
    out, st = swx.simulate_serving(arr, ql, rl, cells_per_us=2e5, batch_us=50.0, request_us=0.5,
                                   **cfg)
    budget = cfg["mem_budget"] or (4 << 30)
    ok = out["status"] == 0
    # every accepted request ran once, after it arrived
    assert (out["start_us"][ok] >= arr[ok]).all() and (out["done_us"][ok] > out["start_us"][ok]).all()
    # the budget, and the long requests' share, hold at every batch start
    # (unless a single request runs alone)
    for t, _, _ in _intervals(out):
        run = ok & (out["start_us"] <= t) & (out["done_us"] > t)
        tot = int(out["footprint"][run].sum())
        lng = int(out["footprint"][run & (out["cls"] == 1)].sum())
        assert tot <= budget or run.sum() == 1, (t, tot)
        assert lng <= budget // 4 * 3 or (run & (out["cls"] == 1)).sum() == 1, (t, lng)
    # worker 0 serves only short requests when there are other workers
    if cfg["workers"] > 1:
        assert (out["cls"][ok & (out["worker"] == 0)] == 0).all()
    # FIFO per class: batch order follows arrival order
    for c in (0, 1):
        ids = out["batch_id"][ok & (out["cls"] == c)]
        assert (np.diff(ids) >= 0).all()
    # batch size limit
    if cfg["max_batch"]:
        assert st["max_batch_seen"] <= cfg["max_batch"]
    if cfg["mem_budget"] == 1:
        assert (out["batch_size"][ok] == 1).all()


def test_pending_limit_on_a_burst():
    # one worker, everything arrives at once: the first request starts, then
    # max_pending wait, and the rest are refused
    n = 50
    out, st = swx.simulate_serving(np.zeros(n), [100] * n, [1000] * n, cells_per_us=1e5,
                                   workers=1, max_pending=7)
    assert int((out["status"] == 0).sum()) == 8 and st["deferred"] == n - 8
    assert (out["status"][8:] == swx.SWX_EBUSY).all()
    assert out["batch_size"][0] == 1 and (out["batch_size"][1:8] == 7).all()


def test_short_requests_do_not_wait_behind_long_ones():
    # long requests back to back keep workers 1.. busy; short ones keep
    # flowing through worker 0 with a wait below one short batch
    g = np.random.Generator(np.random.PCG64(7))
    n = 2000
    arr = np.sort(g.uniform(0, 2e5, size=n))
    is_long = g.random(n) < 0.3
    ql = np.where(is_long, 10000, 150)
    rl = np.where(is_long, 20000, 1000)
    out, _ = swx.simulate_serving(arr, ql, rl, cells_per_us=5e5, batch_us=100.0, workers=3)
    short = out["cls"] == 0
    wait = out["start_us"][short] - arr[short]
    dur = (out["done_us"] - out["start_us"])[short]
    assert wait.max() <= dur.max() + 1e-6
    assert (out["done_us"][~short] - arr[~short]).max() > 10 * wait.max()   # the long queue backs up


def test_simulator_rejects_bad_input():
    with pytest.raises(swx.SwxError) as ei:
        swx.simulate_serving([1.0, 0.5], [10, 10], [10, 10], cells_per_us=1.0)
    assert ei.value.status == SWX_EINVAL
    with pytest.raises(swx.SwxError) as ei:
        swx.simulate_serving([0.0], [10], [10], cells_per_us=0.0)
    assert ei.value.status == SWX_EINVAL
    with pytest.raises(swx.SwxError) as ei:
        swx.simulate_serving([0.0], [-1], [10], cells_per_us=1.0)
    assert ei.value.status == SWX_EINVAL


def test_long_request_above_its_share_runs_under_steady_short_traffic():
    # a long request whose footprint exceeds the long share (3/4 of the budget)
    # can only start on an idle device; short requests arrive faster than one
    # batch lasts, so without the drain rule the device would never be idle
    # before the arrivals stop
    budget = 64 << 20
    assert _footprint(10000, 20000, 4) > budget // 4 * 3
    n_short = 4000
    arr = list(np.arange(n_short) * 25.0)          # 0 .. 100 ms, one every 25 us
    ql, rl = [150] * n_short, [1000] * n_short
    arr.append(1000.0)
    ql.append(10000)
    rl.append(20000)
    order = np.argsort(arr, kind="stable")
    arr, ql, rl = np.asarray(arr)[order], np.asarray(ql)[order], np.asarray(rl)[order]
    out, _ = swx.simulate_serving(arr, ql, rl, cells_per_us=5e5, batch_us=100.0,
                                  mem_budget=budget, workers=3)
    assert (out["status"] == 0).all()
    k = int(np.nonzero(ql == 10000)[0][0])
    assert out["batch_size"][k] == 1
    # it starts within a few short batches of its arrival, long before the
    # short arrivals end
    assert out["start_us"][k] - arr[k] < 1000.0
    assert out["start_us"][k] < arr[-1] / 10
    # short requests keep being served after it starts
    later = (arr > out["start_us"][k]) & (ql == 150)
    assert (out["start_us"][later] < out["done_us"][k]).any()
