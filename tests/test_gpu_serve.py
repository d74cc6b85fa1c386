"""Continuous-batching server: queries admitted while others run, admission by
device-pool bytes, cancellation of waiting and running queries, idle exit and
relaunch, non-finite results, arrival-based latency, and each served result
equal to the query run alone."""
import os
import time

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import assert_rel, say, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2001_10635_amd")


def host_queries(queries):
    """Host arrays and reach_query structs (host pointers) for workload queries."""
    items = []
    for q in queries:
        p = q.problem
        lo, hi = p.box()
        pl, ph = p.inputs()
        r_lo = np.full(p.n, np.nan)
        r_hi = np.full(p.n, np.nan)
        rq = R.make_query(p.kind, p.n, p.prm, R.REACH_F64, lo.ctypes.data, hi.ctypes.data,
                          r_lo.ctypes.data, r_hi.ctypes.data, p.dt, p.nsteps,
                          None if pl is None else pl.ctypes.data,
                          None if ph is None else ph.ctypes.data, n_in=p.n_in)
        items.append(dict(p=p, lo=lo, hi=hi, pl=pl, ph=ph, r_lo=r_lo, r_hi=r_hi, q=rq))
    return items


def alone(rc, d):
    p = d["p"]
    dev = lambda a: None if a is None else to_dev(a)
    r_lo, r_hi = rc.embed(p.kind, p.prm, to_dev(d["lo"]), to_dev(d["hi"]), p.dt, p.nsteps,
                          p_lo=dev(d["pl"]), p_hi=dev(d["ph"]))
    assert rc.sync() == R.REACH_OK
    return to_host(r_lo), to_host(r_hi)


def drain(rc, tickets, timeout_s=120.0):
    status = {}
    t_end = time.time() + timeout_s
    pending = set(tickets)
    while pending and time.time() < t_end:
        for t in list(pending):
            st, res = R.reach_poll(rc.ctx, t)
            if st == R.REACH_OK:
                status[t] = res
                pending.discard(t)
        if pending:
            time.sleep(0.0005)
    assert not pending, f"{len(pending)} queries did not finish"
    return status


@pytest.fixture
def rc():
    r = R.Reach(0)
    yield r
    r.close()


@pytest.mark.parametrize("mode", [0, 1], ids=["persistent", "launch_per_query"])
def test_served_results_equal_alone(rc, mode):
    items = host_queries(workloads.query_stream(600, 5.0e4, seed=99))
    rc.set_option("serve.mode", mode)
    pool = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    say(f"serve mode {mode}")
    R.reach_server_start(rc.ctx, pool, pool.numel(), 256)
    try:
        tickets = []
        for k, d in enumerate(items):
            tickets.append(R.reach_submit(rc.ctx, d["q"]))
            if k % 50 == 0:
                time.sleep(0.001)      # arrivals while earlier queries run
        status = drain(rc, tickets)
        stats = R.reach_server_stats(rc.ctx)
    finally:
        R.reach_server_stop(rc.ctx)
    assert all(s == R.REACH_OK for s in status.values())
    assert stats["completed"] == len(items) and stats["p99_us"] >= stats["p50_us"] > 0
    for k, d in enumerate(items):
        a = alone(rc, d)
        assert np.array_equal(d["r_lo"], a[0]) and np.array_equal(d["r_hi"], a[1]), f"query {k}"
    for k in range(0, len(items), 37):
        d = items[k]
        p = d["p"]
        o_lo, o_hi = oracle.embed_rk4(p.kind, p.prm, d["lo"], d["hi"], d["pl"], d["ph"], dt=p.dt,
                                      nsteps=p.nsteps)
        assert_rel(d["r_lo"], o_lo, 1e-12, f"query {k} lower")
        assert_rel(d["r_hi"], o_hi, 1e-12, f"query {k} upper")


def test_admission_limited_by_pool_bytes(rc):
    """A pool that holds two 512-cell boxes at a time still serves everything."""
    qs = [q for q in workloads.query_stream(400, 5.0e4, seed=7) if q.problem.n > 200][:40]
    items = host_queries(qs)
    footprint = (8 * (2 * 512 + 2) + 255) // 256 * 256     # x_lo, x_hi, u_lo, u_hi
    pool = torch.empty(2 * footprint, dtype=torch.uint8, device="cuda")
    R.reach_server_start(rc.ctx, pool, pool.numel(), 64)
    try:
        big = workloads.small_problem(workloads.KIND_CTM, 512, 1, 10)
        huge = host_queries([workloads.Query(0, 0.0, big)])[0]
        tiny_pool_q = huge["q"]
        tickets = [R.reach_submit(rc.ctx, d["q"]) for d in items]
        status = drain(rc, tickets)
    finally:
        R.reach_server_stop(rc.ctx)
    assert all(s == R.REACH_OK for s in status.values())
    for d in items:
        a = alone(rc, d)
        assert np.array_equal(d["r_lo"], a[0]) and np.array_equal(d["r_hi"], a[1])
    # a query bigger than the whole pool can never be admitted
    pool2 = torch.empty(1024, dtype=torch.uint8, device="cuda")
    R.reach_server_start(rc.ctx, pool2, pool2.numel(), 4)
    try:
        with pytest.raises(R.ReachError) as e:
            R.reach_submit(rc.ctx, tiny_pool_q)
        assert e.value.status == R.REACH_E_NOMEM
    finally:
        R.reach_server_stop(rc.ctx)


def test_cancel_pending_queries(rc):
    items = host_queries(workloads.query_stream(300, 5.0e4, seed=5))
    pool = torch.empty(8 << 20, dtype=torch.uint8, device="cuda")
    R.reach_server_start(rc.ctx, pool, pool.numel(), 2)     # 2 slots: most queries wait
    try:
        tickets = [R.reach_submit(rc.ctx, d["q"]) for d in items]
        cancelled = [t for t in tickets[150:] if R.reach_cancel(rc.ctx, t) == R.REACH_OK]
        status = drain(rc, tickets)
    finally:
        R.reach_server_stop(rc.ctx)
    assert len(cancelled) > 0
    for t in cancelled:
        assert status[t] == R.REACH_E_CANCELLED
    done = [t for t in tickets if status[t] == R.REACH_OK]
    assert len(done) + len(cancelled) == len(tickets)
    for k, t in enumerate(tickets):
        if status[t] == R.REACH_OK and k % 10 == 0:
            a = alone(rc, items[k])
            assert np.array_equal(items[k]["r_lo"], a[0])


@pytest.mark.parametrize("mode", [0, 1], ids=["persistent", "launch_per_query"])
def test_cancel_at_submission_does_not_hold_up_later_queries(rc, mode):
    """Every other query is cancelled the moment it is submitted, while all of
    them have slots (each is admitted at once and so already owns a ring
    sequence): the cancelled ones report REACH_E_CANCELLED (or REACH_OK when
    they finished first) and every other query completes and equals its alone
    run, so no cancelled sequence holds up those after it."""
    rc.set_option("serve.mode", mode)
    items = host_queries(workloads.query_stream(200, 5.0e4, seed=77))
    pool = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    say(f"serve cancel at submission, mode {mode}")
    R.reach_server_start(rc.ctx, pool, pool.numel(), 256)
    try:
        tickets = []
        for k, d in enumerate(items):
            t = R.reach_submit(rc.ctx, d["q"])
            tickets.append(t)
            if k % 2:
                assert R.reach_cancel(rc.ctx, t) in (R.REACH_OK, R.REACH_E_BUSY)
        status = drain(rc, tickets, timeout_s=60.0)
    finally:
        R.reach_server_stop(rc.ctx)
    for k, t in enumerate(tickets):
        if k % 2:
            assert status[t] in (R.REACH_E_CANCELLED, R.REACH_OK)
        else:
            assert status[t] == R.REACH_OK
            a = alone(rc, items[k])
            assert np.array_equal(items[k]["r_lo"], a[0])
            assert np.array_equal(items[k]["r_hi"], a[1])


def long_query(kind, n, nsteps, seed):
    p = workloads.small_problem(kind, n, seed, nsteps)
    return host_queries([workloads.Query(0, 0.0, p)])[0]


@pytest.mark.parametrize("mode", [0, 1], ids=["persistent", "launch_per_query"])
def test_cancel_running_queries(rc, mode):
    """Queries of 2e6 RK4 steps (about a second each) are cancelled while they
    run: each stops within a few milliseconds and reports REACH_E_CANCELLED,
    and the short queries served beside them still equal their alone runs."""
    rc.set_option("serve.mode", mode)
    longs = [long_query(workloads.KIND_RD if k % 2 else workloads.KIND_CTM, 40 + 30 * k,
                        2_000_000, 50 + k) for k in range(4)]
    items = host_queries(workloads.query_stream(80, 5.0e4, seed=21))
    pool = torch.empty(16 << 20, dtype=torch.uint8, device="cuda")
    say(f"serve cancel running, mode {mode}")
    R.reach_server_start(rc.ctx, pool, pool.numel(), 64)
    try:
        lt = [R.reach_submit(rc.ctx, d["q"]) for d in longs]
        st = [R.reach_submit(rc.ctx, d["q"]) for d in items]
        time.sleep(0.05)                   # the long queries are well under way
        t_cancel = time.perf_counter()
        assert all(R.reach_cancel(rc.ctx, t) == R.REACH_OK for t in lt)
        lstatus = drain(rc, lt, timeout_s=30.0)
        waited = time.perf_counter() - t_cancel
        status = drain(rc, st)
    finally:
        R.reach_server_stop(rc.ctx)
    assert all(lstatus[t] == R.REACH_E_CANCELLED for t in lt), lstatus
    say(f"cancelled running queries finished {waited * 1e3:.1f} ms after the request")
    assert waited < 0.3
    for d in longs:                        # no box is written for a cancelled query
        assert np.all(np.isnan(d["r_lo"])) and np.all(np.isnan(d["r_hi"]))
    assert all(v == R.REACH_OK for v in status.values())
    for d in items:
        a = alone(rc, d)
        assert np.array_equal(d["r_lo"], a[0]) and np.array_equal(d["r_hi"], a[1])


@pytest.mark.parametrize("mode", [0, 1], ids=["persistent", "launch_per_query"])
def test_served_nonfinite_reported(rc, mode):
    """A reaction-diffusion query that overflows is reported REACH_E_NONFINITE
    in both serving modes; a finite query served with it is REACH_OK."""
    rc.set_option("serve.mode", mode)
    bad = long_query(workloads.KIND_RD, 70, 40, 3)
    bad["lo"][:] = 1e100
    bad["hi"][:] = 2e100
    good = long_query(workloads.KIND_RD, 70, 40, 4)
    pool = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    say(f"serve non-finite, mode {mode}")
    R.reach_server_start(rc.ctx, pool, pool.numel(), 8)
    try:
        tb = R.reach_submit(rc.ctx, bad["q"])
        tg = R.reach_submit(rc.ctx, good["q"])
        status = drain(rc, [tb, tg])
    finally:
        R.reach_server_stop(rc.ctx)
    assert status[tb] == R.REACH_E_NONFINITE and status[tg] == R.REACH_OK
    a = alone(rc, good)
    assert np.array_equal(good["r_lo"], a[0]) and np.array_equal(good["r_hi"], a[1])
    assert rc.sync() == R.REACH_OK


def test_latency_counts_from_the_stated_arrival(rc):
    """reach_submit_at: a query stated to have arrived 50 ms before its submit
    call has a latency of at least 50 ms."""
    d = long_query(workloads.KIND_CTM, 30, 20, 5)
    pool = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    R.reach_server_start(rc.ctx, pool, pool.numel(), 4)
    try:
        t = R.reach_submit_at(rc.ctx, d["q"], R.reach_clock_us() - 50_000.0)
        drain(rc, [t])
        stats = R.reach_server_stats(rc.ctx)
        with pytest.raises(R.ReachError) as e:
            R.reach_submit_at(rc.ctx, d["q"], float("nan"))
        assert e.value.status == R.REACH_E_INVAL
    finally:
        R.reach_server_stop(rc.ctx)
    assert stats["completed"] == 1 and 50_000.0 <= stats["p50_us"] < 1_000_000.0


def test_idle_exit_of_part_of_the_grid_does_not_stall(rc, monkeypatch):
    """With a 1 s idle limit: a query at 0.9 s keeps two waves busy while the
    rest of the grid reaches its limit at 1 s; the whole grid leaves then, so a
    query at 1.2 s is served by a new grid at once instead of waiting for the
    last two waves to time out at 1.9 s."""
    monkeypatch.setenv("REACH_SERVER_IDLE_S", "1")
    items = host_queries(workloads.query_stream(2, 5.0e4, seed=17))
    pool = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    say("serve partial idle exit")
    t0 = time.perf_counter()
    R.reach_server_start(rc.ctx, pool, pool.numel(), 32)
    try:
        time.sleep(max(0.0, 0.9 - (time.perf_counter() - t0)))
        drain(rc, [R.reach_submit(rc.ctx, items[0]["q"])])
        time.sleep(max(0.0, 1.2 - (time.perf_counter() - t0)))
        t1 = time.perf_counter()
        drain(rc, [R.reach_submit(rc.ctx, items[1]["q"])])
        waited = time.perf_counter() - t1
    finally:
        R.reach_server_stop(rc.ctx)
    say(f"query after the partial idle exit took {waited * 1e3:.1f} ms")
    assert waited < 0.3
    a = alone(rc, items[1])
    assert np.array_equal(items[1]["r_lo"], a[0]) and np.array_equal(items[1]["r_hi"], a[1])


def test_idle_exit_and_relaunch(rc, monkeypatch):
    """With a 1 s idle limit every serving wave leaves; the server starts a new
    grid for the next arrivals and still returns the same boxes."""
    monkeypatch.setenv("REACH_SERVER_IDLE_S", "1")
    items = host_queries(workloads.query_stream(60, 5.0e4, seed=11))
    pool = torch.empty(8 << 20, dtype=torch.uint8, device="cuda")
    R.reach_server_start(rc.ctx, pool, pool.numel(), 32)
    try:
        first = [R.reach_submit(rc.ctx, d["q"]) for d in items[:30]]
        drain(rc, first)
        time.sleep(2.5)                          # the grid drains on its idle limit
        say("serve after idle exit")
        second = [R.reach_submit(rc.ctx, d["q"]) for d in items[30:]]
        status = drain(rc, second)
    finally:
        R.reach_server_stop(rc.ctx)
    assert all(s == R.REACH_OK for s in status.values())
    for d in items:
        a = alone(rc, d)
        assert np.array_equal(d["r_lo"], a[0]) and np.array_equal(d["r_hi"], a[1])


def test_stop_drains_everything(rc):
    items = host_queries(workloads.query_stream(200, 5.0e4, seed=13))
    pool = torch.empty(16 << 20, dtype=torch.uint8, device="cuda")
    R.reach_server_start(rc.ctx, pool, pool.numel(), 16)
    for d in items:
        R.reach_submit(rc.ctx, d["q"])
    R.reach_server_stop(rc.ctx)
    for d in items:
        assert np.all(np.isfinite(d["r_lo"])) and np.all(np.isfinite(d["r_hi"]))
    with pytest.raises(R.ReachError) as e:
        R.reach_submit(rc.ctx, items[0]["q"])
    assert e.value.status == R.REACH_E_BUSY
