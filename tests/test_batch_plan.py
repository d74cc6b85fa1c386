"""The batch schedule (reach_plan_batch), computed on the host: no GPU.

Every query runs exactly once; packs hold 2..16 short cooperative queries with
identical constants and step counts within 1/16 octave in at most 64 lanes;
items come longest first; the plan is deterministic.  Results of packed
queries are compared with single runs bit for bit in the GPU batch tests."""
import math

import numpy as np
import pytest

import workloads

R = pytest.importorskip("paper_2001_10635_amd")

FAKE = 1 << 20     # device addresses are never dereferenced by the planner


def queries_of(stream):
    out = []
    for k, q in enumerate(stream):
        p = q.problem
        base = FAKE + 4096 * k
        out.append(R.make_query(p.kind, p.n, p.prm, R.REACH_F64, base, base + 8, base + 16,
                                base + 24, p.dt, p.nsteps, base + 32 if p.n_in else None,
                                base + 40 if p.n_in else None, n_in=p.n_in))
    return out


def bucket(cost):
    """1/16-octave class of a wave time (larger = longer)."""
    c = cost + 1
    msb = c.bit_length() - 1
    frac = (c >> (msb - 4)) & 15 if msb >= 4 else (c << (4 - msb)) & 15
    return msb * 16 + frac


def check_plan(qs, plan):
    seen = sorted(i for item in plan for i in item)
    assert seen == list(range(len(qs))), "every query exactly once"
    costs = []
    for item in plan:
        if len(item) > 1:
            assert 2 <= len(item) <= 16
            assert sum(qs[i].sys.n for i in item) <= 64
            lead = qs[item[0]]
            for i in item:
                q = qs[i]
                assert q.sys.kind in (R.REACH_CTM, R.REACH_RD) and q.sys.n <= 32
                assert (q.sys.kind, q.dt, tuple(q.sys.prm)) == \
                    (lead.sys.kind, lead.dt, tuple(lead.sys.prm))
                assert bucket(q.nsteps) == bucket(lead.nsteps), "step counts within 1/16 octave"
            costs.append(bucket(max(qs[i].nsteps for i in item)))
        else:
            q = qs[item[0]]
            costs.append(bucket(math.ceil(q.sys.n / 64) * q.nsteps))
    assert all(a >= b for a, b in zip(costs, costs[1:])), "longest item first"


@pytest.mark.parametrize("nq", [1, 7, 400, 20000])
def test_plan_covers_every_query_once_and_packs_validly(nq):
    qs = queries_of(workloads.query_stream(nq, 5.0e4, seed=4242 + nq))
    plan = R.reach_plan_batch(None, qs)
    check_plan(qs, plan)
    assert plan == R.reach_plan_batch(None, qs), "deterministic"


def test_short_queries_are_packed():
    qs = queries_of(workloads.query_stream(4000, 5.0e4, seed=99))
    plan = R.reach_plan_batch(None, qs)
    packs = [it for it in plan if len(it) > 1]
    short = sum(1 for q in qs if q.sys.n <= 32)
    in_packs = sum(len(it) for it in packs)
    assert packs and in_packs > 0.5 * short
    lanes = [sum(qs[i].sys.n for i in it) for it in packs]
    assert np.mean(lanes) > 32


def test_only_identical_constants_share_a_wave():
    p = workloads.small_problem(workloads.KIND_CTM, 10, 3, 50)
    qs = []
    for k in range(12):
        dt = 0.01 if k % 3 else 0.02          # two step sizes
        steps = 50 if k % 4 else 49           # two step counts, same 1/16 octave
        qs.append(R.make_query(p.kind, 10, p.prm, R.REACH_F64, FAKE, FAKE, FAKE, FAKE, dt, steps))
    lin = R.make_query(R.REACH_LIN3, 8, (0.1, -0.5, 0.2, 1.0), R.REACH_F64, FAKE, FAKE, FAKE,
                       FAKE, 0.01, 50)
    qs.append(lin)
    plan = R.reach_plan_batch(None, qs)
    check_plan(qs, plan)
    assert [len(it) for it in plan if 12 in it] == [1], "LIN3 runs alone"
    for it in plan:
        assert len({qs[i].dt for i in it}) == 1
    assert any(len({qs[i].nsteps for i in it}) == 2 for it in plan), "49 and 50 steps share packs"


def test_long_and_wide_queries_run_alone():
    qs = []
    for n in (33, 64, 65, 512):
        p = workloads.small_problem(workloads.KIND_RD, n, 5, 20)
        for _ in range(3):
            qs.append(R.make_query(p.kind, n, p.prm, R.REACH_F64, FAKE, FAKE, FAKE, FAKE, p.dt,
                                   20, FAKE, FAKE, n_in=1))
    plan = R.reach_plan_batch(None, qs)
    check_plan(qs, plan)
    assert all(len(it) == 1 for it in plan)


def test_plan_rejects_what_the_batch_rejects():
    p = workloads.small_problem(workloads.KIND_CTM, 600, 3, 10)
    bad = R.make_query(p.kind, 600, p.prm, R.REACH_F64, FAKE, FAKE, FAKE, FAKE, p.dt, 10)
    with pytest.raises(R.ReachError) as e:
        R.reach_plan_batch(None, [bad])
    assert e.value.status == R.REACH_E_UNSUPPORTED
    neg = R.make_query(p.kind, 20, p.prm, R.REACH_F64, FAKE, FAKE, FAKE, FAKE, -0.1, 10)
    with pytest.raises(R.ReachError) as e:
        R.reach_plan_batch(None, [neg])
    assert e.value.status == R.REACH_E_INVAL
    assert R.reach_plan_batch(None, []) == []


def test_large_plan_without_context_rejects_a_bad_query_deep_inside():
    """20000 queries are planned by several host threads (a pool of the
    call's own when there is no context); one bad query anywhere fails the
    whole plan with that query's status."""
    qs = queries_of(workloads.query_stream(20000, 5.0e4, seed=99))
    p = workloads.small_problem(workloads.KIND_CTM, 20, 3, 10)
    qs[15001] = R.make_query(p.kind, 20, p.prm, R.REACH_F64, FAKE, FAKE, FAKE, FAKE, -0.1, 10)
    with pytest.raises(R.ReachError) as e:
        R.reach_plan_batch(None, qs)
    assert e.value.status == R.REACH_E_INVAL
